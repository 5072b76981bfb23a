"""Host-side checks of the specialised pass kernels (no GPU): every pass of a
few circuit families generates source that hipRTC compiles for gfx950, with
the descriptor layout the library uses, and without packed FP32."""

import ctypes
import os
import subprocess

import numpy as np
import pytest

import synth

HIPRTC = "/opt/rocm/lib/libhiprtc.so"
OBJDUMP = "/opt/rocm/llvm/bin/llvm-objdump"


@pytest.fixture(scope="module")
def sv():
    import paper_quant_ph_0201042_amd as sv

    return sv


@pytest.fixture(scope="module")
def rtc():
    if not os.path.exists(HIPRTC):
        pytest.skip("hipRTC not installed")
    return ctypes.CDLL(HIPRTC)


def compile_src(rtc, src):
    prog = ctypes.c_void_p()
    assert rtc.hiprtcCreateProgram(ctypes.byref(prog), src.encode(), b"p.hip", 0, None, None) == 0
    opts = [b"--offload-arch=gfx950", b"-O3", b"-Xclang", b"-target-feature", b"-Xclang", b"-packed-fp32-ops"]
    arr = (ctypes.c_char_p * len(opts))(*opts)
    rc = rtc.hiprtcCompileProgram(prog, len(opts), arr)
    n = ctypes.c_size_t()
    rtc.hiprtcGetProgramLogSize(prog, ctypes.byref(n))
    log = ctypes.create_string_buffer(max(n.value, 1))
    rtc.hiprtcGetProgramLog(prog, log)
    code = b""
    if rc == 0:
        rtc.hiprtcGetCodeSize(prog, ctypes.byref(n))
        buf = ctypes.create_string_buffer(n.value)
        rtc.hiprtcGetCode(prog, buf)
        code = buf.raw
    rtc.hiprtcDestroyProgram(ctypes.byref(prog))
    return rc, log.value.decode(errors="replace"), code


CASES = [
    ("brickwork_c128", 14, "c128", lambda: synth.brickwork_circuit(14, 6, seed=3).array()),
    ("qft_c64", 14, "c64", lambda: synth.qft_circuit(14).array()),
    ("grover_c128", 13, "c128", lambda: synth.grover_circuit(13, 77, 1).array()),
    ("mix_c64", 9, "c64", lambda: synth.random_gate_mix(9, 60, seed=4).array()),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
def test_every_pass_compiles(sv, rtc, case, tmp_path):
    name, n, dtype, make = case
    g = make()
    _, _, masks = sv.plan_fused(n, dtype, g)
    srcs = {sv.jit_source(n, dtype, g, p) for p in range(len(masks))}
    for src in sorted(srcs)[:4]:
        rc, log, code = compile_src(rtc, src)
        assert rc == 0, log
        if os.path.exists(OBJDUMP):
            f = tmp_path / "pass.co"
            f.write_bytes(code)
            dis = subprocess.run([OBJDUMP, "-d", str(f)], capture_output=True, text=True).stdout
            assert "v_pk_fma_f32" not in dis and "v_pk_mul_f32" not in dis and "v_pk_add_f32" not in dis


def test_source_is_specialised(sv):
    # a pass of a brickwork circuit: straight-line code, one block per op,
    # no run-time op dispatch
    g = synth.brickwork_circuit(12, 2, seed=1).array()
    src = sv.jit_source(12, "c128", g, 0)
    assert "sv_pass" in src and "switch" not in src
    assert src.count("// op ") >= 10


def test_source_rejects_bad_pass(sv):
    g = synth.qft_circuit(6).array()
    _, _, masks = sv.plan_fused(6, "c128", g)
    with pytest.raises(sv.SVError):
        sv.jit_source(6, "c128", g, len(masks))


@pytest.mark.parametrize("reg_bits", [2, 3])
def test_other_register_bits_compile(sv, rtc, reg_bits):
    old = sv.config_get("fused_reg_bits")
    sv.config_set("fused_reg_bits", reg_bits)
    try:
        g = synth.brickwork_circuit(14, 6, seed=3).array()
        src = sv.jit_source(14, "c128", g, 0)
        assert "__launch_bounds__(%d)" % (1 << (12 - reg_bits)) in src
        rc, log, _ = compile_src(rtc, src)
        assert rc == 0, log
    finally:
        sv.config_set("fused_reg_bits", old)
