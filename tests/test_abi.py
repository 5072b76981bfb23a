"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/sv.h declares, rejects bad arguments before touching a
device, and builds the same gate matrices as the oracle."""

import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for f in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not f.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", f)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"static inline[^{]*\{[^}]*\}", "", src)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z_0-9]*\s*\*?\s*(svb?_[a-z0-9_]+)\s*\(", src, re.M):
            names.append(m.group(1))
    return names


@pytest.fixture(scope="module")
def L():
    from paper_quant_ph_0201042_amd import _lib

    return _lib.load()


def test_every_declared_symbol_exported(L):
    from paper_quant_ph_0201042_amd import _lib

    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
        assert name in _lib.SIGNATURES, name


def test_strerror(L):
    for code in (0, -1, -2, -3, -4, -99):
        assert isinstance(L.sv_strerror(code), bytes)


def _fake_handle(L, n, dtype=16):
    h = ctypes.c_void_p()
    assert L.sv_wrap(n, dtype, ctypes.c_void_p(0x10000), None, ctypes.byref(h)) == 0
    return h


def test_validation_before_device(L):
    EINVAL = -1
    h = ctypes.c_void_p()
    assert L.sv_wrap(0, 16, ctypes.c_void_p(0x10000), None, ctypes.byref(h)) == EINVAL
    assert L.sv_wrap(37, 16, ctypes.c_void_p(0x10000), None, ctypes.byref(h)) == EINVAL
    assert L.sv_wrap(4, 12, ctypes.c_void_p(0x10000), None, ctypes.byref(h)) == EINVAL
    assert L.sv_wrap(4, 16, None, None, ctypes.byref(h)) == EINVAL
    assert L.sv_wrap(4, 16, ctypes.c_void_p(0x10008), None, ctypes.byref(h)) == EINVAL  # misaligned
    assert L.sv_create(0, 16, None, ctypes.byref(h)) == EINVAL
    h = _fake_handle(L, 5)
    U = np.array([1, 0, 0, 0, 0, 0, 1, 0], dtype=np.float64)
    Up = U.ctypes.data_as(ctypes.c_void_p)
    assert L.sv_apply_1q(h, -1, Up) == EINVAL
    assert L.sv_apply_1q(h, 5, Up) == EINVAL
    assert L.sv_apply_1q(h, 0, None) == EINVAL
    assert L.sv_apply_1q(None, 0, Up) == EINVAL
    bad = U.copy()
    bad[3] = np.nan
    assert L.sv_apply_1q(h, 0, bad.ctypes.data_as(ctypes.c_void_p)) == EINVAL
    bad[3] = np.inf
    assert L.sv_apply_ctrl(h, 1, 0, bad.ctypes.data_as(ctypes.c_void_p)) == EINVAL
    assert L.sv_apply_ctrl(h, 1 << 5, 0, Up) == EINVAL  # control bit >= n
    assert L.sv_apply_ctrl(h, 1 << 4, 0, Up) == EINVAL  # target inside the mask
    assert L.sv_apply_swap(h, 0, 5) == EINVAL
    out = ctypes.c_double()
    assert L.sv_prob(h, 1 << 5, 0, ctypes.byref(out)) == EINVAL
    assert L.sv_prob(h, 0b1, 0b10, ctypes.byref(out)) == EINVAL  # value outside mask
    assert L.sv_prob(h, 0, 0, None) == EINVAL
    assert L.sv_reset(h, 32) == EINVAL
    assert L.sv_qft(h, -1, 2, 0) == EINVAL
    assert L.sv_qft(h, 0, 0, 0) == EINVAL
    assert L.sv_qft(h, 2, 4, 0) == EINVAL  # q0 + m > n
    assert L.sv_qft(None, 0, 1, 0) == EINVAL
    idx = ctypes.c_uint64()
    assert L.sv_measure(h, -0.1, ctypes.byref(idx)) == EINVAL
    assert L.sv_measure(h, float("nan"), ctypes.byref(idx)) == EINVAL
    assert L.sv_measure(h, float("inf"), ctypes.byref(idx)) == EINVAL
    assert L.sv_measure(h, 0.5, None) == EINVAL
    assert L.sv_measure(None, 0.5, ctypes.byref(idx)) == EINVAL
    assert L.sv_collapse(h, 1 << 5, 0, None) == EINVAL  # mask bit >= n
    assert L.sv_collapse(h, 0b1, 0b10, None) == EINVAL  # value outside mask
    assert L.sv_collapse(None, 1, 1, None) == EINVAL
    qs = np.array([0, 0], dtype=np.int32)
    M4 = np.eye(4, dtype=np.complex128)
    assert L.sv_apply_fused(h, 2, qs.ctypes.data_as(ctypes.c_void_p), M4.ctypes.data_as(ctypes.c_void_p)) == EINVAL
    qs = np.array([0, 5], dtype=np.int32)
    assert L.sv_apply_fused(h, 2, qs.ctypes.data_as(ctypes.c_void_p), M4.ctypes.data_as(ctypes.c_void_p)) == EINVAL
    assert L.sv_apply_fused(h, 7, qs.ctypes.data_as(ctypes.c_void_p), M4.ctypes.data_as(ctypes.c_void_p)) == EINVAL
    h2 = _fake_handle(L, 6)
    o2 = np.zeros(2)
    assert L.sv_inner(h, h2, o2.ctypes.data_as(ctypes.c_void_p)) == EINVAL
    n_, d_ = ctypes.c_int(), ctypes.c_int()
    assert L.sv_info(h, ctypes.byref(n_), ctypes.byref(d_), None) == 0 and n_.value == 5 and d_.value == 16
    # gate lists are validated as a whole before any launch
    g = synth.GateList().add(synth.KIND_H, 0).add(synth.KIND_X, 1, ctrl=1 << 2).add(synth.KIND_H, 7).array()
    badi = ctypes.c_int64(-5)
    assert L.sv_run(h, g.ctypes.data_as(ctypes.c_void_p), len(g), 0, ctypes.byref(badi)) == EINVAL
    assert badi.value == 2
    g = synth.GateList().add(synth.KIND_SWAP, 0, target2=1, ctrl=1).array()
    assert L.sv_run(h, g.ctypes.data_as(ctypes.c_void_p), len(g), 0, ctypes.byref(badi)) == EINVAL
    g = synth.GateList().add(synth.KIND_RK, 0, iarg=63).array()
    assert L.sv_run(h, g.ctypes.data_as(ctypes.c_void_p), len(g), 0, ctypes.byref(badi)) == EINVAL
    g = synth.GateList().add(synth.KIND_SU2, 0, p=[0, 0, 0, 0]).array()
    assert L.sv_run(h, g.ctypes.data_as(ctypes.c_void_p), len(g), 0, ctypes.byref(badi)) == EINVAL
    assert L.sv_run(h, g.ctypes.data_as(ctypes.c_void_p), 1, 7, ctypes.byref(badi)) == EINVAL
    assert L.sv_destroy(h) == 0 and L.sv_destroy(h2) == 0 and L.sv_destroy(None) == 0


def test_library_gate_matrices_match_oracle(orc):
    """a9 on the host: the library's gate construction against the oracle's,
    for every kind, exact and perturbed."""
    from paper_quant_ph_0201042_amd import gate_matrix

    rng = np.random.default_rng(0)
    gl = synth.random_gate_mix(8, 400, seed=1)
    arr = gl.array()
    extra = synth.GateList()
    for k in range(0, 63):
        extra.add(synth.KIND_RK, 0, iarg=k, p=[0, rng.standard_normal() * 0.1 if k % 2 else 0.0])
    arr = np.concatenate([arr, extra.array()])
    for rec in arr:
        if rec["kind"] == synth.KIND_SWAP:
            continue
        lib_U = gate_matrix(rec)
        orc_U = orc.gate_matrix(int(rec["kind"]), int(rec["iarg"]), rec["p"])
        assert np.max(np.abs(lib_U - orc_U)) <= 1e-15, rec
        if (rec["p"][:2] == 0).all() and rec["kind"] in (synth.KIND_H, synth.KIND_X, synth.KIND_Z, synth.KIND_Y):
            assert np.array_equal(lib_U, orc_U)


def test_library_gate_derivatives_match_oracle(orc):
    from paper_quant_ph_0201042_amd import gate_dmatrix

    gl = synth.GateList()
    rng = np.random.default_rng(3)
    for kind in (synth.KIND_H, synth.KIND_X, synth.KIND_ROT, synth.KIND_Z, synth.KIND_RK):
        for _ in range(5):
            gl.add(kind, 0, iarg=int(rng.integers(1, 20)), p=list(rng.standard_normal(2) * 0.3))
    for rec in gl.array():
        for which in (0, 1):
            try:
                ref = orc.gate_dmatrix(int(rec["kind"]), int(rec["iarg"]), rec["p"], which)
            except ValueError:
                from paper_quant_ph_0201042_amd import SVError

                with pytest.raises(SVError):
                    gate_dmatrix(rec, which)
                continue
            assert np.max(np.abs(gate_dmatrix(rec, which) - ref)) <= 1e-15


def test_config_keys_bounds_and_defaults():
    import paper_quant_ph_0201042_amd as sv

    # every documented key, its default and its accepted range
    keys = {
        "fused_tile_bits_c128": (12, 1, 12),
        "fused_tile_bits_c64": (12, 1, 13),
        "fused_low_bits": (4, 1, 12),
        "fused_max_ops": (512, 1, 4096),
        "block_qubits": (5, 1, 6),
        "fused_jit": (1, 0, 1),
        "fused_pairs": (1, 0, 1),
        "swap_runs": (1, 0, 1),
        "perm_low_bits": (6, 1, 6),
        "perm_low_bits_c64": (5, 1, 6),
        "perm_workgroups": (16384, 1, 1 << 20),
        "fused_plan_search": (1, 0, 1),
        "fused_reg_bits": (4, 2, 4),
        "fused_jit_max_ops": (384, 1, 4096),
        "qft_fft": (1, 0, 1),
        "mfma_workgroups": (256, 1, 1 << 20),
        "fused_mfma": (0, 0, 1),
        "fused_rotations": (1, 0, 1),
        "gate_pairs_min_bit": (0, 0, 6),
        "gate_cached_low": (1, 0, 1),
        "batch_mfma": (1, 0, 1),
        "batch_waves": (4, 0, 8),
        "batch_const_bits": (1, 0, 1),
        "gate_spread_bits": (4, 0, 8),
    }
    for k, (default, lo, hi) in keys.items():
        assert sv.config_get(k) == default, k
        for bad in (lo - 1, hi + 1):
            with pytest.raises(sv.SVError):
                sv.config_set(k, bad)
        assert sv.config_get(k) == default, k
        sv.config_set(k, lo)
        assert sv.config_get(k) == lo
        sv.config_set(k, default)
    with pytest.raises(sv.SVError):
        sv.config_get("no_such_key")
    with pytest.raises(sv.SVError):
        sv.config_set("no_such_key", 1)
    # the header documents each key
    hdr = open(os.path.join(ROOT, "include", "sv.h")).read()
    for k in keys:
        assert '"%s"' % k in hdr, k


def test_shor_validation_before_device(L):
    EINVAL = -1
    h = _fake_handle(L, 8)
    c = ctypes.c_uint64()
    assert L.sv_shor_prepare(h, 1, 2, 0, ctypes.byref(c)) == EINVAL          # N < 2
    assert L.sv_shor_prepare(h, 1 << 32, 2, 0, ctypes.byref(c)) == EINVAL    # N >= 2^32
    assert L.sv_shor_prepare(h, 15, 7, 256, ctypes.byref(c)) == EINVAL       # a_star >= 2^n
    assert L.sv_shor_prepare(None, 15, 7, 0, ctypes.byref(c)) == EINVAL
    from paper_quant_ph_0201042_amd import shor

    res = shor.Result()
    V = ctypes.c_void_p
    x = np.array([5], dtype=np.uint64)
    a = np.array([0], dtype=np.uint64)
    u = np.array([0.5])
    args = (x.ctypes.data_as(V), a.ctypes.data_as(V), u.ctypes.data_as(V))
    assert L.sv_shor_factor(h, 21, *args, 1, 0, None, ctypes.byref(res)) == EINVAL   # 21 needs 10 qubits
    assert L.sv_shor_factor(h, 15, *args, 1, 2, None, ctypes.byref(res)) == EINVAL   # unknown flag
    assert L.sv_shor_factor(h, 15, *args, -1, 0, None, ctypes.byref(res)) == EINVAL
    # step 2 settles the run before any device work: gcd(5, 15) = 5
    ys = np.zeros(1, dtype=np.uint64)
    assert L.sv_shor_factor(h, 15, *args, 1, 0, ys.ctypes.data_as(V), ctypes.byref(res)) == 0
    assert (res.iterations, res.factor, res.stage) == (1, 5, shor.GCDX)
    assert ys[0] == np.uint64(2**64 - 1)
    x[0] = 0  # x outside [1, N-1]
    assert L.sv_shor_factor(h, 15, *args, 1, 0, None, ctypes.byref(res)) == EINVAL
    # a bad draw in a later run is rejected before the first run starts
    x2 = np.array([7, 0], dtype=np.uint64)
    a2 = np.array([1, 0], dtype=np.uint64)
    u2 = np.array([0.5, 0.5])
    args2 = (x2.ctypes.data_as(V), a2.ctypes.data_as(V), u2.ctypes.data_as(V))
    assert L.sv_shor_factor(h, 15, *args2, 2, 0, None, ctypes.byref(res)) == EINVAL
    u2[1] = 1.0
    x2[1] = 2
    assert L.sv_shor_factor(h, 15, *args2, 2, 0, None, ctypes.byref(res)) == EINVAL
    out = shor.Outcome()
    assert L.sv_shor_classical(15, 7, 256, 8, 0, 0, ctypes.byref(out)) == EINVAL    # y >= 2^m
    assert L.sv_shor_classical(15, 7, 0, 0, 0, 0, ctypes.byref(out)) == EINVAL      # m < 1
    assert L.sv_shor_classical(15, 7, 0, 63, 0, 0, ctypes.byref(out)) == EINVAL     # m > 62
    assert L.sv_shor_classical(1, 7, 0, 8, 0, 0, ctypes.byref(out)) == EINVAL
    assert L.sv_shor_classical(15, 7, 0, 8, 4, 0, ctypes.byref(out)) == EINVAL
    assert L.sv_shor_classical(15, 7, 0, 8, 0, 0, None) == EINVAL
    L.sv_destroy(h)


def test_batch_start_and_noise_validation(L):
    EINVAL = -1
    assert L.svb_set_start(None, 0) == EINVAL
    assert L.svb_set_noise_kinds(None, 1) == EINVAL


def test_qft_flags_validation(L):
    h = _fake_handle(L, 6)
    assert L.sv_qft(h, 0, 6, 4) == -1
    assert L.sv_qft(h, 0, 6, -1) == -1
    assert L.sv_qft(h, 1, 6, 0) == -1
    L.sv_destroy(h)


def test_missing_library_fails_loudly():
    """Without the built HIP library the binding raises instead of falling
    back to anything (there is no CPU path); the package loads it at import."""
    from paper_quant_ph_0201042_amd import _lib

    saved = (_lib._lib, _lib.LIB_PATH)
    try:
        _lib._lib = None
        _lib.LIB_PATH = os.path.join(ROOT, "no_such_dir", "libsv.so")
        with pytest.raises(ImportError, match="not built"):
            _lib.load()
    finally:
        _lib._lib, _lib.LIB_PATH = saved
    assert _lib.load() is saved[0]
