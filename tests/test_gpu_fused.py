"""GPU parity of the fused-pass path (SV_RUN_FUSED) against the CPU oracle,
under several tile shapes so that plans have many passes, ragged small
registers (tile wider than the register) and every gate kind."""

import math
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

NPDT = {"c128": np.complex128, "c64": np.complex64}


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def sv():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_quant_ph_0201042_amd as sv

    return sv


@pytest.fixture
def tiles(sv):
    keys = ["fused_tile_bits_c128", "fused_tile_bits_c64", "fused_low_bits"]
    old = {k: sv.config_get(k) for k in keys}

    def setter(k128, k64, low):
        sv.config_set("fused_tile_bits_c128", k128)
        sv.config_set("fused_tile_bits_c64", k64)
        sv.config_set("fused_low_bits", low)

    yield setter
    for k, v in old.items():
        sv.config_set(k, v)


def relerr(g, o):
    return float(np.max(np.abs(g.astype(np.complex128) - o)) / max(np.max(np.abs(o)), 1e-300))


def run_both(sv, orc, n, dtype, g, a=None):
    if a is None:
        a = synth.random_state(n, 1000 + n)
    s = sv.State(n, dtype).load(a.astype(NPDT[dtype]))
    s.run(g, fused=True)
    ref = orc.run(a.astype(NPDT[dtype]).astype(np.complex128), g)
    return s, s.numpy(), ref


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("shape", [(12, 13, 6), (8, 8, 4), (5, 5, 2), (10, 11, 8)])
@pytest.mark.parametrize("n", [1, 3, 7, 12, 17])
def test_fused_random_mix(sv, orc, tiles, dtype, shape, n):
    tiles(*shape)
    g = synth.random_gate_mix(n, 200, seed=7 * n + shape[0], max_ctrl=3).array()
    say("fused mix", dtype, shape, n)
    _, got, ref = run_both(sv, orc, n, dtype, g)
    tol = 1e-12 if dtype == "c128" else 200 * 1e-6
    assert relerr(got, ref) <= tol


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_fused_many_controls(sv, orc, tiles, dtype):
    tiles(9, 9, 5)
    n = 14
    g = synth.random_gate_mix(n, 200, seed=3, max_ctrl=13).array()
    say("fused ctrl", dtype)
    _, got, ref = run_both(sv, orc, n, dtype, g)
    assert relerr(got, ref) <= (1e-12 if dtype == "c128" else 2e-4)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_fused_permutations_bit_exact(sv, orc, tiles, dtype):
    """X, CNOT, Toffoli and swaps only: the fused path must move amplitudes
    without arithmetic."""
    tiles(8, 8, 3)
    n = 13
    rng = np.random.default_rng(4)
    gl = synth.GateList()
    for _ in range(300):
        t = int(rng.integers(0, n))
        r = rng.random()
        if r < 0.15:
            t2 = int(rng.integers(0, n))
            if t2 != t:
                gl.add(synth.KIND_SWAP, t, target2=t2)
            continue
        others = [q for q in range(n) if q != t]
        nc = 0 if r < 0.4 else (1 if r < 0.75 else 2)
        ctrl = 0
        for c in rng.choice(others, size=nc, replace=False):
            ctrl |= 1 << (n - 1 - int(c))
        gl.add(synth.KIND_X, t, ctrl=ctrl)
    g = gl.array()
    say("fused perm", dtype)
    _, got, ref = run_both(sv, orc, n, dtype, g)
    assert np.array_equal(got.view(np.uint8), ref.astype(NPDT[dtype]).view(np.uint8))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_fused_brickwork_n20(sv, orc, dtype):
    n = 20
    g = synth.brickwork_circuit(n, 20, seed=0).array()
    say("fused brick20", dtype)
    s = sv.State(n, dtype).reset(0)
    s.run(g, fused=True)
    ref = orc.run(orc.zero_state(n), g)
    assert relerr(s.numpy(), ref) <= (1e-12 if dtype == "c128" else 1e-4)


def test_fused_qft_n16_and_grover(sv, orc):
    n = 16
    a = synth.random_state(n, 16)
    g = synth.qft_circuit(n).array()
    say("fused qft16")
    s = sv.State(n, "c128").load(a)
    s.run(g, fused=True)
    assert relerr(s.numpy(), orc.run(a, g)) <= 1e-12
    n = 14
    for seed in (0, 1, "last"):
        marked = (1 << n) - 1 if seed == "last" else synth.grover_marked(n, seed)
        g = synth.grover_circuit(n, marked, 100).array()
        say("fused grover14", seed)
        s = sv.State(n, "c128").reset(0)
        s.run(g, fused=True)
        assert abs(s.prob((1 << n) - 1, marked) - math.sin(201 * math.asin(2**-7)) ** 2) <= 1e-12
        assert relerr(s.numpy(), orc.run(orc.zero_state(n), g)) <= 1e-12


def test_fused_qft_n28_sampled(sv, orc):
    import torch

    n = 28
    say("fused qft28 input")
    a = synth.random_state(n, 0)
    s = sv.State(n, "c128").load(a)
    say("fused qft28 run")
    s.run(synth.qft_circuit(n).array(), fused=True)
    assert abs(s.norm2() - 1.0) <= 1e-12
    rng = np.random.default_rng(29)
    xs = [0, (1 << n) - 1] + [int(x) for x in rng.integers(0, 1 << n, 4)]
    got = s.tensor[torch.tensor(xs, device=s.tensor.device)].cpu().numpy()
    max_o = math.sqrt(2 * math.log(2.0**n)) * 2.0 ** (-n / 2)
    for x, gx in zip(xs, got):
        say("fused qft28 sample", x)
        assert abs(gx - orc.dft_element(a, x)) <= 1e-12 * max_o


def test_profile_records_steps(sv):
    n = 16
    g = synth.brickwork_circuit(n, 4, seed=2).array()
    s = sv.State(n, "c128").reset(0)
    s.run(g, fused=True, profile=True)
    ms, kind = s.run_profile()
    order, pass_of, masks = sv.plan_fused(n, "c128", g)
    assert len(ms) == len(masks) and (kind == 0).all() and (ms > 0).all()
    s.run(g, profile=True)
    ms, kind = s.run_profile()
    assert len(ms) == len(g) and (kind == 2).all()


@pytest.fixture
def engine(sv):
    keys = ["fused_jit", "fused_pairs"]
    old = {k: sv.config_get(k) for k in keys}

    def setter(jit, pairs):
        sv.config_set("fused_jit", jit)
        sv.config_set("fused_pairs", pairs)

    yield setter
    for k, v in old.items():
        sv.config_set(k, v)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("case", ["brickwork", "qft", "mix", "grover"])
def test_pass_engines_agree_with_oracle(sv, orc, engine, dtype, case):
    # the generic pass kernel, the specialised kernels, and the specialised
    # kernels with composed register-slot runs all match the oracle
    n = 13
    g = {
        "brickwork": lambda: synth.brickwork_circuit(n, 10, seed=8).array(),
        "qft": lambda: synth.qft_circuit(n).array(),
        "mix": lambda: synth.random_gate_mix(n, 300, seed=12, max_ctrl=4).array(),
        "grover": lambda: synth.grover_circuit(n, 4321, 2).array(),
    }[case]()
    tol = 1e-12 if dtype == "c128" else 1e-6 * len(g)
    for jit, pairs in [(0, 0), (1, 0), (1, 1)]:
        engine(jit, pairs)
        say("engine", case, dtype, "jit", jit, "pairs", pairs)
        _, got, ref = run_both(sv, orc, n, dtype, g)
        assert relerr(got, ref) < tol, (case, dtype, jit, pairs)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("cap", [1, 40, 100])
def test_long_passes_fall_back_to_generic_kernel(sv, orc, engine, dtype, cap):
    # passes longer than fused_jit_max_ops run on the generic kernel, the
    # others specialised (with composed runs): mixed in one run, same result
    old = sv.config_get("fused_jit_max_ops")
    engine(1, 1)
    n = 13
    g = synth.random_gate_mix(n, 400, seed=31, max_ctrl=3).array()
    tol = 1e-12 if dtype == "c128" else 1e-6 * len(g)
    try:
        sv.config_set("fused_jit_max_ops", cap)
        say("jit cap", cap, dtype)
        _, got, ref = run_both(sv, orc, n, dtype, g)
        assert relerr(got, ref) < tol
        b = sv.Batch(8, 4, dtype)
        init = synth.hadamard_transform(8).array()
        it = synth.grover_iteration(8, 77).array()
        prob, _ = b.run_noisy(init, it, 5, 0.02, 0.01, 3, target=77)
        ref_b = [orc.noisy_grover_traj(8, 77, 5, 0.02, 0.01, 3, r, init, it) for r in range(4)]
        assert np.max(np.abs(prob - ref_b)) < (1e-11 if dtype == "c128" else 5e-5)
    finally:
        sv.config_set("fused_jit_max_ops", old)


def test_permutation_circuit_bit_exact_with_pairs(sv, orc, engine):
    # X, CNOT, Toffoli and swaps only: never composed, so bit for bit
    engine(1, 1)
    n = 12
    gl = synth.GateList()
    rng = np.random.default_rng(3)
    for _ in range(200):
        q = int(rng.integers(0, n))
        others = [x for x in range(n) if x != q]
        nc = int(rng.integers(0, 3))
        ctrl = 0
        for c in rng.choice(others, nc, replace=False):
            ctrl |= synth.qubit_bit(n, int(c))
        gl.add(synth.KIND_X, q, ctrl=ctrl)
    g = gl.array()
    for dtype in ("c128", "c64"):
        _, got, ref = run_both(sv, orc, n, dtype, g)
        assert np.array_equal(got.astype(np.complex128), ref)


@pytest.fixture
def swap_runs(sv):
    old = sv.config_get("swap_runs")
    yield lambda v: sv.config_set("swap_runs", v)
    sv.config_set("swap_runs", old)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [2, 3, 7, 12, 17])
def test_swap_runs_bit_exact(sv, orc, swap_runs, dtype, n):
    # runs of swaps: disjoint ones (an involution: one bit-permutation pass),
    # the QFT bit reversal, and a 3-cycle (not an involution: one kernel per
    # swap), each between dense gates so that they form separate runs
    rng = np.random.default_rng(n)
    gl = synth.GateList()
    gl.add(synth.KIND_SU2, 0, p=list(rng.standard_normal(4)))
    perm = rng.permutation(n)
    for i in range(n // 2):
        gl.add(synth.KIND_SWAP, int(perm[2 * i]), target2=int(perm[2 * i + 1]))
    gl.add(synth.KIND_SU2, n - 1, p=list(rng.standard_normal(4)))
    for q in range(n // 2):
        gl.add(synth.KIND_SWAP, q, target2=n - 1 - q)
    if n >= 3:
        gl.add(synth.KIND_SU2, 1, p=list(rng.standard_normal(4)))
        gl.add(synth.KIND_SWAP, 0, target2=1)
        gl.add(synth.KIND_SWAP, 1, target2=2)
    g = gl.array()
    a = synth.random_state(n, 77)
    outs = []
    for runs in (1, 0):
        swap_runs(runs)
        say("swap runs", dtype, n, runs)
        _, got, ref = run_both(sv, orc, n, dtype, g, a)
        tol = 1e-12 if dtype == "c128" else 1e-5
        assert relerr(got, ref) < tol
        outs.append(got)
    # the permutation pass and the per-swap kernels move the same values
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_bit_reversal_full_size(sv, swap_runs, dtype):
    # |j> under the QFT's final swaps becomes |reverse(j)>
    n = 30
    swap_runs(1)
    gl = synth.GateList()
    for q in range(n // 2):
        gl.add(synth.KIND_SWAP, q, target2=n - 1 - q)
    g = gl.array()
    s = sv.State(n, dtype)
    for j in [1, 0b1011, (1 << 29) | 6, 0x2AAAAAAA]:
        rev = int(format(j, "030b")[::-1], 2)
        s.reset(j)
        say("bit reversal", dtype, hex(j))
        s.run(g, fused=True)
        assert s.prob((1 << n) - 1, rev) == 1.0


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("low", [1, 3, 5, 6])
@pytest.mark.parametrize("n", [7, 12, 17])
def test_permutation_pass_tile_widths(sv, orc, swap_runs, dtype, low, n):
    # the bit-permutation pass with contiguous runs of 2^low amplitudes
    # (tiles up to 2^12 amplitudes: one tile in LDS, one in registers) moves the
    # same values as one kernel per swap
    key = "perm_low_bits" if dtype == "c128" else "perm_low_bits_c64"
    old = sv.config_get(key)
    rng = np.random.default_rng(100 + n + low)
    gl = synth.GateList()
    perm = rng.permutation(n)
    for i in range(n // 2):
        gl.add(synth.KIND_SWAP, int(perm[2 * i]), target2=int(perm[2 * i + 1]))
    gl.add(synth.KIND_SU2, 0, p=list(rng.standard_normal(4)))
    for q in range(n // 2):
        gl.add(synth.KIND_SWAP, q, target2=n - 1 - q)
    g = gl.array()
    a = synth.random_state(n, 5)
    try:
        sv.config_set(key, low)
        swap_runs(1)
        say("perm tile", dtype, n, low)
        _, got, ref = run_both(sv, orc, n, dtype, g, a)
        swap_runs(0)
        _, got0, _ = run_both(sv, orc, n, dtype, g, a)
    finally:
        sv.config_set(key, old)
    assert np.array_equal(got, got0)
    tol = 1e-12 if dtype == "c128" else 1e-5
    assert relerr(got, ref) < tol
