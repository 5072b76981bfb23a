"""GPU parity of the per-gate HIP path against the FP64 CPU oracle.

Every comparison runs both sides on the same seeded input.  Tolerances:
  - complex128: max_j |gpu_j - oracle_j| <= 1e-12 * max_j |oracle_j| (the
    normwise-in-max relative error; per-amplitude ratios are undefined near
    zero amplitudes);
  - complex64: one gate rounds U and each product/sum once in FP32 (unit
    roundoff 2^-24 ~ 6e-8); a 2-term complex dot product has at most ~8 such
    roundings, so 1e-6 * max|o| per gate, times the gate count for circuits;
  - permutation gates (X, CNOT, Toffoli, swaps) must match bit for bit.
"""

import math
import sys

import numpy as np
import pytest

import synth
from synth import KIND_H, KIND_RK, KIND_SU2, KIND_U, KIND_X

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-6}
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


def relerr(g, o):
    return float(np.max(np.abs(g.astype(np.complex128) - o)) / max(np.max(np.abs(o)), 1e-300))


def gpu_state(sv, amps, dtype):
    s = sv.State(int(np.log2(len(amps))), dtype)
    s.load(np.asarray(amps).astype(NPDT[dtype]))
    return s


def oracle_input(amps, dtype):
    """The oracle starts from exactly the values the GPU holds."""
    return np.asarray(amps).astype(NPDT[dtype]).astype(np.complex128)


def rand_U(rng):
    return np.array(synth.random_unitary_params(rng)).view(np.complex128).reshape(2, 2)


# ------------------------------------------------------------ a1


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_create_reset_load_store(sv, dtype):
    for n in (1, 5, 6, 7, 13):
        say("reset", dtype, n)
        s = sv.State(n, dtype).reset(0)
        e = np.zeros(1 << n)
        e[0] = 1
        assert np.array_equal(s.numpy(), e.astype(NPDT[dtype]))
        j = (1 << n) - 1
        s.reset(j)
        e = np.zeros(1 << n)
        e[j] = 1
        assert np.array_equal(s.numpy(), e.astype(NPDT[dtype]))
        a = synth.random_state(n, n).astype(NPDT[dtype])
        s.load(a)
        assert np.array_equal(s.numpy(), a)


# ------------------------------------------------------------ a2


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 6, 7, 9, 12, 20])
def test_apply_1q_every_target(sv, orc, dtype, n):
    rng = np.random.default_rng(1000 + n)
    a = synth.random_state(n, n)
    ao = oracle_input(a, dtype)
    s = gpu_state(sv, a, dtype)
    for q in range(n):
        for label, U in (("dense", rand_U(rng)), ("general", rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))),
                         ("diag", np.diag([np.exp(0.3j), np.exp(-1.1j)])), ("rk", orc.gate_matrix(KIND_RK, 5)),
                         ("z", np.diag([1.0, -1.0]))):
            say("1q", dtype, n, q, label)
            s.load(a.astype(NPDT[dtype]))
            s.apply_1q(q, U)
            ref = orc.apply_1q(ao, q, U.astype(NPDT[dtype]).astype(np.complex128) if dtype == "c64" else U)
            assert relerr(s.numpy(), ref) <= TOL[dtype] * (4 if label == "general" else 1), (q, label)
        say("1q", dtype, n, q, "x")
        s.load(a.astype(NPDT[dtype]))
        s.apply_1q(q, orc.gate_matrix(KIND_X))
        ref = orc.apply_1q(ao, q, orc.gate_matrix(KIND_X)).astype(NPDT[dtype])
        assert np.array_equal(s.numpy().view(np.uint8), ref.view(np.uint8))


# ------------------------------------------------------------ a3


def _random_mask(rng, n, q, nc):
    others = [k for k in range(n) if k != q]
    cq = rng.choice(others, size=min(nc, len(others)), replace=False)
    m = 0
    for c in cq:
        m |= 1 << (n - 1 - int(c))
    return m


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [2, 3, 7, 10, 14])
def test_apply_ctrl(sv, orc, dtype, n):
    rng = np.random.default_rng(2000 + n)
    a = synth.random_state(n, 100 + n)
    ao = oracle_input(a, dtype)
    s = gpu_state(sv, a, dtype)
    X = orc.gate_matrix(KIND_X)
    cases = []
    for q in range(n):
        for nc in sorted({1, 2, n - 1}):
            if nc <= n - 1:
                cases.append((q, _random_mask(rng, n, q, nc)))
    # controls right next to a low target and a high target
    if n >= 3:
        cases += [(n - 1, 0b10), (n - 2, 0b1), (0, 1), (0, 1 << (n - 2))]
    for q, m in cases:
        for label, U in (("dense", rand_U(rng)), ("rk", orc.gate_matrix(KIND_RK, 3)), ("z", np.diag([1.0, -1.0]))):
            say("ctrl", dtype, n, q, hex(m), label)
            s.load(a.astype(NPDT[dtype]))
            s.apply_ctrl(m, q, U)
            ref = orc.apply_ctrl(ao, m, q, U.astype(NPDT[dtype]).astype(np.complex128) if dtype == "c64" else U)
            assert relerr(s.numpy(), ref) <= TOL[dtype], (q, m, label)
        say("ctrl", dtype, n, q, hex(m), "x")
        s.load(a.astype(NPDT[dtype]))
        s.apply_ctrl(m, q, X)
        ref = orc.apply_ctrl(ao, m, q, X).astype(NPDT[dtype])
        assert np.array_equal(s.numpy().view(np.uint8), ref.view(np.uint8)), (q, m)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_ctrl_spread_order(sv, orc, dtype):
    # controls (and a diagonal gate's fixed target) at byte address bits
    # 10..12 and 20..21 run with the spread block order (gate_spread_bits,
    # default 4): the same results as the plain order, bit for bit, and the
    # oracle's
    n = 20
    sh = 4 if dtype == "c128" else 3
    win = [b for b in range(n) if 10 <= b + sh <= 12 or 20 <= b + sh <= 21]
    rng = np.random.default_rng(7)
    a = synth.random_state(n, 31)
    ao = oracle_input(a, dtype)
    s = gpu_state(sv, a, dtype)
    X = orc.gate_matrix(KIND_X)
    cases = []
    for cb in win:
        # target index bit tb (qubit n - 1 - tb), control mask in index bits
        for tb in (0, 3, cb - 1, cb + 1, 12, n - 1):
            if tb != cb:
                cases.append((n - 1 - tb, 1 << cb))
        cases.append((n - 1 - 15, (1 << cb) | (1 << 2)))
        if cb + 1 < n - 1:
            cases.append((n - 1 - (cb + 1), (1 << cb) | (1 << (n - 1))))
    old = sv.config_get("gate_spread_bits")
    try:
        for q, m in cases:
            for label, U in (("dense", rand_U(rng)), ("rk", orc.gate_matrix(KIND_RK, 2)), ("x", X)):
                say("spread", dtype, q, hex(m), label)
                out = []
                for k in (4, 0):
                    sv.config_set("gate_spread_bits", k)
                    s.load(a.astype(NPDT[dtype]))
                    s.apply_ctrl(m, q, U)
                    out.append(s.numpy())
                assert np.array_equal(out[0].view(np.uint8), out[1].view(np.uint8)), (q, m, label)
                ref = orc.apply_ctrl(ao, m, q, U.astype(NPDT[dtype]).astype(np.complex128) if dtype == "c64" else U)
                if label == "x":
                    assert np.array_equal(out[0].view(np.uint8), ref.astype(NPDT[dtype]).view(np.uint8)), (q, m)
                else:
                    assert relerr(out[0], ref) <= TOL[dtype], (q, m, label)
    finally:
        sv.config_set("gate_spread_bits", old)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_swap_all_pairs_bit_exact(sv, orc, dtype):
    for n in (2, 7, 11):
        a = synth.random_state(n, 300 + n)
        ao = oracle_input(a, dtype)
        s = gpu_state(sv, a, dtype)
        for q1 in range(n):
            for q2 in range(n):
                say("swap", dtype, n, q1, q2)
                s.load(a.astype(NPDT[dtype]))
                s.swap(q1, q2)
                ref = orc.swap(ao, q1, q2).astype(NPDT[dtype])
                assert np.array_equal(s.numpy().view(np.uint8), ref.view(np.uint8))


# ------------------------------------------------------------ a6


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_prob_and_inner(sv, orc, dtype):
    rng = np.random.default_rng(7)
    for n in (1, 4, 9, 13, 21):
        a = synth.random_state(n, 400 + n)
        b = synth.random_state(n, 500 + n)
        ao, bo = oracle_input(a, dtype), oracle_input(b, dtype)
        sa, sb = gpu_state(sv, a, dtype), gpu_state(sv, b, dtype)
        masks = [(0, 0), ((1 << n) - 1, int(rng.integers(0, 1 << n)))]
        for _ in range(6):
            m = int(rng.integers(0, 1 << n))
            v = int(rng.integers(0, 1 << n)) & m
            masks.append((m, v))
        for m, v in masks:
            say("prob", dtype, n, hex(m), hex(v))
            ref = orc.prob(ao, m, v)
            got = sa.prob(m, v)
            assert abs(got - ref) <= 1e-13 * max(1.0, ref) + 1e-300
            assert sa.prob(m, v) == got  # bitwise reproducible
        say("inner", dtype, n)
        ref = orc.inner(ao, bo)
        got = sa.inner(sb)
        assert abs(got - ref) <= 1e-13
        assert sa.inner(sb) == got


def test_inner_mixed_dtype(sv, orc):
    n = 12
    a = synth.random_state(n, 1)
    b = synth.random_state(n, 2)
    s64 = gpu_state(sv, a, "c64")
    s128 = gpu_state(sv, b, "c128")
    ref = orc.inner(oracle_input(a, "c64"), b)
    assert abs(s64.inner(s128) - ref) <= 1e-13
    assert abs(s128.inner(s64) - np.conj(ref)) <= 1e-13


# ------------------------------------------------------------ circuits


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [3, 8, 13])
def test_random_gate_mix(sv, orc, dtype, n):
    gl = synth.random_gate_mix(n, 150, seed=n)
    g = gl.array()
    a = synth.random_state(n, 600 + n)
    say("mix", dtype, n)
    s = gpu_state(sv, a, dtype)
    s.run(g)
    ref = orc.run(oracle_input(a, dtype), g)
    tol = 1e-12 if dtype == "c128" else 150 * 1e-6
    assert relerr(s.numpy(), ref) <= tol


@pytest.mark.parametrize("seed", list(range(16)) + ["first", "last"])
def test_grover_n14(sv, orc, seed):
    """Grover search, n=14, complex128, 100 iterations; final probability of
    the marked index against sin^2(201 asin 2^-7) and the oracle state."""
    n = 14
    marked = 0 if seed == "first" else ((1 << n) - 1 if seed == "last" else synth.grover_marked(n, seed))
    g = synth.grover_circuit(n, marked, synth.grover_iterations(n)).array()
    say("grover14", seed, marked)
    s = sv.State(n, "c128").reset(0)
    s.run(g)
    p = s.prob((1 << n) - 1, marked)
    assert abs(p - math.sin(201 * math.asin(2**-7)) ** 2) <= 1e-12
    ref = orc.run(orc.zero_state(n), g)
    assert relerr(s.numpy(), ref) <= 1e-12


@pytest.mark.parametrize("n", [1, 2, 6, 12, 16])
def test_qft_small_vs_oracle(sv, orc, n):
    a = synth.random_state(n, 700 + n)
    g = synth.qft_circuit(n).array()
    say("qft", n)
    s = gpu_state(sv, a, "c128")
    s.run(g)
    ref = orc.run(a, g)
    assert relerr(s.numpy(), ref) <= 1e-12


def test_qft_n28_sampled(sv, orc):
    """QFT circuit at n=28, complex128, on a seeded Gaussian state: sampled
    outputs against the oracle's direct DFT elements, and the norm."""
    import torch

    n = 28
    say("qft28 input")
    a = synth.random_state(n, 0)
    s = gpu_state(sv, a, "c128")
    g = synth.qft_circuit(n).array()
    say("qft28 run")
    s.run(g)
    assert abs(s.norm2() - 1.0) <= 1e-12
    rng = np.random.default_rng(28)
    xs = [0, 1, (1 << n) - 1] + [int(x) for x in rng.integers(0, 1 << n, 5)]
    got = s.tensor[torch.tensor(xs, device=s.tensor.device)].cpu().numpy()
    # the output is again a unit Gaussian-like state: max_j |beta_j| is about
    # sqrt(2 ln 2^n) 2^{-n/2}, the scale the 1e-12 normwise-in-max bound uses
    max_o = math.sqrt(2 * math.log(2.0**n)) * 2.0 ** (-n / 2)
    for x, gx in zip(xs, got):
        say("qft28 sample", x)
        ref = orc.dft_element(a, x)
        assert abs(gx - ref) <= 1e-12 * max_o, (x, gx, ref)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_brickwork_small_vs_oracle(sv, orc, dtype):
    n, depth = 12, 20
    g = synth.brickwork_circuit(n, depth, seed=0).array()
    say("brick", dtype)
    s = sv.State(n, dtype).reset(0)
    s.run(g)
    ref = orc.run(orc.zero_state(n), g)
    tol = 1e-12 if dtype == "c128" else len(g) * 1e-6
    assert relerr(s.numpy(), ref) <= tol
