"""GPU parity of measurement (sv_measure: the sampling rule of sec. 2.2.3)
and of projective collapse onto an outcome of a subset of qubits
(sv_collapse) against the CPU oracle.

sv_measure is an index decision taken in FP64 on both sides from the same
amplitudes; the GPU sums chunks in a tree where the oracle sums in index
order, so draws r within 1e-9 (relative to the total) of a cumulative
boundary are skipped and every other draw must give the same index.
Collapse: complex128 to 1e-12 of the largest amplitude; complex64 rounds the
scale to FP32 and one product, so 1e-6.
"""

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


def load(sv, amps, dtype):
    s = sv.State(int(np.log2(len(amps))), dtype)
    s.load(np.asarray(amps).astype(NPDT[dtype]))
    return s


def draws_away_from_boundaries(w, count, seed):
    cum = np.cumsum(w)
    tot = cum[-1]
    rng = np.random.default_rng(seed)
    out = []
    for r in rng.random(4 * count) * tot:
        k = np.searchsorted(cum, r)
        near = min(abs(cum[max(k - 1, 0)] - r), abs(cum[min(k, len(cum) - 1)] - r))
        if near > 1e-9 * tot:
            out.append(float(r))
        if len(out) == count:
            break
    return out


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 5, 12, 13, 17, 20])
def test_measure_matches_oracle(sv, orc, dtype, n):
    psi = synth.random_state(n, seed=n).astype(NPDT[dtype])
    ref = psi.astype(np.complex128)
    s = load(sv, psi, dtype)
    w = np.abs(ref) ** 2
    say("measure", dtype, n)
    for r in draws_away_from_boundaries(w, 60, seed=n):
        assert s.measure(r) == orc.measure(ref, r), (n, r)
    # the register is not modified
    assert np.array_equal(s.numpy(), psi)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_measure_edges(sv, orc, dtype):
    n = 14
    N = 1 << n
    # sparse weights in far-apart chunks, with all-zero chunks between
    psi = np.zeros(N, dtype=np.complex128)
    for i, amp in [(3, 0.5), (4099, 0.5j), (9000, -0.5), (N - 2, 0.5)]:
        psi[i] = amp
    s = load(sv, psi, dtype)
    ref = psi.astype(NPDT[dtype]).astype(np.complex128)
    for r in [0.0, 0.1, 0.25 - 1e-6, 0.3, 0.6, 0.74, 0.9999, 1.0, 5.0]:
        assert s.measure(r) == orc.measure(ref, r), r
    assert s.measure(1.0) == N - 2  # beyond the total: last nonzero weight
    # a basis state is measured with certainty
    s.reset(12345)
    for r in [0.0, 0.5, 0.999999, 1.0]:
        assert s.measure(r) == 12345
    # an all-zero register gives index 0
    s.load(np.zeros(N, dtype=NPDT[dtype]))
    assert s.measure(0.3) == 0


@pytest.mark.parametrize("dtype,n", [("c64", 30), ("c128", 30), ("c64", 32)])
def test_measure_full_size(sv, dtype, n):
    # H on qubits 0, 9, 19, n-1 of |0...0>: weight 1/16 on each of the 16
    # patterns of those bits; draw (k + 1/2)/16 picks the k-th pattern in
    # increasing index order
    qs = [0, 9, 19, n - 1]
    s = sv.State(n, dtype).reset(0)
    h = np.array([[1, 1], [1, -1]]) / np.sqrt(2)
    for q in qs:
        s.apply_1q(q, h)
    bits = sorted(n - 1 - q for q in qs)
    pats = sorted(sum(((k >> i) & 1) << b for i, b in enumerate(bits)) for k in range(16))
    say("measure full size", dtype, n)
    for k in [0, 1, 7, 8, 15]:
        assert s.measure((k + 0.5) / 16) == pats[k]
    # measuring qubit 9 alone: outcome 1 with probability 1/2, then certain
    m9 = 1 << (n - 1 - 9)
    v, p = s.measure_qubits(m9, 0.8)  # pattern 12 = 0b1100: qubit 9 is 1
    assert v == m9 and abs(p - 0.5) < 1e-6
    assert abs(s.prob(m9, m9) - 1.0) < 1e-6 and abs(s.norm2() - 1.0) < 1e-6


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [3, 11, 16])
def test_collapse_matches_oracle(sv, orc, dtype, n):
    psi = synth.random_state(n, seed=100 + n).astype(NPDT[dtype])
    ref = psi.astype(np.complex128)
    rng = np.random.default_rng(n)
    tol = 1e-12 if dtype == "c128" else 1e-6
    for _ in range(4):
        mask = int(rng.integers(1, 1 << n))
        value = int(rng.integers(0, 1 << n)) & mask
        s = load(sv, psi, dtype)
        say("collapse", dtype, n, hex(mask), hex(value))
        p = s.collapse(mask, value)
        want, pw = orc.collapse(ref, mask, value)
        assert abs(p - pw) <= 1e-13 * max(pw, 1e-300) + 1e-15
        got = s.numpy().astype(np.complex128)
        assert np.max(np.abs(got - want)) <= tol * np.max(np.abs(want))
        # off-outcome amplitudes are exactly zero
        idx = np.arange(1 << n)
        assert np.all(got[(idx & mask) != value] == 0)


def test_collapse_impossible_outcome(sv):
    n = 6
    s = sv.State(n, "c128").reset(5)
    before = s.numpy()
    with pytest.raises(sv.SVError):
        s.collapse(0b111, 0b001)
    assert np.array_equal(s.numpy(), before)


def test_measure_then_reset_is_sec_2_2_3(sv, orc):
    # the full measurement: index from the sampling rule, then the register
    # is that basis state
    n = 10
    psi = synth.random_state(n, seed=3)
    s = load(sv, psi, "c128")
    i = s.measure(0.4321)
    assert i == orc.measure(psi, 0.4321)
    s.reset(i)
    assert s.prob((1 << n) - 1, i) == 1.0
