"""GPU parity of sv_qft (the QFT of sec. 2.3.2 on a qubit range, and its
inverse) against the CPU oracle running the same gate list, and against the
definition beta_y = 2^{-m/2} sum_x e^{+2 pi i x y / 2^m} alpha_x along the
sub-register axis (the oracle's QFT is pinned to it).  Tolerances as for the
fused path: 1e-12 (complex128), 1e-6 per gate (complex64)."""

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


def qft_gates(n, q0, m, inverse):
    g = synth.GateList()
    bit = lambda q: synth.qubit_bit(n, q)
    if not inverse:
        for i in range(m):
            g.add(synth.KIND_H, q0 + i)
            for c in range(i + 1, m):
                g.add(synth.KIND_RK, q0 + i, ctrl=bit(q0 + c), iarg=c - i + 1)
        for i in range(m // 2):
            g.add(synth.KIND_SWAP, q0 + i, target2=q0 + m - 1 - i)
    else:
        for i in range(m // 2):
            g.add(synth.KIND_SWAP, q0 + i, target2=q0 + m - 1 - i)
        for i in reversed(range(m)):
            for c in reversed(range(i + 1, m)):
                k = c - i + 1
                g.add(synth.KIND_RK, q0 + i, ctrl=bit(q0 + c), iarg=k, p=[0.0, -2.0 * (2 * np.pi / 2.0**k)])
            g.add(synth.KIND_H, q0 + i)
    return g.array()


def by_definition(a, n, q0, m, inverse):
    x = a.reshape(1 << q0, 1 << m, 1 << (n - q0 - m))
    f = np.fft.fft if inverse else np.fft.ifft
    return f(x, axis=1, norm="ortho").reshape(-1)


def relerr(g, o):
    return float(np.max(np.abs(g.astype(np.complex128) - o)) / max(np.max(np.abs(o)), 1e-300))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,q0,m", [(1, 0, 1), (2, 0, 2), (5, 0, 5), (12, 0, 12), (16, 0, 16), (14, 3, 7), (13, 0, 6),
                                    (13, 7, 6), (17, 2, 13)])
@pytest.mark.parametrize("inverse", [False, True])
def test_qft_matches_oracle_and_definition(sv, orc, dtype, n, q0, m, inverse):
    a = synth.random_state(n, 40 + n + q0 + m).astype(NPDT[dtype])
    s = sv.State(n, dtype).load(a)
    say("qft", dtype, n, q0, m, inverse)
    s.qft(q0, m, inverse=inverse)
    got = s.numpy()
    ref = orc.run(a.astype(np.complex128), qft_gates(n, q0, m, inverse))
    ng = m * (m + 1) // 2 + m // 2
    tol = 1e-12 if dtype == "c128" else 1e-6 * ng
    assert relerr(got, ref) < tol
    assert relerr(got, by_definition(a.astype(np.complex128), n, q0, m, inverse)) < tol


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_qft_round_trip(sv, dtype):
    n = 15
    a = synth.random_state(n, 5).astype(NPDT[dtype])
    s = sv.State(n, dtype).load(a)
    s.qft(2, 11).qft(2, 11, inverse=True)
    tol = 1e-12 if dtype == "c128" else 1e-5
    assert relerr(s.numpy(), a.astype(np.complex128)) < tol


@pytest.mark.parametrize("dtype,n", [("c128", 30), ("c64", 30), ("c64", 32)])
def test_qft_full_size(sv, dtype, n):
    # QFT |0> is the uniform superposition; the inverse brings back |0>
    s = sv.State(n, dtype).reset(0)
    say("qft full size", dtype, n)
    s.qft()
    full = (1 << n) - 1
    eps = 1e-12 if dtype == "c128" else 1e-5
    for y in [0, 1, 12345, full >> 1, full]:
        assert abs(s.prob(full, y) * 2.0**n - 1.0) < eps
    s.qft(inverse=True)
    assert abs(s.prob(full, 0) - 1.0) < 10 * eps
