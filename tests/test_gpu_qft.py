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


@pytest.fixture
def qft_engine(sv):
    old = sv.config_get("qft_fft")
    yield lambda v: sv.config_set("qft_fft", v)
    sv.config_set("qft_fft", old)


def bitrev_range(v, n, q0, m):
    x = v.reshape(1 << q0, 1 << m, 1 << (n - q0 - m))
    r = np.array([synth.bit_reverse(y, m) for y in range(1 << m)])
    out = np.empty_like(x)
    out[:, r, :] = x
    return out.reshape(-1)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,q0,m", [(12, 0, 12), (13, 0, 13), (16, 0, 16), (14, 3, 7), (13, 7, 6), (17, 2, 13),
                                    (20, 0, 20), (15, 0, 5), (14, 13, 1), (18, 5, 9), (20, 2, 12), (24, 0, 24)])
@pytest.mark.parametrize("flags", [0, 1, 2, 3])
def test_fft_and_circuit_engines(sv, qft_engine, dtype, n, q0, m, flags):
    # FFT block passes and the circuit agree with the definition for every
    # flag: inverse (bit 0) and bit-reversed output / input (bit 1)
    inverse, bitrev = bool(flags & 1), bool(flags & 2)
    a = synth.random_state(n, 77 + n + q0 + m).astype(NPDT[dtype])
    a128 = a.astype(np.complex128)
    if not bitrev:
        want = by_definition(a128, n, q0, m, inverse)
    elif not inverse:
        want = bitrev_range(by_definition(a128, n, q0, m, False), n, q0, m)
    else:
        want = by_definition(bitrev_range(a128, n, q0, m), n, q0, m, True)
    ng = m * (m + 1) // 2 + m // 2
    tol = 1e-12 if dtype == "c128" else 1e-6 * ng
    for eng in (1, 0):
        qft_engine(eng)
        say("qft engine", eng, dtype, n, q0, m, flags)
        s = sv.State(n, dtype).load(a)
        s.qft(q0, m, inverse=inverse, bitrev=bitrev)
        assert relerr(s.numpy(), want) < tol, (eng, relerr(s.numpy(), want))


@pytest.mark.parametrize("n", [28, 29])
def test_fft_full_size_sampled(sv, orc, n):
    # random complex128 register at n = 28 (blocks of 8, 8 and 12 bits) and
    # 29 (6, 6, 5 and 12): sampled outputs against the oracle's one-output
    # DFT
    import torch

    a = synth.random_state(n, 0)
    s = sv.State(n, "c128").load(a)
    say("fft sampled", n)
    s.qft()
    ys = [0, 1, 777, (1 << (n - 1)) + 12345, (1 << n) - 1]
    got = s.tensor[torch.tensor(ys, device="cuda")].cpu().numpy()
    mx = float(np.max(np.abs(a)))
    for y, g in zip(ys, got):
        assert abs(g - orc.dft_element(a, y)) < 1e-12 * max(mx, 1e-300) * 4
