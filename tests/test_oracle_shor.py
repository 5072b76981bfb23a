"""Pins of the oracle's Shor pieces (sec. 5.1): the register after the
classical modular exponentiation, the classical steps 4-5 and their
improvements, and the theoretical iteration counts of Table 5.  CPU only."""

import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import shor

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "shor_table5_theoretical.txt")


def _order(x, N):
    r = 1
    while pow(x, r, N) != 1:
        r += 1
    return r


def test_table5_theoretical_iterations():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 7
    for N, p, q, printed in rows:
        N, p, q = int(N), int(p), int(q)
        assert p * q == N
        assert shor.euler_phi(N) == (p - 1) * (q - 1)
        v = 1.0 / shor.prob_succ(N)
        assert math.floor(v * 100) / 100 == pytest.approx(float(printed), abs=1e-9), (N, v)


def test_euler_phi_brute_force():
    for N in range(2, 200):
        assert shor.euler_phi(N) == sum(1 for k in range(1, N + 1) if math.gcd(k, N) == 1)


@pytest.mark.parametrize("N,m", [(15, 8), (21, 10), (33, 12)])
def test_order_candidate_brute_force(N, m):
    # the unique k/r (coprime, 0 < k < r < N) within 1/2^(m+1) of y/2^m, by
    # enumerating every such fraction
    M = 1 << m
    fracs = [(k, r) for r in range(2, N) for k in range(1, r) if math.gcd(k, r) == 1]
    for y in range(M):
        ok = [(k, r) for k, r in fracs if abs(Fraction(y, M) - Fraction(k, r)) <= Fraction(1, 2 * M)]
        assert len(ok) <= 1
        assert shor.order_candidate(y, m, N) == (ok[0] if ok else None), y


def test_convergents_reconstruct_fraction():
    for y, M in [(0, 8), (3, 8), (4096 * 5, 1 << 16), (12345, 1 << 20), (1, 3)]:
        h, k = shor.convergents(y, M)[-1]
        assert Fraction(h, k) == Fraction(y, M)


def test_step5_textbook_cases():
    # N = 15, x = 7: order 4, 7^2 = 4 (mod 15), gcd(15, 3) = 3
    assert _order(7, 15) == 4
    assert shor.step5(15, 7, 4) in (3, 5)
    assert shor.step5(15, 7, 2) == 0          # 7^2 != 1
    assert shor.step5(15, 4, 2) == 3          # 4^1 = 4: gcd(15, 3)
    assert shor.step5(15, 14, 2) == 0         # 14 = -1: x^(r/2) = -1 fails
    assert shor.step5(21, 2, 6) in (3, 7)     # 2^3 = 8: gcd(21, 7), gcd(21, 9)
    assert shor.step5(21, 2, 3) == 0          # odd r


def test_improvements_only_add_successes():
    # the improved checks run only where plain steps 4-5 fail, so every
    # y that succeeds plainly succeeds improved with the same factor
    N, m = 187, 16
    for x in (2, 23, 100, 186):
        for y in range(0, 1 << m, 97):
            a = shor.classical(N, x, y, m, False)
            b = shor.classical(N, x, y, m, True)
            if a.factor:
                assert b.factor == a.factor and b.stage == shor.ST_PLAIN
            for out in (a, b):
                if out.factor:
                    assert N % out.factor == 0 and 1 < out.factor < N


@pytest.mark.parametrize("N,x,m", [(15, 7, 8), (21, 2, 10), (187, 23, 16), (33, 5, 12)])
def test_shor_state_is_periodic_superposition(N, x, m):
    r = _order(x, N)
    M = 1 << m
    for a_star in (0, 1, r - 1, M - 1, 12345 % M):
        v = pow(x, a_star, N)
        a, count = oracle.shor_state(m, N, x, v)
        a0 = a_star % r
        support = np.arange(a0, M, r)
        assert count == len(support) == (M - 1 - a0) // r + 1
        nz = np.nonzero(a)[0]
        assert np.array_equal(nz, support)
        assert np.all(a[nz] == 1.0 / math.sqrt(count))
        assert abs(np.vdot(a, a) - 1.0) < 1e-13
    a, count = oracle.shor_state(m, N, x, N + 1)  # no preimage
    assert count == 0 and not a.any()


def test_modpow_matches_python():
    rng = np.random.default_rng(0)
    for _ in range(200):
        N = int(rng.integers(2, 1 << 31))
        x = int(rng.integers(0, N))
        e = int(rng.integers(0, 1 << 40))
        assert oracle.modpow(x, e, N) == pow(x, e, N)


def test_qft_of_shor_state_peaks():
    # order 16 divides 2^16: the QFT output has weight 1/16 on the multiples
    # of 2^16/16 and zero elsewhere (the textbook period-finding identity)
    N, x, m = 187, 23, 16
    assert _order(x, N) == 16
    g = synth.qft_circuit(m).array()
    a, _ = oracle.shor_state(m, N, x, pow(x, 5, N))
    b = oracle.run(a, g)
    w = np.abs(b) ** 2
    peaks = np.arange(0, 1 << m, 1 << 12)
    assert np.allclose(w[peaks], 1.0 / 16, atol=1e-13)
    w[peaks] = 0
    assert w.max() < 1e-25


def test_qft_of_shor_state_matches_fft_nonpower_order():
    # order 6 does not divide 2^10: compare with numpy's inverse FFT
    N, x, m = 21, 2, 10
    g = synth.qft_circuit(m).array()
    a, _ = oracle.shor_state(m, N, x, pow(x, 4, N))
    assert np.abs(oracle.run(a, g) - np.fft.ifft(a, norm="ortho")).max() < 1e-13


def test_noiseless_success_probability_n187():
    # x = 23, order 16: y = 4096 k with probability 1/16 each; the plain
    # steps 4-5 succeed iff k is odd (r = 16 recovered) and 23^8 != -1
    N, x, m = 187, 23, 16
    assert pow(x, 8, N) not in (1, N - 1)
    ok = [k for k in range(16) if shor.classical(N, x, 4096 * k, m, False).factor]
    assert ok == [1, 3, 5, 7, 9, 11, 13, 15]


def test_experiment_finds_factors():
    for N in (15, 21, 187):
        m = shor.register_qubits(N)
        g = synth.qft_circuit(m, swaps=False).array()
        for improved in (False, True):
            for seed in range(4):
                it, f, st, log, tries = shor.experiment(N, synth.shor_draws(N, m, seed, 100), improved, g, 100)
                assert it >= 1 and 1 < f < N and N % f == 0


def test_noisy_traj_state_noise_free_limit():
    n = 8
    psi = synth.random_state(n, 3)
    g = synth.qft_circuit(n, swaps=False).array()
    out = oracle.noisy_traj_state(psi, 1, 0.0, 0.0, 7, 3, g[:0], g)
    assert np.abs(out - oracle.run(psi, g)).max() < 1e-14


def test_measuring_without_swaps_reads_reversed_index():
    # the final swaps of the QFT only reverse the bit order (sec. 2.3.2): the
    # output without them, read at the reversed index, is the same
    N, x, m = 21, 2, 10
    a, _ = oracle.shor_state(m, N, x, pow(x, 3, N))
    full = oracle.run(a, synth.qft_circuit(m).array())
    part = oracle.run(a, synth.qft_circuit(m, swaps=False).array())
    rev = np.array([synth.bit_reverse(y, m) for y in range(1 << m)])
    assert np.array_equal(part[rev], full)
    g = synth.qft_circuit(m, swaps=False).array()
    cum = np.cumsum(np.abs(full) ** 2)
    for u in (0.0, 0.1, 0.5, 0.77, 0.999):
        y = shor.quantum_step(N, x, m, 3, u, g)
        # y is the reversal of the index measured without swaps
        j = oracle.measure(part, u)
        assert y == synth.bit_reverse(j, m)
        assert abs(full[y]) ** 2 > 0 and cum[-1] > u
