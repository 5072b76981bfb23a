"""Pins of the CPU oracle against facts fixed outside it: dense Kronecker
matrices (sec. 2.2.1 / 2.2.2 definitions), closed forms (Grover's sin^2 law,
the Hadamard transform, the DFT that sec. 2.3.2 defines the QFT to be),
library routines for special cases, brute force on tiny inputs, and the
published Philox known-answer vectors.  No GPU."""

import math
import os

import numpy as np
import pytest

import synth
from synth import KIND_H, KIND_RK, KIND_ROT, KIND_SU2, KIND_SWAP, KIND_U, KIND_X, KIND_Y, KIND_Z

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------ brute force


def dense_1q(n, q, U):
    """X = I^(x)q (x) U (x) I^(x)(n-1-q), qubit 0 leftmost (sec. 2.2.1)."""
    X = np.eye(1, dtype=np.complex128)
    for k in range(n):
        X = np.kron(X, U if k == q else np.eye(2))
    return X


def dense_ctrl(n, ctrl, q, U):
    """CTX[j] = X[j] if every control bit of j is 1, else I[j] (sec. 2.2.2)."""
    X = dense_1q(n, q, U)
    N = 1 << n
    I = np.eye(N, dtype=np.complex128)
    rows = np.array([(j & ctrl) == ctrl for j in range(N)])
    return np.where(rows[:, None], X, I)


def dense_swap(n, q1, q2):
    N = 1 << n
    P = np.zeros((N, N))
    b1, b2 = n - 1 - q1, n - 1 - q2
    for j in range(N):
        x1, x2 = (j >> b1) & 1, (j >> b2) & 1
        k = j & ~((1 << b1) | (1 << b2)) | (x2 << b1) | (x1 << b2)
        P[k, j] = 1
    return P


def rand_state(n, seed):
    return synth.random_state(n, seed)


def rand_U(rng):
    return np.array(synth.random_unitary_params(rng)).view(np.complex128).reshape(2, 2)


# ------------------------------------------------------------ P1: gates


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_apply_1q_matches_kronecker(orc, n):
    rng = np.random.default_rng(100 + n)
    for q in range(n):
        for U in (rand_U(rng), rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))):
            a = rand_state(n, 7 * n + q)
            got = orc.apply_1q(a, q, U)
            ref = dense_1q(n, q, U) @ a
            assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("n", [2, 3, 6, 9])
def test_apply_ctrl_matches_kronecker(orc, n):
    rng = np.random.default_rng(200 + n)
    for trial in range(12):
        q = int(rng.integers(0, n))
        others = [k for k in range(n) if k != q]
        nc = int(rng.integers(1, len(others) + 1))
        cq = rng.choice(others, size=nc, replace=False)
        ctrl = 0
        for c in cq:
            ctrl |= 1 << (n - 1 - int(c))
        U = rand_U(rng)
        a = rand_state(n, 1000 * n + trial)
        got = orc.apply_ctrl(a, ctrl, q, U)
        ref = dense_ctrl(n, ctrl, q, U) @ a
        assert np.max(np.abs(got - ref)) <= 1e-13


def test_apply_10_qubits_every_target(orc):
    n = 10
    rng = np.random.default_rng(10)
    a = rand_state(n, 10)
    for q in range(n):
        U = rand_U(rng)
        ref = dense_1q(n, q, U) @ a
        got = orc.apply_1q(a, q, U)
        assert np.max(np.abs(got - ref)) <= 1e-13
        ctrl = 1 << (n - 1 - ((q + 3) % n))
        ref = dense_ctrl(n, ctrl, q, U) @ a
        got = orc.apply_ctrl(a, ctrl, q, U)
        assert np.max(np.abs(got - ref)) <= 1e-13


def test_swap_matches_permutation(orc):
    n = 5
    a = rand_state(n, 3)
    for q1 in range(n):
        for q2 in range(n):
            got = orc.swap(a, q1, q2)
            ref = dense_swap(n, q1, q2) @ a
            assert np.array_equal(got, ref)


# ------------------------------------------------------------ P9: permutations


def test_permutations_bit_exact(orc):
    n = 6
    X = orc.gate_matrix(KIND_X)
    assert np.array_equal(X, np.array([[0, 1], [1, 0]], dtype=np.complex128))
    a = rand_state(n, 5)
    for q in range(n):
        b = orc.apply_1q(orc.apply_1q(a, q, X), q, X)
        assert np.array_equal(b.view(np.uint64), a.view(np.uint64))
    # CNOT and Toffoli truth tables on basis states
    for j in range(1 << n):
        e = np.zeros(1 << n, dtype=np.complex128)
        e[j] = 1
        # CNOT control qubit 1, target qubit 4
        out = orc.apply_ctrl(e, 1 << (n - 1 - 1), 4, X)
        k = j ^ (1 << (n - 1 - 4)) if (j >> (n - 1 - 1)) & 1 else j
        assert out[k] == 1 and np.count_nonzero(out) == 1
        # Toffoli controls 0 and 5, target 2
        m = (1 << (n - 1)) | 1
        out = orc.apply_ctrl(e, m, 2, X)
        k = j ^ (1 << (n - 1 - 2)) if (j & m) == m else j
        assert out[k] == 1 and np.count_nonzero(out) == 1
    # signed zeros survive moves (0 * x + y would lose -0.0)
    a = np.array([-0.0 + 1j, 0.5 - 0.0j], dtype=np.complex128)
    b = orc.apply_1q(a, 0, X)
    assert np.array_equal(b.view(np.uint64), a[::-1].copy().view(np.uint64))


# ------------------------------------------------------------ a9: gate matrices


def test_gate_matrices_definitions(orc):
    r = math.sqrt(0.5)  # correctly rounded 1/sqrt(2)
    H = orc.gate_matrix(KIND_H)
    assert np.array_equal(H, np.array([[r, r], [r, -r]]))
    assert np.array_equal(orc.gate_matrix(KIND_Z), np.diag([1.0, -1.0]).astype(complex))
    assert np.array_equal(orc.gate_matrix(KIND_Y), np.array([[0, -1j], [1j, 0]]))
    # sec. 3.2: H = U_R(pi/4) U_P1(pi), NOT = U_R(pi/2) U_P1(pi)
    UR = lambda t: np.array([[math.cos(t), -math.sin(t)], [math.sin(t), math.cos(t)]])
    UP = lambda f: np.diag([1.0, np.exp(1j * f)])
    assert np.allclose(orc.gate_matrix(KIND_ROT, 0, [math.pi / 4, math.pi]), H, atol=1e-15)
    assert np.allclose(orc.gate_matrix(KIND_ROT, 0, [math.pi / 2, math.pi]), [[0, 1], [1, 0]], atol=1e-15)
    for th, ph in [(0.3, -1.1), (2.0, 0.25)]:
        assert np.allclose(orc.gate_matrix(KIND_ROT, 0, [th, ph]), UR(th) @ UP(ph), atol=1e-15)
    # over-rotated H and NOT
    x, y = 0.01, -0.02
    assert np.allclose(orc.gate_matrix(KIND_H, 0, [x, y]), UR(math.pi / 4 + x) @ UP(math.pi + y), atol=1e-15)
    assert np.allclose(orc.gate_matrix(KIND_X, 0, [x, y]), UR(math.pi / 2 + x) @ UP(math.pi + y), atol=1e-15)
    assert np.allclose(orc.gate_matrix(KIND_Z, 0, [0, y]), UP(math.pi + y), atol=1e-15)
    # R_k = diag(1, e^{2 pi i / 2^k})
    for k in range(1, 12):
        Rk = orc.gate_matrix(KIND_RK, k)
        assert np.allclose(Rk, np.diag([1, np.exp(2j * math.pi / 2**k)]), atol=1e-15)
        assert Rk[0, 1] == 0 and Rk[1, 0] == 0 and Rk[0, 0] == 1
    # Haar SU(2) from quaternion: unitary, det 1
    rng = np.random.default_rng(0)
    for _ in range(20):
        qv = rng.standard_normal(4)
        S = orc.gate_matrix(KIND_SU2, 0, qv)
        assert np.allclose(S.conj().T @ S, np.eye(2), atol=1e-15)
        assert abs(np.linalg.det(S) - 1) < 1e-15
        qn = qv / np.linalg.norm(qv)
        assert np.allclose(S[0, 0], qn[0] + 1j * qn[1]) and np.allclose(S[0, 1], qn[2] + 1j * qn[3])


def test_gate_dmatrix_is_derivative(orc):
    h = 1e-6
    cases = [(KIND_H, 0, [0.01, -0.02]), (KIND_X, 0, [0.0, 0.03]), (KIND_ROT, 0, [0.7, 1.3]),
             (KIND_Z, 0, [0.0, 0.05]), (KIND_RK, 4, [0.0, 0.01])]
    for kind, iarg, p in cases:
        for which in (0, 1):
            if which == 0 and kind in (KIND_Z, KIND_RK):
                with pytest.raises(ValueError):
                    orc.gate_dmatrix(kind, iarg, p, which)
                continue
            pp, pm = list(p), list(p)
            pp[which] += h
            pm[which] -= h
            fd = (orc.gate_matrix(kind, iarg, pp) - orc.gate_matrix(kind, iarg, pm)) / (2 * h)
            assert np.allclose(orc.gate_dmatrix(kind, iarg, p, which), fd, atol=1e-9)


# ------------------------------------------------------------ a5: dense blocks


def test_apply_kq_matches_kronecker_and_sequence(orc):
    n = 7
    rng = np.random.default_rng(3)
    a = rand_state(n, 11)
    for k in (1, 2, 3, 4, 5):
        qs = [int(x) for x in rng.choice(n, size=k, replace=False)]
        M = rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))
        got = orc.apply_kq(a, qs, M)
        # brute force: permute qubits so the k targets lead (in order qs), apply
        # kron(M, I), permute back
        rest = [q for q in range(n) if q not in qs]
        order = qs + rest
        t = a.reshape([2] * n).transpose(order).reshape(1 << k, -1)
        t = (M @ t).reshape([2] * n)
        ref = t.transpose(np.argsort(order)).reshape(-1)
        assert np.max(np.abs(got - ref)) <= 1e-12
    # a product of one-qubit gates on the block equals their sequence
    qs = [4, 1, 6]
    Us = [rand_U(rng) for _ in qs]
    M = np.kron(np.kron(Us[0], Us[1]), Us[2])
    seq = a
    for q, U in zip(qs, Us):
        seq = orc.apply_1q(seq, q, U)
    assert np.max(np.abs(orc.apply_kq(a, qs, M) - seq)) <= 1e-14


# ------------------------------------------------------------ a6: reductions


def test_prob_inner_measure(orc):
    n = 9
    a = rand_state(n, 21)
    b = rand_state(n, 22)
    w = np.abs(a) ** 2
    idx = np.arange(1 << n)
    for mask, value in [(0, 0), (1, 1), (0b101000000, 0b100000000), ((1 << n) - 1, 300), (0b11, 0b10)]:
        assert abs(orc.prob(a, mask, value) - w[(idx & mask) == value].sum()) <= 1e-14
    assert abs(orc.prob(a) - 1.0) <= 1e-14
    assert abs(orc.inner(a, b) - np.vdot(a, b)) <= 1e-14
    assert abs(orc.inner(a, a) - 1.0) <= 1e-14
    cum = np.cumsum(w)
    rng = np.random.default_rng(5)
    for r in rng.random(200):
        assert orc.measure(a, r) == int(np.searchsorted(cum, r, side="right"))
    # r at or beyond the total returns the last index with nonzero weight
    e = np.zeros(8, dtype=np.complex128)
    e[3] = 1.0
    assert orc.measure(e, 0.0) == 3 and orc.measure(e, 0.999999) == 3 and orc.measure(e, 1.0) == 3


def test_collapse_invariants(orc):
    # projective measurement of a subset of qubits (sec. 2.2.3 applied to the
    # qubits in a mask): pinned by the laws it must obey, not by its formula
    n = 8
    a = rand_state(n, 31)
    full = (1 << n) - 1
    m1, m2 = 0b10010000, 0b00000101
    # (1) the outcome probabilities of a mask sum to the squared norm
    vals = [v for v in range(1 << n) if v & ~m1 == 0]
    assert abs(sum(orc.collapse(a, m1, v)[1] for v in vals) - 1.0) <= 1e-14
    # (2) the post-measurement register is normalised, lives on its outcome,
    #     and a second identical measurement is certain and changes nothing
    b, p = orc.collapse(a, m1, 0b10000000)
    idx = np.arange(1 << n)
    assert abs(orc.prob(b) - 1.0) <= 1e-14
    assert np.all(b[(idx & m1) != 0b10000000] == 0)
    c, p2 = orc.collapse(b, m1, 0b10000000)
    assert abs(p2 - 1.0) <= 1e-14 and np.max(np.abs(c - b)) <= 1e-15
    # (3) measuring disjoint masks one after the other equals measuring their
    #     union, and the probabilities multiply (chain rule)
    x, px = orc.collapse(a, m1, 0b00010000)
    y, py = orc.collapse(x, m2, 0b00000100)
    z, pz = orc.collapse(a, m1 | m2, 0b00010100)
    assert abs(px * py - pz) <= 1e-15 and np.max(np.abs(y - z)) <= 1e-14
    # (4) all qubits measured: the basis state with the amplitude's phase,
    #     with probability |alpha_v|^2
    e, pe = orc.collapse(a, full, 77)
    assert abs(pe - abs(a[77]) ** 2) <= 1e-16
    assert abs(e[77] - a[77] / abs(a[77])) <= 1e-15 and np.count_nonzero(e) == 1
    # (5) an impossible outcome has probability 0 and leaves the register
    z0 = a.copy()
    z0[(idx & m2) == 0b101] = 0
    q, pq = orc.collapse(z0, m2, 0b101)
    assert pq == 0.0 and np.array_equal(q, z0)


# ------------------------------------------------------------ P4, P5


def test_norm_and_round_trip(orc):
    n = 10
    gl = synth.random_gate_mix(n, 200, seed=4)
    a = rand_state(n, 4)
    g = gl.array()
    # keep only unitary gates for the norm check
    out = orc.run(a, g)
    assert abs(orc.prob(out) - 1.0) <= 1e-13
    back = out.copy()
    for rec in g[::-1]:
        orc.lib().orc_apply_gate_inverse(back.ctypes.data, n, rec.tobytes())
    assert np.max(np.abs(back - a)) <= 1e-13


def test_hadamard_transform(orc):
    for n in (1, 4, 11):
        out = orc.run(orc.zero_state(n), synth.hadamard_transform(n).array())
        assert np.max(np.abs(out - 2 ** (-n / 2))) <= 1e-15
        a = rand_state(n, n)
        b = orc.run(orc.run(a, synth.hadamard_transform(n).array()), synth.hadamard_transform(n).array())
        assert np.max(np.abs(a - b)) <= 1e-14
    # sec. 2.3.1: H_n|x> = 2^{-n/2} sum_y (-1)^{x.y} |y>
    n = 5
    for x in (0, 7, 21, 31):
        e = np.zeros(1 << n, dtype=np.complex128)
        e[x] = 1
        out = orc.run(e, synth.hadamard_transform(n).array())
        ref = np.array([(-1) ** bin(x & y).count("1") for y in range(1 << n)]) * 2 ** (-n / 2)
        assert np.max(np.abs(out - ref)) <= 1e-15


# ------------------------------------------------------------ P3: QFT


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 10])
def test_qft_equals_direct_dft(orc, n):
    """sec. 2.3.2: beta_x = 2^{-n/2} sum_y omega^{xy} alpha_y, omega = e^{2 pi i/2^n}."""
    N = 1 << n
    a = rand_state(n, 50 + n)
    out = orc.run(a, synth.qft_circuit(n).array())
    x = np.arange(N)
    W = np.exp(2j * np.pi * np.outer(x, x) / N) / math.sqrt(N)
    ref = W @ a
    assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("n", [12, 16])
def test_qft_equals_library_fft(orc, n):
    a = rand_state(n, 60 + n)
    out = orc.run(a, synth.qft_circuit(n).array())
    ref = np.fft.ifft(a, norm="ortho")
    assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_dft_element_matches_library_fft(orc):
    for n in (1, 5, 11, 16):
        a = rand_state(n, 70 + n)
        ref = np.fft.ifft(a, norm="ortho")
        rng = np.random.default_rng(n)
        for x in list(rng.integers(0, 1 << n, 6)) + [0, (1 << n) - 1]:
            assert abs(orc.dft_element(a, int(x)) - ref[int(x)]) <= 1e-13


def test_qft_gate_count():
    for n in (5, 24, 28):
        gl = synth.qft_circuit(n, swaps=False)
        assert len(gl) == n * (n + 1) // 2
    assert len(synth.qft_circuit(24, swaps=False)) == 300


# ------------------------------------------------------------ P2: Grover


@pytest.mark.parametrize("n,seed", [(4, 0), (7, 1), (10, 2), (10, 3)])
def test_grover_sin2_every_iteration(orc, n, seed):
    """Noise-free success probability follows sin^2((2k+1) theta),
    theta = asin(2^{-n/2}) (the sine curve of sec. 5.3.1)."""
    marked = synth.grover_marked(n, seed)
    theta = math.asin(2 ** (-n / 2))
    a = orc.run(orc.zero_state(n), synth.hadamard_transform(n).array())
    it = synth.grover_iteration(n, marked).array()
    for k in range(1, 2 * synth.grover_iterations(n) + 2):
        a = orc.run(a, it)
        assert abs(orc.prob(a, (1 << n) - 1, marked) - math.sin((2 * k + 1) * theta) ** 2) <= 1e-12


@pytest.mark.parametrize("marked", [0, 16383, None])
def test_grover_n14_full(orc, marked):
    n = 14
    if marked is None:
        marked = synth.grover_marked(n, 0)
    iters = synth.grover_iterations(n)
    assert iters == 100
    a = orc.run(orc.zero_state(n), synth.grover_circuit(n, marked, iters).array())
    ref = math.sin(201 * math.asin(2**-7)) ** 2
    assert abs(ref - 0.999999781114231) < 1e-15
    assert abs(orc.prob(a, (1 << n) - 1, marked) - ref) <= 1e-12


# ------------------------------------------------------------ Philox


def test_philox_known_answers(orc):
    rows = 0
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        assert list(orc.philox4x32_10(w[0:4], w[4:6])) == w[6:]
        rows += 1
    assert rows == 3


def test_pauli_threshold(orc):
    assert orc.pauli_threshold(0.0) == 0
    assert orc.pauli_threshold(1e-4) == math.floor(1e-4 * 2**32)
    assert orc.pauli_threshold(1e-5) == math.floor(1e-5 * 2**32)
    assert orc.pauli_threshold(1.0) == 2**32 - 1


# ------------------------------------------------------------ P6, P7: noise statistics


def _ht_mean(orc, n, k, sigma, p, trajectories, seed):
    init = np.zeros(0, dtype=synth.GATE_DTYPE)
    it = synth.hadamard_transform(n).array()
    vals = np.array([orc.noisy_grover_traj(n, 0, k, sigma, p, seed, t, init, it) for t in range(trajectories)])
    return vals.mean(), vals.std(ddof=1) / math.sqrt(len(vals))


def test_ht_depolarizing_closed_form(orc):
    """sec. 4.3.1: <0|rho_k|0> = ((1 + (1 - 4p/3)^k) / 2)^n for even k."""
    n, k, p = 3, 10, 0.05
    mean, se = _ht_mean(orc, n, k, 0.0, p, 6000, seed=11)
    ref = ((1 + (1 - 4 * p / 3) ** k) / 2) ** n
    assert abs(mean - ref) <= 4 * se, (mean, ref, se)


def test_ht_operational_closed_form(orc):
    """sec. 4.3.1: <0|rho_k|0> = ((1 + exp(-9 k sigma^2 / 4)) / 2)^n for even k."""
    n, k, sigma = 2, 10, 0.15
    mean, se = _ht_mean(orc, n, k, sigma, 0.0, 6000, seed=12)
    ref = ((1 + math.exp(-9 * k * sigma**2 / 4)) / 2) ** n
    assert abs(mean - ref) <= 4 * se, (mean, ref, se)


def _ht_with_identity_sites(n, sites):
    """One HT application followed by `sites` explicit identity gates (kind
    U) on every qubit."""
    g = synth.hadamard_transform(n)
    eye = [1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0]
    for _ in range(sites):
        for q in range(n):
            g.add(KIND_U, q, p=eye)
    return g.array()


def _masked_ht_mean(orc, n, k, p, kinds, trajectories, seed, sites=2):
    zero = orc.zero_state(n)
    it = _ht_with_identity_sites(n, sites)
    init = np.zeros(0, dtype=synth.GATE_DTYPE)
    vals = np.array([abs(orc.noisy_traj_state(zero, k, 0.0, p, seed, t, init, it, depol_kinds=kinds)[0]) ** 2
                     for t in range(trajectories)])
    return vals.mean(), vals.std(ddof=1) / math.sqrt(len(vals))


@pytest.mark.parametrize("kinds,sites_per_qubit", [(1 << KIND_U, 2), (1 << KIND_H, 1), (0xFFFFFFFF, 3)])
def test_depolarizing_follows_only_the_selected_kinds(orc, kinds, sites_per_qubit):
    """sec. 3.1 channel at the sites the kind mask selects: each HT
    application is followed by two identity gates per qubit, so depolarizing
    after the identities alone gives 2 channel uses per qubit and
    application, after the H gates alone 1, after every gate 3; the closed
    form of sec. 4.3.1 with k replaced by the number of channel uses,
    ((1 + (1 - 4p/3)^(k s)) / 2)^n, must hold within 4 SE.  n = 4, k = 10,
    p = 0.05 gives 0.318, 0.153 and 0.101 for s = 1, 2, 3, more than 6 SE
    apart at 4000 trajectories, so an inverted or shifted mask fails."""
    n, k, p = 4, 10, 0.05
    mean, se = _masked_ht_mean(orc, n, k, p, kinds, 4000, seed=13)
    ref = ((1 + (1 - 4 * p / 3) ** (k * sites_per_qubit)) / 2) ** n
    assert abs(mean - ref) <= 4 * se, (mean, ref, se)
    others = [((1 + (1 - 4 * p / 3) ** (k * s)) / 2) ** n for s in (1, 2, 3) if s != sites_per_qubit]
    assert all(abs(mean - o) > 6 * se for o in others)


def test_depolarizing_mask_without_listed_kinds_is_noise_free(orc):
    # a mask that selects no kind present in the list (R_k, Y) draws no
    # Pauli: bit for bit the p = 0 run, which is the plain run of the list
    n, k = 4, 6
    zero = orc.zero_state(n)
    it = _ht_with_identity_sites(n, 2)
    init = np.zeros(0, dtype=synth.GATE_DTYPE)
    plain = orc.noisy_traj_state(zero, k, 0.0, 0.0, 21, 0, init, it)
    for t in range(20):
        got = orc.noisy_traj_state(zero, k, 0.0, 0.5, 21, t, init, it,
                                   depol_kinds=(1 << KIND_RK) | (1 << KIND_Y))
        assert np.array_equal(got, plain)
    # the same p with the identity sites selected does change trajectories
    changed = sum(not np.array_equal(orc.noisy_traj_state(zero, k, 0.0, 0.5, 21, t, init, it,
                                                           depol_kinds=1 << KIND_U), plain) for t in range(20))
    assert changed >= 15
    ref = orc.run(zero, np.concatenate([it] * k))
    assert np.array_equal(plain, ref)


def test_noise_free_limit_equals_plain_run(orc):
    n, seed = 8, 5
    marked = synth.grover_marked(n, seed)
    iters = synth.grover_iterations(n)
    init = synth.hadamard_transform(n).array()
    it = synth.grover_iteration(n, marked).array()
    p_noisy, st = orc.noisy_grover_traj(n, marked, iters, 0.0, 0.0, 9, 3, init, it, want_state=True)
    plain = orc.run(orc.zero_state(n), synth.grover_circuit(n, marked, iters).array())
    assert np.array_equal(st, plain)
    assert p_noisy == orc.prob(plain, (1 << n) - 1, marked)


def test_noisy_trajectories_reproducible_and_distinct(orc):
    n = 6
    marked = 5
    init = synth.hadamard_transform(n).array()
    it = synth.grover_iteration(n, marked).array()
    a = orc.noisy_grover_traj(n, marked, 6, 0.05, 1e-2, 123, 7, init, it)
    b = orc.noisy_grover_traj(n, marked, 6, 0.05, 1e-2, 123, 7, init, it)
    c = orc.noisy_grover_traj(n, marked, 6, 0.05, 1e-2, 123, 8, init, it)
    assert a == b and a != c


# ------------------------------------------------------------ P8: adjoint


def _loss(orc, psi0, phi, gates):
    out = orc.run(psi0, gates)
    return 1.0 - abs(orc.inner(phi, out)) ** 2


def test_adjoint_against_parameter_shift_and_fd(orc):
    """Gradient of 1 - |<QFT psi0 | QFT(eps) psi0>|^2 w.r.t. every gate's
    deviation at n = 10 (55 gates): exact parameter-shift rule
    (R_k phase: shift pi/2, factor 1/2; H rotation U_R = exp(-i theta Y):
    shift pi/4, factor 1) and central differences with h = 1e-6."""
    n = 10
    ng = n * (n + 1) // 2
    eps = synth.qft_eps(ng, seed=1, sigma=1e-2)
    psi0 = rand_state(n, 0)
    phi = orc.run(psi0, synth.qft_circuit(n).array())
    gates = synth.qft_perturbed(n, eps).array()
    dparam = np.array([0 if g["kind"] == KIND_H else (1 if g["kind"] == KIND_RK else -1) for g in gates], np.int32)
    grad, A, _ = orc.adjoint(psi0, phi, gates, dparam)
    assert np.all(grad[len(eps):] == 0)
    for gi in range(ng):
        which = dparam[gi]
        shift, fac = (math.pi / 4, 1.0) if which == 0 else (math.pi / 2, 0.5)
        gp, gm = gates.copy(), gates.copy()
        gp[gi]["p"][which] += shift
        gm[gi]["p"][which] -= shift
        ps = fac * (_loss(orc, psi0, phi, gp) - _loss(orc, psi0, phi, gm))
        assert abs(grad[gi] - ps) <= 1e-11, (gi, grad[gi], ps)
        if gi % 5 == 0:
            h = 1e-6
            gp, gm = gates.copy(), gates.copy()
            gp[gi]["p"][which] += h
            gm[gi]["p"][which] -= h
            fd = (_loss(orc, psi0, phi, gp) - _loss(orc, psi0, phi, gm)) / (2 * h)
            assert abs(grad[gi] - fd) <= 1e-8
