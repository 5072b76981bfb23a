"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and
the benchmark.

This module holds no simulation arithmetic: it draws random numbers and writes
gate lists as symbolic records (kind, qubits, raw parameters).  Turning a record
into a 2x2 matrix, applying it, and any reduction are done separately by the
plain CPU oracle and by the HIP library, each with its own code.

Gate record layout (88 bytes, little endian, 8-byte aligned)::

    int32  kind      gate kind code (KIND_* below)
    int32  target    target qubit (qubit 0 = most significant index bit)
    int32  target2   second qubit of a SWAP, else -1
    int32  iarg      integer argument (k of R_k), else 0
    uint64 ctrl      control mask over basis-index bits (bit b <-> qubit n-1-b)
    float64 p[8]     real parameters, meaning by kind:
        U    p = (u11re,u11im,u12re,u12im,u21re,u21im,u22re,u22im)
        H    p[0] = dtheta, p[1] = dphi   (over-rotation of U_R(pi/4) U_P1(pi))
        X    p[0] = dtheta, p[1] = dphi   (over-rotation of U_R(pi/2) U_P1(pi))
        Y    none (Pauli sigma_y)
        Z    p[1] = dphi                   (U_P1(pi + dphi))
        RK   iarg = k, p[1] = dphi         (U_P1(2 pi / 2^k + dphi))
        ROT  p[0] = theta, p[1] = phi      (U_R(theta) U_P1(phi))
        SU2  p[0..3] = raw N(0,1) quaternion (normalised by the consumer)
        SWAP target, target2
"""

from __future__ import annotations

import math

import numpy as np

KIND_U, KIND_H, KIND_X, KIND_Y, KIND_Z, KIND_RK, KIND_ROT, KIND_SU2, KIND_SWAP = range(9)
KIND_NAMES = ["U", "H", "X", "Y", "Z", "RK", "ROT", "SU2", "SWAP"]

GATE_DTYPE = np.dtype(
    [
        ("kind", "<i4"),
        ("target", "<i4"),
        ("target2", "<i4"),
        ("iarg", "<i4"),
        ("ctrl", "<u8"),
        ("p", "<f8", (8,)),
    ],
    align=True,
)
assert GATE_DTYPE.itemsize == 88


def qubit_bit(n: int, q: int) -> int:
    """Basis-index bit mask of qubit q (qubit 0 is the most significant bit)."""
    return 1 << (n - 1 - q)


class GateList:
    """Append-only builder of gate records."""

    def __init__(self):
        self._rows = []

    def add(self, kind, target, ctrl=0, target2=-1, iarg=0, p=None):
        pp = [0.0] * 8
        if p is not None:
            for i, v in enumerate(p):
                pp[i] = float(v)
        self._rows.append((int(kind), int(target), int(target2), int(iarg), int(ctrl), pp))
        return self

    def extend(self, other: "GateList"):
        self._rows.extend(other._rows)
        return self

    def __len__(self):
        return len(self._rows)

    def array(self) -> np.ndarray:
        a = np.zeros(len(self._rows), dtype=GATE_DTYPE)
        for i, (k, t, t2, ia, c, p) in enumerate(self._rows):
            a[i]["kind"] = k
            a[i]["target"] = t
            a[i]["target2"] = t2
            a[i]["iarg"] = ia
            a[i]["ctrl"] = c
            a[i]["p"] = p
        return a


# ---------------------------------------------------------------- states


def random_state(n: int, seed: int) -> np.ndarray:
    """i.i.d. complex Gaussian amplitudes, scaled to unit 2-norm (complex128)."""
    rng = np.random.default_rng(seed)
    N = 1 << n
    v = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    v /= math.sqrt(float(np.vdot(v, v).real))
    return v.astype(np.complex128)


def random_unitary_params(rng) -> list:
    """Eight doubles (row-major, re/im interleaved) of a Haar-random 2x2
    unitary: QR of a complex Ginibre matrix with the phases of R's diagonal
    moved into Q.  Used only to make test inputs."""
    z = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    qm, r = np.linalg.qr(z)
    d = np.diag(r)
    qm = qm * (d / np.abs(d))
    out = []
    for i in range(2):
        for j in range(2):
            out += [float(qm[i, j].real), float(qm[i, j].imag)]
    return out


def random_matrix_params(rng) -> list:
    """Eight doubles of a random (non-unitary) complex 2x2 matrix."""
    return list(rng.standard_normal(8))


# ---------------------------------------------------------------- circuits


def hadamard_transform(n: int) -> GateList:
    """H on every qubit, qubit 0 first."""
    g = GateList()
    for q in range(n):
        g.add(KIND_H, q)
    return g


def grover_marked(n: int, seed: int) -> int:
    """Marked index for a seeded Grover search."""
    return int(np.random.default_rng(seed).integers(0, 1 << n))


def grover_iterations(n: int) -> int:
    """floor(pi/4 * sqrt(2^n))."""
    return int(math.floor(math.pi / 4 * math.sqrt(float(1 << n))))


def grover_iteration(n: int, marked: int) -> GateList:
    """One ancilla-free Grover iteration on n qubits.

    oracle    : X on each qubit whose bit of `marked` is 0, C^{n-1}Z, same X's
    diffusion : H^n, X^n, C^{n-1}Z, X^n, H^n
    C^{n-1}Z is a Z on qubit n-1 controlled by every other qubit."""
    g = GateList()
    allc = ((1 << n) - 1) & ~1  # every basis bit except bit 0 (qubit n-1)
    zeros = [q for q in range(n) if not (marked >> (n - 1 - q)) & 1]
    for q in zeros:
        g.add(KIND_X, q)
    g.add(KIND_Z, n - 1, ctrl=allc)
    for q in zeros:
        g.add(KIND_X, q)
    for q in range(n):
        g.add(KIND_H, q)
    for q in range(n):
        g.add(KIND_X, q)
    g.add(KIND_Z, n - 1, ctrl=allc)
    for q in range(n):
        g.add(KIND_X, q)
    for q in range(n):
        g.add(KIND_H, q)
    return g


def grover_circuit(n: int, marked: int, iters: int) -> GateList:
    g = hadamard_transform(n)
    it = grover_iteration(n, marked)
    for _ in range(iters):
        g.extend(it)
    return g


def qft_circuit(n: int, swaps: bool = True) -> GateList:
    """Textbook QFT: for q = 0..n-1: H(q), then R_k on target q controlled by
    qubit c for c = q+1..n-1 with k = c-q+1; finally swap(q, n-1-q)."""
    g = GateList()
    for q in range(n):
        g.add(KIND_H, q)
        for c in range(q + 1, n):
            g.add(KIND_RK, q, ctrl=qubit_bit(n, c), iarg=c - q + 1)
    if swaps:
        for q in range(n // 2):
            g.add(KIND_SWAP, q, target2=n - 1 - q)
    return g


def qft_eps(n_gates: int, seed: int, sigma: float) -> np.ndarray:
    """Per-gate over-rotation angles eps_g ~ N(0, sigma^2)."""
    return np.random.default_rng(seed).standard_normal(n_gates) * sigma


def qft_perturbed(n: int, eps) -> GateList:
    """QFT with one over-rotation per H (on theta) and per R_k (on phi); the
    final swaps are exact.  len(eps) must be n(n+1)/2."""
    g = GateList()
    i = 0
    for q in range(n):
        g.add(KIND_H, q, p=[eps[i], 0.0])
        i += 1
        for c in range(q + 1, n):
            g.add(KIND_RK, q, ctrl=qubit_bit(n, c), iarg=c - q + 1, p=[0.0, eps[i]])
            i += 1
    assert i == len(eps)
    for q in range(n // 2):
        g.add(KIND_SWAP, q, target2=n - 1 - q)
    return g


def brickwork_circuit(n: int, depth: int, seed: int) -> GateList:
    """Brickwork random circuit: each layer applies a Haar SU(2) (raw Gaussian
    quaternion, normalised by the consumer) on every qubit, then CNOTs with the
    lower-numbered qubit as control: pairs (2j, 2j+1) in even layers and
    (2j+1, 2j+2) in odd layers."""
    rng = np.random.default_rng(seed)
    g = GateList()
    for layer in range(depth):
        quats = rng.standard_normal((n, 4))
        for q in range(n):
            g.add(KIND_SU2, q, p=list(quats[q]))
        first = 0 if layer % 2 == 0 else 1
        for c in range(first, n - 1, 2):
            g.add(KIND_X, c + 1, ctrl=qubit_bit(n, c))
    return g


def random_gate_mix(n: int, count: int, seed: int, max_ctrl: int = 3) -> GateList:
    """A random mix of every gate kind with random controls (test workload)."""
    rng = np.random.default_rng(seed)
    g = GateList()
    for _ in range(count):
        kind = int(rng.integers(0, 9))
        t = int(rng.integers(0, n))
        others = [q for q in range(n) if q != t]
        nc = int(rng.integers(0, min(max_ctrl, len(others)) + 1)) if others else 0
        cq = list(rng.choice(others, size=nc, replace=False)) if nc else []
        ctrl = 0
        for c in cq:
            ctrl |= qubit_bit(n, int(c))
        if kind == KIND_SWAP:
            if n < 2:
                continue
            t2 = int(rng.choice(others))
            g.add(KIND_SWAP, t, target2=t2)
        elif kind == KIND_U:
            g.add(KIND_U, t, ctrl=ctrl, p=random_unitary_params(rng))
        elif kind in (KIND_H, KIND_X):
            p = [0.0, 0.0] if rng.random() < 0.5 else list(rng.standard_normal(2) * 0.1)
            g.add(kind, t, ctrl=ctrl, p=p)
        elif kind == KIND_Y:
            g.add(KIND_Y, t, ctrl=ctrl)
        elif kind == KIND_Z:
            p = [0.0, 0.0] if rng.random() < 0.5 else [0.0, float(rng.standard_normal() * 0.1)]
            g.add(KIND_Z, t, ctrl=ctrl, p=p)
        elif kind == KIND_RK:
            g.add(KIND_RK, t, ctrl=ctrl, iarg=int(rng.integers(1, 12)), p=[0.0, 0.0])
        elif kind == KIND_ROT:
            g.add(KIND_ROT, t, ctrl=ctrl, p=list(rng.uniform(-math.pi, math.pi, 2)))
        else:
            g.add(KIND_SU2, t, ctrl=ctrl, p=list(rng.standard_normal(4)))
    return g


def shor_draws(N: int, m: int, seed: int, iters: int):
    """Random choices of repeated runs of Shor's algorithm on N: per run i,
    x[i] uniform in [1, N-1] (step 1), a_star[i] uniform in [0, 2^m) (the
    first-register measurement is the value x^a_star mod N of a uniform a,
    which has the same law), u[i] uniform in [0, 1) (the measurement of the
    second register)."""
    rng = np.random.default_rng(seed)
    x = rng.integers(1, N, size=iters, dtype=np.int64)
    a = rng.integers(0, 1 << m, size=iters, dtype=np.int64)
    u = rng.random(iters)
    return x, a, u


def qft_register_noise(n: int) -> GateList:
    """The gates of qft_circuit(n, swaps=False) (the output is in bit-reversed
    order), with an explicit identity on every qubit after each controlled
    R_k: the points at which the QFT experiment on Shor's register
    depolarizes the whole register."""
    ident = [1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0]
    g = GateList()
    for q in range(n):
        g.add(KIND_H, q)
        for c in range(q + 1, n):
            g.add(KIND_RK, q, ctrl=qubit_bit(n, c), iarg=c - q + 1)
            for t in range(n):
                g.add(KIND_U, t, p=ident)
    return g


def bit_reverse(v: int, n: int) -> int:
    """v with its n low bits in reverse order."""
    r = 0
    for _ in range(n):
        r = (r << 1) | (v & 1)
        v >>= 1
    return r


def grover_iteration_noise_sites(n: int, marked: int) -> GateList:
    """grover_iteration followed by an explicit identity on every qubit: the
    points at which the Grover robustness study depolarizes each qubit once
    per G-iteration."""
    g = GateList()
    g.extend(grover_iteration(n, marked))
    ident = [1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0]
    for t in range(n):
        g.add(KIND_U, t, p=ident)
    return g
