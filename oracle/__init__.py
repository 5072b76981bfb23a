"""Plain single-threaded FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never calls it and shares no code
with it.  The arithmetic lives in ``sv_oracle.c`` (plain C, FP64, built with
``-ffp-contract=off`` and no fast-math); this module only marshals numpy
arrays into it and builds it with gcc when the shared object is missing or
older than its source.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sv_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GCC_FLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (seconds)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, u64, dbl = ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        sig = {
            "orc_gate_matrix": (i32, [i32, i32, P, P]),
            "orc_gate_dmatrix": (i32, [i32, i32, P, i32, P]),
            "orc_apply_ctrl": (None, [P, i32, u64, i32, P]),
            "orc_apply_1q": (None, [P, i32, i32, P]),
            "orc_apply_ctrl_derivative": (None, [P, i32, u64, i32, P]),
            "orc_swap": (None, [P, i32, i32, i32]),
            "orc_apply_kq": (i32, [P, i32, i32, P, P]),
            "orc_prob": (dbl, [P, i32, u64, u64]),
            "orc_inner": (None, [P, P, i32, P]),
            "orc_measure": (u64, [P, i32, dbl]),
            "orc_collapse": (dbl, [P, i32, u64, u64]),
            "orc_run": (i32, [P, i32, P, i64]),
            "orc_apply_gate_inverse": (i32, [P, i32, P]),
            "orc_philox4x32_10": (None, [P, P, P]),
            "orc_pauli_threshold": (ctypes.c_uint32, [dbl]),
            "orc_noisy_grover_traj": (dbl, [i32, u64, i32, dbl, dbl, u64, u64, P, i64, P, i64, P]),
            "orc_adjoint": (i32, [P, P, i32, P, i64, P, P, P]),
            "orc_dft_element": (None, [P, i32, u64, P]),
            "orc_noisy_traj_state": (None, [P, i32, i32, dbl, dbl, u64, u64, P, i64, P, i64, ctypes.c_uint32]),
            "orc_modpow": (u64, [u64, u64, u64]),
            "orc_shor_state": (u64, [P, i32, u64, u64, u64]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _state(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a


def _n_of(a: np.ndarray) -> int:
    n = int(a.size).bit_length() - 1
    if a.size != 1 << n:
        raise ValueError("state length must be a power of two")
    return n


def _mat(U) -> np.ndarray:
    U = np.asarray(U)
    if U.dtype.kind == "c" or U.size == 4:
        U = np.ascontiguousarray(U.astype(np.complex128).reshape(2, 2)).view(np.float64).reshape(8)
    return np.ascontiguousarray(U, dtype=np.float64).reshape(8)


# ---------------------------------------------------------------- API


def zero_state(n: int) -> np.ndarray:
    a = np.zeros(1 << n, dtype=np.complex128)
    a[0] = 1.0
    return a


def gate_matrix(kind: int, iarg: int = 0, p=None) -> np.ndarray:
    pp = np.zeros(8, dtype=np.float64)
    if p is not None:
        pp[: len(p)] = p
    U = np.zeros(8, dtype=np.float64)
    if lib().orc_gate_matrix(kind, iarg, _ptr(pp), _ptr(U)):
        raise ValueError("bad gate kind/argument")
    return U.view(np.complex128).reshape(2, 2).copy()


def gate_dmatrix(kind: int, iarg: int, p, which: int) -> np.ndarray:
    pp = np.zeros(8, dtype=np.float64)
    pp[: len(p)] = p
    D = np.zeros(8, dtype=np.float64)
    if lib().orc_gate_dmatrix(kind, iarg, _ptr(pp), which, _ptr(D)):
        raise ValueError("gate has no such parameter")
    return D.view(np.complex128).reshape(2, 2).copy()


def apply_1q(a, q: int, U) -> np.ndarray:
    a = _state(a).copy()
    lib().orc_apply_1q(_ptr(a), _n_of(a), q, _ptr(_mat(U)))
    return a


def apply_ctrl(a, ctrl_mask: int, q: int, U) -> np.ndarray:
    a = _state(a).copy()
    lib().orc_apply_ctrl(_ptr(a), _n_of(a), ctrl_mask, q, _ptr(_mat(U)))
    return a


def swap(a, q1: int, q2: int) -> np.ndarray:
    a = _state(a).copy()
    lib().orc_swap(_ptr(a), _n_of(a), q1, q2)
    return a


def apply_kq(a, qubits, M) -> np.ndarray:
    a = _state(a).copy()
    k = len(qubits)
    qs = np.ascontiguousarray(qubits, dtype=np.int32)
    Mf = np.ascontiguousarray(np.asarray(M, dtype=np.complex128).reshape(1 << k, 1 << k))
    if lib().orc_apply_kq(_ptr(a), _n_of(a), k, _ptr(qs), _ptr(Mf)):
        raise ValueError("bad k")
    return a


def prob(a, mask: int = 0, value: int = 0) -> float:
    a = _state(a)
    return float(lib().orc_prob(_ptr(a), _n_of(a), mask, value))


def inner(a, b) -> complex:
    a, b = _state(a), _state(b)
    out = np.zeros(2)
    lib().orc_inner(_ptr(a), _ptr(b), _n_of(a), _ptr(out))
    return complex(out[0], out[1])


def measure(a, r: float) -> int:
    a = _state(a)
    return int(lib().orc_measure(_ptr(a), _n_of(a), r))


def collapse(a, mask: int, value: int):
    """(post-measurement register, probability) for outcome value of the
    qubits in mask; the input is not modified."""
    a = _state(a).copy()
    p = float(lib().orc_collapse(_ptr(a), _n_of(a), int(mask), int(value)))
    return a, p


def dft_element(a, x: int) -> complex:
    """beta_x of the DFT that defines the QFT (one output, O(2^n))."""
    a = _state(a)
    out = np.zeros(2)
    lib().orc_dft_element(_ptr(a), _n_of(a), int(x), _ptr(out))
    return complex(out[0], out[1])


def run(a, gates: np.ndarray) -> np.ndarray:
    """Apply a gate-record array (synth.GATE_DTYPE) to a copy of state a."""
    a = _state(a).copy()
    g = np.ascontiguousarray(gates)
    rc = lib().orc_run(_ptr(a), _n_of(a), _ptr(g), len(g))
    if rc:
        raise ValueError("bad gate at index %d" % (rc - 1))
    return a


def run_inplace(a: np.ndarray, gates: np.ndarray) -> None:
    assert a.dtype == np.complex128 and a.flags.c_contiguous
    g = np.ascontiguousarray(gates)
    rc = lib().orc_run(_ptr(a), _n_of(a), _ptr(g), len(g))
    if rc:
        raise ValueError("bad gate at index %d" % (rc - 1))


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def pauli_threshold(p: float) -> int:
    return int(lib().orc_pauli_threshold(p))


def noisy_grover_traj(n, marked, iters, sigma, p, seed, traj, init_gates, iter_gates, want_state=False):
    """One noisy Grover trajectory; returns |alpha_marked|^2 (and the state)."""
    gi = np.ascontiguousarray(init_gates)
    gt = np.ascontiguousarray(iter_gates)
    out = np.zeros(1 << n, dtype=np.complex128) if want_state else None
    pr = lib().orc_noisy_grover_traj(
        n, marked, iters, sigma, p, seed, traj, _ptr(gi), len(gi), _ptr(gt), len(gt),
        _ptr(out) if out is not None else None,
    )
    return (float(pr), out) if want_state else float(pr)


def noisy_traj_state(a, iters, sigma, p, seed, traj, init_gates, iter_gates, depol_kinds=0xFFFFFFFF) -> np.ndarray:
    """The noisy trajectory of noisy_grover_traj applied to a copy of register
    a; depolarizing follows only gates whose kind bit is set in depol_kinds."""
    a = _state(a).copy()
    gi = np.ascontiguousarray(init_gates)
    gt = np.ascontiguousarray(iter_gates)
    lib().orc_noisy_traj_state(_ptr(a), _n_of(a), iters, sigma, p, seed, traj, _ptr(gi), len(gi), _ptr(gt), len(gt),
                               int(depol_kinds))
    return a


def modpow(x: int, e: int, N: int) -> int:
    return int(lib().orc_modpow(x, e, N))


def shor_state(m: int, N: int, x: int, v: int):
    """(register of m qubits after the classical modular exponentiation and a
    first-register outcome v, number of a with x^a mod N = v)."""
    if not (1 <= N < 1 << 32):
        raise ValueError("N must be in [1, 2^32)")
    a = np.zeros(1 << m, dtype=np.complex128)
    c = int(lib().orc_shor_state(_ptr(a), m, N, x, v))
    return a, c


def adjoint(psi0, phi, gates: np.ndarray, dparam):
    """Adjoint gradient of 1 - |<phi|U(eps) psi0>|^2 per gate deviation.

    Returns (grad[ng], A = <phi|psi_L>, psi_L)."""
    psi = run(psi0, gates)
    psiL = psi.copy()
    phi = _state(phi)
    g = np.ascontiguousarray(gates)
    dp = np.ascontiguousarray(dparam, dtype=np.int32)
    grad = np.zeros(len(g))
    A = np.zeros(2)
    rc = lib().orc_adjoint(_ptr(psi), _ptr(phi), _n_of(psi), _ptr(g), len(g), _ptr(dp), _ptr(grad), _ptr(A))
    if rc:
        raise ValueError("bad gate at index %d" % (rc - 1))
    return grad, complex(A[0], A[1]), psiL
