"""Python handle over a device state vector.

Device memory comes from PyTorch (a contiguous complex tensor on the current
GPU) and work is enqueued on torch's current stream; every operation is a call
into libsv.so.  This module only marshals arguments."""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import SV_C64, SV_C128, check

_DT = {"c64": (SV_C64, torch.complex64, np.complex64), "c128": (SV_C128, torch.complex128, np.complex128)}


def _mat8(U) -> np.ndarray:
    U = np.asarray(U)
    if U.dtype.kind == "c" or U.size == 4:
        U = np.ascontiguousarray(U.astype(np.complex128).reshape(2, 2)).view(np.float64).reshape(8)
    return np.ascontiguousarray(U, dtype=np.float64).reshape(8)


def _stream_ptr():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class State:
    """An n-qubit register in HBM (qubit 0 = most significant index bit)."""

    def __init__(self, n: int, dtype: str = "c128", tensor: torch.Tensor | None = None, *, _ptr=None, _owner=None):
        if dtype not in _DT:
            raise ValueError("dtype must be 'c64' or 'c128'")
        self.n = int(n)
        self.dtype = dtype
        code, tdt, _ = _DT[dtype]
        if _ptr is not None:
            # a view of device memory owned by _owner (a batch register)
            self.tensor = None
            self._owner = _owner
            self._addr = int(_ptr)
        else:
            if tensor is None:
                tensor = torch.empty(1 << self.n, dtype=tdt, device="cuda")
            if tensor.dtype != tdt or not tensor.is_contiguous() or tensor.numel() != (1 << self.n):
                raise ValueError("tensor must be a contiguous %s vector of 2^n elements" % tdt)
            self.tensor = tensor
            self._addr = tensor.data_ptr()
        self._h = ctypes.c_void_p()
        L = _lib.load()
        check(L.sv_wrap(self.n, code, ctypes.c_void_p(self._addr), _stream_ptr(), ctypes.byref(self._h)), "sv_wrap")

    # -- lifetime
    def close(self):
        if self._h:
            _lib.load().sv_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def _bind_stream(self):
        _lib.load().sv_set_stream(self._h, _stream_ptr())

    # -- set-up
    def reset(self, basis_index: int = 0) -> "State":
        self._bind_stream()
        check(_lib.load().sv_reset(self._h, int(basis_index)), "sv_reset")
        return self

    def load(self, amps) -> "State":
        a = np.ascontiguousarray(amps, dtype=_DT[self.dtype][2])
        if a.size != 1 << self.n:
            raise ValueError("need 2^n amplitudes")
        self._bind_stream()
        check(_lib.load().sv_load(self._h, a.ctypes.data_as(ctypes.c_void_p), 0), "sv_load")
        return self

    def numpy(self) -> np.ndarray:
        out = np.empty(1 << self.n, dtype=_DT[self.dtype][2])
        self._bind_stream()
        check(_lib.load().sv_store(self._h, out.ctypes.data_as(ctypes.c_void_p), 0), "sv_store")
        return out

    # -- evolution
    def apply_1q(self, q: int, U) -> "State":
        m = _mat8(U)
        self._bind_stream()
        check(_lib.load().sv_apply_1q(self._h, int(q), m.ctypes.data_as(ctypes.c_void_p)), "sv_apply_1q")
        return self

    def apply_ctrl(self, ctrl_mask: int, q: int, U) -> "State":
        m = _mat8(U)
        self._bind_stream()
        check(_lib.load().sv_apply_ctrl(self._h, int(ctrl_mask), int(q), m.ctypes.data_as(ctypes.c_void_p)),
              "sv_apply_ctrl")
        return self

    def apply_block(self, qubits, M) -> "State":
        """Dense 2^k x 2^k block on the given qubits (qubits[0] = MSB of the
        block index)."""
        k = len(qubits)
        qs = np.ascontiguousarray(qubits, dtype=np.int32)
        Mf = np.ascontiguousarray(np.asarray(M, dtype=np.complex128).reshape(1 << k, 1 << k))
        self._bind_stream()
        check(_lib.load().sv_apply_fused(self._h, k, qs.ctypes.data_as(ctypes.c_void_p),
                                         Mf.ctypes.data_as(ctypes.c_void_p)), "sv_apply_fused")
        return self

    def swap(self, q1: int, q2: int) -> "State":
        self._bind_stream()
        check(_lib.load().sv_apply_swap(self._h, int(q1), int(q2)), "sv_apply_swap")
        return self

    def run(self, gates: np.ndarray, fused: bool = False, profile: bool = False, blocks: bool = False) -> "State":
        """Apply a gate-record array: per gate (default), as fused LDS passes
        (fused=True) or as dense blocks (blocks=True)."""
        g = np.ascontiguousarray(gates)
        if g.dtype.itemsize != 88:
            raise ValueError("gate records must be 88 bytes")
        bad = ctypes.c_int64(-1)
        flags = (_lib.SV_RUN_FUSED if fused else _lib.SV_RUN_PER_GATE) | (_lib.SV_RUN_PROFILE if profile else 0)
        if blocks:
            flags |= _lib.SV_RUN_BLOCKS
        self._bind_stream()
        rc = _lib.load().sv_run(self._h, g.ctypes.data_as(ctypes.c_void_p), len(g), flags, ctypes.byref(bad))
        check(rc, "sv_run (gate %d)" % bad.value if bad.value >= 0 else "sv_run")
        return self

    def qft(self, q0: int = 0, m: int | None = None, inverse: bool = False, bitrev: bool = False) -> "State":
        """QFT (or its inverse) on qubits q0 .. q0 + m - 1 (default: all);
        bitrev leaves out the final bit reversal."""
        if m is None:
            m = self.n - q0
        self._bind_stream()
        flags = (1 if inverse else 0) | (2 if bitrev else 0)
        check(_lib.load().sv_qft(self._h, int(q0), int(m), flags), "sv_qft")
        return self

    def shor_prepare(self, N: int, x: int, a_star: int) -> int:
        """Register left by step 3(c) of Shor's algorithm with first-register
        outcome x^a_star mod N (sec. 5.1); returns the number of a with
        x^a mod N equal to it."""
        c = ctypes.c_uint64()
        self._bind_stream()
        check(_lib.load().sv_shor_prepare(self._h, int(N), int(x), int(a_star), ctypes.byref(c)), "sv_shor_prepare")
        return c.value

    def run_profile(self):
        """(ms[], kind[]) per launched step of the last profiled run."""
        L = _lib.load()
        cnt = ctypes.c_int64()
        check(L.sv_run_profile(self._h, None, None, 0, ctypes.byref(cnt)), "sv_run_profile")
        ms = np.zeros(max(cnt.value, 1))
        kind = np.zeros(max(cnt.value, 1), dtype=np.int32)
        check(L.sv_run_profile(self._h, ms.ctypes.data_as(ctypes.c_void_p), kind.ctypes.data_as(ctypes.c_void_p),
                               cnt.value, ctypes.byref(cnt)), "sv_run_profile")
        return ms[: cnt.value], kind[: cnt.value]

    # -- reductions
    def prob(self, mask: int = 0, value: int = 0) -> float:
        out = ctypes.c_double()
        self._bind_stream()
        check(_lib.load().sv_prob(self._h, int(mask), int(value), ctypes.byref(out)), "sv_prob")
        return out.value

    def norm2(self) -> float:
        return self.prob(0, 0)

    # -- measurement
    def measure(self, r: float) -> int:
        """Basis index i with sum_{j<i}|a_j|^2 <= r < sum_{j<=i}|a_j|^2; the
        register is left unchanged."""
        out = ctypes.c_uint64()
        self._bind_stream()
        check(_lib.load().sv_measure(self._h, float(r), ctypes.byref(out)), "sv_measure")
        return out.value

    def collapse(self, mask: int, value: int) -> float:
        """Project onto (j & mask) == value and renormalise; returns the
        outcome's probability."""
        p = ctypes.c_double()
        self._bind_stream()
        check(_lib.load().sv_collapse(self._h, int(mask), int(value), ctypes.byref(p)), "sv_collapse")
        return p.value

    def measure_qubits(self, mask: int, r: float):
        """Measure the qubits of a basis-index mask with the draw r: returns
        (value, probability) and leaves the collapsed register."""
        v = self.measure(r) & int(mask)
        return v, self.collapse(mask, v)

    def inner(self, other: "State") -> complex:
        """<self|other> accumulated in FP64."""
        out = np.zeros(2)
        self._bind_stream()
        other._bind_stream()
        check(_lib.load().sv_inner(self._h, other._h, out.ctypes.data_as(ctypes.c_void_p)), "sv_inner")
        return complex(out[0], out[1])

    def fidelity(self, other: "State") -> float:
        """|<self|other>|^2 / (<self|self> <other|other>), FP64."""
        out = ctypes.c_double()
        self._bind_stream()
        other._bind_stream()
        check(_lib.load().sv_fidelity(self._h, other._h, ctypes.byref(out)), "sv_fidelity")
        return out.value

    def copy_from(self, other: "State") -> "State":
        """Device-to-device copy of another state of the same n and dtype."""
        if other.n != self.n or other.dtype != self.dtype:
            raise ValueError("shape/dtype mismatch")
        self._bind_stream()
        check(_lib.load().sv_load(self._h, ctypes.c_void_p(other._addr), 1), "sv_load")
        return self

    def sync(self):
        check(_lib.load().sv_sync(self._h), "sv_sync")


def gate_matrix(record) -> np.ndarray:
    """2x2 matrix of one gate record (library-side construction)."""
    r = np.ascontiguousarray(np.asarray(record).reshape(1))
    U = np.zeros(8)
    check(_lib.load().sv_gate_matrix(r.ctypes.data_as(ctypes.c_void_p), U.ctypes.data_as(ctypes.c_void_p)),
          "sv_gate_matrix")
    return U.view(np.complex128).reshape(2, 2).copy()


def plan_fused(n: int, dtype: str, gates: np.ndarray):
    """Host-side fusion plan: (order, pass_of, tile_masks) as numpy arrays."""
    g = np.ascontiguousarray(gates)
    ng = len(g)
    order = np.zeros(max(ng, 1), dtype=np.int64)
    pass_of = np.zeros(max(ng, 1), dtype=np.int32)
    masks = np.zeros(max(ng, 1), dtype=np.uint64)
    npass = ctypes.c_int64()
    check(_lib.load().sv_plan_fused(n, _DT[dtype][0], g.ctypes.data_as(ctypes.c_void_p), ng,
                                    order.ctypes.data_as(ctypes.c_void_p), pass_of.ctypes.data_as(ctypes.c_void_p),
                                    masks.ctypes.data_as(ctypes.c_void_p), ctypes.byref(npass)), "sv_plan_fused")
    return order[:ng], pass_of[:ng], masks[: npass.value]


def config_set(key: str, value: int) -> None:
    check(_lib.load().sv_config_set(key.encode(), int(value)), "sv_config_set(%s)" % key)


def config_get(key: str) -> int:
    v = ctypes.c_int()
    check(_lib.load().sv_config_get(key.encode(), ctypes.byref(v)), "sv_config_get(%s)" % key)
    return v.value


def gate_dmatrix(record, which: int) -> np.ndarray:
    """Derivative of a gate record's matrix w.r.t. its p[which] deviation."""
    r = np.ascontiguousarray(np.asarray(record).reshape(1))
    D = np.zeros(8)
    check(_lib.load().sv_gate_dmatrix(r.ctypes.data_as(ctypes.c_void_p), int(which),
                                      D.ctypes.data_as(ctypes.c_void_p)), "sv_gate_dmatrix")
    return D.view(np.complex128).reshape(2, 2).copy()


def overlap_loss(phi: State, psi: State):
    """(1 - |<phi|psi>|^2, <phi|psi>)."""
    loss = ctypes.c_double()
    A = np.zeros(2)
    phi._bind_stream()
    psi._bind_stream()
    check(_lib.load().sv_overlap_loss(phi._h, psi._h, ctypes.byref(loss), A.ctypes.data_as(ctypes.c_void_p)),
          "sv_overlap_loss")
    return loss.value, complex(A[0], A[1])


def adjoint(psi: State, lam: State, gates: np.ndarray, dparam):
    """Adjoint sweep (sv_adjoint): psi holds psi_L, lam holds phi on entry.
    Returns (grad[ng] float64, A)."""
    g = np.ascontiguousarray(gates)
    dp = np.ascontiguousarray(dparam, dtype=np.int32)
    if len(dp) != len(g):
        raise ValueError("one dparam entry per gate")
    grad = np.zeros(len(g))
    A = np.zeros(2)
    psi._bind_stream()
    lam._bind_stream()
    check(_lib.load().sv_adjoint(psi._h, lam._h, g.ctypes.data_as(ctypes.c_void_p), len(g),
                                 dp.ctypes.data_as(ctypes.c_void_p), grad.ctypes.data_as(ctypes.c_void_p),
                                 A.ctypes.data_as(ctypes.c_void_p)), "sv_adjoint")
    return grad, complex(A[0], A[1])


def plan_blocks(n: int, gates: np.ndarray, kmax: int = 5):
    """Host-side dense-block plan: list of ("block", qubits, M) or ("gate", index)."""
    g = np.ascontiguousarray(gates)
    L = _lib.load()
    nst = ctypes.c_int64()
    check(L.sv_plan_blocks(n, g.ctypes.data_as(ctypes.c_void_p), len(g), kmax, ctypes.byref(nst), None, None, 0),
          "sv_plan_blocks")
    info = np.zeros((max(nst.value, 1), 8), dtype=np.int32)
    msz = 2 << (2 * kmax)
    mats = np.zeros((max(nst.value, 1), msz))
    check(L.sv_plan_blocks(n, g.ctypes.data_as(ctypes.c_void_p), len(g), kmax, ctypes.byref(nst),
                           info.ctypes.data_as(ctypes.c_void_p), mats.ctypes.data_as(ctypes.c_void_p), nst.value),
          "sv_plan_blocks")
    out = []
    for i in range(nst.value):
        if info[i, 0] == 1:
            out.append(("gate", int(info[i, 1])))
        else:
            k = int(info[i, 1])
            D = 1 << k
            M = mats[i, : 2 * D * D].view(np.complex128).reshape(D, D).copy()
            out.append(("block", [int(q) for q in info[i, 2:2 + k]], M))
    return out


def jit_source(n: int, dtype: str, gates: np.ndarray, pass_index: int) -> str:
    """Source of the specialised kernel of one fused pass (host only)."""
    g = np.ascontiguousarray(gates)
    L = _lib.load()
    ln = ctypes.c_int64()
    dt = _DT[dtype][0]
    check(L.sv_jit_source(n, dt, g.ctypes.data_as(ctypes.c_void_p), len(g), pass_index, None, 0, ctypes.byref(ln)),
          "sv_jit_source")
    buf = ctypes.create_string_buffer(ln.value + 1)
    check(L.sv_jit_source(n, dt, g.ctypes.data_as(ctypes.c_void_p), len(g), pass_index, buf, ln.value + 1,
                          ctypes.byref(ln)), "sv_jit_source")
    return buf.value.decode()


def model_fused(n: int, dtype: str, gates: np.ndarray, amps) -> np.ndarray:
    """Host model of the fused engine: the plan and op rewrites sv_run would
    use for an n-qubit register of dtype, applied in FP64 on the host (no
    device).  Returns the evolved copy of amps."""
    g = np.ascontiguousarray(gates)
    a = np.array(amps, dtype=np.complex128, copy=True)
    if a.shape != (1 << n,):
        raise ValueError("amps must hold 2^n values")
    check(_lib.load().sv_model_fused(n, _DT[dtype][0], g.ctypes.data_as(ctypes.c_void_p), len(g),
                                     a.ctypes.data_as(ctypes.c_void_p)), "sv_model_fused")
    return a
