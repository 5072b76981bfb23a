"""Python handle over a batch of noisy-trajectory registers (svb_* in
include/sv.h).  Argument marshalling only."""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import SV_C64, SV_C128, check

_CODE = {"c64": SV_C64, "c128": SV_C128}
_NP = {"c64": np.complex64, "c128": np.complex128}


class Batch:
    """B registers of n qubits (c64 or c128) for noisy trajectories."""

    def __init__(self, n: int, batch: int, dtype: str = "c64"):
        if dtype not in _CODE:
            raise ValueError("dtype must be 'c64' or 'c128'")
        self.n, self.B, self.dtype = int(n), int(batch), dtype
        self._h = ctypes.c_void_p()
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        check(_lib.load().svb_create(self.n, self.B, _CODE[dtype], stream, ctypes.byref(self._h)), "svb_create")

    def close(self):
        if self._h:
            _lib.load().svb_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_start(self, keep: bool) -> None:
        """keep=True: later runs start from the registers' current contents
        (written through register()); False: from |0...0>."""
        check(_lib.load().svb_set_start(self._h, 1 if keep else 0), "svb_set_start")

    def set_noise_kinds(self, kinds_mask: int) -> None:
        """Depolarizing only after gates whose kind bit is set."""
        check(_lib.load().svb_set_noise_kinds(self._h, int(kinds_mask) & 0xFFFFFFFF), "svb_set_noise_kinds")

    def register(self, reg: int):
        """A State viewing register reg in place (valid while the batch lives)."""
        from .state import State

        ptr = ctypes.c_void_p()
        check(_lib.load().svb_state(self._h, int(reg), ctypes.byref(ptr)), "svb_state")
        return State(self.n, self.dtype, _ptr=ptr.value, _owner=self)

    def set_group(self, regs_per_launch: int) -> None:
        check(_lib.load().svb_set_group(self._h, int(regs_per_launch)), "svb_set_group")

    def run_noisy(self, init: np.ndarray, iteration: np.ndarray, iters: int, sigma: float, p: float, seed: int,
                  traj_offset: int = 0, target: int = 0):
        """Returns (prob[B], norm2[B]) as float64 arrays."""
        gi = np.ascontiguousarray(init)
        gt = np.ascontiguousarray(iteration)
        prob = np.zeros(self.B)
        nrm = np.zeros(self.B)
        rc = _lib.load().svb_run_noisy(self._h, gi.ctypes.data_as(ctypes.c_void_p), len(gi),
                                       gt.ctypes.data_as(ctypes.c_void_p), len(gt), int(iters), float(sigma),
                                       float(p), int(seed), int(traj_offset), int(target),
                                       prob.ctypes.data_as(ctypes.c_void_p), nrm.ctypes.data_as(ctypes.c_void_p))
        check(rc, "svb_run_noisy")
        return prob, nrm

    def fidelity(self, other: "Batch"):
        """(fid[B], overlap[B] complex): per register |<self_r|other_r>|^2 /
        (|self_r|^2 |other_r|^2) and <self_r|other_r>, one launch."""
        fid = np.zeros(self.B)
        ov = np.zeros(2 * self.B)
        check(_lib.load().svb_fidelity(self._h, other._h, fid.ctypes.data_as(ctypes.c_void_p),
                                       ov.ctypes.data_as(ctypes.c_void_p)), "svb_fidelity")
        return fid, ov.view(np.complex128)

    def measure(self, draws) -> np.ndarray:
        """Per register, the basis index sampled with draw r[reg] (sec. 2.2.3);
        registers unchanged."""
        r = np.ascontiguousarray(draws, dtype=np.float64)
        if r.shape != (self.B,):
            raise ValueError("one draw per register")
        idx = np.zeros(self.B, dtype=np.uint64)
        check(_lib.load().svb_measure(self._h, r.ctypes.data_as(ctypes.c_void_p), idx.ctypes.data_as(ctypes.c_void_p)),
              "svb_measure")
        return idx

    def last_run_ms(self) -> float:
        v = ctypes.c_double()
        check(_lib.load().svb_last_run_ms(self._h, ctypes.byref(v)), "svb_last_run_ms")
        return v.value

    def state(self, reg: int) -> np.ndarray:
        """Copy of register reg (host)."""
        ptr = ctypes.c_void_p()
        check(_lib.load().svb_state(self._h, int(reg), ctypes.byref(ptr)), "svb_state")
        nb = (1 << self.n) * (16 if self.dtype == "c128" else 8)
        out = np.empty(1 << self.n, dtype=_NP[self.dtype])
        torch.cuda.synchronize()
        hip = ctypes.CDLL("libamdhip64.so")
        hip.hipMemcpy.restype = ctypes.c_int
        hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        rc = hip.hipMemcpy(out.ctypes.data_as(ctypes.c_void_p), ptr, nb, 2)  # device to host
        if rc != 0:
            raise RuntimeError("hipMemcpy failed (%d)" % rc)
        return out


def plan(n: int, dtype: str, init: np.ndarray, iteration: np.ndarray, iters: int):
    """(passes, matrix slots) of the program run_noisy builds (host only)."""
    gi, gt = np.ascontiguousarray(init), np.ascontiguousarray(iteration)
    npass, nslot = ctypes.c_int64(), ctypes.c_int64()
    check(_lib.load().svb_plan(int(n), _CODE[dtype], gi.ctypes.data_as(ctypes.c_void_p), len(gi),
                               gt.ctypes.data_as(ctypes.c_void_p), len(gt), int(iters), ctypes.byref(npass),
                               ctypes.byref(nslot)), "svb_plan")
    return npass.value, nslot.value


def jit_source(n: int, dtype: str, init: np.ndarray, iteration: np.ndarray, iters: int, pass_index: int) -> str:
    """Source of the specialised kernel of one pass of run_noisy's program."""
    gi, gt = np.ascontiguousarray(init), np.ascontiguousarray(iteration)
    L = _lib.load()
    ln = ctypes.c_int64()
    args = (int(n), _CODE[dtype], gi.ctypes.data_as(ctypes.c_void_p), len(gi), gt.ctypes.data_as(ctypes.c_void_p),
            len(gt), int(iters), int(pass_index))
    check(L.svb_jit_source(*args, None, 0, ctypes.byref(ln)), "svb_jit_source")
    buf = ctypes.create_string_buffer(ln.value + 1)
    check(L.svb_jit_source(*args, buf, ln.value + 1, ctypes.byref(ln)), "svb_jit_source")
    return buf.value.decode()


def trajectory_gates(n: int, init: np.ndarray, iteration: np.ndarray, iters: int, sigma: float, p: float, seed: int,
                     traj: int, depolarize_kinds: int = 0xFFFFFFFF) -> np.ndarray:
    """Trajectory traj of Batch.run_noisy's error model as an explicit gate
    list for the per-gate path (svb_trajectory_gates)."""
    gi = np.ascontiguousarray(init)
    gt = np.ascontiguousarray(iteration)
    L = _lib.load()
    cnt = ctypes.c_int64()
    args = (int(iters), float(sigma), float(p), int(seed), int(traj), int(depolarize_kinds) & 0xFFFFFFFF)
    check(L.svb_trajectory_gates(int(n), gi.ctypes.data_as(ctypes.c_void_p), len(gi), gt.ctypes.data_as(ctypes.c_void_p),
                                 len(gt), *args, None, 0, ctypes.byref(cnt)), "svb_trajectory_gates")
    out = np.zeros(cnt.value, dtype=gi.dtype if gi.dtype.itemsize == 88 else gt.dtype)
    check(L.svb_trajectory_gates(int(n), gi.ctypes.data_as(ctypes.c_void_p), len(gi), gt.ctypes.data_as(ctypes.c_void_p),
                                 len(gt), *args, out.ctypes.data_as(ctypes.c_void_p), len(out), ctypes.byref(cnt)),
          "svb_trajectory_gates")
    return out
