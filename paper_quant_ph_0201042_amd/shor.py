"""Shor's factoring algorithm as sec. 5.1 runs it (sv_shor_* in
include/sv.h): classical modular exponentiation, QFT and measurement on the
register, classical steps 4-5 with the four improvements.  Argument
marshalling only."""

from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import check

FAIL, PLAIN, NEIGHBOR, GCD, SMALL, LCM, GCDX = -1, 0, 1, 2, 3, 4, 5
STAGE_NAMES = {FAIL: "fail", PLAIN: "plain", NEIGHBOR: "neighbor", GCD: "gcd", SMALL: "small_factor", LCM: "lcm",
               GCDX: "gcd_x"}
IMPROVED = 1


class Outcome(ctypes.Structure):
    _fields_ = [("factor", ctypes.c_uint64), ("r", ctypes.c_uint64), ("stage", ctypes.c_int32),
                ("checks", (ctypes.c_int32 * 2) * 4)]

    def checks_list(self):
        return [[self.checks[i][0], self.checks[i][1]] for i in range(4)]


class Result(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("factor", ctypes.c_uint64), ("stage", ctypes.c_int32),
                ("checks", (ctypes.c_int32 * 2) * 4)]

    def checks_list(self):
        return [[self.checks[i][0], self.checks[i][1]] for i in range(4)]


def register_qubits(N: int) -> int:
    """2l, l the bit length of N."""
    return 2 * int(N).bit_length()


def classical(N: int, x: int, y: int, m: int, improved: bool = False, r_prev: int = 0) -> Outcome:
    """Steps 4-5 for one measured y of an m-qubit register (host code)."""
    out = Outcome()
    check(_lib.load().sv_shor_classical(int(N), int(x), int(y), int(m), IMPROVED if improved else 0, int(r_prev),
                                        ctypes.byref(out)), "sv_shor_classical")
    return out


def factor(state, N: int, x, a_star, u, improved: bool = False):
    """Repeats steps 1-5 on state (2l qubits) with the given random choices
    per run until a factor is found; returns (Result, y per run)."""
    xs = np.ascontiguousarray(x, dtype=np.uint64)
    a = np.ascontiguousarray(a_star, dtype=np.uint64)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    if not (len(xs) == len(a) == len(uu)):
        raise ValueError("x, a_star and u need one entry per run")
    ys = np.zeros(len(xs), dtype=np.uint64)
    res = Result()
    state._bind_stream()
    V = ctypes.c_void_p
    check(_lib.load().sv_shor_factor(state.handle, int(N), xs.ctypes.data_as(V), a.ctypes.data_as(V),
                                     uu.ctypes.data_as(V), len(xs), IMPROVED if improved else 0, ys.ctypes.data_as(V),
                                     ctypes.byref(res)), "sv_shor_factor")
    return res, ys
