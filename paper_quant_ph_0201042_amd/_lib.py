"""ctypes loader of libsv.so, the gfx950 HIP library declared in include/sv.h.

There is no fallback: if the library is missing, importing the package raises
so that no caller silently runs anything else."""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsv.so")

SV_OK, SV_EINVAL, SV_ENOMEM, SV_EDEVICE, SV_ENOTSUP = 0, -1, -2, -3, -4
SV_C64, SV_C128 = 8, 16
SV_RUN_PER_GATE, SV_RUN_FUSED, SV_RUN_PROFILE, SV_RUN_BLOCKS = 0, 1, 2, 4

P = ctypes.c_void_p
PP = ctypes.POINTER(ctypes.c_void_p)
i32, i64, u64, dbl = ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double

# name -> (restype, argtypes); every function declared in include/sv.h
SIGNATURES = {
    "sv_strerror": (ctypes.c_char_p, [i32]),
    "sv_last_error": (ctypes.c_char_p, []),
    "sv_create": (i32, [i32, i32, P, PP]),
    "sv_wrap": (i32, [i32, i32, P, P, PP]),
    "sv_destroy": (i32, [P]),
    "sv_set_stream": (i32, [P, P]),
    "sv_reset": (i32, [P, u64]),
    "sv_load": (i32, [P, P, i32]),
    "sv_store": (i32, [P, P, i32]),
    "sv_info": (i32, [P, ctypes.POINTER(i32), ctypes.POINTER(i32), PP]),
    "sv_apply_1q": (i32, [P, i32, P]),
    "sv_apply_ctrl": (i32, [P, u64, i32, P]),
    "sv_apply_swap": (i32, [P, i32, i32]),
    "sv_apply_fused": (i32, [P, i32, P, P]),
    "sv_prob": (i32, [P, u64, u64, ctypes.POINTER(dbl)]),
    "sv_measure": (i32, [P, ctypes.c_double, ctypes.POINTER(u64)]),
    "sv_collapse": (i32, [P, u64, u64, ctypes.POINTER(ctypes.c_double)]),
    "sv_inner": (i32, [P, P, P]),
    "sv_sync": (i32, [P]),
    "sv_fidelity": (i32, [P, P, ctypes.POINTER(dbl)]),
    "sv_overlap_loss": (i32, [P, P, ctypes.POINTER(dbl), P]),
    "sv_gate_dmatrix": (i32, [P, i32, P]),
    "sv_adjoint": (i32, [P, P, P, i64, P, P, P]),
    "sv_gate_matrix": (i32, [P, P]),
    "sv_run": (i32, [P, P, i64, i32, ctypes.POINTER(i64)]),
    "sv_qft": (i32, [P, i32, i32, i32]),
    "sv_qft_plan": (i32, [i32, i32, i32, P, i64, ctypes.POINTER(i64)]),
    "sv_run_profile": (i32, [P, P, P, i64, ctypes.POINTER(i64)]),
    "svb_create": (i32, [i32, i32, i32, P, PP]),
    "svb_destroy": (i32, [P]),
    "svb_set_group": (i32, [P, i32]),
    "svb_state": (i32, [P, i32, PP]),
    "svb_info": (i32, [P, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]),
    "svb_get_group": (i32, [P, ctypes.POINTER(i32)]),
    "svb_run_noisy": (i32, [P, P, i64, P, i64, i32, dbl, dbl, u64, u64, u64, P, P]),
    "svb_last_run_ms": (i32, [P, ctypes.POINTER(dbl)]),
    "svb_set_start": (i32, [P, i32]),
    "svb_set_noise_kinds": (i32, [P, ctypes.c_uint32]),
    "svb_fidelity": (i32, [P, P, P, P]),
    "svb_measure": (i32, [P, P, P]),
    "svb_fidelity_noalloc": (i32, [i32, i32, i32, P, i32, P, P, P, P]),
    "svb_plan": (i32, [i32, i32, P, i64, P, i64, i32, ctypes.POINTER(i64), ctypes.POINTER(i64)]),
    "svb_jit_source": (i32, [i32, i32, P, i64, P, i64, i32, i64, P, i64, ctypes.POINTER(i64)]),
    "svb_trajectory_gates": (i32, [i32, P, i64, P, i64, i32, dbl, dbl, u64, u64, ctypes.c_uint32, P, i64,
                                   ctypes.POINTER(i64)]),
    "sv_shor_prepare": (i32, [P, u64, u64, u64, ctypes.POINTER(u64)]),
    "sv_shor_classical": (i32, [u64, u64, u64, i32, i32, u64, P]),
    "sv_shor_factor": (i32, [P, u64, P, P, P, i64, i32, P, P]),
    "sv_jit_source": (i32, [i32, i32, P, i64, i64, P, i64, ctypes.POINTER(i64)]),
    "sv_model_fused": (i32, [i32, i32, P, i64, P]),
    "sv_plan_blocks": (i32, [i32, P, i64, i32, ctypes.POINTER(i64), P, P, i64]),
    "sv_plan_fused": (i32, [i32, i32, P, i64, P, P, P, ctypes.POINTER(i64)]),
    "sv_config_set": (i32, [ctypes.c_char_p, i32]),
    "sv_config_get": (i32, [ctypes.c_char_p, ctypes.POINTER(i32)]),
    "sv_tune_fused": (i32, [P, P, i64, i32, P]),
    "svb_tune_group": (i32, [P, P, i64, P, i64, i32, i32, P]),
}



class TuneResult(ctypes.Structure):
    """sv_tune_result of include/sv.h."""

    _fields_ = [("nkeys", ctypes.c_int32), ("tried", ctypes.c_int32), ("key", (ctypes.c_char * 24) * 8),
                ("start", ctypes.c_int32 * 8), ("best", ctypes.c_int32 * 8), ("start_ms", ctypes.c_double),
                ("best_ms", ctypes.c_double)]


_lib = None


class SVError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = load().sv_strerror(status).decode()
        detail = load().sv_last_error().decode()
        if status == SV_EDEVICE and detail:
            msg += " [" + detail + "]"
        super().__init__(f"{what}: {msg} ({status})" if what else f"{msg} ({status})")


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                "libsv.so is not built (expected at %s); run __graft_entry__.build() "
                "or python -m paper_quant_ph_0201042_amd.build" % LIB_PATH
            )
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status: int, what: str = "") -> None:
    if status != SV_OK:
        raise SVError(status, what)
