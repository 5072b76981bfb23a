"""Autotuned tile and fusion widths: runs the library's tuner (sv_tune_fused,
svb_tune_group) on a workload and keeps the chosen values in a small JSON
file, keyed by the device architecture and the workload's shape (qubits,
element type and the gate list's kinds, targets and controls, not its
angles), so later runs of the same workload start from them.  The search and
the timing run in the library; this module marshals arguments and reads and
writes the file."""

from __future__ import annotations

import ctypes
import hashlib
import json
import os

import numpy as np

from . import _lib
from ._lib import TuneResult, check

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")
ARCH = "gfx950"


def workload_key(n: int, dtype: str, gates: np.ndarray, extra: str = "") -> str:
    """Key of a workload's shape: n, dtype and the structure of its gates."""
    g = np.ascontiguousarray(gates)
    h = hashlib.sha256()
    h.update(("%s|%d|%s|%s|" % (ARCH, n, dtype, extra)).encode())
    for f in ("kind", "target", "target2", "ctrl"):
        h.update(np.ascontiguousarray(g[f]).tobytes())
    return "%s:n%d:%s:%s" % (ARCH, n, dtype, h.hexdigest()[:16])


def _result(r: TuneResult) -> dict:
    keys = [r.key[i].value.decode() for i in range(r.nkeys)]
    return {"keys": keys, "start": {k: int(r.start[i]) for i, k in enumerate(keys)},
            "best": {k: int(r.best[i]) for i, k in enumerate(keys)}, "start_ms": r.start_ms, "best_ms": r.best_ms,
            "tried": int(r.tried)}


def tune_fused(state, gates: np.ndarray, reps: int = 3) -> dict:
    """Searches the fused-pass knobs for running gates on state (its
    contents are overwritten) and leaves the fastest values set."""
    g = np.ascontiguousarray(gates)
    r = TuneResult()
    state._bind_stream()
    check(_lib.load().sv_tune_fused(state.handle, g.ctypes.data_as(ctypes.c_void_p), len(g), int(reps),
                                    ctypes.byref(r)), "sv_tune_fused")
    return _result(r)


def tune_group(batch, init: np.ndarray, iteration: np.ndarray, iters: int, reps: int = 2) -> dict:
    """Searches the registers per launch of batch.run_noisy for this program
    and leaves the fastest set on the batch."""
    gi, gt = np.ascontiguousarray(init), np.ascontiguousarray(iteration)
    r = TuneResult()
    check(_lib.load().svb_tune_group(batch._h, gi.ctypes.data_as(ctypes.c_void_p), len(gi),
                                     gt.ctypes.data_as(ctypes.c_void_p), len(gt), int(iters), int(reps),
                                     ctypes.byref(r)), "svb_tune_group")
    return _result(r)


def load(path: str = CACHE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save(key: str, result: dict, path: str = CACHE, note: str = "") -> None:
    data = load(path)
    data[key] = {"best": result["best"], "start": result["start"], "start_ms": result["start_ms"],
                 "best_ms": result["best_ms"], "tried": result["tried"], "note": note}
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
        f.write("\n")


def apply(key: str, path: str = CACHE, batch=None):
    """Sets the values stored for key (engine keys through sv_config_set,
    "svb_group" on the given batch); returns them, or None if the file has
    no entry for key."""
    from .state import config_set

    ent = load(path).get(key)
    if ent is None:
        return None
    for k, v in ent["best"].items():
        if k == "svb_group":
            if batch is not None:
                batch.set_group(int(v))
        else:
            config_set(k, int(v))
    return dict(ent["best"])
