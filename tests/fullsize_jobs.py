"""Oracle runs that the full-size GPU parity tests compare against.

Each job is one plain run of the CPU oracle (single-threaded C, FP64) on a
register of the benchmark's size.  They take between one and three minutes,
so they start in host threads as soon as the GPU tests that need them are
collected (ctypes releases the GIL during the oracle call) and run while
other GPU tests use the device."""

from __future__ import annotations

import concurrent.futures as cf
import threading

import numpy as np

import synth

_lock = threading.Lock()
_pool = None
_futures = {}

BRICK30_LAYERS = 2


def brick30_gates() -> np.ndarray:
    """The first two layers of the n = 30, depth-20 brickwork circuit (seed
    0): 60 Haar SU(2) gates and 29 CNOTs."""
    n = 30
    full = synth.brickwork_circuit(n, 20, seed=0).array()
    per_layer = [n + len(range(0 if l % 2 == 0 else 1, n - 1, 2)) for l in range(BRICK30_LAYERS)]
    return full[: sum(per_layer)]


def _brick30():
    import oracle

    return oracle.run(oracle.zero_state(30), brick30_gates())


def _brick26():
    import oracle

    return oracle.run(oracle.zero_state(26), synth.brickwork_circuit(26, 20, seed=0).array())


def _qft28():
    import oracle

    return oracle.run(synth.random_state(28, 0), synth.qft_circuit(28).array())


JOBS = {"brick30": _brick30, "brick26": _brick26, "qft28": _qft28}


def start() -> None:
    """Submits every job once (idempotent)."""
    global _pool
    with _lock:
        if _pool is None:
            _pool = cf.ThreadPoolExecutor(max_workers=len(JOBS), thread_name_prefix="oracle")
        for name, fn in JOBS.items():
            if name not in _futures:
                _futures[name] = _pool.submit(fn)


def result(name: str) -> np.ndarray:
    start()
    return _futures[name].result()


def release(name: str) -> None:
    """Drops a finished job's state (they are 1 to 16 GiB)."""
    with _lock:
        f = _futures.get(name)
        if f is not None and f.done():
            _futures[name] = _Done()


class _Done:
    def done(self):
        return True

    def result(self):
        raise RuntimeError("oracle result already released")
