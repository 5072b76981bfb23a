"""Benchmark of the MI355X state-vector gate engine.

One step = the brickwork random circuit of depth 20 on an n=30 register
(every layer: a Haar SU(2) on each of the 30 qubits, then CNOTs on (2j,2j+1)
in even layers and (2j+1,2j+2) in odd layers; 600 one-qubit gates and 290
CNOTs), complex128, applied gate by gate by the HIP kernels from |0...0>,
followed by the FP64 norm reduction.  Inputs are seeded and synthetic.

Metric: gate-amplitude updates per second (a one-qubit gate updates 2^n
amplitudes, a CNOT 2^{n-1}), plus the HBM GB/s of the dominant kernel (the
dense one-qubit pair kernel) against the MI355X peak of 8 TB/s, measured with
HIP events on the stream the kernels are launched on.  The plain CPU oracle
is timed on a bounded sample of the same workload on the host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

PEAK_HBM_GBS = 8000.0
METRIC = "gate-amp updates/s + HBM GB/s at n=30; batched fp32 vs plain fp64 speedup"


def prepared_gates(sv, gl_array, n):
    """(kind, q, ctrl, U[8], amps_updated, is_dominant) per gate; matrices built
    by the library's host-side constructor."""
    import ctypes

    from paper_quant_ph_0201042_amd import _lib

    L = _lib.load()
    out = []
    for rec in gl_array:
        r = np.ascontiguousarray(rec.reshape(1))
        U = np.zeros(8)
        _lib.check(L.sv_gate_matrix(r.ctypes.data_as(ctypes.c_void_p), U.ctypes.data_as(ctypes.c_void_p)))
        q = int(rec["target"])
        ctrl = int(rec["ctrl"])
        nc = bin(ctrl).count("1")
        amps = 1 << (n - nc)
        # dominant kernel: dense pair stream (no controls, target bit >= 6)
        dominant = ctrl == 0 and (n - 1 - q) >= 6 and not (U[2] == 0 and U[3] == 0 and U[4] == 0 and U[5] == 0)
        out.append((q, ctrl, U, amps, dominant))
    return out


def run_step(s, gates, ev_pairs=None):
    s.reset(0)
    for q, ctrl, U, _, dom in gates:
        if ev_pairs is not None and dom:
            e0, e1 = ev_pairs.pop()
            e0.record()
            s.apply_1q(q, U)
            e1.record()
            ev_pairs_done.append((e0, e1))
        elif ctrl:
            s.apply_ctrl(ctrl, q, U)
        else:
            s.apply_1q(q, U)
    return s.norm2()


ev_pairs_done = []


def cpu_baseline(gl_array, n, budget_s=20.0):
    """The plain oracle on the host: the first gates of the same circuit on an
    n-qubit FP64 register, single-threaded, until about budget_s of work."""
    import oracle

    L = oracle.lib()
    a = np.empty(1 << n, dtype=np.complex128)
    a[:] = 0.0  # touch every page (untimed) so the timed gates pay no first-touch faults
    a[0] = 1.0
    ptr = a.ctypes.data
    done_amps = 0
    gates_done = 0
    t0 = time.perf_counter()
    for rec in gl_array:
        one = np.ascontiguousarray(rec.reshape(1))
        rc = L.orc_run(ptr, n, one.ctypes.data, 1)
        assert rc == 0
        done_amps += 1 << (n - bin(int(rec["ctrl"])).count("1"))
        gates_done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {
        "value": done_amps / dt,
        "unit": "gate-amp updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": "first %d gates of the same n=%d brickwork circuit (seed 0), complex128, "
        "single-threaded plain C oracle, %.1f s" % (gates_done, n, dt),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--depth", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the engine has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    import paper_quant_ph_0201042_amd as sv

    n, depth = args.n, args.depth
    gl = synth.brickwork_circuit(n, depth, seed=0).array()
    gates = prepared_gates(sv, gl, n)
    updates_per_step = sum(g[3] for g in gates)
    n_dom = sum(1 for g in gates if g[4])

    s = sv.State(n, "c128")
    for _ in range(args.warmup):
        nrm = run_step(s, gates)
    torch.cuda.synchronize()

    global ev_pairs_done
    ev_pairs_done = []
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(n_dom * args.steps)]
    t0 = time.perf_counter()
    for _ in range(args.steps):
        nrm = run_step(s, gates, evs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = t1 - t0
    if abs(nrm - 1.0) > 1e-10:
        raise RuntimeError("norm drifted: %r" % nrm)

    durs_ms = [e0.elapsed_time(e1) for e0, e1 in ev_pairs_done]
    avg_ms = float(np.mean(durs_ms))
    bytes_per_launch = 2 * (1 << n) * 16
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    step_bytes = 2 * 16 * updates_per_step  # algorithmic: read+write each updated amplitude

    rec = {
        "metric": METRIC,
        "value": updates_per_step * args.steps / dt,
        "unit": "gate-amp updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "brickwork random circuit, n=%d, depth %d, complex128, per-gate kernels" % (n, depth),
            "n": n,
            "depth": depth,
            "gates_per_step": len(gates),
            "seed": 0,
        },
        "hbm_gbps_algorithmic": step_bytes * args.steps / dt / 1e9,
        "roofline": {
            "kernel": "k_pairs<double2> dense one-qubit gate, target bit >= 6",
            "bound": "hbm",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": None,
            "avg_launch_ms": avg_ms,
            "launches": len(durs_ms),
            "bytes_per_launch": bytes_per_launch,
        },
    }
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(gl, n, args.cpu_budget)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
