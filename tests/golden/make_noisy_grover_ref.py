"""Writes noisy_grover_n20_oracle.txt: FP64 oracle trajectories of the noisy
Grover search on 20 qubits (804 iterations), the batched workload of the
error-model study (sec. 3.1 depolarizing channel, sec. 3.2 operational error,
robustness of Grover's search in sec. 5.3.1).

Inputs: marked index synth.grover_marked(20, 0); the initial Hadamard
transform and the ancilla-free Grover iteration from synth; Philox seed 0;
the (sigma, p) grid sigma in {1e-3, 5e-3, 1e-2, 5e-2} x p in {1e-5, 1e-4,
1e-3}.  Trajectory ids: 0..255 plus 3584 and 4095 at sigma = 1e-2,
p = 1e-4; 0..7 plus 4095 at every other point.

Every value is computed by the plain C oracle (oracle.noisy_grover_traj, one
trajectory per process, single-threaded); nothing here comes from the GPU
library.  Per trajectory the file keeps |alpha_marked|^2, the squared norm
and the amplitudes at SAMPLE_INDICES (the marked index first), so a GPU
run of the same draws can be compared amplitude by amplitude.

Run from the repository root:
    python tests/golden/make_noisy_grover_ref.py [--procs 6]
Lines are appended as trajectories finish; a rerun skips those present.
"""

from __future__ import annotations

import argparse
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

OUT = os.path.join(HERE, "noisy_grover_n20_oracle.txt")
N_QUBITS = 20
ITERS = 804
SEED = 0
SIGMAS = (1e-3, 5e-3, 1e-2, 5e-2)
PS = (1e-5, 1e-4, 1e-3)
HEADLINE = (1e-2, 1e-4)


def marked() -> int:
    return synth.grover_marked(N_QUBITS, 0)


def sample_indices() -> list:
    rng = np.random.default_rng(20020131)
    rest = [int(v) for v in rng.integers(0, 1 << N_QUBITS, 15)]
    return [marked()] + rest


def jobs() -> list:
    """Every trajectory the file is to hold, in the order they are run: a
    first sample of every grid point comes before the bulk of the headline
    point, so that a partial file already covers the whole grid."""
    head = [(HEADLINE[0], HEADLINE[1], t) for t in range(256)]
    others = [(s, p) for s in SIGMAS for p in PS if (s, p) != HEADLINE]
    out = head[:36] + [(HEADLINE[0], HEADLINE[1], t) for t in (3584, 4095)]
    out += [(s, p, t) for s, p in others for t in (0, 1, 4095)]
    out += head[36:128]
    out += [(s, p, t) for s, p in others for t in range(2, 8)]
    out += head[128:]
    return out


def one(job):
    import oracle

    sigma, p, traj = job
    n = N_QUBITS
    m = marked()
    init = synth.hadamard_transform(n).array()
    it = synth.grover_iteration(n, m).array()
    t0 = time.perf_counter()
    pr, a = oracle.noisy_grover_traj(n, m, ITERS, sigma, p, SEED, traj, init, it, want_state=True)
    dt = time.perf_counter() - t0
    nrm = float(np.vdot(a, a).real)
    amps = a[sample_indices()]
    fields = ["%.17g" % sigma, "%.17g" % p, "%d" % traj, "%.17g" % pr, "%.17g" % nrm]
    for z in amps:
        fields += ["%.17g" % z.real, "%.17g" % z.imag]
    return " ".join(fields), dt


def header() -> str:
    idx = " ".join(str(i) for i in sample_indices())
    return "\n".join([
        "# FP64 oracle trajectories of noisy Grover search (written by make_noisy_grover_ref.py; oracle only).",
        "# n=%d marked=%d iterations=%d philox_seed=%d; init = H on every qubit; iteration = synth.grover_iteration"
        % (N_QUBITS, marked(), ITERS, SEED),
        "# sample_indices: %s" % idx,
        "# columns: sigma p traj prob_marked norm2 then (re im) of the amplitude at each sample index",
    ]) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=6)
    args = ap.parse_args()
    done = set()
    if os.path.exists(OUT):
        with open(OUT) as f:
            for line in f:
                if line.startswith("#") or not line.strip():
                    continue
                s, p, t = line.split()[:3]
                done.add((float(s), float(p), int(t)))
    else:
        with open(OUT, "w") as f:
            f.write(header())
    todo = [j for j in jobs() if j not in done]
    print("%d trajectories to run on %d processes" % (len(todo), args.procs), flush=True)
    with mp.Pool(args.procs) as pool:
        for k, (line, dt) in enumerate(pool.imap(one, todo)):
            with open(OUT, "a") as f:
                f.write(line + "\n")
            print("%d/%d  %s  %.1f s" % (k + 1, len(todo), " ".join(line.split()[:4]), dt), flush=True)


if __name__ == "__main__":
    main()
