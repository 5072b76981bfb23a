"""The QFT robustness experiment of sec. 5.1.1 on the batched engine: Shor's
register for N (after the classical modular exponentiation and a
first-register outcome per trajectory) goes through a noisy QFT; each
trajectory reports its fidelity with the noise-free output, its measured y
and whether steps 4-5 find a factor from it.  Every step is a call into
libsv.so; this module only strings the calls together."""

from __future__ import annotations

import numpy as np

from .batch import Batch
from .shor import classical, register_qubits

KIND_U = 0


def _bit_reverse(v: int, n: int) -> int:
    r = 0
    for _ in range(n):
        r = (r << 1) | (v & 1)
        v >>= 1
    return r


class QftShorNoise:
    """B trajectories of the noisy QFT on Shor's register for (N, x).

    gates: the QFT without its final swaps (output in bit-reversed order),
    with an explicit identity on every qubit after each controlled R_k, the
    sites where the register is depolarized.  a_star[t] fixes trajectory
    t's first-register outcome x^a_star mod N; u[t] is its measurement draw."""

    def __init__(self, N: int, x: int, gates: np.ndarray, a_star, u, dtype: str = "c128", group: int = 0):
        self.N, self.x = int(N), int(x)
        self.m = register_qubits(N)
        self.gates = np.ascontiguousarray(gates)
        self.a_star = [int(a) for a in a_star]
        self.u = [float(v) for v in u]
        if len(self.a_star) != len(self.u):
            raise ValueError("one a_star and one u per trajectory")
        self.B = len(self.a_star)
        self.noisy = Batch(self.m, self.B, dtype)
        self.ideal = Batch(self.m, self.B, dtype)
        for b in (self.noisy, self.ideal):
            b.set_start(True)
            b.set_noise_kinds(1 << KIND_U)
            if group:
                b.set_group(group)
        self.noisy_regs = [self.noisy.register(t) for t in range(self.B)]
        self.ideal_regs = [self.ideal.register(t) for t in range(self.B)]
        self._prepare(self.ideal_regs)
        self.ideal.run_noisy(self.gates, self.gates[:0], 0, 0.0, 0.0, 0)
        self.ms = 0.0

    def _prepare(self, regs):
        for t, s in enumerate(regs):
            s.shor_prepare(self.N, self.x, self.a_star[t])

    def run(self, sigma: float, p: float, seed: int, traj_offset: int = 0):
        """One noisy pass over every trajectory; returns a dict of per-
        trajectory arrays: fidelity, y (natural bit order), success (plain
        steps 4-5 give a factor), norm2."""
        self._prepare(self.noisy_regs)
        _, nrm = self.noisy.run_noisy(self.gates, self.gates[:0], 0, sigma, p, seed, traj_offset=traj_offset)
        self.ms = self.noisy.last_run_ms()
        fid, _ = self.ideal.fidelity(self.noisy)
        raw = self.noisy.measure(self.u)
        ys = np.array([_bit_reverse(int(v), self.m) for v in raw], dtype=np.int64)
        ok = np.array([classical(self.N, self.x, int(y), self.m, False).factor != 0 for y in ys], dtype=bool)
        return {"fidelity": fid, "y": ys, "success": ok, "norm2": nrm}

    def close(self):
        self.noisy_regs = self.ideal_regs = []
        self.noisy.close()
        self.ideal.close()


def iterations_needed(success) -> float:
    """Mean number of runs until the first success when each run succeeds
    with the observed rate (geometric law): 1 / rate (inf if none)."""
    rate = float(np.mean(success))
    return 1.0 / rate if rate > 0 else float("inf")

