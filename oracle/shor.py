"""Classical steps of Shor's factoring algorithm as run in sec. 5.1 (test
infrastructure only, like the rest of this package: the product library never
imports it and shares no code with it).

Plain Python integers throughout, so every decision here is exact.  The
quantum step 3 (register after the classical modular exponentiation, QFT,
measurement) is in ``sv_oracle.c``; ``quantum_step`` and ``experiment`` string the
two together for small registers.

Readings of the paper taken here (the paper states the checks, not their
order or bounds):
  * step 4 tests |y/2^m - k/r| <= 1/2^(m+1) exactly, as 2|y r - k 2^m| <= r,
    over the convergents of y/2^m with denominator below N (a fraction that
    close is a convergent, and with 2^m >= N^2 at most one qualifies);
  * step 5 outputs gcd(N, x^(r/2) - 1) when it is a nontrivial factor, else
    gcd(N, x^(r/2) + 1);
  * the improved variant tries, in the paper's order: neighbour y (y+1, y-1,
    y+2, y-2, first with a candidate) when y has none; then, only when
    x^r != 1 (mod N): the GCD check on r (r even), multiples c r for
    c = 2, 3, ... while c r < N (the first with x^(c r) = 1 is tested), and
    lcm(r1, r) with r1 the candidate of the experiment's previous quantum
    iteration; the first check that yields a factor ends the iteration.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

# stage codes of a successful iteration
ST_FAIL = -1
ST_PLAIN = 0      # steps 4-5 as stated
ST_NEIGHBOR = 1   # candidate from y +- 1, 2, then steps 4-5
ST_GCD = 2        # gcd(N, x^(r/2) +- 1) although x^r != 1
ST_SMALL = 3      # multiple c r of the candidate
ST_LCM = 4        # lcm of two candidates
ST_GCDX = 5       # step 2: gcd(x, N) > 1

EULER_GAMMA = 0.57721566490153286061


def convergents(y: int, M: int):
    """Convergents h/k of the continued fraction of y/M, in order."""
    h0, h1, k0, k1 = 0, 1, 1, 0
    num, den = y, M
    out = []
    while den:
        q = num // den
        num, den = den, num - q * den
        h0, h1 = h1, q * h1 + h0
        k0, k1 = k1, q * k1 + k0
        out.append((h1, k1))
    return out


def order_candidate(y: int, m: int, N: int):
    """Step 4: the coprime (k, r), 0 < k < r < N, with |y/2^m - k/r| <=
    1/2^(m+1), found among the convergents of y/2^m; None if there is none."""
    M = 1 << m
    found = None
    for h, k in convergents(y, M):
        if k >= N:
            break
        if 0 < h < k and 2 * abs(y * k - h * M) <= k:
            found = (h, k)
    return found


def step5(N: int, x: int, r: int) -> int:
    """Steps 4 (the three failure tests) and 5 for candidate r; returns a
    nontrivial factor of N or 0."""
    if r <= 0 or r % 2 or pow(x, r, N) != 1:
        return 0
    h = pow(x, r // 2, N)
    if h == 1 or h == N - 1:
        return 0
    for d in (math.gcd(N, h - 1), math.gcd(N, h + 1)):
        if 1 < d < N:
            return d
    return 0


def gcd_check(N: int, x: int, r: int) -> int:
    """Improvement 2: gcd(N, x^(r/2) -+ 1) for even r whatever x^r is."""
    if r <= 0 or r % 2:
        return 0
    h = pow(x, r // 2, N)
    for d in (math.gcd(N, h - 1), math.gcd(N, h + 1)):
        if 1 < d < N:
            return d
    return 0


@dataclass
class Outcome:
    factor: int = 0
    stage: int = ST_FAIL
    r: int = 0                      # candidate from y (0: none)
    # tries[i] = (successes, failures) of improvement i+1 in this iteration
    tries: list = field(default_factory=lambda: [[0, 0] for _ in range(4)])


def classical(N: int, x: int, y: int, m: int, improved: bool, r_prev: int = 0) -> Outcome:
    """Steps 4-5 (and, if improved, the four checks) for one measured y."""
    out = Outcome()
    cand = order_candidate(y, m, N)
    stage = ST_PLAIN
    if cand is None and improved:
        for d in (1, -1, 2, -2):
            yy = y + d
            if 0 <= yy < (1 << m):
                cand = order_candidate(yy, m, N)
                if cand is not None:
                    break
        out.tries[0][0 if cand is not None else 1] += 1
        stage = ST_NEIGHBOR
    if cand is None:
        return out
    r = cand[1]
    out.r = r
    if pow(x, r, N) == 1 or not improved:
        f = step5(N, x, r)
        if f:
            out.factor, out.stage = f, stage
        return out
    # x^r != 1 (mod N)
    if r % 2 == 0:
        f = gcd_check(N, x, r)
        out.tries[1][0 if f else 1] += 1
        if f:
            out.factor, out.stage = f, ST_GCD
            return out
    c = 2
    f = 0
    while c * r < N:
        if pow(x, c * r, N) == 1:
            f = step5(N, x, c * r)
            break
        c += 1
    out.tries[2][0 if f else 1] += 1
    if f:
        out.factor, out.stage = f, ST_SMALL
        return out
    if r_prev and r_prev != r:
        L = r_prev * r // math.gcd(r_prev, r)
        f = step5(N, x, L)
        out.tries[3][0 if f else 1] += 1
        if f:
            out.factor, out.stage = f, ST_LCM
    return out


def euler_phi(N: int) -> int:
    """Euler's totient by trial division (N small)."""
    res, n, p = N, N, 2
    while p * p <= n:
        if n % p == 0:
            while n % p == 0:
                n //= p
            res -= res // p
        p += 1
    if n > 1:
        res -= res // n
    return res


def prob_succ(N: int) -> float:
    """Lower bound on the success probability of one run of steps 1-5
    (sec. 5.1): p_step2 + (1 - p_step2) p_step3-4 with
    p_step2 = 1 - phi(N)/(N-1) and p_step3-4 = (1/2)(4/pi^2) e^-gamma / log log N
    (natural logarithms)."""
    f = euler_phi(N) / (N - 1)
    p34 = 0.5 * (4.0 / math.pi ** 2) * math.exp(-EULER_GAMMA) / math.log(math.log(N))
    return (1.0 - f) + f * p34


def register_qubits(N: int) -> int:
    """2l, l the bit length of N (step 3(a))."""
    return 2 * N.bit_length()


def quantum_step(N: int, x: int, m: int, a_star: int, u: float, gates) -> int:
    """Step 3 on the plain FP64 oracle: register after the classical modular
    exponentiation with first-register outcome x^a_star mod N, the QFT gate
    list ``gates`` (m qubits) WITHOUT its final swaps, and a measurement with
    uniform draw u whose index, read with its m bits reversed, is y.  The
    swaps only reverse the bit order of the output (sec. 2.3.2), so y has
    the law of a measurement after them."""
    from . import measure, modpow, run, shor_state

    a, _ = shor_state(m, N, x, modpow(x, a_star, N))
    j = measure(run(a, gates), u)
    return int(format(j, "0%db" % m)[::-1], 2)


def experiment(N: int, draws, improved: bool, gates, max_iters: int):
    """Repeats steps 1-5 until a nontrivial factor is found (sec. 5.1).
    draws = (x[i], a_star[i], u[i]) per iteration i; gates is the QFT
    without its final swaps (see quantum_step).  Returns (iterations,
    factor, stage, [(x, y, Outcome) per quantum iteration], tries summed)."""
    xs, astar, us = draws
    m = register_qubits(N)
    r_prev = 0
    log = []
    tries = [[0, 0] for _ in range(4)]
    for i in range(min(max_iters, len(xs))):
        x = int(xs[i])
        d = math.gcd(x, N)
        if d > 1:
            return i + 1, d, ST_GCDX, log, tries
        y = quantum_step(N, x, m, int(astar[i]), float(us[i]), gates)
        out = classical(N, x, y, m, improved, r_prev)
        log.append((x, y, out))
        for j in range(4):
            tries[j][0] += out.tries[j][0]
            tries[j][1] += out.tries[j][1]
        if out.r:
            r_prev = out.r
        if out.factor:
            return i + 1, out.factor, out.stage, log, tries
    return 0, 0, ST_FAIL, log, tries
