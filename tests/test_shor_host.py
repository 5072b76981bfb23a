"""The library's host code for steps 4-5 of Shor's algorithm (sec. 5.1)
against the oracle's, decision by decision (exact integers on both sides,
so the outcomes must agree bit for bit).  No GPU: sv_shor_classical is host
code."""

import numpy as np
import pytest

from oracle import shor as oshor


def _same(N, x, y, m, improved, r_prev):
    from paper_quant_ph_0201042_amd import shor

    a = shor.classical(N, x, y, m, improved, r_prev)
    b = oshor.classical(N, x, y, m, improved, r_prev)
    assert (a.factor, a.r, a.stage) == (b.factor, b.r, b.stage), (N, x, y, improved, r_prev)
    assert a.checks_list() == b.tries, (N, x, y, improved, r_prev)


@pytest.mark.parametrize("improved", [False, True])
def test_every_y_n15_n21(improved):
    for N, m, xs in ((15, 8, (2, 4, 7, 11, 13, 14)), (21, 10, (2, 5, 8, 13, 20))):
        for x in xs:
            for r_prev in (0, 2, 6):
                for y in range(1 << m):
                    _same(N, x, y, m, improved, r_prev)


@pytest.mark.parametrize("x", [23, 100, 2])
def test_every_y_n187(x):
    for y in range(0, 1 << 16, 3):
        _same(187, x, y, 16, True, 0)
    for y in range(1, 1 << 16, 7):
        _same(187, x, y, 16, False, 0)
        _same(187, x, y, 16, True, 12)


def test_sampled_y_table5_sizes():
    # 15-bit N of the paper's table, 30-qubit registers: y near the peaks
    # j 2^30 / r (where the candidates are) and uniform y
    rng = np.random.default_rng(7)
    for N in (21311, 22999, 23129):
        m = 30
        for _ in range(6):
            x = int(rng.integers(2, N))
            r = next(k for k in range(1, N) if pow(x, k, N) == 1)
            for _ in range(150):
                j = int(rng.integers(0, r))
                y = (j << m) // r + int(rng.integers(-3, 4))
                y = min(max(y, 0), (1 << m) - 1)
                _same(N, x, y, m, bool(rng.integers(0, 2)), int(rng.integers(0, 3)) * 2 * int(rng.integers(1, 50)))
            for _ in range(50):
                _same(N, x, int(rng.integers(0, 1 << m)), m, True, 0)
