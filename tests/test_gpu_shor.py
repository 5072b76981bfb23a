"""GPU parity of Shor's algorithm with classical modular exponentiation
(sec. 5.1) and of the noisy QFT experiment on its register (sec. 5.1.1)
against the CPU oracle: the register after step 3(c) bit for bit, whole
factoring runs decision by decision on the same draws, noisy trajectories
state by state; at the paper's 30-qubit size, the closed form of the QFT
output of a periodic register."""

import math
import sys

import numpy as np
import pytest

import synth
from oracle import shor as oshor

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def sv():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_quant_ph_0201042_amd as sv

    return sv


def _order(x, N):
    r = 1
    while pow(x, r, N) != 1:
        r += 1
    return r


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("N,x,m", [(15, 7, 8), (21, 2, 10), (187, 23, 16), (33, 5, 12), (35, 4, 7), (2, 1, 3),
                                   (23129, 7, 13), (4294967291, 3, 18)])
def test_prepare_bit_exact(sv, orc, dtype, N, x, m):
    s = sv.State(m, dtype)
    M = 1 << m
    for a_star in sorted({0, 1, 5 % M, M - 1, (M * 2) // 3}):
        say("shor_prepare", dtype, N, x, m, a_star)
        c = s.shor_prepare(N, x, a_star)
        ref, rc = orc.shor_state(m, N, x, orc.modpow(x, a_star, N))
        assert c == rc
        got = s.numpy()
        want = ref.astype(np.complex64 if dtype == "c64" else np.complex128)
        assert np.array_equal(got.view(np.uint8), want.view(np.uint8))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_prepare_full_size_n30(sv, dtype):
    import torch

    N, m = 23129, 30
    M = 1 << m
    s = sv.State(m, dtype)
    rng = np.random.default_rng(3)
    for x in (int(rng.integers(2, N)), 2):
        if math.gcd(x, N) != 1:
            continue
        r = _order(x, N)
        a_star = int(rng.integers(0, M))
        say("shor_prepare n30", dtype, N, x, r, a_star)
        c = s.shor_prepare(N, x, a_star)
        a0 = a_star % r
        assert c == (M - 1 - a0) // r + 1
        amp = 1.0 / math.sqrt(c)
        if dtype == "c64":
            amp = float(np.float32(amp))
        j = rng.integers(0, c - 1, size=200)  # a0 + j r + k < M for 0 < k < r
        on = torch.from_numpy((a0 + j * r).astype(np.int64)).cuda()
        off = torch.from_numpy(((a0 + j * r + rng.integers(1, r, size=200)) % M).astype(np.int64)).cuda()
        got_on = s.tensor[on].cpu().numpy()
        got_off = s.tensor[off].cpu().numpy()
        assert np.all(got_on.real == amp) and np.all(got_on.imag == 0)
        assert np.all(got_off == 0)
        assert abs(s.norm2() - 1.0) < (1e-12 if dtype == "c128" else 1e-5)


def test_qft_of_register_closed_form_n30(sv):
    # uniform over a0 + j r, j < c: |beta_y|^2 = sin^2(pi c r y / M) / (c M sin^2(pi r y / M))
    import torch

    N, m, x = 21311, 30, 2
    M = 1 << m
    r = _order(x, N)
    s = sv.State(m, "c128")
    c = s.shor_prepare(N, x, 123456789)
    s.qft()
    rng = np.random.default_rng(11)
    j = rng.integers(0, r, size=100)
    ys = np.unique(np.clip((j * M) // r + rng.integers(-2, 3, size=100), 0, M - 1))
    got = s.tensor[torch.from_numpy(ys.astype(np.int64)).cuda()].cpu().numpy()
    for y, b in zip(ys, got):
        # phases reduced exactly in integers, and folded to [0, M/2] (sin(pi k / M)
        # = sin(pi (M - k) / M)), before the sines
        ph = (int(r) * int(y)) % M
        fold = lambda k: min(k, M - k)  # noqa: E731
        if ph == 0:
            w = c / M
        else:
            w = math.sin(math.pi * fold((c * ph) % M) / M) ** 2 / (c * M * math.sin(math.pi * fold(ph) / M) ** 2)
        assert abs(abs(b) ** 2 - w) < 1e-12, (y, abs(b) ** 2, w)


@pytest.mark.parametrize("improved", [False, True])
@pytest.mark.parametrize("N", [15, 21, 143, 187])
def test_factor_runs_match_oracle(sv, N, improved):
    m = sv.shor.register_qubits(N)
    s = sv.State(m, "c128")
    g = synth.qft_circuit(m, swaps=False).array()
    for seed in range(3):
        say("shor_factor", N, improved, seed)
        draws = synth.shor_draws(N, m, seed, 60)
        res, ys = sv.shor.factor(s, N, *draws, improved=improved)
        it, f, st, log, tries = oshor.experiment(N, draws, improved, g, 60)
        assert (res.iterations, res.factor, res.stage) == (it, f, st)
        assert res.checks_list() == tries
        upto = res.iterations if res.iterations else len(ys)
        quantum = [int(y) for y in ys[:upto] if y != np.uint64(2**64 - 1)]
        assert quantum == [y for (_, y, _) in log]


def test_factor_full_size_n30(sv):
    N = 21311
    m = sv.shor.register_qubits(N)
    assert m == 30
    s = sv.State(m, "c128")
    draws = synth.shor_draws(N, m, 5, 64)
    say("shor_factor n30", N)
    res, ys = sv.shor.factor(s, N, *draws, improved=True)
    assert res.iterations >= 1 and N % res.factor == 0 and 1 < res.factor < N
    # replay the host decisions on the measured y with the oracle
    r_prev = 0
    for i in range(res.iterations):
        x = int(draws[0][i])
        if math.gcd(x, N) > 1:
            assert i == res.iterations - 1 and res.stage == oshor.ST_GCDX
            break
        out = oshor.classical(N, x, int(ys[i]), m, True, r_prev)
        if out.r:
            r_prev = out.r
        assert bool(out.factor) == (i == res.iterations - 1)
        if out.factor:
            assert (out.factor, out.stage) == (res.factor, res.stage)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("sigma,p", [(0.05, 0.01), (0.0, 0.03), (0.02, 0.0)])
def test_keep_start_noise_sites_match_oracle(sv, orc, dtype, sigma, p):
    N, x, m = 33, 5, 12
    g = synth.qft_register_noise(m).array()
    B, seed, off = 8, 99, 1000
    draws = synth.shor_draws(N, m, 4, B)
    say("keep start", dtype, sigma, p)
    b = sv.Batch(m, B, dtype)
    b.set_start(True)
    b.set_noise_kinds(1 << synth.KIND_U)
    regs = [b.register(t) for t in range(B)]
    for t in range(B):
        regs[t].shor_prepare(N, x, int(draws[1][t]))
    b.run_noisy(g, g[:0], 0, sigma, p, seed, traj_offset=off)
    tol = 1e-11 if dtype == "c128" else 5e-5
    for t in range(B):
        start, _ = orc.shor_state(m, N, x, orc.modpow(x, int(draws[1][t]), N))
        want = orc.noisy_traj_state(start, 0, sigma, p, seed, off + t, g, g[:0], depol_kinds=1 << synth.KIND_U)
        got = regs[t].numpy().astype(np.complex128)
        assert np.max(np.abs(got - want)) <= tol, (t, np.max(np.abs(got - want)))
    # a second run starts again from what the caller writes
    for t in range(B):
        regs[t].shor_prepare(N, x, int(draws[1][t]))
    b.run_noisy(g, g[:0], 0, sigma, p, seed, traj_offset=off)
    start, _ = orc.shor_state(m, N, x, orc.modpow(x, int(draws[1][0]), N))
    want = orc.noisy_traj_state(start, 0, sigma, p, seed, off, g, g[:0], depol_kinds=1 << synth.KIND_U)
    assert np.max(np.abs(regs[0].numpy().astype(np.complex128) - want)) <= tol


def test_qft_experiment_matches_oracle_n187(sv, orc):
    N, x, m = 187, 23, 16
    g = synth.qft_register_noise(m).array()
    B = 24
    _, a_star, u = synth.shor_draws(N, m, 8, B)
    exp = sv.experiments.QftShorNoise(N, x, g, a_star, u, "c128")
    for sigma, p, seed in ((0.0, 0.0, 1), (1e-2, 1e-3, 2), (1e-3, 1e-2, 3)):
        say("qft experiment", sigma, p)
        out = exp.run(sigma, p, seed)
        for t in range(B):
            start, _ = orc.shor_state(m, N, x, orc.modpow(x, int(a_star[t]), N))
            ideal = orc.run(start, g)
            noisy = orc.noisy_traj_state(start, 0, sigma, p, seed, t, g, g[:0], depol_kinds=1 << synth.KIND_U)
            f = abs(np.vdot(ideal, noisy)) ** 2 / (np.vdot(ideal, ideal).real * np.vdot(noisy, noisy).real)
            assert abs(out["fidelity"][t] - f) < 1e-10
            y = synth.bit_reverse(orc.measure(noisy, float(u[t])), m)
            assert out["y"][t] == y
            assert out["success"][t] == bool(oshor.classical(N, x, y, m, False).factor)
        if p == 0.0 and sigma == 0.0:
            assert np.all(np.abs(out["fidelity"] - 1.0) < 1e-12)
            assert np.all(out["y"] % 4096 == 0)   # peaks of the order-16 register
    exp.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [9, 14])
def test_qft_bitrev_flag(sv, dtype, n):
    a = synth.random_state(n, n + 40)
    rev = np.array([synth.bit_reverse(y, n) for y in range(1 << n)])
    tol = 1e-12 if dtype == "c128" else 2e-6
    say("qft bitrev", dtype, n)
    s = sv.State(n, dtype).load(a)
    got = s.qft(bitrev=True).numpy().astype(np.complex128)
    assert np.max(np.abs(got - np.fft.ifft(a, norm="ortho")[rev])) <= tol
    s.load(a)
    got = s.qft(inverse=True, bitrev=True).numpy().astype(np.complex128)
    assert np.max(np.abs(got - np.fft.fft(a[rev], norm="ortho"))) <= tol
