"""GPU parity of the batched noisy-trajectory engine (svb_run_noisy) against
the CPU oracle's trajectories, which use the same counter-based draws; plus
the closed forms of the paper's Hadamard-transform noise study and the
noise-free Grover law, evaluated on the GPU engine."""

import math
import sys

import numpy as np
import pytest

import synth

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


def grover_lists(n, marked):
    return synth.hadamard_transform(n).array(), synth.grover_iteration(n, marked).array()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,iters,sigma,p", [(6, 6, 0.05, 0.01), (9, 12, 0.02, 0.002), (5, 3, 0.0, 0.05),
                                            (7, 5, 0.1, 0.0)])
def test_trajectories_match_oracle(sv, orc, dtype, n, iters, sigma, p):
    marked = synth.grover_marked(n, n)
    init, it = grover_lists(n, marked)
    B, seed, off = 24, 1234 + n, 77
    say("batched", dtype, n, iters, sigma, p)
    b = sv.Batch(n, B, dtype)
    prob, nrm = b.run_noisy(init, it, iters, sigma, p, seed, traj_offset=off, target=marked)
    ref = np.array([orc.noisy_grover_traj(n, marked, iters, sigma, p, seed, off + r, init, it) for r in range(B)])
    tol = 1e-11 if dtype == "c128" else 5e-5
    assert np.max(np.abs(prob - ref)) <= tol, np.max(np.abs(prob - ref))
    assert np.max(np.abs(nrm - 1.0)) <= (1e-12 if dtype == "c128" else 1e-4)
    # whole final state of one trajectory
    _, st = orc.noisy_grover_traj(n, marked, iters, sigma, p, seed, off + 5, init, it, want_state=True)
    got = b.state(5).astype(np.complex128)
    assert np.max(np.abs(got - st)) <= (1e-11 if dtype == "c128" else 5e-5)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_noise_free_limit_is_grover_law(sv, dtype):
    n = 10
    marked = 700
    init, it = grover_lists(n, marked)
    iters = synth.grover_iterations(n)
    b = sv.Batch(n, 8, dtype)
    prob, _ = b.run_noisy(init, it, iters, 0.0, 0.0, 5, target=marked)
    ref = math.sin((2 * iters + 1) * math.asin(2 ** (-n / 2))) ** 2
    assert np.max(np.abs(prob - ref)) <= (1e-12 if dtype == "c128" else 2e-5)


def test_ht_closed_forms_on_gpu(sv):
    """sec. 4.3.1: <0|rho_k|0> after k Hadamard transforms with depolarizing
    probability p is ((1 + (1 - 4p/3)^k)/2)^n; with operational error sigma it
    is ((1 + exp(-9 k sigma^2 / 4))/2)^n."""
    n, k, B = 4, 10, 8192
    init = np.zeros(0, dtype=synth.GATE_DTYPE)
    it = synth.hadamard_transform(n).array()
    b = sv.Batch(n, B, "c64")
    for sigma, p, ref in [(0.0, 0.05, ((1 + (1 - 4 * 0.05 / 3) ** k) / 2) ** n),
                          (0.15, 0.0, ((1 + math.exp(-9 * k * 0.15**2 / 4)) / 2) ** n)]:
        say("ht", sigma, p)
        prob, _ = b.run_noisy(init, it, k, sigma, p, seed=99, target=0)
        se = prob.std(ddof=1) / math.sqrt(B)
        assert abs(prob.mean() - ref) <= 4 * se, (prob.mean(), ref, se)


def test_reproducible_by_trajectory_id(sv):
    n, iters = 8, 10
    init, it = grover_lists(n, 3)
    b64 = sv.Batch(n, 64, "c64")
    b64.set_group(16)
    p_all, _ = b64.run_noisy(init, it, iters, 0.02, 1e-3, 42, traj_offset=1000, target=3)
    b1 = sv.Batch(n, 1, "c64")
    for r in (0, 17, 63):
        p1, _ = b1.run_noisy(init, it, iters, 0.02, 1e-3, 42, traj_offset=1000 + r, target=3)
        assert p1[0] == p_all[r]
    # a second call replays the captured graph with new parameters
    p_again, _ = b64.run_noisy(init, it, iters, 0.02, 1e-3, 42, traj_offset=1000, target=3)
    assert np.array_equal(p_again, p_all)
    p_other, _ = b64.run_noisy(init, it, iters, 0.02, 1e-3, 43, traj_offset=1000, target=3)
    assert not np.array_equal(p_other, p_all)


def test_unsupported_programs(sv):
    from paper_quant_ph_0201042_amd import SVError

    n = 4
    b = sv.Batch(n, 2, "c64")
    cnot = synth.GateList().add(synth.KIND_X, 1, ctrl=1 << 3).array()
    with pytest.raises(SVError):
        b.run_noisy(np.zeros(0, dtype=synth.GATE_DTYPE), cnot, 1, 0.1, 0.0, 1)
    sw = synth.GateList().add(synth.KIND_SWAP, 0, target2=1).array()
    with pytest.raises(SVError):
        b.run_noisy(np.zeros(0, dtype=synth.GATE_DTYPE), sw, 1, 0.1, 0.0, 1)


def test_n20_sampled_trajectories(sv, orc):
    """The batched workload's register size (n = 20, complex64) with a
    shortened iteration count the oracle can replay: trajectories 0, 1 and
    B-1 of a 512-trajectory batch against the oracle."""
    n, iters, B = 20, 4, 512
    marked = synth.grover_marked(n, 0)
    init, it = grover_lists(n, marked)
    b = sv.Batch(n, B, "c64")
    say("n20 batch")
    prob, nrm = b.run_noisy(init, it, iters, 1e-2, 1e-4, seed=0, target=marked)
    assert np.max(np.abs(nrm - 1.0)) <= 1e-4
    for r in (0, 1, B - 1):
        say("n20 oracle traj", r)
        ref = orc.noisy_grover_traj(n, marked, iters, 1e-2, 1e-4, 0, r, init, it)
        assert abs(prob[r] - ref) <= 1e-5


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_grover_depolarized_once_per_iteration(sv, orc, dtype):
    # depolarizing only at the identity sites that close each G-iteration
    n, iters, sigma, p = 6, 5, 0.03, 0.05
    marked = synth.grover_marked(n, 9)
    init = synth.hadamard_transform(n).array()
    it = synth.grover_iteration_noise_sites(n, marked).array()
    B, seed = 16, 4242
    b = sv.Batch(n, B, dtype)
    b.set_noise_kinds(1 << synth.KIND_U)
    prob, _ = b.run_noisy(init, it, iters, sigma, p, seed, target=marked)
    zero = np.zeros(1 << n, dtype=np.complex128)
    zero[0] = 1.0
    tol = 1e-11 if dtype == "c128" else 5e-5
    for r in range(B):
        st = orc.noisy_traj_state(zero, iters, sigma, p, seed, r, init, it, depol_kinds=1 << synth.KIND_U)
        assert abs(prob[r] - abs(st[marked]) ** 2) <= tol


@pytest.mark.parametrize("da,db", [("c64", "c128"), ("c128", "c128"), ("c64", "c64"), ("c128", "c64")])
def test_batched_fidelity_matches_register_states(sv, da, db):
    # svb_fidelity against the per-register definition on host copies
    n, B, iters = 9, 12, 6
    marked = synth.grover_marked(n, 2)
    init, it = grover_lists(n, marked)
    a = sv.Batch(n, B, da)
    b = sv.Batch(n, B, db)
    a.run_noisy(init, it, iters, 0.03, 0.01, 8, target=marked)
    b.run_noisy(init, it, iters, 0.03, 0.01, 8 if da != db else 9, target=marked)
    fid, ov = a.fidelity(b)
    for r in range(B):
        x = a.state(r).astype(np.complex128)
        y = b.state(r).astype(np.complex128)
        ip = np.vdot(x, y)
        ref = abs(ip) ** 2 / (np.vdot(x, x).real * np.vdot(y, y).real)
        assert abs(fid[r] - ref) <= 1e-12 and abs(ov[r] - ip) <= 1e-12
    if da != db:
        assert np.max(1 - fid) <= 1e-9  # same draws, c64 against c128
    from paper_quant_ph_0201042_amd import SVError

    with pytest.raises(SVError):
        a.fidelity(a)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [4, 8, 11])
def test_batched_measure_matches_oracle(sv, orc, dtype, n):
    # svb_measure against the oracle's sequential rule on every register,
    # draws kept away from cumulative boundaries (reading of sec. 2.2.3)
    B = 16
    marked = synth.grover_marked(n, 5)
    init, it = grover_lists(n, marked)
    b = sv.Batch(n, B, dtype)
    b.run_noisy(init, it, 3, 0.1, 0.05, 17, target=marked)
    rng = np.random.default_rng(n)
    draws = np.zeros(B)
    states = [b.state(r).astype(np.complex128) for r in range(B)]
    for r in range(B):
        c = np.cumsum(np.abs(states[r]) ** 2)
        while True:
            u = float(rng.random()) * c[-1]
            if np.min(np.abs(c - u)) > 1e-9:
                break
        draws[r] = u
    draws[0] = 2.0  # past the total: last index of nonzero weight
    idx = b.measure(draws)
    for r in range(B):
        assert int(idx[r]) == orc.measure(states[r], draws[r]), r
