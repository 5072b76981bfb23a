"""svb_trajectory_gates (host only, no GPU): the library's explicit gate list
of one noisy trajectory (sec. 3.1 depolarizing channel, sec. 3.2 operational
error), applied by the CPU oracle as a plain gate list, reproduces the
oracle's own noisy trajectory with the same draws.  The two sides draw from
independent Philox4x32-10 implementations."""

import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def sv():
    import paper_quant_ph_0201042_amd as sv

    return sv


@pytest.mark.parametrize("n,iters,sigma,p,kinds", [
    (6, 6, 0.05, 0.02, 0xFFFFFFFF),
    (5, 9, 0.0, 0.08, 0xFFFFFFFF),
    (7, 4, 0.1, 0.0, 0xFFFFFFFF),
    (6, 5, 0.03, 0.05, 1 << synth.KIND_U),
])
def test_trajectory_list_reproduces_oracle(sv, orc, n, iters, sigma, p, kinds):
    marked = synth.grover_marked(n, n + 1)
    init = synth.hadamard_transform(n).array()
    it = (synth.grover_iteration_noise_sites(n, marked) if kinds != 0xFFFFFFFF
          else synth.grover_iteration(n, marked)).array()
    zero = orc.zero_state(n)
    seed = 900 + n
    lens = set()
    for traj in (0, 1, 17, 4095):
        gl = sv.trajectory_gates(n, init, it, iters, sigma, p, seed, traj, kinds)
        lens.add(len(gl))
        got = orc.run(zero, gl)
        ref = orc.noisy_traj_state(zero, iters, sigma, p, seed, traj, init, it, depol_kinds=kinds)
        assert np.max(np.abs(got - ref)) <= 1e-13
        # the list is the gate sequence plus the drawn Paulis
        base = len(init) + iters * len(it)
        assert len(gl) >= base and (p > 0 or len(gl) == base)
    if p > 0:
        assert len(lens) > 1  # trajectories draw different Pauli events


def test_noise_free_list_is_the_gate_sequence(sv):
    n = 5
    init = synth.hadamard_transform(n).array()
    it = synth.grover_iteration(n, 3).array()
    gl = sv.trajectory_gates(n, init, it, 3, 0.0, 0.0, 1, 0)
    assert np.array_equal(gl, np.concatenate([init, it, it, it]))


def test_validation(sv):
    from paper_quant_ph_0201042_amd import SVError

    n = 4
    init = synth.hadamard_transform(n).array()
    it = synth.grover_iteration(n, 3).array()
    with pytest.raises(SVError):
        sv.trajectory_gates(n, init, it, 2, -1.0, 0.0, 1, 0)
    with pytest.raises(SVError):
        sv.trajectory_gates(n, init, it, 2, 0.1, 1.5, 1, 0)
    with pytest.raises(SVError):
        sv.trajectory_gates(n, init, it, 2, 0.1, 0.1, 1, 1 << 32)
    sw = synth.GateList().add(synth.KIND_SWAP, 0, target2=1).array()
    with pytest.raises(SVError):
        sv.trajectory_gates(n, init, sw, 2, 0.1, 0.1, 1, 0)
    bad = synth.GateList().add(synth.KIND_H, n).array()
    with pytest.raises(SVError):
        sv.trajectory_gates(n, init, bad, 2, 0.1, 0.1, 1, 0)


def test_batched_plan_two_passes_per_grover_iteration():
    """svb_plan (host only): the noisy Grover program at n = 20 folds each
    qubit's one-qubit gates and Paulis between the two C^19 Z of an
    iteration into one matrix, so an iteration is two layers of 20 dense
    ops around diagonal gates: two passes of 12-bit tiles per iteration,
    one 20-qubit layer of matrix slots per layer."""
    from paper_quant_ph_0201042_amd import batch

    n = 20
    marked = synth.grover_marked(n, 0)
    init = synth.hadamard_transform(n).array()
    it = synth.grover_iteration(n, marked).array()
    p1, s1 = batch.plan(n, "c64", init, it, 1)
    p804, s804 = batch.plan(n, "c64", init, it, 804)
    assert p804 - p1 == 2 * 803
    assert (s804 - s1) % 803 == 0
