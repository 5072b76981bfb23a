"""Host-side checks of the dense-block planner (no GPU).  Replaying the plan
through the CPU oracle (blocks with the generic k-qubit update, single gates
with the per-gate update) must reproduce the circuit in program order."""

import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def sv():
    import paper_quant_ph_0201042_amd as sv

    return sv


def replay(orc, n, g, plan, psi):
    a = psi.copy()
    for st in plan:
        if st[0] == "gate":
            a = orc.run(a, g[st[1]:st[1] + 1])
        else:
            a = orc.apply_kq(a, st[1], st[2])
    return a


def circuits():
    rng = np.random.default_rng(71)
    yield "brickwork", 9, synth.brickwork_circuit(9, 6, seed=5).array()
    yield "qft", 8, synth.qft_circuit(8).array()
    yield "mix", 9, synth.random_gate_mix(9, 120, seed=int(rng.integers(1 << 30))).array()
    yield "grover", 7, synth.grover_circuit(7, 37, 2).array()
    yield "qft_perturbed", 7, synth.qft_perturbed(7, synth.qft_eps(28, seed=3, sigma=0.05)).array()


@pytest.mark.parametrize("kmax", [1, 2, 3, 5, 6])
@pytest.mark.parametrize("case", list(circuits()), ids=lambda c: c[0])
def test_plan_replays_program_order(sv, orc, case, kmax):
    name, n, g = case
    plan = sv.plan_blocks(n, g, kmax)
    psi = synth.random_state(n, seed=17)
    want = orc.run(psi, g)
    got = replay(orc, n, g, plan, psi)
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    assert err < 1e-12, (name, kmax, err)
    for st in plan:
        if st[0] == "block":
            qs, M = st[1], st[2]
            assert 1 <= len(qs) <= kmax
            assert qs == sorted(qs) and len(set(qs)) == len(qs)
            D = 1 << len(qs)
            assert np.max(np.abs(M.conj().T @ M - np.eye(D))) < 1e-12


def test_large_gates_run_alone(sv):
    # the Grover oracle C^{n-1}Z touches every qubit: it cannot join a block
    n = 7
    g = synth.grover_circuit(n, 5, 1).array()
    plan = sv.plan_blocks(n, g, 5)
    singles = [st[1] for st in plan if st[0] == "gate"]
    assert singles
    for i in singles:
        assert bin(int(g[i]["ctrl"])).count("1") + 1 > 5


def test_blocks_absorb_gates(sv):
    # a depth-8 brickwork on 10 qubits has far more gates than 5-qubit blocks
    g = synth.brickwork_circuit(10, 8, seed=2).array()
    plan = sv.plan_blocks(10, g, 5)
    assert all(st[0] == "block" for st in plan)
    assert len(plan) * 4 < len(g)


def test_plan_rejects_bad_args(sv):
    g = synth.qft_circuit(4).array()
    with pytest.raises(sv.SVError):
        sv.plan_blocks(4, g, 0)
    with pytest.raises(sv.SVError):
        sv.plan_blocks(4, g, 7)
