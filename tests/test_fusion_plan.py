"""Host-side checks of the fused-pass planner (no GPU).  The planner may
reorder gates only where they commute; running the gates in the planned
order through the CPU oracle must reproduce program order."""

import numpy as np
import pytest

import synth
from synth import KIND_SWAP


@pytest.fixture(scope="module")
def sv():
    import paper_quant_ph_0201042_amd as sv

    return sv


def is_diag(orc, rec):
    if rec["kind"] == KIND_SWAP:
        return False
    U = orc.gate_matrix(int(rec["kind"]), int(rec["iarg"]), rec["p"])
    return U[0, 1] == 0 and U[1, 0] == 0


def check_plan(sv, orc, n, dtype, g):
    order, pass_of, masks = sv.plan_fused(n, dtype, g)
    assert sorted(order.tolist()) == list(range(len(g)))
    # passes run in order; a SWAP (pass -1) sits between passes
    last = -1
    for p in pass_of:
        if p >= 0:
            assert p >= last
            last = p
    for i, gi in enumerate(order):
        rec = g[gi]
        if rec["kind"] == KIND_SWAP:
            assert pass_of[i] == -1
            continue
        assert pass_of[i] >= 0
        tb = 1 << (n - 1 - int(rec["target"]))
        if not is_diag(orc, rec):
            assert int(masks[pass_of[i]]) & tb, (gi, hex(int(masks[pass_of[i]])))
    return order, pass_of, masks


@pytest.mark.parametrize("case", ["mix8", "mix12", "brick12", "qft11", "grover9", "ctrl10"])
@pytest.mark.parametrize("tile", [(5, 2), (8, 4), (12, 6)])
def test_plan_order_equivalent(sv, orc, case, tile):
    K, low = tile
    old = (sv.config_get("fused_tile_bits_c128"), sv.config_get("fused_low_bits"))
    sv.config_set("fused_tile_bits_c128", K)
    sv.config_set("fused_low_bits", low)
    try:
        if case.startswith("mix"):
            n = int(case[3:])
            g = synth.random_gate_mix(n, 300, seed=n, max_ctrl=3).array()
        elif case == "brick12":
            n = 12
            g = synth.brickwork_circuit(n, 8, seed=1).array()
        elif case == "qft11":
            n = 11
            g = synth.qft_circuit(n).array()
        elif case == "grover9":
            n = 9
            g = synth.grover_circuit(n, 300, 4).array()
        else:
            n = 10
            g = synth.random_gate_mix(n, 300, seed=99, max_ctrl=9).array()
        order, pass_of, masks = check_plan(sv, orc, n, "c128", g)
        a = synth.random_state(n, 5)
        ref = orc.run(a, g)
        got = orc.run(a, g[order])
        assert np.max(np.abs(got - ref)) <= 1e-12
        # fusion must pay: far fewer sweeps than gates when the tile is wide
        if K >= 8 and case != "mix8":
            assert len(masks) < len(g) / 3
    finally:
        sv.config_set("fused_tile_bits_c128", old[0])
        sv.config_set("fused_low_bits", old[1])


def test_plan_brickwork_n30_pass_count(sv, orc):
    n = 30
    g = synth.brickwork_circuit(n, 20, seed=0).array()
    order, pass_of, masks = check_plan(sv, orc, n, "c128", g)
    # 30 one-qubit targets per layer, 6 new high bits per 12-bit tile
    assert len(masks) <= 20 * 5
    g64 = check_plan(sv, orc, n, "c64", g)[2]
    assert len(g64) <= len(masks)


def test_plan_qft_n28_swaps_last(sv, orc):
    n = 28
    g = synth.qft_circuit(n).array()
    order, pass_of, masks = check_plan(sv, orc, n, "c128", g)
    nsw = n // 2
    assert (pass_of[-nsw:] == -1).all()
    assert len(masks) <= 10


def test_config_validation(sv):
    from paper_quant_ph_0201042_amd import SVError

    with pytest.raises(SVError):
        sv.config_set("fused_tile_bits_c128", 13)
    with pytest.raises(SVError):
        sv.config_set("no_such_key", 1)
    assert sv.config_get("fused_max_ops") >= 1
