"""Host-side checks of the pass rewrites (no GPU): the fused plan of a gate
list, with its ops rewritten as the specialised kernels get them (unitary
2x2 as phase, real rotation, phase; phases merged into runs and moved
across controlled NOTs; or 2x2/4x4 composition when the split is off), is
applied by the library's host model in FP64 and compared with the CPU
oracle.  Tile shapes are varied so that controls and phase targets fall
inside and outside the tiles, on register and on thread bits."""

import numpy as np
import pytest

import synth

CIRCUITS = [
    ("brickwork", 13, lambda: synth.brickwork_circuit(13, 8, seed=1).array()),
    ("qft", 12, lambda: synth.qft_circuit(12).array()),
    ("mix", 11, lambda: synth.random_gate_mix(11, 400, seed=4).array()),
    ("grover", 10, lambda: synth.grover_circuit(10, 77, 2).array()),
]

KEYS = ["fused_rotations", "fused_pairs", "fused_tile_bits_c128", "fused_tile_bits_c64", "fused_low_bits",
        "fused_reg_bits"]


@pytest.fixture
def sv():
    import paper_quant_ph_0201042_amd as sv

    saved = {k: sv.config_get(k) for k in KEYS}
    yield sv
    for k, v in saved.items():
        sv.config_set(k, v)


@pytest.mark.parametrize("case", CIRCUITS, ids=lambda c: c[0])
@pytest.mark.parametrize("rot", [1, 0])
@pytest.mark.parametrize("shape", [(12, 4, 4), (8, 3, 4), (6, 2, 3)], ids=lambda s: "K%d_low%d_M%d" % s)
def test_model_matches_oracle(sv, orc, case, rot, shape):
    name, n, make = case
    K, low, M = shape
    sv.config_set("fused_rotations", rot)
    sv.config_set("fused_tile_bits_c128", K)
    sv.config_set("fused_tile_bits_c64", K)
    sv.config_set("fused_low_bits", low)
    sv.config_set("fused_reg_bits", M)
    gl = make()
    a = synth.random_state(n, 11)
    ref = orc.run(a, gl)
    for dtype in ("c128", "c64"):
        got = sv.model_fused(n, dtype, gl, a)
        err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
        assert err <= 1e-13, (name, dtype, err)


def test_split_is_used_and_merges_phases(sv):
    """The brickwork passes carry rotation ops and far fewer phase runs than
    rotations (the runs are merged across layers and controlled NOTs)."""
    sv.config_set("fused_rotations", 1)
    n = 16
    gl = synth.brickwork_circuit(n, 6, seed=2).array()
    _, _, masks = sv.plan_fused(n, "c128", gl)
    rots = runs = 0
    for p in range(len(masks)):
        src = sv.jit_source(n, "c128", gl, p)
        rots += src.count("kind %d\n" % 6)
        runs += src.count("{ // phase run")
    assert rots == 6 * n
    assert 0 < runs <= rots / 3


def test_non_unitary_dense_stays_dense(sv, orc):
    """A projector-like matrix is not split (it is applied as a dense op)."""
    sv.config_set("fused_rotations", 1)
    n = 6
    gl = synth.random_gate_mix(n, 40, seed=8).array()
    g = gl.copy()
    # a general matrix gate that is not unitary
    rec = synth.GateList().add(synth.KIND_U, 2, p=[0.5, 0.0, 0.0, 0.25, 0.1, 0.0, 0.75, 0.0]).array()
    g = np.concatenate([g[:20], rec, g[20:]])
    a = synth.random_state(n, 3)
    got = sv.model_fused(n, "c128", g, a)
    ref = orc.run(a, g)
    assert float(np.max(np.abs(got - ref))) <= 1e-13


@pytest.mark.parametrize("diag", [(1e-3, 1.0), (1.0, 0.0), (1e-200, 1.0), (4.0, 0.25)],
                         ids=["scale", "projector", "tiny", "stretch"])
def test_non_unit_diagonal_stays_an_op(sv, orc, diag):
    """A diagonal gate whose entries are not phases is applied where it
    stands: phase runs divide by entries, so only near-unit ones join them."""
    sv.config_set("fused_rotations", 1)
    n = 8
    gl = synth.brickwork_circuit(n, 4, seed=5).array()
    d0, d1 = diag
    rec = synth.GateList().add(synth.KIND_U, 3, p=[d0, 0.0, 0.0, 0.0, 0.0, 0.0, d1, 0.0]).array()
    g = np.concatenate([gl[: len(gl) // 2], rec, gl[len(gl) // 2:]])
    a = synth.random_state(n, 6)
    ref = orc.run(a, g)
    got = sv.model_fused(n, "c128", g, a)
    assert float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))) <= 1e-13
