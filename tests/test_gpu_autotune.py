"""The autotuner on the device: it times candidates, leaves its choice set,
and the circuit still matches the oracle under the chosen values."""

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


@pytest.fixture
def keep_config(sv):
    keys = ["fused_tile_bits_c128", "fused_tile_bits_c64", "fused_low_bits", "fused_reg_bits", "fused_mfma"]
    old = {k: sv.config_get(k) for k in keys}
    yield
    for k, v in old.items():
        sv.config_set(k, v)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_tune_fused_sets_its_choice(sv, orc, keep_config, dtype):
    n = 14
    g = synth.brickwork_circuit(n, 6, seed=5).array()
    s = sv.State(n, dtype).reset(0)
    say("tune fused", dtype)
    r = sv.autotune.tune_fused(s, g, reps=2)
    assert r["tried"] >= 1 + len(r["keys"]) and r["best_ms"] <= r["start_ms"] and r["best_ms"] > 0
    for k, v in r["best"].items():
        assert sv.config_get(k) == v
    s.reset(0)
    s.run(g, fused=True)
    ref = orc.run(orc.zero_state(n), g)
    got = s.numpy().astype(np.complex128)
    tol = 1e-12 if dtype == "c128" else 1e-6 * 6
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))


def test_tune_group_sets_its_choice(sv):
    n, B = 10, 256
    marked = synth.grover_marked(n, 1)
    init = synth.hadamard_transform(n).array()
    it = synth.grover_iteration(n, marked).array()
    b = sv.Batch(n, B, "c64")
    say("tune group")
    r = sv.autotune.tune_group(b, init, it, 4, reps=2)
    assert r["keys"] == ["svb_group", "batch_waves"] and r["tried"] >= 4
    assert r["best"]["batch_waves"] in (0, 3, 4) and sv.config_get("batch_waves") == r["best"]["batch_waves"]
    g = r["best"]["svb_group"]
    assert g == 0 or B % g == 0
    from paper_quant_ph_0201042_amd import _lib
    import ctypes

    v = ctypes.c_int()
    assert _lib.load().svb_get_group(b._h, ctypes.byref(v)) == 0 and v.value == g
    # results do not depend on the group size
    p1, _ = b.run_noisy(init, it, 6, 0.02, 0.01, 3, target=marked)
    b.set_group(0)
    sv.config_set("batch_waves", 4)
    p0, _ = b.run_noisy(init, it, 6, 0.02, 0.01, 3, target=marked)
    assert np.array_equal(p0, p1)
