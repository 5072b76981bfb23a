"""Autotuner host logic (no GPU): workload keys, the tuned-value file, and
that a stored choice is what later runs use; argument checks of the tuner
entry points."""

import ctypes
import json

import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def sv():
    import paper_quant_ph_0201042_amd as sv

    return sv


def test_workload_key_follows_structure_not_angles(sv):
    a = synth.brickwork_circuit(12, 4, seed=0).array()
    b = synth.brickwork_circuit(12, 4, seed=1).array()  # same shape, other angles
    c = synth.brickwork_circuit(12, 5, seed=0).array()
    k = sv.autotune.workload_key
    assert k(12, "c128", a) == k(12, "c128", b)
    assert k(12, "c128", a) != k(12, "c128", c)
    assert k(12, "c128", a) != k(12, "c64", a)
    assert k(12, "c128", a) != k(13, "c128", a)
    assert k(12, "c128", a).startswith("gfx950:n12:c128:")


def test_stored_choice_is_applied(sv, tmp_path):
    path = str(tmp_path / "tuned.json")
    g = synth.brickwork_circuit(10, 3, seed=0).array()
    key = sv.autotune.workload_key(10, "c64", g)
    assert sv.autotune.apply(key, path) is None  # nothing stored yet
    keys = ["fused_tile_bits_c64", "fused_low_bits", "fused_reg_bits", "fused_mfma"]
    old = {k: sv.config_get(k) for k in keys}
    res = {"keys": keys, "start": old, "best": {"fused_tile_bits_c64": 11, "fused_low_bits": 5, "fused_reg_bits": 3,
                                                "fused_mfma": 1},
           "start_ms": 10.0, "best_ms": 8.0, "tried": 7}
    try:
        sv.autotune.save(key, res, path, note="test")
        data = json.load(open(path))
        assert data[key]["best"] == res["best"] and data[key]["best_ms"] == 8.0
        got = sv.autotune.apply(key, path)
        assert got == res["best"]
        for k, v in res["best"].items():
            assert sv.config_get(k) == v
    finally:
        for k, v in old.items():
            sv.config_set(k, v)


def test_committed_tuned_file_is_valid(sv):
    # every stored entry names known keys with values the library accepts
    data = sv.autotune.load()
    for key, ent in data.items():
        assert key.startswith("gfx950:n")
        assert ent["best_ms"] <= ent["start_ms"] + 1e-9
        for k, v in ent["best"].items():
            if k == "svb_group":
                assert v >= 0
                continue
            old = sv.config_get(k)
            sv.config_set(k, int(v))  # raises if out of range
            sv.config_set(k, old)


def test_tuner_argument_checks(sv):
    from paper_quant_ph_0201042_amd import _lib

    L = _lib.load()
    r = _lib.TuneResult()
    g = synth.brickwork_circuit(4, 1, seed=0).array()
    assert L.sv_tune_fused(None, g.ctypes.data_as(ctypes.c_void_p), len(g), 2, ctypes.byref(r)) == _lib.SV_EINVAL
    assert L.svb_tune_group(None, None, 0, None, 0, 1, 2, ctypes.byref(r)) == _lib.SV_EINVAL
    assert ctypes.sizeof(_lib.TuneResult) == 4 + 4 + 8 * 24 + 8 * 4 + 8 * 4 + 8 + 8
