"""complex64 fused passes with dense ops on the matrix cores
(fused_mfma = 1, v_mfma_f32_4x4x1_16b) against the oracle: plain passes
(with and without composed 4x4 ops), controls on register bits, thread bits
(vector fallback) and outside the tile, and trajectory batches with
per-register matrices (batch_mfma = 1, the default, and 0)."""

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
def mfma(sv):
    keys = ["fused_mfma", "batch_mfma", "fused_pairs", "fused_jit", "fused_tile_bits_c64", "fused_low_bits"]
    old = {k: sv.config_get(k) for k in keys}
    sv.config_set("fused_mfma", 1)
    sv.config_set("fused_jit", 1)
    yield
    for k, v in old.items():
        sv.config_set(k, v)


def relerr(g, o):
    return float(np.max(np.abs(g.astype(np.complex128) - o)) / max(np.max(np.abs(o)), 1e-300))


@pytest.mark.parametrize("pairs", [0, 1])
@pytest.mark.parametrize("case", ["brickwork", "mix", "grover", "qft", "ctrl"])
def test_mfma_passes_match_oracle(sv, orc, mfma, pairs, case):
    sv.config_set("fused_pairs", pairs)
    n = 13
    g = {
        "brickwork": lambda: synth.brickwork_circuit(n, 10, seed=8).array(),
        "mix": lambda: synth.random_gate_mix(n, 300, seed=12, max_ctrl=4).array(),
        "grover": lambda: synth.grover_circuit(n, 4321, 2).array(),
        "qft": lambda: synth.qft_circuit(n).array(),
        "ctrl": lambda: synth.random_gate_mix(n, 200, seed=3, max_ctrl=12).array(),
    }[case]()
    a = synth.random_state(n, 77)
    say("mfma pass", case, pairs)
    s = sv.State(n, "c64").load(a.astype(np.complex64))
    s.run(g, fused=True)
    ref = orc.run(a.astype(np.complex64).astype(np.complex128), g)
    assert relerr(s.numpy(), ref) <= 1e-6 * len(g)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 6, 7, 9])
def test_mfma_small_registers(sv, orc, mfma, n):
    # tiles of fewer than 4 threads fall back to the vector units; 4 to 16
    # threads form whole groups of four lanes
    g = synth.random_gate_mix(n, 120, seed=40 + n, max_ctrl=2).array()
    a = synth.random_state(n, 5)
    s = sv.State(n, "c64").load(a.astype(np.complex64))
    s.run(g, fused=True)
    ref = orc.run(a.astype(np.complex64).astype(np.complex128), g)
    assert relerr(s.numpy(), ref) <= 1e-6 * len(g)


@pytest.mark.parametrize("shape", [(12, 4), (13, 5), (11, 3), (8, 2)])
def test_mfma_tile_shapes(sv, orc, mfma, shape):
    sv.config_set("fused_tile_bits_c64", shape[0])
    sv.config_set("fused_low_bits", shape[1])
    n = 17
    g = synth.brickwork_circuit(n, 8, seed=shape[0]).array()
    say("mfma tiles", shape)
    s = sv.State(n, "c64").reset(0)
    s.run(g, fused=True)
    ref = orc.run(orc.zero_state(n), g)
    assert relerr(s.numpy(), ref) <= 1e-6 * 8


def test_mfma_brickwork_n20_infidelity(sv, orc, mfma):
    n = 20
    g = synth.brickwork_circuit(n, 20, seed=0).array()
    s = sv.State(n, "c64").reset(0)
    s.run(g, fused=True)
    got = s.numpy().astype(np.complex128)
    ref = orc.run(orc.zero_state(n), g)
    ip = np.vdot(ref, got)
    infid = 1 - abs(ip) ** 2 / (np.vdot(got, got).real * np.vdot(ref, ref).real)
    assert relerr(got, ref) <= 1e-4 and infid <= 1e-6


@pytest.mark.parametrize("bm", [1, 0])
@pytest.mark.parametrize("n,iters,sigma,p", [(6, 6, 0.05, 0.01), (9, 12, 0.02, 0.002), (12, 3, 0.03, 0.01)])
def test_mfma_batched_trajectories(sv, orc, mfma, n, iters, sigma, p, bm):
    # batch_mfma = 1 (default): dense ops of the batches on the matrix
    # cores; 0: the vector units
    sv.config_set("batch_mfma", bm)
    marked = synth.grover_marked(n, n)
    init = synth.hadamard_transform(n).array()
    it = synth.grover_iteration(n, marked).array()
    B = 24
    b = sv.Batch(n, B, "c64")
    say("mfma batched", n)
    prob, nrm = b.run_noisy(init, it, iters, sigma, p, 1234 + n, traj_offset=77, target=marked)
    ref = np.array([orc.noisy_grover_traj(n, marked, iters, sigma, p, 1234 + n, 77 + r, init, it) for r in range(B)])
    assert np.max(np.abs(prob - ref)) <= 5e-5
    _, st = orc.noisy_grover_traj(n, marked, iters, sigma, p, 1234 + n, 77 + 5, init, it, want_state=True)
    assert np.max(np.abs(b.state(5).astype(np.complex128) - st)) <= 5e-5


@pytest.mark.parametrize("waves", [0, 3])
def test_batch_register_budget_same_results(sv, orc, mfma, waves):
    # batch_waves only changes how the compiler budgets registers (default
    # 4): the trajectories must come out bit for bit the same, and match
    # the oracle
    n, iters, sigma, p = 10, 5, 0.03, 0.005
    marked = synth.grover_marked(n, 2)
    init = synth.hadamard_transform(n).array()
    it = synth.grover_iteration(n, marked).array()
    B = 16
    b = sv.Batch(n, B, "c64")
    old = sv.config_get("batch_waves")
    say("batch waves", waves)
    try:
        sv.config_set("batch_waves", 4)
        p4, n4 = b.run_noisy(init, it, iters, sigma, p, 77, traj_offset=3, target=marked)
        s4 = b.state(B - 1).copy()
        sv.config_set("batch_waves", waves)
        pw, nw = b.run_noisy(init, it, iters, sigma, p, 77, traj_offset=3, target=marked)
        assert np.array_equal(p4, pw) and np.array_equal(n4, nw)
        assert np.array_equal(b.state(B - 1), s4)
    finally:
        sv.config_set("batch_waves", old)
    ref = np.array([orc.noisy_grover_traj(n, marked, iters, sigma, p, 77, 3 + r, init, it) for r in (0, B - 1)])
    assert np.max(np.abs(pw[[0, B - 1]] - ref)) <= 5e-5
