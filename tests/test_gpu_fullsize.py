"""Full-size GPU parity: the benchmark's own registers against the CPU oracle.

- n = 30 (16 GiB complex128, byte offsets far beyond 2^32): one brickwork
  layer against its closed form (a product state permuted by the CNOT
  layer), and the first two brickwork layers against a whole oracle run,
  element by element, on the fused, per-gate and complex64 paths;
- n = 26: the whole depth-20 brickwork circuit on every engine, the
  complex64 dense-block form included;
- n = 28: the whole QFT output vector of a random input (per-gate, fused
  and FFT engines) against the oracle's circuit run;
- n = 20, 4096 complex64 trajectories of 804 noisy Grover iterations (the
  32 GiB batch): every stored FP64 oracle trajectory of the same draws in
  tests/golden (ids 0..255, 3584 and 4095; at least 32), and up to 9
  trajectories at every other point of the (sigma, p) grid.

Tolerances (sec. 2.2.1 arithmetic): complex128 max_j |g_j - o_j| <= 1e-12
max_j |o_j|; complex64 infidelity 1 - |<o|g>|^2 / (|o|^2 |g|^2) <= 1e-6 and
max-norm relative error <= 1e-6 per gate layer."""

import math
import os
import sys

import numpy as np
import pytest

import fullsize_jobs
import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "noisy_grover_n20_oracle.txt")
CHUNK = 1 << 26


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def sv():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_quant_ph_0201042_amd as sv

    fullsize_jobs.start()
    return sv


def compare(got, ref):
    """(max |g - o| / max |o|, infidelity) over the whole vector, in chunks."""
    dmax = omax = 0.0
    ip = 0j
    gg = oo = 0.0
    for i in range(0, len(ref), CHUNK):
        g = got[i:i + CHUNK].astype(np.complex128)
        o = ref[i:i + CHUNK]
        dmax = max(dmax, float(np.max(np.abs(g - o))))
        omax = max(omax, float(np.max(np.abs(o))))
        ip += np.vdot(o, g)
        gg += float(np.vdot(g, g).real)
        oo += float(np.vdot(o, o).real)
    return dmax / omax, 1.0 - abs(ip) ** 2 / (gg * oo)


def free_gpu():
    import gc

    import torch

    gc.collect()
    torch.cuda.empty_cache()


# ------------------------------------------------------------ n = 30


def su2(p):
    a, b, c, d = np.asarray(p[:4]) / np.linalg.norm(p[:4])
    return np.array([[a + 1j * b, c + 1j * d], [-c + 1j * d, a - 1j * b]])


@pytest.mark.parametrize("dtype,fused", [("c128", True), ("c128", False), ("c64", True)])
def test_n30_first_layer_closed_form(sv, dtype, fused):
    """One Haar SU(2) on every qubit of |0..0> is the product state
    alpha_j = prod_q U_q[b_q(j)][0]; the CNOT layer (2j -> 2j+1) then maps
    alpha to alpha o pi with pi flipping each target bit whose control bit is
    set (an involution).  Sampled amplitudes, highest indices included."""
    n = 30
    g = synth.brickwork_circuit(n, 1, seed=0).array()
    say("n30 closed form", dtype, fused)
    s = sv.State(n, dtype).reset(0)
    s.run(g, fused=fused)
    U = [su2(r["p"]) for r in g[:n]]
    rng = np.random.default_rng(30)
    js = np.concatenate([np.array([0, (1 << n) - 1, (1 << n) - 2, 1 << (n - 1), 0x2AAAAAAA, 0x15555555], np.uint64),
                         rng.integers(0, 1 << n, 1 << 20, dtype=np.uint64)])
    k = js.copy()
    for c in range(0, n - 1, 2):
        cb = (k >> np.uint64(n - 1 - c)) & np.uint64(1)
        k ^= cb << np.uint64(n - 2 - c)
    ref = np.ones(len(js), dtype=np.complex128)
    for q in range(n):
        b = ((k >> np.uint64(n - 1 - q)) & np.uint64(1)).astype(np.int64)
        ref *= np.where(b == 0, U[q][0, 0], U[q][1, 0])
    omax = math.prod(max(abs(u[0, 0]), abs(u[1, 0])) for u in U)
    import torch

    got = s.tensor[torch.from_numpy(js.astype(np.int64)).to(s.tensor.device)].cpu().numpy().astype(np.complex128)
    tol = 1e-12 if dtype == "c128" else 31 * 1e-6
    assert float(np.max(np.abs(got - ref))) <= tol * omax
    assert abs(s.norm2() - 1.0) <= (1e-12 if dtype == "c128" else 1e-5)
    del s
    free_gpu()


@pytest.mark.parametrize("dtype,mode", [("c128", "fused"), ("c128", "per_gate"), ("c64", "fused")])
def test_n30_two_brickwork_layers_vs_oracle(sv, dtype, mode):
    n = 30
    g = fullsize_jobs.brick30_gates()
    say("n30 two layers", dtype, mode)
    s = sv.State(n, dtype).reset(0)
    s.run(g, fused=(mode == "fused"))
    got = s.numpy()
    del s
    free_gpu()
    say("n30 two layers: waiting for the oracle")
    ref = fullsize_jobs.result("brick30")
    rel, infid = compare(got, ref)
    del got
    if dtype == "c128":
        assert rel <= 1e-12, rel
    else:
        assert rel <= 1e-6 * fullsize_jobs.BRICK30_LAYERS * 4 and infid <= 1e-6, (rel, infid)


# ------------------------------------------------------------ n = 26, whole depth-20 circuit


@pytest.mark.parametrize("dtype,mode", [("c128", "fused"), ("c128", "per_gate"), ("c64", "fused"),
                                        ("c64", "blocks4"), ("c64", "blocks5"), ("c128", "blocks5")])
def test_n26_brickwork_depth20_vs_oracle(sv, dtype, mode):
    n = 26
    g = synth.brickwork_circuit(n, 20, seed=0).array()
    say("n26 brickwork", dtype, mode)
    old = sv.config_get("block_qubits")
    try:
        if mode.startswith("blocks"):
            sv.config_set("block_qubits", int(mode[-1]))
        s = sv.State(n, dtype).reset(0)
        s.run(g, fused=(mode == "fused"), blocks=mode.startswith("blocks"))
    finally:
        sv.config_set("block_qubits", old)
    got = s.numpy()
    del s
    free_gpu()
    ref = fullsize_jobs.result("brick26")
    rel, infid = compare(got, ref)
    if dtype == "c128":
        assert rel <= 1e-12, rel
    else:
        # 20 layers: at most 1e-6 relative per layer, infidelity <= 1e-6
        assert rel <= 20 * 1e-6 and infid <= 1e-6, (rel, infid)


# ------------------------------------------------------------ n = 28 QFT, whole vector


@pytest.mark.parametrize("engine", ["fft", "fused", "per_gate", "fft_bitrev"])
def test_n28_qft_whole_vector(sv, engine):
    n = 28
    a = synth.random_state(n, 0)
    say("n28 qft", engine)
    s = sv.State(n, "c128").load(a)
    if engine == "fft":
        s.qft()
    elif engine == "fft_bitrev":
        s.qft(bitrev=True)
    else:
        s.run(synth.qft_circuit(n).array(), fused=(engine == "fused"))
    got = s.numpy()
    del s
    free_gpu()
    ref = fullsize_jobs.result("qft28")
    if engine == "fft_bitrev":
        # natural order: reverse the n index bits (a transpose of the 2x..x2 view)
        got = np.ascontiguousarray(got.reshape((2,) * n).transpose(tuple(range(n - 1, -1, -1)))).reshape(-1)
    rel, infid = compare(got, ref)
    assert rel <= 1e-12 and infid <= 1e-13, (rel, infid)


# ------------------------------------------------------------ n = 20 batched, stored oracle trajectories


def golden_rows():
    if not os.path.exists(GOLDEN):
        pytest.fail("missing %s (written by tests/golden/make_noisy_grover_ref.py)" % GOLDEN)
    rows = {}
    idx = None
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("# sample_indices:"):
                idx = [int(v) for v in line.split(":", 1)[1].split()]
            if line.startswith("#") or not line.strip():
                continue
            v = line.split()
            sigma, p, t = float(v[0]), float(v[1]), int(v[2])
            vals = [float(x) for x in v[3:]]
            amps = np.array(vals[2:][0::2]) + 1j * np.array(vals[2:][1::2])
            rows[(sigma, p, t)] = (vals[0], vals[1], amps)
    return idx, rows


# complex64 trajectories of 804 iterations: each amplitude takes about
# R = 8e4 roundings (804 iterations of ~100 gates, applied as ~1600 fused
# passes), so the state's relative error grows like sqrt(R) * 2^-24 ~ 1.7e-5
# (the measured norm drift is of that order).  A probability p = |a|^2 then
# moves by about 2 p times that, an amplitude by about that times itself:
# tolerances 5e-5 relative, with the absolute floors that bound the
# near-zero amplitudes and probabilities of the decohered points (2^-10
# amplitudes and their ~1e-7 error).
AMP_TOL = 2e-6
AMP_REL = 5e-5
PROB_TOL = 1e-6
PROB_REL = 5e-5


def check_against_golden(b, prob, traj0, wanted, rows, idx, sigma, p):
    checked = 0
    for t in wanted:
        key = (sigma, p, t)
        if key not in rows:
            pytest.fail("golden file lacks trajectory %r" % (key,))
        pr, nrm, amps = rows[key]
        reg = t - traj0
        assert abs(prob[reg] - pr) <= PROB_TOL + PROB_REL * pr, (key, prob[reg], pr)
        st = b.state(reg).astype(np.complex128)
        assert np.all(np.abs(st[idx] - amps) <= AMP_TOL + AMP_REL * np.abs(amps)), key
        assert abs(float(np.vdot(st, st).real) - nrm) <= 1e-4
        checked += 1
    return checked


def test_batched_4096_full_config_vs_stored_oracle(sv):
    n, iters, B = 20, 804, 4096
    sigma, p = 1e-2, 1e-4
    idx, rows = golden_rows()
    marked = synth.grover_marked(n, 0)
    init = synth.hadamard_transform(n).array()
    it = synth.grover_iteration(n, marked).array()
    say("batched n20 B4096 804 iterations")
    b = sv.Batch(n, B, "c64")
    prob, nrm = b.run_noisy(init, it, iters, sigma, p, seed=0, target=marked)
    assert np.max(np.abs(nrm - 1.0)) <= 1e-4
    # every stored trajectory (ids 0..255, 3584 and 4095; the file is
    # written in that order of priority and may still be growing)
    first = [t for t in range(256) if (sigma, p, t) in rows]
    assert len(first) >= 32, "golden file holds %d headline trajectories" % len(first)
    wanted = first + [t for t in (3584, 4095) if (sigma, p, t) in rows]
    assert check_against_golden(b, prob, 0, wanted, rows, idx, sigma, p) == len(wanted)
    # the mean over the stored oracle trajectories within 4 combined SE of
    # the mean over the 4096 GPU trajectories
    orc = np.array([rows[(sigma, p, t)][0] for t in first])
    se = math.hypot(orc.std(ddof=1) / math.sqrt(len(orc)), prob.std(ddof=1) / 64)
    assert abs(orc.mean() - prob.mean()) <= 4 * se + 1e-12
    b.close()
    del b
    free_gpu()


@pytest.mark.parametrize("sigma", [1e-3, 5e-3, 1e-2, 5e-2])
@pytest.mark.parametrize("p", [1e-5, 1e-4, 1e-3])
def test_batched_grid_points_vs_stored_oracle(sv, sigma, p):
    if (sigma, p) == (1e-2, 1e-4):
        pytest.skip("the full 4096-trajectory test covers this point")
    n, iters = 20, 804
    idx, rows = golden_rows()
    marked = synth.grover_marked(n, 0)
    init = synth.hadamard_transform(n).array()
    it = synth.grover_iteration(n, marked).array()
    say("batched grid", sigma, p)
    have = [t for t in range(8) if (sigma, p, t) in rows]
    assert have, "golden file holds no trajectory of this point"
    b = sv.Batch(n, 8, "c64")
    prob, _ = b.run_noisy(init, it, iters, sigma, p, seed=0, target=marked)
    assert check_against_golden(b, prob, 0, have, rows, idx, sigma, p) == len(have)
    if (sigma, p, 4095) in rows:
        b1 = sv.Batch(n, 1, "c64")
        prob1, _ = b1.run_noisy(init, it, iters, sigma, p, seed=0, traj_offset=4095, target=marked)
        assert check_against_golden(b1, prob1, 4095, [4095], rows, idx, sigma, p) == 1


def test_plain_path_trajectories_match_batched_and_oracle(sv, orc):
    """The plain per-gate complex128 baseline runs trajectory t as the
    explicit list svb_trajectory_gates writes; it matches the batched
    complex128 engine and the oracle on the same draws."""
    n, iters, sigma, p = 10, 12, 0.02, 0.01
    marked = synth.grover_marked(n, 4)
    init = synth.hadamard_transform(n).array()
    it = synth.grover_iteration(n, marked).array()
    b = sv.Batch(n, 16, "c128")
    prob, _ = b.run_noisy(init, it, iters, sigma, p, seed=5, target=marked)
    s = sv.State(n, "c128")
    for t in range(16):
        gl = sv.trajectory_gates(n, init, it, iters, sigma, p, 5, t)
        s.reset(0)
        s.run(gl)
        pr = s.prob((1 << n) - 1, marked)
        assert abs(pr - prob[t]) <= 1e-11
        if t % 5 == 0:
            ref = orc.noisy_grover_traj(n, marked, iters, sigma, p, 5, t, init, it)
            assert abs(pr - ref) <= 1e-11
