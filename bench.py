"""Benchmark of the MI355X state-vector gate engine.

One step = the brickwork random circuit of depth 20 on an n=30 register
(every layer: a Haar SU(2) on each of the 30 qubits, then CNOTs on (2j,2j+1)
in even layers and (2j+1,2j+2) in odd layers; 600 one-qubit gates and 290
CNOTs), complex128, from |0...0> (register reset), through the HIP kernels,
followed by the FP64 norm reduction.  Inputs are seeded and synthetic.

The headline runs the circuit as fused passes (SV_RUN_FUSED): each pass is a
kernel specialised to its op list and compiled with hipRTC on first use; the
first run of the circuit does that compilation and is not timed
("jit_prepare_s").  The same circuit is also timed gate by gate (one HBM
sweep per gate) and reported under "per_gate_path".

Metric: gate-amplitude updates per second (a one-qubit gate updates 2^n
amplitudes, a CNOT 2^{n-1}), plus the dominant kernel against its roofline:
its algorithmic FP64 flops and HBM bytes per launch over its mean duration,
against the MI355X peaks (78.6 TFLOP/s FP64 vector, 8 TB/s HBM), timed with
HIP events on the stream the kernels are launched on (the library's
profiled run records them around each pass); "bound" names the ceiling
whose time is the larger one.  The plain CPU oracle is timed on a bounded sample of the same
workload on the host.

Every form (complex64 precision form, batched trajectories, per-gate
microbench matrix, adjoint, dense blocks, QFT, robustness experiments, Shor)
writes its whole record to a side file (--forms-out); the last stdout line
is one compact JSON object with the headline keys.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-forms]
       [--pg-steps 0] [--copy-probe] [--only-form NAME]
"""

from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

PEAK_HBM_GBS = 8000.0
METRIC = "gate-amp updates/s + HBM GB/s at n=30; batched fp32 vs plain fp64 speedup"


def prepared_gates(sv, gl_array, n):
    """(kind, q, ctrl, U[8], amps_updated, is_dominant) per gate; matrices built
    by the library's host-side constructor."""
    import ctypes

    from paper_quant_ph_0201042_amd import _lib

    L = _lib.load()
    out = []
    for rec in gl_array:
        r = np.ascontiguousarray(rec.reshape(1))
        U = np.zeros(8)
        _lib.check(L.sv_gate_matrix(r.ctypes.data_as(ctypes.c_void_p), U.ctypes.data_as(ctypes.c_void_p)))
        q = int(rec["target"])
        ctrl = int(rec["ctrl"])
        nc = bin(ctrl).count("1")
        amps = 1 << (n - nc)
        # dominant kernel: dense pair stream (no controls, target bit >= 6)
        dominant = ctrl == 0 and (n - 1 - q) >= 6 and not (U[2] == 0 and U[3] == 0 and U[4] == 0 and U[5] == 0)
        out.append((q, ctrl, U, amps, dominant))
    return out


def run_step_per_gate(s, gates, ev_pairs=None):
    s.reset(0)
    for q, ctrl, U, _, dom in gates:
        if ev_pairs is not None and dom:
            e0, e1 = ev_pairs.pop()
            e0.record()
            s.apply_1q(q, U)
            e1.record()
            ev_pairs_done.append((e0, e1))
        elif ctrl:
            s.apply_ctrl(ctrl, q, U)
        else:
            s.apply_1q(q, U)
    return s.norm2()


ev_pairs_done = []


def run_step_fused(s, gl, profile=False):
    s.reset(0)
    s.run(gl, fused=True, profile=profile)
    return s.norm2()


TUNED_KEYS = ("fused_tile_bits_c128", "fused_tile_bits_c64", "fused_low_bits", "fused_reg_bits", "fused_mfma")


def time_headline(s, gl, steps, warmup, torch):
    """The fused circuit on s: one untimed run that compiles the pass kernels
    (hipRTC, cached for the process; preparation, not a step), warmup runs,
    then steps timed runs with per-pass HIP events."""
    t0 = time.perf_counter()
    run_step_fused(s, gl)
    torch.cuda.synchronize()
    jit_prepare_s = time.perf_counter() - t0
    nrm = None
    for _ in range(warmup):
        nrm = run_step_fused(s, gl)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pass_ms = []
    for _ in range(steps):
        nrm = run_step_fused(s, gl, profile=True)
        ms, kind = s.run_profile()
        pass_ms += [float(m) for m, k in zip(ms, kind) if k == 0]
    torch.cuda.synchronize()
    return {"dt": time.perf_counter() - t0, "pass_ms": pass_ms, "nrm": nrm, "jit_prepare_s": jit_prepare_s}


def precision_form(sv, torch, n, depth, steps):
    """The same circuit on a complex64 register beside the complex128 result:
    as fused passes, and as dense blocks of at most 4 and 5 qubits (composed
    on the host in FP64, applied on FP32 MFMA); time per step, infidelity
    1 - |<psi32|psi64>|^2 and the largest amplitude error."""
    gl = synth.brickwork_circuit(n, depth, seed=0).array()
    s64 = sv.State(n, "c128").reset(0)
    s64.run(gl, fused=True)
    s32 = sv.State(n, "c64")
    upd = sum(1 << (n - bin(int(r["ctrl"])).count("1")) for r in gl)
    out = {"workload": "brickwork n=%d depth %d from |0..0>, complex64 vs complex128 (fused passes)" % (n, depth)}
    old_k = sv.config_get("block_qubits")
    saved = {k: sv.config_get(k) for k in TUNED_KEYS}
    out["autotuned"] = sv.autotune.apply(sv.autotune.workload_key(n, "c64", gl))
    try:
        for key, kw, kq in (("fused", {"fused": True}, None), ("blocks5", {"blocks": True}, 5),
                            ("blocks4", {"blocks": True}, 4)):
            if kq:
                sv.config_set("block_qubits", kq)
            s32.reset(0)
            s32.run(gl, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                s32.reset(0)
                s32.run(gl, **kw)
                s32.norm2()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            fid = s32.fidelity(s64)
            rec = {"ms_per_step": dt * 1e3, "gate_amp_updates_per_s": upd / dt, "infidelity": 1.0 - fid,
                   "norm2_c64": s32.norm2()}
            if kq:
                plan = sv.plan_blocks(n, gl, kq)
                rec["blocks"] = sum(1 for st in plan if st[0] == "block")
                rec["path"] = "dense blocks of <= %d qubits, FP32 MFMA (v_mfma_f32_32x32x2f32)" % kq
            else:
                rec["path"] = "fused LDS passes, FP32 vector"
            out[key] = rec
    finally:
        sv.config_set("block_qubits", old_k)
        for k, v in saved.items():
            sv.config_set(k, v)
    del s64, s32
    torch.cuda.empty_cache()
    return out


def dense_block_form(sv, torch, n):
    """Dense k-qubit blocks (sv_apply_fused) on an n-qubit register: complex64
    k = 4, 5 on FP32 MFMA, complex128 on the vector path; time per launch
    (HIP events on the launch stream), HBM rate and real FLOP rate (the real
    embedding of a 2^k block costs 8 * 2^k real flops per amplitude)."""
    out = {"workload": "one dense block of random unitary entries, n=%d: complex128 on qubits 0, 7, 15, 22, 29 "
           "(first k); complex64 LDS tiles on qubits 0, 7, 15, 22, 29 (last k, so index bit 0 is a block bit); "
           "c64_k*_direct: qubits 0, 7, 15, 22, 24 (first k; every block bit >= 5, the LDS-free MFMA form)" % n}
    rng = np.random.default_rng(1)
    for dt_, ks in (("c64", (4, 5, "4_direct", "5_direct")), ("c128", (3, 4, 5))):
        s = sv.State(n, dt_).reset(0)
        B = 8 if dt_ == "c64" else 16
        for kk in ks:
            k = int(str(kk)[0])
            D = 1 << k
            z = rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D))
            M, _ = np.linalg.qr(z)
            if "direct" in str(kk):
                qs = [0, 7, 15, 22, 24][:k]
            elif dt_ == "c64":
                qs = [0, 7, 15, 22, 29][-k:]
            else:
                qs = [0, 7, 15, 22, 29][:k]
            s.apply_block(qs, M)
            torch.cuda.synchronize()
            ts = []
            for _ in range(5):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                s.apply_block(qs, M)
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            ms = float(np.median(ts))
            out["%s_k%s" % (dt_, kk)] = {
                "path": ("mfma f32 32x32x2, no LDS" if "direct" in str(kk) else "mfma f32 32x32x2, LDS tiles")
                if dt_ == "c64" else "vector fp64",
                "ms": ms,
                "hbm_gbps": 2 * (1 << n) * B / (ms * 1e-3) / 1e9,
                "tflops": 8 * D * (1 << n) / (ms * 1e-3) / 1e12,
            }
        del s
        torch.cuda.empty_cache()
    return out


def qft_form(sv, torch, n):
    """The QFT circuit of sec. 2.3.2 (n Hadamards, n(n-1)/2 controlled R_k,
    floor(n/2) swaps) on a random complex128 state, as fused passes, with the
    final swaps as one bit-permutation pass (default) or one kernel each;
    and sv_qft's FFT block passes (blocks of 8 index bits), with and without
    the final bit reversal."""
    g = synth.qft_circuit(n).array()
    s = sv.State(n, "c128").load(synth.random_state(n, 0))
    out = {"workload": "QFT n=%d, complex128, random normalised input (seed 0), fused passes" % n}
    for runs in (1, 0):
        sv.config_set("swap_runs", runs)
        s.run(g, fused=True)
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            s.run(g, fused=True)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        s.run(g, fused=True, profile=True)
        ms, kind = s.run_profile()
        out["bit_permutation_pass" if runs else "swap_per_kernel"] = {
            "ms": min(ts) * 1e3, "passes": int(np.sum(kind == 0)), "swap_launches": int(np.sum(kind == 1)),
            "swap_ms": float(np.sum(ms[kind == 1]))}
    sv.config_set("swap_runs", 1)
    # sv_qft as FFT block passes (the default engine for n >= 12): with the
    # bit reversal (one bit-permutation pass) and without it
    cnt = ctypes.c_int64()
    sv.load_library().sv_qft_plan(n, 0, n, None, 0, ctypes.byref(cnt))
    passes = int(cnt.value)
    for key, bitrev in (("fft", False), ("fft_bitrev", True)):
        s.qft(bitrev=bitrev)
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            s.qft(bitrev=bitrev)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        out[key] = {"ms": min(ts) * 1e3, "block_passes": passes}
    out["fft_bitrev"]["hbm_gbps"] = passes * 2 * (1 << n) * 16 / (out["fft_bitrev"]["ms"] * 1e-3) / 1e9
    del s
    torch.cuda.empty_cache()
    return out


def ht_robustness_form(sv, torch, n=20, k=100, B=2048):
    """The Hadamard-transform robustness experiment of sec. 4.3.1 on the
    batched engine: the HT applied k times (k even) to |0...0> of an n-qubit
    register under depolarizing noise p and operational error sigma; the
    |0><0| term of the density matrix is the mean of |alpha_0|^2 over B
    complex64 trajectories.  The closed forms of sec. 4.3.1 are
    ((1 + (1 - 4p/3)^k)/2)^n and ((1 + e^{-9 k sigma^2 / 4})/2)^n; for both
    errors together their product is listed."""
    init = synth.GateList().array()
    it = synth.hadamard_transform(n).array()
    b = sv.Batch(n, B, "c64")
    rows = []
    t0 = time.perf_counter()
    for p in (0.0, 1e-5, 1e-4, 1e-3):
        for sigma in (0.0, 1e-5, 1e-4, 1e-3):
            prob, _ = b.run_noisy(init, it, k, sigma, p, seed=11, target=0)
            dep = ((1 + (1 - 4 * p / 3) ** k) / 2) ** n
            op = ((1 + math.exp(-9 * k * sigma * sigma / 4)) / 2) ** n
            rows.append({"p": p, "sigma": sigma, "mean": float(prob.mean()),
                         "se": float(prob.std(ddof=1) / math.sqrt(B)), "closed_form": dep * op})
    dt = time.perf_counter() - t0
    b.close()
    del b
    torch.cuda.empty_cache()
    return {"workload": "HT applied %d times to |0...0>, n=%d, %d complex64 trajectories per point, Philox seed 11"
            % (k, n, B), "seconds": dt, "table": rows}


# Table 7 of sec. 5.1.1: fidelity of the QFT on Shor's register (N = 187,
# x = 23, 16 qubits) under decoherence p (rows) and operational error sigma
# (columns), and the iterations of Shor's algorithm needed (Fig. qft16 over
# p at sigma = 0, Fig. qft16o over sigma at p = 0); 1000 runs per point.
PAPER_QFT_LEVELS = (0.0, 1e-5, 1e-4, 1e-3, 1e-2)
PAPER_TABLE7 = ((1.0000, 0.9999, 0.9999, 0.9999, 0.9998), (0.9880, 0.9840, 0.9860, 0.9880, 0.9848),
                (0.8837, 0.8897, 0.8827, 0.8801, 0.8980), (0.3287, 0.3399, 0.3332, 0.3209, 0.3363),
                (0.0027, 0.0015, 0.0019, 0.0017, 0.0031))
PAPER_QFT_ITERS_P = (1.9569, 2.1000, 2.3201, 6.0606, 327.00)
PAPER_QFT_ITERS_SIGMA = (1.9569, 1.9841, 2.0283, 1.9015, 1.9607)
# Table 5 of sec. 5.1: N, theoretical 1/Prob_succ, mean iterations of the
# original and the improved algorithm over 100 experiments.
PAPER_TABLE5 = ((21311, 15.79, 6.690, 1.760), (21733, 15.85, 8.990, 2.356), (22999, 16.00, 6.360, 1.730),
                (22523, 15.88, 5.480, 1.770), (22927, 15.91, 3.790, 1.470), (22969, 15.94, 8.050, 2.070),
                (23129, 15.92, 7.133, 1.636))


def qft_robustness_form(sv, torch, B=1000, N=187, x=23):
    """The QFT experiment of sec. 5.1.1 on the batched engine (complex128):
    Shor's register for N = 187, x = 23 (16 qubits; each trajectory its own
    first-register outcome), QFT with depolarizing noise on every qubit after
    each controlled R_k and Gaussian deviations on the H and R_k angles.  Per
    (p, sigma): mean fidelity with the noise-free output and the iterations
    needed (1 / rate at which the plain steps 4-5 find a factor)."""
    m = sv.shor.register_qubits(N)
    g = synth.qft_register_noise(m).array()
    _, a_star, u = synth.shor_draws(N, m, 21, B)
    t0 = time.perf_counter()
    exp = sv.experiments.QftShorNoise(N, x, g, a_star, u, "c128")
    setup_s = time.perf_counter() - t0
    rows, run_ms = [], []
    t0 = time.perf_counter()
    for i, p in enumerate(PAPER_QFT_LEVELS):
        for j, sigma in enumerate(PAPER_QFT_LEVELS):
            out = exp.run(sigma, p, seed=1000 + 10 * i + j)
            run_ms.append(exp.ms)
            f = out["fidelity"]
            rows.append({"p": p, "sigma": sigma, "fidelity": float(f.mean()),
                         "se": float(f.std(ddof=1) / math.sqrt(B)),
                         "iterations": (lambda v: v if math.isfinite(v) else None)(
                             sv.experiments.iterations_needed(out["success"])),
                         "success_rate": float(out["success"].mean()),
                         "paper_fidelity": PAPER_TABLE7[i][j],
                         "paper_iterations": PAPER_QFT_ITERS_P[i] if j == 0 else
                         (PAPER_QFT_ITERS_SIGMA[j] if i == 0 else None)})
    dt = time.perf_counter() - t0
    exp.close()
    del exp
    torch.cuda.empty_cache()
    return {"workload": "QFT on Shor's register, N=%d x=%d, %d qubits, %d complex128 trajectories per point, "
                        "depolarizing on every qubit after each controlled R_k" % (N, x, m, B),
            "setup_s": setup_s, "seconds": dt, "graph_ms_mean": float(np.mean(run_ms)), "table": rows}


def shor_form(sv, torch, experiments=10, Ns=None):
    """Shor's algorithm as sec. 5.1 runs it on 15-bit N (30-qubit complex128
    register, classical modular exponentiation): per N of Table 5, the mean
    number of runs until a factor is found, original and improved
    algorithm on the same random choices, beside 1/Prob_succ; plus the time
    of one run's steps at this size."""
    Ns = Ns or [row[0] for row in PAPER_TABLE5]
    m = 30
    s = sv.State(m, "c128")
    # one run's steps, timed on their own (HIP events around each)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    st = []
    for i in range(4):
        ev[0].record()
        s.shor_prepare(Ns[0], 2, 1000 + i)
        ev[1].record()
        s.qft(bitrev=True)
        ev[2].record()
        s.measure(0.5)
        ev[3].record()
        torch.cuda.synchronize()
        st.append([ev[k].elapsed_time(ev[k + 1]) for k in range(3)])
    st = np.array(st[1:])
    rows = []
    t0 = time.perf_counter()
    total_runs = 0
    for N in Ns:
        paper = next((r for r in PAPER_TABLE5 if r[0] == N), None)
        rec = {"N": N}
        for improved in (False, True):
            its, checks = [], np.zeros((4, 2), dtype=np.int64)
            for e in range(experiments):
                draws = synth.shor_draws(N, m, 7919 * N + e, 400)
                res, _ = sv.shor.factor(s, N, *draws, improved=improved)
                if res.iterations == 0:
                    raise RuntimeError("no factor of %d within 400 runs" % N)
                its.append(res.iterations)
                checks += np.array(res.checks_list())
            key = "improved" if improved else "original"
            total_runs += int(sum(its))
            rec[key] = {"mean_iterations": float(np.mean(its)),
                        "se": float(np.std(its, ddof=1) / math.sqrt(len(its))) if len(its) > 1 else None,
                        "checks_success_failure": checks.tolist() if improved else None}
        rec["theoretical"] = 1.0 / prob_succ_theory(N)
        if paper:
            rec["paper"] = {"theoretical": paper[1], "original": paper[2], "improved": paper[3]}
        rows.append(rec)
    dt = time.perf_counter() - t0
    del s
    torch.cuda.empty_cache()
    return {"workload": "Shor's algorithm with classical modular exponentiation, 15-bit N, 30-qubit complex128 "
                        "register, %d experiments per N and variant" % experiments,
            "step_ms": {"prepare": float(st[:, 0].mean()), "qft_bitrev": float(st[:, 1].mean()),
                        "measure": float(st[:, 2].mean())},
            "seconds": dt, "runs": total_runs, "ms_per_run": dt / max(total_runs, 1) * 1e3, "table": rows}


def prob_succ_theory(N):
    """Prob_succ(N) of sec. 5.1 for N = p q (natural logarithms)."""
    phi, n, f = N, N, 2
    while f * f <= n:
        if n % f == 0:
            while n % f == 0:
                n //= f
            phi -= phi // f
        f += 1
    if n > 1:
        phi -= phi // n
    r = phi / (N - 1)
    return (1 - r) + r * 0.5 * (4 / math.pi ** 2) * math.exp(-0.5772156649015329) / math.log(math.log(N))


def ht_curves_form(sv, torch, n=20, B=2048):
    """Figs. 20d and 20o of sec. 4.3.1: the |0><0| term after the HT applied k
    times (k even) to |0...0> of 20 qubits, for p = 1e-5 .. 1e-2 (sigma = 0)
    and sigma = 1e-5 .. 1e-2 (p = 0), B complex64 trajectories per point,
    beside the closed forms.  Runs of one-qubit gates fold into one matrix
    per qubit and trajectory, so a point costs one pass whatever k is."""
    init = synth.GateList().array()
    it = synth.hadamard_transform(n).array()
    b = sv.Batch(n, B, "c64")
    ks = (2, 4, 8, 16, 32, 50, 64, 80, 100)
    curves = []
    t0 = time.perf_counter()
    for kind, levels in (("p", (1e-5, 1e-4, 1e-3, 1e-2)), ("sigma", (1e-5, 1e-4, 1e-3, 1e-2))):
        for lv in levels:
            pts = []
            for k in ks:
                p, sigma = (lv, 0.0) if kind == "p" else (0.0, lv)
                prob, _ = b.run_noisy(init, it, k, sigma, p, seed=23, target=0)
                cf = (((1 + (1 - 4 * p / 3) ** k) / 2) ** n if kind == "p"
                      else ((1 + math.exp(-9 * k * sigma * sigma / 4)) / 2) ** n)
                pts.append({"k": k, "mean": float(prob.mean()), "se": float(prob.std(ddof=1) / math.sqrt(B)),
                            "closed_form": cf})
            curves.append({kind: lv, "points": pts})
    dt = time.perf_counter() - t0
    b.close()
    del b
    torch.cuda.empty_cache()
    return {"workload": "HT applied k times to |0...0>, n=%d, %d complex64 trajectories per point, Philox seed 23"
            % (n, B), "seconds": dt, "curves": curves}


def grover_robustness_form(sv, torch, n=10, B=1000, max_iter=50):
    """Figs. g10d and g10o of sec. 5.3: mean probability of the marked
    element after j = 0 .. max_iter G-iterations on 10 qubits, B complex128
    trajectories, with depolarizing noise once per G-iteration on every
    qubit (p, sigma = 0) or Gaussian deviations on the H, NOT and phase
    angles (sigma, p = 0); the noise-free curve is sin^2((2j+1) theta),
    theta = asin 2^{-n/2}."""
    marked = synth.grover_marked(n, 3)
    init = synth.hadamard_transform(n).array()
    it = synth.grover_iteration_noise_sites(n, marked).array()
    b = sv.Batch(n, B, "c128")
    b.set_noise_kinds(1 << synth.KIND_U)
    theta = math.asin(2.0 ** (-n / 2))
    js = list(range(0, max_iter + 1, 2))
    curves = []
    t0 = time.perf_counter()
    for kind, levels in (("p", (1e-3, 1e-2, 3e-2)), ("sigma", (1e-2, 3e-2, 1e-1))):
        for lv in levels:
            p, sigma = (lv, 0.0) if kind == "p" else (0.0, lv)
            pts = []
            for j in js:
                prob, _ = b.run_noisy(init, it, j, sigma, p, seed=31, target=marked)
                pts.append({"j": j, "mean": float(prob.mean()), "se": float(prob.std(ddof=1) / math.sqrt(B)),
                            "noise_free": math.sin((2 * j + 1) * theta) ** 2})
            curves.append({kind: lv, "points": pts})
    dt = time.perf_counter() - t0
    b.close()
    del b
    torch.cuda.empty_cache()
    return {"workload": "Grover, n=%d, marked %d, %d complex128 trajectories per point, depolarizing once per "
                        "G-iteration, Philox seed 31" % (n, marked, B), "seconds": dt, "curves": curves}


GOLDEN_GROVER = os.path.join(ROOT, "tests", "golden", "noisy_grover_n20_oracle.txt")


def golden_grover(sigma, p):
    """FP64 oracle trajectories of the noisy Grover workload stored by
    tests/golden/make_noisy_grover_ref.py (written by the oracle alone):
    {traj: (prob_marked, norm2, sampled amplitudes)} and the sample indices."""
    if not os.path.exists(GOLDEN_GROVER):
        return None, {}
    idx, rows = None, {}
    with open(GOLDEN_GROVER) as f:
        for line in f:
            if line.startswith("# sample_indices:"):
                idx = [int(v) for v in line.split(":", 1)[1].split()]
            if line.startswith("#") or not line.strip():
                continue
            v = line.split()
            if float(v[0]) != sigma or float(v[1]) != p:
                continue
            vals = [float(x) for x in v[3:]]
            rows[int(v[2])] = (vals[0], vals[1], np.array(vals[2::2]) + 1j * np.array(vals[3::2]))
    return idx, rows


BATCHED_SIGMAS = (1e-3, 5e-3, 1e-2, 5e-2)
BATCHED_PS = (1e-5, 1e-4, 1e-3)


def batched_form(sv, torch, n, B, iters, sigma, p, n_plain=64, n_ref=256, grid_b=1024):
    """Noisy Grover trajectories on the batched complex64 engine (one HIP
    graph per run) against the plain complex128 per-gate path on the same
    draws; per-trajectory infidelity of complex64 against complex128; the
    stored FP64 oracle trajectories; the (sigma, p) grid."""
    marked = synth.grover_marked(n, 0)
    init = synth.hadamard_transform(n).array()
    it = synth.grover_iteration(n, marked).array()
    b = sv.Batch(n, B, "c64")
    tuned_group = sv.autotune.apply(sv.autotune.workload_key(n, "c64", it, extra="batched B=%d" % B), batch=b)
    # first call: captures the graph (and compiles the pass kernels) on the
    # grid's first point; the graph does not depend on sigma, p or the seed
    t0 = time.perf_counter()
    g0_prob, _ = b.run_noisy(init, it, iters, BATCHED_SIGMAS[0], BATCHED_PS[0], seed=0, target=marked)
    capture_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    prob, nrm = b.run_noisy(init, it, iters, sigma, p, seed=0, target=marked)
    dt = time.perf_counter() - t0
    dev_ms = b.last_run_ms()
    # same draws on n_ref trajectories with complex128 registers
    bref = sv.Batch(n, n_ref, "c128")
    pref, _ = bref.run_noisy(init, it, iters, sigma, p, seed=0, target=marked)
    sub = sv.Batch(n, n_ref, "c64")
    psub, _ = sub.run_noisy(init, it, iters, sigma, p, seed=0, target=marked)
    fid, _ = sub.fidelity(bref)
    infid = 1.0 - fid
    same_as_full = bool(np.array_equal(psub, prob[:n_ref]))
    # stored FP64 oracle trajectories (same draws)
    idx, rows = golden_grover(sigma, p)
    oracle_check = None
    ids = sorted(t for t in rows if t < B)
    first = [t for t in ids if t < n_ref]
    if len(first) >= 16:
        # every stored FP64 oracle trajectory (ids 0..255 in order, then
        # 3584 and 4095; the file may still be growing)
        orc_p = np.array([rows[t][0] for t in first])
        dprob = max(abs(prob[t] - rows[t][0]) for t in ids)
        damp = 0.0
        for t in ids[:: max(1, len(ids) // 32)] + [ids[-1]]:
            st = b.state(t).astype(np.complex128)
            damp = max(damp, float(np.max(np.abs(st[idx] - rows[t][2]))))
        oracle_check = {"trajectories": len(ids), "oracle_mean": float(orc_p.mean()),
                        "oracle_se": float(orc_p.std(ddof=1) / math.sqrt(len(first))),
                        "gpu_mean_same_ids": float(prob[first].mean()),
                        "gpu_mean_all": float(prob.mean()),
                        "max_abs_dprob": float(dprob), "max_abs_damp_sampled": damp,
                        "source": "tests/golden/noisy_grover_n20_oracle.txt (FP64 oracle, same draws)"}
    b.close()
    sub.close()
    bref.close()
    del b, sub, bref
    torch.cuda.empty_cache()
    # plain complex128 per-gate path, one trajectory at a time, same draws:
    # the explicit gate list of each trajectory (perturbed gates + drawn
    # Paulis) through one kernel per gate
    s = sv.State(n, "c128")
    warm = sv.trajectory_gates(n, init, it, 2, sigma, p, 0, B - 1)
    s.reset(0)
    s.run(warm)
    torch.cuda.synchronize()
    plain_p = []
    ngates = 0
    t0 = time.perf_counter()
    for t in range(n_plain):
        gl = sv.trajectory_gates(n, init, it, iters, sigma, p, 0, t)
        ngates += len(gl)
        s.reset(0)
        s.run(gl)
        plain_p.append(s.prob((1 << n) - 1, marked))
    torch.cuda.synchronize()
    pg_per_traj = (time.perf_counter() - t0) / n_plain
    plain_p = np.array(plain_p)
    del s
    torch.cuda.empty_cache()
    theta = math.asin(2 ** (-n / 2))
    rec = {
        "workload": "noisy Grover n=%d, %d complex64 trajectories, %d iterations, sigma=%g, p=%g, Philox seed 0"
        % (n, B, iters, sigma, p),
        "seconds": dt,
        "device_ms": dev_ms,
        "autotuned": tuned_group,
        "capture_and_first_run_s": capture_s,
        "trajectories_per_s": B / dt,
        "success_mean": float(prob.mean()),
        "success_se": float(prob.std(ddof=1) / math.sqrt(B)),
        "noise_free_success": math.sin((2 * iters + 1) * theta) ** 2,
        "max_norm_deviation_c64": float(np.max(np.abs(nrm - 1.0))),
        "infidelity_c64_vs_c128": {"trajectories": n_ref, "max": float(infid.max()), "mean": float(infid.mean()),
                                   "c64_subbatch_bit_identical_to_full_batch": same_as_full},
        "oracle_check": oracle_check,
        "plain_c128": {
            "seconds_per_trajectory": pg_per_traj,
            "trajectories_per_s": 1.0 / pg_per_traj,
            "measured_trajectories": n_plain,
            "gates_per_trajectory": ngates / n_plain,
            "max_abs_dprob_vs_batched_c128": float(np.max(np.abs(plain_p - pref[:n_plain]))),
            "note": "same draws: svb_trajectory_gates lists (perturbed gates plus drawn Paulis), one kernel per gate, "
                    "host list generation included; rate measured on %d trajectories and applied per trajectory" % n_plain,
        },
        "speedup_vs_plain_c128": (B / dt) * pg_per_traj,
        "speedup_holds_at_infidelity_1e-6": bool(infid.max() <= 1e-6),
    }
    # (sigma, p) grid: mean and SE per point (the capture run gave the first)
    grid = []
    gb = sv.Batch(n, grid_b, "c64")
    t0 = time.perf_counter()
    for sg in BATCHED_SIGMAS:
        for pp in BATCHED_PS:
            if grid_b == B and (sg, pp) == (BATCHED_SIGMAS[0], BATCHED_PS[0]):
                pr = g0_prob
            elif grid_b == B and (sg, pp) == (sigma, p):
                pr = prob
            else:
                pr, _ = gb.run_noisy(init, it, iters, sg, pp, seed=0, target=marked)
            _, grows = golden_grover(sg, pp)
            og = [grows[t][0] for t in range(min(grid_b, 8)) if t in grows]
            grid.append({"sigma": sg, "p": pp, "mean": float(pr.mean()),
                         "se": float(pr.std(ddof=1) / math.sqrt(len(pr))),
                         "max_abs_dprob_vs_oracle_ids_0_7": float(np.max(np.abs(pr[:len(og)] - og))) if og else None})
    rec["grid"] = {"trajectories_per_point": grid_b, "seconds": time.perf_counter() - t0, "points": grid}
    gb.close()
    del gb
    torch.cuda.empty_cache()
    return rec


def adjoint_form(sv, torch, n):
    ng = n * (n + 1) // 2
    eps = synth.qft_eps(ng, 1, 1e-2)
    gates = synth.qft_perturbed(n, eps).array()
    dparam = np.array([0 if r["kind"] == synth.KIND_H else (1 if r["kind"] == synth.KIND_RK else -1) for r in gates],
                      np.int32)
    psi0 = synth.random_state(n, 0)
    out = {"workload": "QFT n=%d, %d gates with one over-rotation each, loss 1 - |<QFT psi0|QFT(eps) psi0>|^2" % (n, ng)}
    for dt_ in ("c128", "c64"):
        NP = np.complex128 if dt_ == "c128" else np.complex64
        p0 = sv.State(n, dt_).load(psi0.astype(NP))
        phi = sv.State(n, dt_).copy_from(p0)
        phi.run(synth.qft_circuit(n).array(), fused=True)
        psi = sv.State(n, dt_)
        lam = sv.State(n, dt_)
        times = []
        for rep in range(3):
            psi.copy_from(p0)
            lam.copy_from(phi)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            psi.run(gates)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            grad, A = sv.adjoint(psi, lam, gates, dparam)
            t2 = time.perf_counter()
            times.append((t1 - t0, t2 - t1))
        fw = min(t[0] for t in times)
        bw = min(t[1] for t in times)
        out[dt_] = {"forward_ms": fw * 1e3, "gradient_ms": bw * 1e3, "loss": 1 - abs(A) ** 2,
                    "max_abs_grad": float(np.max(np.abs(grad)))}
        del p0, phi, psi, lam
        torch.cuda.empty_cache()
    return out


# HBM traffic of the dominant kernel from rocprofv3 counter runs (FETCH_SIZE,
# then WRITE_SIZE, separate runs), each scaled by what the same counter reads
# for a plain copy of known size.  Valid only for the pass generator and
# planner sources they were measured with; otherwise reported as null.
TRAFFIC = {
    "sources": "cbccbcd0f9adbf47",
    "bytes_per_launch": 3.4366e+10,
    "fetch_bytes_per_launch": 1.7180e+10,
    "write_bytes_per_launch": 1.7186e+10,
    "calibration": "FETCH_SIZE x 2.0000, WRITE_SIZE x 1.0000 (plain 4 GiB copy)",
    "profile": "profiles/sv_pass_brickwork_n30_c128.md",
}


def source_digest():
    import hashlib

    h = hashlib.sha256()
    for f in ("jit.hip", "fused.hip", "rotations.cpp"):
        with open(os.path.join(ROOT, "paper_quant_ph_0201042_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_record():
    if TRAFFIC is None or TRAFFIC["sources"] != source_digest():
        return None
    return TRAFFIC["bytes_per_launch"]


def traffic_detail():
    if TRAFFIC is None or TRAFFIC["sources"] != source_digest():
        return None
    return {k: v for k, v in TRAFFIC.items() if k != "sources"}


PEAK_FP64_TFLOPS = 78.6  # MI355X FP64 vector: 256 CUs x 2.4 GHz x 64 FMA lanes x 2


def algorithmic_flops(n, gl):
    """Real flops the circuit needs per step: 14 per amplitude a dense
    one-qubit gate changes (2^(n-c) with c controls; four complex products
    and two complex additions per pair), 6 per amplitude a diagonal gate
    changes (2^(n-1-c)), 0 for permutations (exact X, CNOT, swaps)."""
    import paper_quant_ph_0201042_amd as sv

    total = 0.0
    for r in gl:
        if r["kind"] == synth.KIND_SWAP:
            continue
        c = bin(int(r["ctrl"])).count("1")
        U = sv.gate_matrix(r)
        if U[0, 1] == 0 and U[1, 0] == 0:
            total += 6.0 * 2 ** (n - 1 - c)
        elif U[0, 0] == 0 and U[1, 1] == 0 and U[0, 1] == 1 and U[1, 0] == 1:
            continue
        else:
            total += 14.0 * 2 ** (n - c)
    return total


def fp64_share(n, gl, n_passes, avg_pass_ms):
    """Busy share of the FP64 vector units in the average pass: 16 FP64
    multiply/FMA instructions per amplitude pair of a dense gate (wave64,
    4 cycles each on a SIMD16) against 1024 SIMDs at 2.4 GHz."""
    dense = 0
    for r in gl:
        if r["kind"] in (synth.KIND_SU2, synth.KIND_U, synth.KIND_H, synth.KIND_ROT):
            dense += 1 << (n - 1 - bin(int(r["ctrl"])).count("1"))
    fma_per_pass = 16.0 * dense / n_passes
    peak_fma_per_s = PEAK_FP64_TFLOPS * 1e12 / 2
    return fma_per_pass / peak_fma_per_s / (avg_pass_ms * 1e-3)


def roofline_record(n, gl, n_passes, avg_pass_ms, n_launches, bytes_per_pass):
    """The pass kernel against both of its ceilings.  Per launch it moves
    2 * 2^n * 16 B and does the step's algorithmic flops / passes; the bound
    is the ceiling whose time (work / peak) is the larger one."""
    flops_per_pass = algorithmic_flops(n, gl) / n_passes
    t_hbm = bytes_per_pass / (PEAK_HBM_GBS * 1e9)
    t_alu = flops_per_pass / (PEAK_FP64_TFLOPS * 1e12)
    sec = avg_pass_ms * 1e-3
    hbm = {"achieved": bytes_per_pass / sec / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": bytes_per_pass / sec / 1e9 / PEAK_HBM_GBS, "per_launch": bytes_per_pass}
    alu = {"achieved": flops_per_pass / sec / 1e12, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
           "frac": flops_per_pass / sec / 1e12 / PEAK_FP64_TFLOPS, "per_launch": flops_per_pass}
    main, other, bound = (alu, hbm, "alu") if t_alu >= t_hbm else (hbm, alu, "hbm")
    return {
        "kernel": "sv_pass: fused pass specialised to its op list (hipRTC, gfx950), one read + one write "
        "of the register per launch",
        "bound": bound,
        "achieved": main["achieved"],
        "peak": main["peak"],
        "unit": main["unit"],
        "frac": main["frac"],
        "traffic": traffic_record(),
        "avg_launch_ms": avg_pass_ms,
        "launches": n_launches,
        "work_per_launch": main["per_launch"],
        "other_ceiling": {"bound": "hbm" if bound == "alu" else "alu", **other},
        "fp64_busy_share": fp64_share(n, gl, n_passes, avg_pass_ms),
        "traffic_detail": traffic_detail(),
    }


def copy_probe(torch, gib=4, reps=3):
    """A plain device copy of known size, for calibrating HBM byte counters."""
    n = (gib << 30) // 16
    x = torch.ones(n, dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 16, "copy_probe_bytes_written": n * 16, "reps": reps}))


def perm_probe(torch, sv, n=28):
    """One dense gate on the top qubit (the streaming pair kernel) and one
    bit reversal of the index (the permutation pass) on an n-qubit
    complex128 register, twice each, for counter comparisons."""
    s = sv.State(n, "c128").reset(5)
    H = np.array([[1, 1], [1, -1]]) / math.sqrt(2)
    gl = synth.GateList()
    for q in range(n // 2):
        gl.add(synth.KIND_SWAP, q, target2=n - 1 - q)
    g = gl.array()
    for _ in range(2):
        s.apply_1q(0, H)
        s.run(g, fused=True)
    torch.cuda.synchronize()
    print(json.dumps({"perm_probe_n": n, "bytes_per_launch": 2 * (1 << n) * 16}))


def batch_probe(torch, sv, iters, B, n=20):
    """Noisy Grover on the batched complex64 engine (the batched form's
    workload, sigma = 1e-2, p = 1e-4) for a few iterations, twice: the
    first run captures the graph, the second is the one to read."""
    marked = synth.grover_marked(n, 0)
    init = synth.hadamard_transform(n).array()
    it = synth.grover_iteration(n, marked).array()
    b = sv.Batch(n, B, "c64")
    npass, _ = sv.batch.plan(n, "c64", init, it, iters)
    for _ in range(2):
        b.run_noisy(init, it, iters, 1e-2, 1e-4, seed=0, target=marked)
    torch.cuda.synchronize()
    print(json.dumps({"batch_probe_n": n, "registers": B, "iterations": iters, "passes_per_run": npass,
                      "run_ms": round(b.last_run_ms(), 3), "bytes_per_pass": 2 * B * (1 << n) * 8}))
    b.close()


def autotune_run(torch, sv, out):
    """Runs the library's autotuner on the benchmark workloads (the n=30
    brickwork in both dtypes, the batched noisy Grover) and writes the
    chosen values to out, in the format of the package's tuned.json."""
    from paper_quant_ph_0201042_amd import autotune

    n = 30
    gl = synth.brickwork_circuit(n, 20, seed=0).array()
    keys = ("fused_tile_bits_c128", "fused_tile_bits_c64", "fused_low_bits", "fused_reg_bits", "fused_mfma")
    for dt in ("c128", "c64"):
        defaults = {k: sv.config_get(k) for k in keys}
        s = sv.State(n, dt)
        t0 = time.perf_counter()
        res = autotune.tune_fused(s, gl, reps=3)
        print(dt, "tuned in %.1f s" % (time.perf_counter() - t0), json.dumps(res), flush=True)
        autotune.save(autotune.workload_key(n, dt, gl), res, out,
                      note="n=30 brickwork depth 20 (seed-independent key), sv_tune_fused reps=3")
        for k, v in defaults.items():
            sv.config_set(k, v)
        del s
        torch.cuda.empty_cache()
    nb, B = 20, 4096
    marked = synth.grover_marked(nb, 0)
    init = synth.hadamard_transform(nb).array()
    it = synth.grover_iteration(nb, marked).array()
    b = sv.Batch(nb, B, "c64")
    t0 = time.perf_counter()
    res = autotune.tune_group(b, init, it, 8, reps=2)
    print("batched tuned in %.1f s" % (time.perf_counter() - t0), json.dumps(res), flush=True)
    autotune.save(autotune.workload_key(nb, "c64", it, extra="batched B=%d" % B), res, out,
                  note="noisy Grover n=20, B=4096, svb_tune_group over 8 iterations")
    b.close()


def form_oracle_timings():
    """The plain oracle on the host beside each form, on bounded samples
    (single thread; every sample stated)."""
    import oracle

    out = {}
    # noisy Grover: one trajectory, the first 20 of 804 iterations, scaled
    n, iters_s, iters = 20, 20, 804
    marked = synth.grover_marked(n, 0)
    init = synth.hadamard_transform(n).array()
    it = synth.grover_iteration(n, marked).array()
    t0 = time.perf_counter()
    oracle.noisy_grover_traj(n, marked, iters_s, 1e-2, 1e-4, 0, 0, init, it)
    dt = time.perf_counter() - t0
    per_traj = dt * iters / iters_s
    out["batched"] = {"trajectories_per_s": 1.0 / per_traj, "cores": 1, "kind": "oracle",
                      "sample": "one trajectory, first %d of %d iterations (%.1f s), scaled to %d" % (iters_s, iters, dt, iters)}
    # adjoint: the full 300-parameter sweep at n = 20 (the form runs n = 24)
    na = 20
    ng = na * (na + 1) // 2
    gates = synth.qft_perturbed(na, synth.qft_eps(ng, 1, 1e-2)).array()
    dparam = np.array([0 if r["kind"] == synth.KIND_H else (1 if r["kind"] == synth.KIND_RK else -1) for r in gates],
                      np.int32)
    psi0 = synth.random_state(na, 0)
    phi = oracle.run(psi0, synth.qft_circuit(na).array())
    t0 = time.perf_counter()
    oracle.adjoint(psi0, phi, gates, dparam)
    dt = time.perf_counter() - t0
    out["adjoint"] = {"seconds": dt, "cores": 1, "kind": "oracle",
                      "sample": "forward run + adjoint sweep of QFT n=%d (%d parameters); the form uses n=24" % (na, ng)}
    # one dense 5-qubit block at n = 22
    nb = 22
    rng = np.random.default_rng(1)
    M, _ = np.linalg.qr(rng.standard_normal((32, 32)) + 1j * rng.standard_normal((32, 32)))
    a = synth.random_state(nb, 2)
    t0 = time.perf_counter()
    oracle.apply_kq(a, [0, 7, 15, 19, 21], M)
    dt = time.perf_counter() - t0
    out["dense_blocks"] = {"amplitudes_per_s": (1 << nb) / dt, "cores": 1, "kind": "oracle",
                           "sample": "one 5-qubit complex128 block at n=%d (%.2f s)" % (nb, dt)}
    return out


def host_facts():
    """Host core count, CPU model and this process's CPU set."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = sorted(os.sched_getaffinity(0))
    except AttributeError:
        allowed = list(range(os.cpu_count() or 1))
    return {"nproc": os.cpu_count(), "cpus_allowed": len(allowed), "cpu_model": model}, allowed


def cpu_baseline(gl_array, n, budget_s=20.0):
    """The plain oracle on the host: the first gates of the same circuit on an
    n-qubit FP64 register, single-threaded and pinned to one core, until
    about budget_s of work; then one gate of each microbench class at the
    lowest and highest target."""
    import oracle

    facts, allowed = host_facts()
    core = allowed[0]
    pinned = False
    try:
        os.sched_setaffinity(0, {core})
        pinned = True
    except (AttributeError, OSError):
        pass
    L = oracle.lib()
    a = np.empty(1 << n, dtype=np.complex128)
    a[:] = 0.0  # touch every page (untimed) so the timed gates pay no first-touch faults
    a[0] = 1.0
    ptr = a.ctypes.data
    done_amps = 0
    gates_done = 0
    t0 = time.perf_counter()
    for rec in gl_array:
        one = np.ascontiguousarray(rec.reshape(1))
        rc = L.orc_run(ptr, n, one.ctypes.data, 1)
        assert rc == 0
        done_amps += 1 << (n - bin(int(rec["ctrl"])).count("1"))
        gates_done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    per_class = {}
    for cls in MB_CLASSES:
        rates = []
        for q in (0, n - 1):
            g = synth.GateList()
            kind, ctrl, iarg, par = mb_gate(cls, n, q)
            g.add(kind, q, ctrl=ctrl, iarg=iarg, p=par)
            one = g.array()
            t1 = time.perf_counter()
            assert L.orc_run(ptr, n, one.ctypes.data, 1) == 0
            rates.append(mb_updates(cls, n) / (time.perf_counter() - t1))
        per_class[cls] = rates
    if pinned:
        os.sched_setaffinity(0, set(allowed))
    return {
        "value": done_amps / dt,
        "unit": "gate-amp updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": "first %d gates of the same n=%d brickwork circuit (seed 0), complex128, "
        "single-threaded plain C oracle, %.1f s" % (gates_done, n, dt),
        **facts,
        "pinning": ("sched_setaffinity to core %d" % core) if pinned else "none",
        "per_class_q0_q%d" % (n - 1): per_class,
    }


# ---------------------------------------------------------------- microbench

MB_CLASSES = ("haar1q", "cnot", "cp", "x")


def mb_gate(cls, n, q):
    """(kind, ctrl, iarg, p) of one microbench gate on target q: a fixed Haar SU(2),
    CNOT with the neighbouring qubit as control, the controlled phase R_2
    (diag(1, i)) with that control, and an exact NOT."""
    c = q - 1 if q > 0 else 1
    cbit = 1 << (n - 1 - c)
    if cls == "haar1q":
        return synth.KIND_SU2, 0, 0, [0.3, -0.5, 0.7, 0.2]
    if cls == "cnot":
        return synth.KIND_X, cbit, 0, None
    if cls == "cp":
        return synth.KIND_RK, cbit, 2, None
    return synth.KIND_X, 0, 0, None


def mb_updates(cls, n):
    """Amplitudes the gate changes (gate-amp updates)."""
    return {"haar1q": 1 << n, "cnot": 1 << (n - 1), "cp": 1 << (n - 2), "x": 1 << n}[cls]


def mb_bytes(cls, n, q, w):
    """max(algorithmic, 128-B-line-granular) HBM bytes of one gate: the
    changed amplitudes read and written, or every line holding one."""
    line_bits = {16: 3, 8: 4}[w]
    c = q - 1 if q > 0 else 1
    fixed = {"haar1q": [], "x": [], "cnot": [n - 1 - c], "cp": [n - 1 - c, n - 1 - q]}[cls]
    frac_lines = 1.0
    for b in fixed:
        if b >= line_bits:
            frac_lines /= 2
    alg = 2.0 * w * mb_updates(cls, n)
    return max(alg, 2.0 * w * (1 << n) * frac_lines)


def measure_copy(torch, gib=4, reps=5):
    """Device-to-device copy of gib GiB (torch copy kernel): (read + write)
    bytes over the median HIP-event time."""
    x = torch.empty((gib << 30) // 8, dtype=torch.float64, device="cuda")
    x.fill_(1.0)
    y = torch.empty_like(x)
    y.copy_(x)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record()
    for i in range(reps):
        y.copy_(x)
        ev[i + 1].record()
    torch.cuda.synchronize()
    ms = float(np.median([ev[i].elapsed_time(ev[i + 1]) for i in range(reps)]))
    del x, y
    torch.cuda.empty_cache()
    return 2.0 * (gib << 30) / (ms * 1e-3) / 1e9


def microbench_form(sv, torch, n=30, reps=10, warm=3):
    """Every target q of an n-qubit register x {Haar 1q, CNOT, CP, X} x
    {complex128, complex64}, one kernel per gate: median of reps HIP-event
    intervals (back-to-back launches, so each interval is one kernel) after
    warm untimed launches; HBM rate against 8 TB/s and a measured copy."""
    copy_gbps = measure_copy(torch)
    table = []
    for dt in ("c128", "c64"):
        w = 16 if dt == "c128" else 8
        s = sv.State(n, dt).reset(0)
        for cls in MB_CLASSES:
            for q in range(n):
                kind, ctrl, iarg, par = mb_gate(cls, n, q)
                g = synth.GateList().add(kind, q, ctrl=ctrl, iarg=iarg, p=par).array()
                U = sv.gate_matrix(g[0])
                call = (lambda: s.apply_ctrl(ctrl, q, U)) if ctrl else (lambda: s.apply_1q(q, U))
                for _ in range(warm):
                    call()
                ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
                ev[0].record()
                for i in range(reps):
                    call()
                    ev[i + 1].record()
                torch.cuda.synchronize()
                ms = float(np.median([ev[i].elapsed_time(ev[i + 1]) for i in range(reps)]))
                by = mb_bytes(cls, n, q, w)
                gbps = by / (ms * 1e-3) / 1e9
                table.append({"dtype": dt, "class": cls, "q": q, "ms": ms, "gbps": gbps,
                              "frac_peak": gbps / PEAK_HBM_GBS, "frac_copy": gbps / copy_gbps,
                              "updates_per_s": mb_updates(cls, n) / (ms * 1e-3)})
        del s
        torch.cuda.empty_cache()
    summary = {}
    for dt in ("c128", "c64"):
        for cls in MB_CLASSES:
            rows = [r for r in table if r["dtype"] == dt and r["class"] == cls]
            fr = np.array([r["frac_peak"] for r in rows])
            worst = rows[int(np.argmin(fr))]
            summary["%s_%s" % (dt, cls)] = {"min": float(fr.min()), "median": float(np.median(fr)),
                                            "max": float(fr.max()), "worst_q": worst["q"],
                                            "below_0.7": int(np.sum(fr < 0.7))}
    return {"workload": "one gate per kernel on an n=%d register, every target q, median of %d HIP-event "
                        "intervals after %d warm-up launches; bytes = max(algorithmic, 128-B line granular)"
                        % (n, reps, warm),
            "copy_gbps": copy_gbps, "summary": summary, "table": table}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--depth", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--pg-steps", type=int, default=1, help="timed steps of the per-gate comparison (0: skip)")
    ap.add_argument("--no-forms", action="store_true", help="skip the complex64, batched and adjoint forms")
    ap.add_argument("--batched-iters", type=int, default=804)
    ap.add_argument("--batched-b", type=int, default=4096)
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--copy-probe", action="store_true", help="only run a plain 4 GiB copy (counter calibration)")
    ap.add_argument("--perm-probe", action="store_true",
                    help="only run one dense gate and one bit reversal at n=28 (counter comparison)")
    ap.add_argument("--autotune", metavar="PATH",
                    help="only run the autotuner on the benchmark workloads and write its choices to PATH")
    ap.add_argument("--batch-probe", type=int, default=0, metavar="ITERS",
                    help="only run ITERS noisy Grover iterations of the batched form's workload, twice (profiling)")
    ap.add_argument("--shor-experiments", type=int, default=10, help="experiments per N and variant")
    ap.add_argument("--plain-trajectories", type=int, default=64,
                    help="trajectories of the plain complex128 per-gate baseline of the batched form")
    ap.add_argument("--grid-b", type=int, default=512, help="trajectories per point of the (sigma, p) grid")
    ap.add_argument("--forms-out", default=os.path.join("bench_out", "bench_forms.json"),
                    help="side file for the forms' whole records ('' for none)")
    ap.add_argument("--only-form", choices=["precision_c64", "batched", "microbench", "adjoint", "dense_blocks", "qft",
                                            "ht_robustness", "qft_robustness", "shor", "ht_curves",
                                            "grover_robustness"],
                    help="only run one form and print its record (for profiling)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the engine has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_probe:
        copy_probe(torch)
        return
    import paper_quant_ph_0201042_amd as sv

    if args.perm_probe:
        perm_probe(torch, sv)
        return
    if args.batch_probe:
        batch_probe(torch, sv, args.batch_probe, args.batched_b)
        return
    if args.autotune:
        autotune_run(torch, sv, args.autotune)
        return

    n, depth = args.n, args.depth
    if args.only_form:
        forms = {
            "precision_c64": lambda: precision_form(sv, torch, n, depth, args.steps),
            "batched": lambda: batched_form(sv, torch, 20, args.batched_b, args.batched_iters, 1e-2, 1e-4,
                                            n_plain=args.plain_trajectories, grid_b=args.grid_b),
            "microbench": lambda: microbench_form(sv, torch, n),
            "adjoint": lambda: adjoint_form(sv, torch, 24),
            "dense_blocks": lambda: dense_block_form(sv, torch, n),
            "qft": lambda: qft_form(sv, torch, 28),
            "ht_robustness": lambda: ht_robustness_form(sv, torch),
            "qft_robustness": lambda: qft_robustness_form(sv, torch),
            "shor": lambda: shor_form(sv, torch, args.shor_experiments),
            "ht_curves": lambda: ht_curves_form(sv, torch),
            "grover_robustness": lambda: grover_robustness_form(sv, torch),
        }
        print(json.dumps({args.only_form: forms[args.only_form]()}))
        return
    gl = synth.brickwork_circuit(n, depth, seed=0).array()
    gates = prepared_gates(sv, gl, n)
    updates_per_step = sum(g[3] for g in gates)
    n_dom = sum(1 for g in gates if g[4])
    _, pass_of, masks = sv.plan_fused(n, "c128", gl)
    n_passes = len(masks)

    s = sv.State(n, "c128")
    # ---- fused path (headline), with the library defaults and, when the
    # tuned-value file holds this workload, with the autotuner's choice
    tkey = sv.autotune.workload_key(n, "c128", gl)
    tuned_ent = sv.autotune.load().get(tkey)
    default_cfg = {k: sv.config_get(k) for k in TUNED_KEYS}
    dflt = time_headline(s, gl, args.steps, args.warmup, torch)
    use = dflt
    autotune_rec = {"key": tkey, "default": {"ms_per_step": dflt["dt"] / args.steps * 1e3, "config": default_cfg},
                    "tuned": None}
    if tuned_ent is not None:
        sv.autotune.apply(tkey)
        _, _, masks_t = sv.plan_fused(n, "c128", gl)
        tuned = time_headline(s, gl, args.steps, args.warmup, torch)
        autotune_rec["tuned"] = {"ms_per_step": tuned["dt"] / args.steps * 1e3, "config": dict(tuned_ent["best"]),
                                 "passes": len(masks_t), "tuner_best_ms": tuned_ent.get("best_ms")}
        if tuned["dt"] < dflt["dt"]:
            use, masks = tuned, masks_t
            n_passes = len(masks)
        else:
            for k, v in default_cfg.items():
                sv.config_set(k, v)
    autotune_rec["headline_uses"] = "tuned" if use is not dflt else "default"
    dt, pass_ms, nrm, jit_prepare_s = use["dt"], use["pass_ms"], use["nrm"], use["jit_prepare_s"]
    if abs(nrm - 1.0) > 1e-10:
        raise RuntimeError("norm drifted: %r" % nrm)
    avg_pass_ms = float(np.mean(pass_ms))
    bytes_per_pass = 2 * (1 << n) * 16
    achieved = bytes_per_pass / (avg_pass_ms * 1e-3) / 1e9

    # ---- per-gate path (every gate its own sweep), same circuit
    global ev_pairs_done
    pg_steps = max(0, args.pg_steps)
    dt_pg, pg_avg_ms, pg_achieved, durs_ms = float("nan"), float("nan"), float("nan"), []
    if pg_steps:
        nrm = run_step_per_gate(s, gates)
        torch.cuda.synchronize()
        ev_pairs_done = []
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(n_dom * pg_steps)]
        t0 = time.perf_counter()
        for _ in range(pg_steps):
            nrm = run_step_per_gate(s, gates, evs)
        torch.cuda.synchronize()
        dt_pg = time.perf_counter() - t0
        if abs(nrm - 1.0) > 1e-10:
            raise RuntimeError("norm drifted (per-gate): %r" % nrm)
        durs_ms = [e0.elapsed_time(e1) for e0, e1 in ev_pairs_done]
        pg_avg_ms = float(np.mean(durs_ms))
        pg_achieved = bytes_per_pass / (pg_avg_ms * 1e-3) / 1e9

    rec = {
        "metric": METRIC,
        "value": updates_per_step * args.steps / dt,
        "unit": "gate-amp updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "brickwork random circuit, n=%d, depth %d, complex128, fused LDS passes" % (n, depth),
            "n": n,
            "depth": depth,
            "gates_per_step": len(gates),
            "fused_passes_per_step": n_passes,
            "seed": 0,
        },
        "hbm_gbps": n_passes * bytes_per_pass * args.steps / dt / 1e9,
        "roofline": roofline_record(n, gl, n_passes, avg_pass_ms, len(pass_ms), bytes_per_pass),
        "jit_prepare_s": jit_prepare_s,
        "autotune": autotune_rec,
        "per_gate_path": None if pg_steps == 0 else {
            "value": updates_per_step * pg_steps / dt_pg,
            "unit": "gate-amp updates/s",
            "ms_per_step": dt_pg / pg_steps * 1e3,
            "dominant_kernel": "k_pairs<c128> dense one-qubit gate, target bit >= 6",
            "achieved_gbps": pg_achieved,
            "frac": pg_achieved / PEAK_HBM_GBS,
            "avg_launch_ms": pg_avg_ms,
            "launches": len(durs_ms),
        },
    }
    forms = {}
    if not args.no_forms:
        del s
        torch.cuda.empty_cache()
        plan = [
            ("precision_c64", lambda: precision_form(sv, torch, n, depth, args.steps)),
            ("batched", lambda: batched_form(sv, torch, 20, args.batched_b, args.batched_iters, 1e-2, 1e-4,
                                             n_plain=args.plain_trajectories, grid_b=args.grid_b)),
            ("microbench", lambda: microbench_form(sv, torch, n)),
            ("adjoint", lambda: adjoint_form(sv, torch, 24)),
            ("dense_blocks", lambda: dense_block_form(sv, torch, n)),
            ("qft", lambda: qft_form(sv, torch, 28)),
            ("ht_robustness", lambda: ht_robustness_form(sv, torch)),
            ("qft_robustness", lambda: qft_robustness_form(sv, torch)),
            ("shor", lambda: shor_form(sv, torch, args.shor_experiments)),
            ("ht_curves", lambda: ht_curves_form(sv, torch)),
        ]
        for name, fn in plan:
            t0 = time.perf_counter()
            forms[name] = fn()
            print("# form %s: %.1f s" % (name, time.perf_counter() - t0), flush=True)
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(gl, n, args.cpu_budget)
        if not args.no_forms:
            forms["cpu_oracle_beside_forms"] = form_oracle_timings()
    side = write_forms(args.forms_out, rec, forms)
    print(json.dumps(final_line(rec, forms, side), separators=(",", ":")))


def write_forms(path, rec, forms):
    """Every form's whole record (tables, curves, per-point values) goes to a
    side file; the last stdout line keeps the headline keys only."""
    if not path:
        return None
    try:
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        with open(path, "w") as f:
            json.dump({"headline": rec, "forms": forms}, f, indent=1)
        return path
    except OSError as e:
        print("# forms file not written: %s" % e, file=sys.stderr)
        return None


def _r(v, d=4):
    """Float rounded to d significant digits (None and ints kept)."""
    if isinstance(v, float) and math.isfinite(v) and v != 0.0:
        return float("%.*g" % (d, v))
    return v


def final_line(rec, forms, side=None):
    """The compact JSON the last stdout line carries (a few KB at most)."""
    roof = rec["roofline"]
    out = {k: rec[k] for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                               "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config")}
    out["value"] = _r(out["value"], 6)
    out["ms_per_step"] = _r(out["ms_per_step"], 6)
    out["hbm_gbps"] = _r(rec["hbm_gbps"])
    out["roofline"] = {"bound": roof["bound"], "achieved": _r(roof["achieved"]), "peak": roof["peak"],
                       "unit": roof["unit"], "frac": _r(roof["frac"]), "traffic": roof["traffic"],
                       "kernel": "sv_pass", "avg_launch_ms": _r(roof["avg_launch_ms"]), "launches": roof["launches"],
                       "hbm_frac": _r(roof["other_ceiling"]["frac"])}
    at = rec.get("autotune")
    if at:
        out["autotune"] = {"default_ms_per_step": _r(at["default"]["ms_per_step"]),
                           "tuned_ms_per_step": _r(at["tuned"]["ms_per_step"]) if at["tuned"] else None,
                           "tuned_config": at["tuned"]["config"] if at["tuned"] else None,
                           "headline_uses": at["headline_uses"]}
    pg = rec.get("per_gate_path")
    if pg:
        out["per_gate_path"] = {"value": _r(pg["value"]), "ms_per_step": _r(pg["ms_per_step"]),
                                "achieved_gbps": _r(pg["achieved_gbps"]), "frac": _r(pg["frac"])}
    mb = forms.get("microbench")
    if mb:
        out["microbench_frac_of_8TBs"] = {
            k: [_r(v["min"], 3), _r(v["median"], 3), v["worst_q"]] for k, v in mb["summary"].items()}
        out["microbench_frac_of_8TBs"]["format"] = "[min, median, worst q] over q = 0..n-1"
        out["copy_gbps"] = _r(mb["copy_gbps"])
    pc = forms.get("precision_c64")
    if pc:
        out["precision_c64"] = {k: {"ms_per_step": _r(v["ms_per_step"]), "infidelity": _r(v["infidelity"], 3)}
                                for k, v in pc.items() if isinstance(v, dict) and "ms_per_step" in v}
    bt = forms.get("batched")
    if bt:
        oc = bt.get("oracle_check") or {}
        out["batched"] = {
            "trajectories_per_s": _r(bt["trajectories_per_s"]),
            "plain_c128_trajectories_per_s": _r(bt["plain_c128"]["trajectories_per_s"]),
            "plain_measured": bt["plain_c128"]["measured_trajectories"],
            "speedup": _r(bt["speedup_vs_plain_c128"]),
            "infidelity_c64_vs_c128_max": _r(bt["infidelity_c64_vs_c128"]["max"], 3),
            "infidelity_c64_vs_c128_mean": _r(bt["infidelity_c64_vs_c128"]["mean"], 3),
            "infidelity_trajectories": bt["infidelity_c64_vs_c128"]["trajectories"],
            "speedup_holds_at_infidelity_1e-6": bt["speedup_holds_at_infidelity_1e-6"],
            "success_mean": _r(bt["success_mean"]), "success_se": _r(bt["success_se"], 2),
            "oracle_mean": _r(oc.get("oracle_mean")), "oracle_se": _r(oc.get("oracle_se"), 2),
            "oracle_trajectories": oc.get("trajectories"),
            "max_abs_dprob_vs_oracle": _r(oc.get("max_abs_dprob"), 2),
            "grid_points": len(bt["grid"]["points"]), "grid_trajectories_per_point": bt["grid"]["trajectories_per_point"],
        }
        out["batched_fp32_vs_plain_fp64_speedup"] = out["batched"]["speedup"]
    ad = forms.get("adjoint")
    if ad:
        out["adjoint_gradient_ms"] = {k: _r(ad[k]["gradient_ms"]) for k in ("c128", "c64") if k in ad}
    cb = rec.get("cpu_baseline")
    if cb:
        out["cpu_baseline"] = {k: (_r(v) if isinstance(v, float) else v) for k, v in cb.items()
                               if not k.startswith("per_class")}
    if side:
        out["forms_file"] = side
    return out


if __name__ == "__main__":
    main()
