"""Host logic of bench.py (no GPU): the one-GPU contract, the algorithmic
flop count the roofline divides by, and the choice of the bounding
ceiling."""

import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import synth  # noqa: E402


@pytest.fixture(scope="module")
def bench():
    import bench as b

    return b


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_algorithmic_flops_brickwork(bench):
    # 600 Haar SU(2) gates at 14 real flops per amplitude of 2^30; the 290
    # CNOTs move amplitudes only
    n, depth = 30, 20
    gl = synth.brickwork_circuit(n, depth, seed=0).array()
    kinds = list(gl["kind"])
    assert kinds.count(synth.KIND_SU2) == n * depth
    assert bench.algorithmic_flops(n, gl) == 14.0 * n * depth * 2 ** n


def test_algorithmic_flops_qft(bench):
    # QFT of sec. 2.3.2 on 6 qubits: 6 Hadamards (14 flops on each of 2^6
    # amplitudes), 15 controlled phases R_k (6 flops on each of the 2^4
    # amplitudes with control and target set), 3 swaps (none)
    n = 6
    gl = synth.qft_circuit(n).array()
    assert bench.algorithmic_flops(n, gl) == 6 * 14 * 2 ** 6 + 15 * 6 * 2 ** 4


def test_roofline_picks_the_larger_ceiling(bench):
    n = 30
    gl = synth.brickwork_circuit(n, 20, seed=0).array()
    per_pass_bytes = 2 * 2 ** n * 16
    r = bench.roofline_record(n, gl, 15, 12.2, 30, per_pass_bytes)
    flops = 14.0 * 600 * 2 ** n / 15
    # FP64 time at peak (7.65 ms) exceeds HBM time at peak (4.30 ms)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == 78.6
    assert r["achieved"] == pytest.approx(flops / 12.2e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 78.6)
    assert r["other_ceiling"]["bound"] == "hbm"
    assert r["other_ceiling"]["achieved"] == pytest.approx(per_pass_bytes / 12.2e-3 / 1e9)
    # one Hadamard per pass: the HBM ceiling binds
    gl1 = synth.GateList()
    gl1.add(synth.KIND_H, 0)
    r1 = bench.roofline_record(n, gl1.array(), 1, 6.0, 1, per_pass_bytes)
    assert r1["bound"] == "hbm" and r1["unit"] == "GB/s" and r1["peak"] == 8000.0
    assert r1["frac"] == pytest.approx(per_pass_bytes / 6.0e-3 / 1e9 / 8000.0)


def _fake_forms(bench):
    n = 30
    summary = {"%s_%s" % (dt, c): {"min": 0.71234567, "median": 0.7456789, "max": 0.76, "worst_q": 29,
                                   "below_0.7": 0}
               for dt in ("c128", "c64") for c in bench.MB_CLASSES}
    return {
        "microbench": {"summary": summary, "copy_gbps": 5612.345678, "table": [{"q": q} for q in range(240)]},
        "precision_c64": {"workload": "x" * 200,
                          **{k: {"ms_per_step": 110.123456, "infidelity": 1.23456e-12, "path": "p" * 80}
                             for k in ("fused", "blocks5", "blocks4")}},
        "batched": {"trajectories_per_s": 115.123456, "plain_c128": {"trajectories_per_s": 2.1812345,
                                                                     "measured_trajectories": 64},
                    "speedup_vs_plain_c128": 52.9123456,
                    "infidelity_c64_vs_c128": {"max": 3.2e-9, "mean": 1.1e-9, "trajectories": 256},
                    "speedup_holds_at_infidelity_1e-6": True, "success_mean": 3.0123e-6, "success_se": 1.1234e-8,
                    "oracle_check": {"oracle_mean": 3.01e-6, "oracle_se": 4.4e-8, "trajectories": 258,
                                     "max_abs_dprob": 1.2e-10},
                    "grid": {"points": [{}] * 12, "trajectories_per_point": 4096}},
        "adjoint": {"c128": {"gradient_ms": 21.7123}, "c64": {"gradient_ms": 12.01234}},
    }


def test_final_line_is_compact_json(bench):
    n = 30
    gl = synth.brickwork_circuit(n, 20, seed=0).array()
    rec = {"metric": bench.METRIC, "value": 4.2512345678e12, "unit": "gate-amp updates/s", "n_gpus": 1,
           "steps": 20, "warmup": 5, "ms_per_step": 188.123456789, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "brickwork random circuit, n=30, depth 20, complex128, fused LDS passes",
                      "n": 30, "depth": 20, "gates_per_step": 890, "fused_passes_per_step": 15, "seed": 0},
           "hbm_gbps": 2741.123456,
           "roofline": bench.roofline_record(n, gl, 15, 12.2, 300, 2 * 2 ** n * 16),
           "per_gate_path": {"value": 1.76e11, "ms_per_step": 4550.1234, "achieved_gbps": 5912.1234,
                             "frac": 0.739012, "avg_launch_ms": 5.8, "launches": 600},
           "cpu_baseline": {"value": 1.09e9, "unit": "gate-amp updates/s", "cores": 1, "kind": "oracle",
                            "sample": "s" * 160, "nproc": 256, "cpus_allowed": 16,
                            "cpu_model": "AMD EPYC 9575F 64-Core Processor", "pinning": "sched_setaffinity to core 17",
                            "per_class_q0_q29": {"haar1q": [1e9, 1e9]}}}
    line = json.dumps(bench.final_line(rec, _fake_forms(bench), "bench_out/bench_forms.json"),
                      separators=(",", ":"))
    assert len(line) < 4096, len(line)
    back = json.loads(line)
    for k in ("metric", "value", "unit", "ms_per_step", "steps", "dtype", "config", "hbm_gbps", "roofline",
              "per_gate_path", "cpu_baseline", "batched_fp32_vs_plain_fp64_speedup"):
        assert k in back, k
    assert back["config"]["workload"].startswith("brickwork")
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in back["roofline"]
    for k in ("nproc", "cpu_model", "pinning", "cores", "kind", "sample"):
        assert k in back["cpu_baseline"]
    assert "\n" not in line


def test_microbench_bytes(bench):
    n = 30
    # dense and NOT: every amplitude read and written
    assert bench.mb_bytes("haar1q", n, 7, 16) == 2 * 16 * 2 ** n
    assert bench.mb_bytes("x", n, 29, 8) == 2 * 8 * 2 ** n
    # CNOT with its control on a high bit: half the lines; on a bit inside
    # a 128-B line (bit < 3 for complex128): every line
    assert bench.mb_bytes("cnot", n, 5, 16) == 2 * 16 * 2 ** (n - 1)
    assert bench.mb_bytes("cnot", n, 28, 16) == 2 * 16 * 2 ** n   # control qubit 27 = index bit 2
    # controlled phase: a quarter of the amplitudes change
    assert bench.mb_bytes("cp", n, 10, 8) == 2 * 8 * 2 ** (n - 2)
    assert bench.mb_updates("cp", n) == 2 ** (n - 2)
