"""Host logic of bench.py (no GPU): the one-GPU contract, the algorithmic
flop count the roofline divides by, and the choice of the bounding
ceiling."""

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
