"""Registers of 2^33 and 2^34 amplitudes (128 GiB: the largest that fit one
MI355X), so basis indices pass 2^32 and every index computation must stay
64-bit.  A brickwork circuit followed by its inverse must return |0...0>
on the fused-pass and on the per-gate engines; the inverse is built from
the oracle's gate matrices (U^dagger as explicit matrix records), and a
layer of Hadamards gives the closed form 2^-k for the probability of any
pattern of k qubits, high index bits included.  The circuit and its
inverse act on the uniform superposition (Hadamards on every qubit before
and after), so amplitudes at every index take part."""

import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

SELF_INVERSE = {synth.KIND_X, synth.KIND_Y, synth.KIND_Z, synth.KIND_H, synth.KIND_SWAP}


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def sv():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < (130 << 30):
        pytest.skip("needs 130 GiB of free device memory")
    import paper_quant_ph_0201042_amd as sv

    return sv


def inverse(orc, gl):
    """The gate list of the inverse circuit: reversed order, each gate
    replaced by its adjoint (self-inverse kinds kept as they are)."""
    out = synth.GateList()
    for r in gl[::-1]:
        k = int(r["kind"])
        if k in SELF_INVERSE:
            out.add(k, int(r["target"]), ctrl=int(r["ctrl"]), target2=int(r["target2"]), iarg=int(r["iarg"]), p=r["p"])
            continue
        U = orc.gate_matrix(k, int(r["iarg"]), r["p"])
        Ud = U.conj().T
        p = [Ud[0, 0].real, Ud[0, 0].imag, Ud[0, 1].real, Ud[0, 1].imag,
             Ud[1, 0].real, Ud[1, 0].imag, Ud[1, 1].real, Ud[1, 1].imag]
        out.add(synth.KIND_U, int(r["target"]), ctrl=int(r["ctrl"]), p=p)
    return out.array()


@pytest.mark.parametrize("dtype,n", [("c64", 34), ("c128", 33)])
@pytest.mark.parametrize("fused", [True, False], ids=["fused", "per_gate"])
def test_circuit_then_inverse_is_identity(sv, orc, dtype, n, fused):
    import torch

    gl = synth.brickwork_circuit(n, 3, seed=5).array()
    # H on every qubit before and after: the circuit acts on the uniform
    # superposition, whose amplitudes sit at every index, high halves included
    hl = synth.GateList()
    for q in range(n):
        hl.add(synth.KIND_H, q)
    hl = hl.array()
    both = np.concatenate([hl, gl, inverse(orc, gl), hl])
    say("large U U^dagger", dtype, n, "fused" if fused else "per gate", len(both))
    s = sv.State(n, dtype).reset(0)
    s.run(both, fused=fused)
    p0 = s.prob((1 << n) - 1, 0)
    tol = 1e-10 if dtype == "c128" else 2e-4
    assert abs(p0 - 1.0) <= tol, p0
    # the norm stayed where the identity leaves it
    assert abs(s.prob(0, 0) - 1.0) <= tol
    del s
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype,n", [("c64", 34), ("c128", 33)])
def test_hadamard_layer_patterns(sv, dtype, n):
    import torch

    gl = synth.GateList()
    for q in range(n):
        gl.add(synth.KIND_H, q)
    say("large H layer", dtype, n)
    s = sv.State(n, dtype).reset(0)
    s.run(gl.array(), fused=True)
    eps = 1e-12 if dtype == "c128" else 1e-5
    top = 1 << (n - 1)
    for mask, value in [(top, top), (top | 1, 1), ((1 << n) - 1, (1 << n) - 1), (0b111 << (n - 3), 0b101 << (n - 3)),
                        (top | (1 << 32) | (1 << 31) | 1, top | (1 << 31) | 1)]:
        k = bin(mask).count("1")
        assert abs(s.prob(mask, value) - 2.0 ** -k) <= eps * max(1.0, 2.0 ** -k), (mask, value)
    # a second layer undoes the first
    s.run(gl.array(), fused=True)
    assert abs(s.prob((1 << n) - 1, 0) - 1.0) <= 100 * eps
    del s
    torch.cuda.empty_cache()
