"""GPU parity of the adjoint sweep (sv_adjoint) against the CPU oracle's
adjoint gradient, which is itself pinned to the parameter-shift rule and
central differences (tests/test_oracle_pins.py).  Workload: the QFT circuit
with one over-rotation per gate (H on theta, R_k on phi), eps_g ~ N(0, 1e-2^2),
on a seeded Gaussian input; loss = 1 - |<QFT psi0 | QFT(eps) psi0>|^2."""

import math
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


def qft_problem(n, eps_seed=1, state_seed=0):
    ng = n * (n + 1) // 2
    eps = synth.qft_eps(ng, eps_seed, 1e-2)
    gates = synth.qft_perturbed(n, eps).array()
    dparam = np.array([0 if r["kind"] == synth.KIND_H else (1 if r["kind"] == synth.KIND_RK else -1) for r in gates],
                      np.int32)
    psi0 = synth.random_state(n, state_seed)
    return gates, dparam, psi0


def gpu_adjoint(sv, orc, n, dtype, gates, dparam, psi0, phi):
    NP = np.complex128 if dtype == "c128" else np.complex64
    psi = sv.State(n, dtype).load(psi0.astype(NP))
    psi.run(gates)
    lam = sv.State(n, dtype).load(phi.astype(NP))
    grad, A = sv.adjoint(psi, lam, gates, dparam)
    return grad, A, psi


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [2, 6, 11, 16])
def test_adjoint_qft_vs_oracle(sv, orc, dtype, n):
    gates, dparam, psi0 = qft_problem(n)
    NP = np.complex128 if dtype == "c128" else np.complex64
    psi0 = psi0.astype(NP).astype(np.complex128)
    phi = orc.run(psi0, synth.qft_circuit(n).array()).astype(NP).astype(np.complex128)
    ref, Aref, _ = orc.adjoint(psi0, phi, gates, dparam)
    say("adjoint qft", dtype, n)
    grad, A, psi = gpu_adjoint(sv, orc, n, dtype, gates, dparam, psi0, phi)
    scale = max(np.max(np.abs(ref)), 1e-3)
    tol = 1e-11 if dtype == "c128" else 2e-5
    assert np.max(np.abs(grad - ref)) <= tol * scale, np.max(np.abs(grad - ref))
    assert abs(A - Aref) <= (1e-13 if dtype == "c128" else 1e-5)
    # the sweep uncomputes: psi returns to psi0
    back = psi.numpy().astype(np.complex128)
    assert np.max(np.abs(back - psi0)) <= (1e-13 if dtype == "c128" else 1e-5)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_adjoint_random_mix_vs_oracle(sv, orc, dtype):
    """Every parameterised kind (H, X, ROT on theta and phi; Z, R_k on phi),
    with controls, mixed with unparameterised gates and swaps."""
    n = 9
    rng = np.random.default_rng(11)
    gl = synth.random_gate_mix(n, 120, seed=5, max_ctrl=3)
    gates = gl.array()
    dparam = np.full(len(gates), -1, np.int32)
    for i, r in enumerate(gates):
        k = int(r["kind"])
        if k in (synth.KIND_H, synth.KIND_X, synth.KIND_ROT) and rng.random() < 0.8:
            dparam[i] = int(rng.integers(0, 2))
            r["p"][0] += 0.01
            r["p"][1] += 0.02
        elif k in (synth.KIND_Z, synth.KIND_RK) and rng.random() < 0.8:
            dparam[i] = 1
            r["p"][1] += 0.03
    NP = np.complex128 if dtype == "c128" else np.complex64
    psi0 = synth.random_state(n, 3).astype(NP).astype(np.complex128)
    phi = synth.random_state(n, 4).astype(NP).astype(np.complex128)
    ref, Aref, _ = orc.adjoint(psi0, phi, gates, dparam)
    say("adjoint mix", dtype)
    grad, A, _ = gpu_adjoint(sv, orc, n, dtype, gates, dparam, psi0, phi)
    scale = max(np.max(np.abs(ref)), 1e-3)
    assert np.max(np.abs(grad - ref)) <= (1e-11 if dtype == "c128" else 1e-4) * scale
    assert (grad[dparam < 0] == 0).all()


@pytest.fixture(scope="module")
def qft24_reference(orc):
    n = 24
    gates, dparam, psi0 = qft_problem(n)
    say("qft24 oracle adjoint (about a minute)")
    phi = orc.run(psi0, synth.qft_circuit(n).array())
    ref, Aref, _ = orc.adjoint(psi0, phi, gates, dparam)
    return n, gates, dparam, psi0, phi, ref, Aref


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_adjoint_qft_n24_vs_oracle(sv, orc, qft24_reference, dtype):
    """The differentiation workload at its full size: n=24, 300 gates,
    complex128 and complex64, all 300 gradient entries against the oracle."""
    n, gates, dparam, psi0, phi, ref, Aref = qft24_reference
    NP = np.complex128 if dtype == "c128" else np.complex64
    say("qft24 gpu adjoint", dtype)
    grad, A, psi = gpu_adjoint(sv, orc, n, dtype, gates, dparam, psi0.astype(NP), phi.astype(NP))
    assert len(grad[dparam >= 0]) == 300
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(grad - ref)) <= (1e-10 if dtype == "c128" else 1e-3) * scale
    back = psi.numpy().astype(np.complex128)
    assert np.max(np.abs(back - psi0)) <= (1e-12 if dtype == "c128" else 1e-5) * np.max(np.abs(psi0))


def test_autograd_function(sv, orc):
    import torch

    n = 10
    gates, dparam, psi0 = qft_problem(n)
    slots = np.nonzero(dparam >= 0)[0]
    which = dparam[slots]
    base = gates.copy()
    for s, w in zip(slots, which):
        base[s]["p"][w] = 0.0
    psi0_s = sv.State(n, "c128").load(psi0)
    phi = orc.run(psi0, synth.qft_circuit(n).array())
    phi_s = sv.State(n, "c128").load(phi)
    eps = torch.tensor(synth.qft_eps(len(slots), 1, 1e-2), dtype=torch.float64, requires_grad=True)
    loss = sv.overlap_loss_fn(eps, base, slots, which, psi0_s, phi_s)
    loss.backward()
    ref, Aref, _ = orc.adjoint(psi0, phi, gates, dparam)
    assert abs(loss.item() - (1 - abs(Aref) ** 2)) <= 1e-13
    assert np.max(np.abs(eps.grad.numpy() - ref[slots])) <= 1e-12


def test_autograd_second_backward_gives_the_same_gradient(sv, orc):
    import torch

    n = 9
    gates, dparam, psi0 = qft_problem(n)
    slots = np.nonzero(dparam >= 0)[0]
    which = dparam[slots]
    psi0_s = sv.State(n, "c128").load(psi0)
    phi_s = sv.State(n, "c128").load(orc.run(psi0, synth.qft_circuit(n).array()))
    eps = torch.tensor(synth.qft_eps(len(slots), 2, 1e-2), dtype=torch.float64, requires_grad=True)
    loss = sv.overlap_loss_fn(eps, gates, slots, which, psi0_s, phi_s)
    loss.backward(retain_graph=True)
    g1 = eps.grad.clone()
    eps.grad = None
    loss.backward()
    assert torch.equal(g1, eps.grad)
