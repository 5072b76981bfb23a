"""torch.autograd binding of the adjoint sweep.

OverlapLoss.apply(eps, gates, slots, psi0, phi) returns
loss = 1 - |<phi| U(eps) psi0>|^2 for a gate list in which gate slots[i]
carries the deviation eps[i] in its parameter p[which].  The forward pass
runs the circuit on the device (sv_run); the backward pass is sv_adjoint,
which uncomputes U^dagger gate by gate and needs no stored intermediate
states.  Writing eps into the gate records is argument marshalling; all
arithmetic happens in libsv.so.
"""

from __future__ import annotations

import numpy as np
import torch

from .state import State, adjoint, overlap_loss


def _records(gates: np.ndarray, slots, which, eps: np.ndarray) -> np.ndarray:
    g = np.array(gates, copy=True)
    for i, (s, w) in enumerate(zip(slots, which)):
        g[int(s)]["p"][int(w)] = float(eps[i])
    return g


class OverlapLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps, gates, slots, which, psi0: State, phi: State, fused: bool = False):
        e = eps.detach().to("cpu", torch.float64).numpy()
        g = _records(gates, slots, which, e)
        psi = State(psi0.n, psi0.dtype).copy_from(psi0)
        psi.run(g, fused=fused)
        loss, A = overlap_loss(phi, psi)
        ctx.save_for_backward(eps)
        ctx.state = (g, np.asarray(slots), np.asarray(which), psi, phi)
        return eps.new_tensor(loss, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_out):
        (eps,) = ctx.saved_tensors
        g, slots, which, psi, phi = ctx.state
        dparam = np.full(len(g), -1, dtype=np.int32)
        dparam[slots] = which
        # the sweep uncomputes its input in place: run it on copies, so the
        # saved forward state survives a second backward (retain_graph)
        work = State(psi.n, psi.dtype).copy_from(psi)
        lam = State(phi.n, phi.dtype).copy_from(phi)
        grad, _ = adjoint(work, lam, g, dparam)
        ge = torch.from_numpy(grad[slots]).to(eps.device, eps.dtype) * grad_out.to(eps.dtype)
        return ge, None, None, None, None, None, None


def overlap_loss_fn(eps: torch.Tensor, gates: np.ndarray, slots, which, psi0: State, phi: State, fused=False):
    return OverlapLoss.apply(eps, gates, slots, which, psi0, phi, fused)
