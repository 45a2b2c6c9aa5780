"""Gradients of a lattice run as a torch.autograd.Function.

LBMLoss.apply(force_mag, G, rho0, lattice, spec) runs the checkpointed forward
pass of the library (lbm_adjoint_forward) on `lattice` and returns the loss as
a 0-d FP64 tensor; its backward runs the library's reverse sweep
(lbm_adjoint_backward) and returns dL/d|F_ext|, dL/dG and dL/drho0 scaled by
the incoming gradient.  `spec` holds the adjoint_forward keywords (n_steps,
loss, window, checkpoint_every, u_target).

The run starts at rest, fbar = f^eq(rho0, 0), with the lattice's current
parameters except the body-force magnitude (direction and mode kept) and G,
which are taken from the inputs.  The gradients are those of the discrete
run: the reverse of every step's streaming, bounce-back, pseudopotential
stencil (Eq. 4) and moment-space collision with the third-order source term
(Eq. 2a with Eqs. 6-8 and Eq. 11, or Eqs. 13 + 42).
"""
from __future__ import annotations

import torch

from .lattice import Lattice


class LBMLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, force_mag: torch.Tensor, G: torch.Tensor, rho0: torch.Tensor, lattice: Lattice, spec: dict):
        lattice.set_force_magnitude(float(force_mag))
        lattice.set_G(float(G))
        value = lattice.adjoint_forward(rho0.detach(), **spec)
        ctx.lattice = lattice
        ctx.devices = (force_mag.device, G.device, rho0.device)
        ctx.dtypes = (force_mag.dtype, G.dtype, rho0.dtype)
        return torch.tensor(value, dtype=torch.float64, device=rho0.device)

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        if not any(ctx.needs_input_grad[:3]):
            return None, None, None, None, None
        g_rho0, g_force, g_G = ctx.lattice.adjoint_backward()
        go = grad_out.to(torch.float64)
        out = []
        for need, g, dev, dt in zip(ctx.needs_input_grad[:3], (g_force, g_G, g_rho0), ctx.devices, ctx.dtypes):
            if not need:
                out.append(None)
                continue
            t = torch.as_tensor(g, dtype=torch.float64, device=go.device) * go
            out.append(t.to(device=dev, dtype=dt))
        return out[0], out[1], out[2], None, None


def lbm_loss(force_mag: torch.Tensor, G: torch.Tensor, rho0: torch.Tensor, lattice: Lattice, **spec) -> torch.Tensor:
    """Differentiable loss of a run; see LBMLoss."""
    return LBMLoss.apply(force_mag, G, rho0, lattice, spec)
