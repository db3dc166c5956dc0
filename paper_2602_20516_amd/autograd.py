"""The action as a differentiable torch function, with the hand-written adjoint.

``LatticeAction.apply(U_real, phi, lattice, beta, kappa, rho, nlevels, params)``
returns S = S_G(U) + phi^dag (D^dag D)^-1 phi with D built on stout^n(U).
U is taken as a float64 real view ``[..., 4, 3, 3, 2]`` of the complex links, so
the backward returns exactly (dS/dRe U, dS/dIm U), the real components the
paper's AD differentiates (S2.12).  The backward is the library's explicit
adjoint (lgt_smeared_force in gradient mode): the fermion adjoint on the
smeared links, then the stout adjoint chain, recomputing the smeared levels
instead of saving them; only U and phi are kept between forward and backward.
"""
from __future__ import annotations

import torch

from .api import Lattice, Params


class LatticeAction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U_real, phi, lattice: Lattice, beta: float, kappa: float, rho: float = 0.0,
                nlevels: int = 0, params: Params = None):
        params = params or Params()
        U = torch.view_as_complex(U_real.detach().contiguous())
        sg, _, _ = lattice.action(U, phi, beta, kappa, params, gauge=True, fermion=False)
        Un = lattice.stout_smear(U, rho, nlevels) if nlevels > 0 else U
        _, sf, _ = lattice.action(Un, phi, beta, kappa, params, gauge=False, fermion=True)
        ctx.save_for_backward(U_real, phi)
        ctx.cfg = (lattice, beta, kappa, rho, nlevels, params)
        return torch.tensor(sg + sf, dtype=torch.float64, device=U_real.device)

    @staticmethod
    def backward(ctx, grad_s):
        U_real, phi = ctx.saved_tensors
        lattice, beta, kappa, rho, nlevels, params = ctx.cfg
        U = torch.view_as_complex(U_real.detach().contiguous())
        G, _, _ = lattice.smeared_force(U, phi, beta, kappa, rho, nlevels, params, mode="grad")
        return grad_s * torch.view_as_real(G), None, None, None, None, None, None, None


def lattice_action(U_real, phi, lattice, beta, kappa, rho=0.0, nlevels=0, params=None):
    return LatticeAction.apply(U_real, phi, lattice, beta, kappa, rho, nlevels, params)
