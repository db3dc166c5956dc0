"""Hybrid Monte Carlo driver over the library's trajectory entry point.

One HMC update (Sec. III B): draw Gaussian momenta Pi = i sum_a p_a T_a
(p_a ~ N(0,1)) and a Gaussian eta (E|eta|^2 = 1 per component), set the
pseudofermion phi = D(V)^dag eta on the operator links V (the thin links, or
stout^n of them), run one molecular-dynamics trajectory with
lgt_md_step_sw (leapfrog for n_inner = 1, Sexton-Weingarten otherwise), and
accept the new links with probability min(1, exp(-Delta H)).

Random numbers come from a seeded torch generator on the GPU (normals for
the momenta, whose algebra element lgt_momenta_from_normals assembles, and
for eta); every step of the trajectory runs in liblgt.so.  This module only
orchestrates (the Metropolis test is a host decision on Delta H).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import torch

from .api import Lattice, Params


def _site_shape(dims):
    lx, ly, lz, lt = dims
    return (lt, lz, ly, lx)


@dataclass
class HMCRecord:
    dH: List[float] = field(default_factory=list)
    accepted: List[bool] = field(default_factory=list)
    plaquette: List[float] = field(default_factory=list)
    cg_iters: List[int] = field(default_factory=list)

    def summary(self) -> dict:
        n = len(self.dH)
        if n == 0:
            return {}
        dh = torch.tensor(self.dH, dtype=torch.float64)
        return {
            "trajectories": n,
            "mean_dH": float(dh.mean()),
            "mean_abs_dH": float(dh.abs().mean()),
            "rms_dH": float(dh.pow(2).mean().sqrt()),
            "mean_exp_minus_dH": float(torch.exp(-dh).mean()),
            "acceptance": sum(self.accepted) / n,
            "mean_plaquette": sum(self.plaquette) / len(self.plaquette) if self.plaquette else None,
            "mean_cg_iters": sum(self.cg_iters) / len(self.cg_iters) if self.cg_iters else None,
        }


class HMC:
    """HMC chain for S = S_G(U) + phi^dag (D(V)^dag D(V))^-1 phi, V = stout^nlevels(U)."""

    def __init__(self, lat: Lattice, beta: float, kappa: float, dt: float, nsteps: int, n_inner: int = 1,
                 rho: float = 0.0, nlevels: int = 0, params: Optional[Params] = None, seed: int = 1234):
        self.lat, self.beta, self.kappa = lat, beta, kappa
        self.dt, self.nsteps, self.n_inner = dt, nsteps, n_inner
        self.rho, self.nlevels = rho, nlevels
        self.params = params or Params(precision="mixed_fp32", tol=1e-10)
        self.dev = torch.device("cuda")
        self.gen = torch.Generator(device=self.dev)
        self.gen.manual_seed(seed)
        self.shape = _site_shape(lat.dims)

    def momenta(self) -> torch.Tensor:
        c = torch.randn(self.shape + (4, 8), generator=self.gen, dtype=torch.float64, device=self.dev)
        return self.lat.momenta_from_normals(c)

    def gaussian_spinor(self) -> torch.Tensor:
        re = torch.randn(self.shape + (4, 3), generator=self.gen, dtype=torch.float64, device=self.dev)
        im = torch.randn(self.shape + (4, 3), generator=self.gen, dtype=torch.float64, device=self.dev)
        return (torch.complex(re, im) / math.sqrt(2.0)).contiguous()

    def update(self, U: torch.Tensor, rec: Optional[HMCRecord] = None, metropolis: bool = True) -> torch.Tensor:
        """One HMC update of U; returns the new (or the old) links."""
        P = self.momenta()
        eta = self.gaussian_spinor()
        V = self.lat.stout_smear(U, self.rho, self.nlevels) if self.nlevels > 0 else U
        phi = self.lat.dslash(V, eta, self.kappa, dagger=True)
        U1 = U.clone()
        dh, st = self.lat.md_step_sw(U1, P, phi, self.beta, self.kappa, self.dt, self.nsteps, self.n_inner,
                                     self.params, self.rho, self.nlevels)
        u = float(torch.rand((), generator=self.gen, dtype=torch.float64, device=self.dev))
        acc = (not metropolis) or dh <= 0.0 or u < math.exp(-dh)
        out = U1 if acc else U
        if rec is not None:
            rec.dH.append(dh)
            rec.accepted.append(acc)
            rec.cg_iters.append(st["iters"])
            rec.plaquette.append(self.lat.mean_plaquette(out))
        return out
