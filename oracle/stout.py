"""Stout smearing and gradients through it, for the oracle (test infrastructure only).

Stout smearing (Morningstar & Peardon, the smearing the paper cites in Sec. I
and uses in Sec. III B), all four directions smeared simultaneously from the
previous level:

  C_mu(x) = rho * sum_{nu != mu} [ U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag
                                  + U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu) ],
  Omega = C U^dag,   Q = (i/2)(Omega^dag - Omega) - (i/6) tr(Omega^dag - Omega),
  U' = exp(i Q) U.

The smeared links enter D only; the gauge action uses the thin links.

The gradient of S(U0) = S_G(U0) + S_f(U_n), U_n = stout^n(U0), is taken the way
the paper takes every force: by reverse-mode automatic differentiation of the
action code -- here PyTorch CPU autograd through a torch transcription of the
definition above (``torch.linalg.matrix_exp``), seeded with the fermion
gradient G_f(U_n) of ``force.fermion_grad``.  The result is in the G = dS/dRe U
+ i dS/dIm U convention of Sec. S2.
"""
from __future__ import annotations

import numpy as np

from .force import fermion_grad, force_from_grad, gauge_grad
from .action import gauge_action, fermion_action
from .lattice import shift
from .su3 import dag, expm_antihermitian, trace, identity_like


def staple_sum(u: np.ndarray, mu: int) -> np.ndarray:
    """sum_{nu != mu} [U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag + U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu)]."""
    s = np.zeros(u.shape[:4] + (3, 3), dtype=np.complex128)
    umu = u[..., mu, :, :]
    for nu in range(4):
        if nu == mu:
            continue
        unu = u[..., nu, :, :]
        s += unu @ shift(umu, nu, +1) @ dag(shift(unu, mu, +1))
        unu_m = shift(unu, nu, -1)
        s += dag(unu_m) @ shift(umu, nu, -1) @ shift(unu_m, mu, +1)
    return s


def stout_level(u: np.ndarray, rho: float) -> np.ndarray:
    out = np.empty_like(u)
    for mu in range(4):
        om = rho * staple_sum(u, mu) @ dag(u[..., mu, :, :])
        d = dag(om) - om
        q = 0.5j * d - (1j / 6.0) * trace(d)[..., None, None] * identity_like(d)
        out[..., mu, :, :] = expm_antihermitian(1j * q) @ u[..., mu, :, :]
    return out


def stout(u: np.ndarray, rho: float, nlevels: int) -> np.ndarray:
    for _ in range(nlevels):
        u = stout_level(u, rho)
    return u


# ---------------------------------------------------------------------------
# torch transcription of the same definition (for autograd)
# ---------------------------------------------------------------------------
_AXIS = {0: 3, 1: 2, 2: 1, 3: 0}


def _t_shift(f, mu, sign):
    import torch
    return torch.roll(f, shifts=-sign, dims=_AXIS[mu])


def _t_dag(m):
    return m.conj().transpose(-1, -2)


def stout_level_torch(u, rho):
    import torch
    outs = []
    eye = torch.eye(3, dtype=u.dtype)
    for mu in range(4):
        umu = u[..., mu, :, :]
        s = torch.zeros_like(umu)
        for nu in range(4):
            if nu == mu:
                continue
            unu = u[..., nu, :, :]
            s = s + unu @ _t_shift(umu, nu, +1) @ _t_dag(_t_shift(unu, mu, +1))
            unu_m = _t_shift(unu, nu, -1)
            s = s + _t_dag(unu_m) @ _t_shift(umu, nu, -1) @ _t_shift(unu_m, mu, +1)
        om = rho * s @ _t_dag(umu)
        d = _t_dag(om) - om
        tr = torch.diagonal(d, dim1=-2, dim2=-1).sum(-1)
        q = 0.5j * d - (1j / 6.0) * tr[..., None, None] * eye
        outs.append(torch.linalg.matrix_exp(1j * q) @ umu)
    return torch.stack(outs, dim=-3)


def stout_vjp(u0: np.ndarray, g_top: np.ndarray, rho: float, nlevels: int) -> np.ndarray:
    """Gradient at U0 of L(U0) = Re tr(G_top^dag U_n(U0)), by torch autograd (real leaves)."""
    import torch
    re = torch.tensor(u0.real, dtype=torch.float64, requires_grad=True)
    im = torch.tensor(u0.imag, dtype=torch.float64, requires_grad=True)
    u = torch.complex(re, im)
    for _ in range(nlevels):
        u = stout_level_torch(u, rho)
    g = torch.tensor(g_top)
    loss = (g.real * u.real + g.imag * u.imag).sum()
    loss.backward()
    return re.grad.numpy() + 1j * im.grad.numpy()


def smeared_fermion_action(u0, phi, kappa, rho, nlevels, bc=-1, tol=1e-12):
    return fermion_action(stout(u0, rho, nlevels), phi, kappa, bc, tol)[0]


def smeared_fermion_grad(u0, phi, kappa, rho, nlevels, bc=-1, tol=1e-12):
    """G at U0 of S_f(stout^n(U0))."""
    un = stout(u0, rho, nlevels)
    return stout_vjp(u0, fermion_grad(un, phi, kappa, bc, tol), rho, nlevels)


def total_action(u0, phi, beta, kappa, rho, nlevels, bc=-1, tol=1e-12):
    """S = S_G(U0) + S_f(stout^n(U0))."""
    return gauge_action(u0, beta) + smeared_fermion_action(u0, phi, kappa, rho, nlevels, bc, tol)


def total_force(u0, phi, beta, kappa, rho, nlevels, bc=-1, tol=1e-12):
    g = gauge_grad(u0, beta) + smeared_fermion_grad(u0, phi, kappa, rho, nlevels, bc, tol)
    return force_from_grad(u0, g)
