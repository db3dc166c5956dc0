"""Gradients and MD forces for the oracle (test infrastructure only).

Conventions (Sec. S2):

* The gradient of a real action is the complex matrix
  G = dS/dU_R + i dS/dU_I (eq. S2.12), so that a first-order variation reads
  delta S = Re tr(G^dag delta U).  (The paper's matrix derivative is
  dS/dU = G^dag / 2, eq. S2.15.)
* Reading of the force: with the left update U -> exp(dt Pi) U, Pi = i sum_a p_a T_a
  and H = 1/2 sum p_a^2 + S, energy conservation needs dp_a/dtau = -d_a S with
  d_a S = d/ds S(exp(i s T_a) U)|_0 = Re tr(G^dag i T_a U).  Writing
  Pi' = -F gives F = i sum_a (d_a S) T_a = -1/2 P_su(3)[U G^dag], i.e. the
  projection of eq. (7) applied to U G^dag (S2 "Why the implementation
  constructs U G^dag"), with the overall factor -1/2.  A momentum update
  P <- P - dt F is then P <- P + (dt/2) P_su(3)[U G^dag], the gauge-force
  listing's step with factor eps*dtau/2.

Gauge gradient: reverse-mode differentiation, written by hand, of the
plaquette sum of ``action.gauge_action``: every plaquette term
-beta/3 Re tr(A B C^dag D^dag) sends one adjoint to each of its four links.

Fermion gradient (Sec. S3): delta S_f = -2 Re[eta^dag (delta D) chi] (S3.12)
with chi = (D^dag D)^-1 phi and eta = D chi, i.e. S_f's gradient is -2 times
the gradient of Re I(U), I(U) = a^dag D(U) b (S3.13) at a = eta, b = chi, with
the solve itself not differentiated.
"""
from __future__ import annotations

import numpy as np

from .action import gauge_action, fermion_action
from .dirac import GAMMA, ONE4
from .lattice import shift
from .solver import solve_ddag_d
from .su3 import T, dag, project_su, expm_antihermitian


def force_from_grad(u: np.ndarray, g: np.ndarray) -> np.ndarray:
    """F = -1/2 P_su(3)[U G^dag]."""
    return -0.5 * project_su(u @ dag(g))


def gauge_grad(u: np.ndarray, beta: float) -> np.ndarray:
    """G of S_G, by reverse-mode over every plaquette term.

    For f = Re tr(W M): the gradient with respect to W is M^dag; for
    f = Re tr(W^dag M) it is M.  With P = A B C^dag D^dag,
    A = U_mu(x), B = U_nu(x+mu), C = U_mu(x+nu), D = U_nu(x):
      dA: (B C^dag D^dag)^dag, dB: (C^dag D^dag A)^dag, dC: D^dag A B, dD: A B C^dag.
    """
    g = np.zeros_like(u)
    c = -beta / 3.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            a = u[..., mu, :, :]
            b = shift(u[..., nu, :, :], mu, +1)
            cc = shift(u[..., mu, :, :], nu, +1)
            d = u[..., nu, :, :]
            ga = dag(b @ dag(cc) @ dag(d))
            gb = dag(dag(cc) @ dag(d) @ a)
            gc = dag(d) @ a @ b
            gd = a @ b @ dag(cc)
            g[..., mu, :, :] += c * ga
            g[..., nu, :, :] += c * shift(gb, mu, -1)   # B(x) is the link at x+mu
            g[..., mu, :, :] += c * shift(gc, nu, -1)   # C(x) is the link at x+nu
            g[..., nu, :, :] += c * gd
    return g


def gauge_force(u: np.ndarray, beta: float) -> np.ndarray:
    return force_from_grad(u, gauge_grad(u, beta))


def bilinear_grad(u: np.ndarray, a: np.ndarray, b: np.ndarray, kappa: float,
                  bc: int = -1) -> np.ndarray:
    """Gradient of Re I(U), I(U) = a^dag D(U) b (eq. S3.13), with respect to the links.

    The link U_mu(x) appears in two hops of D, each with U~ = s U, s the
    fermion boundary sign of that link:
      -kappa s a(x)^dag (1 - gamma_mu) U b(x+mu)    = -kappa s tr(U Z1),
      -kappa s a(x+mu)^dag (1 + gamma_mu) U^dag b(x) = -kappa s tr(U^dag Z2),
    with colour matrices Z1 = sum_{st} (1-gamma_mu)_st b(x+mu)_t a(x)_s^dag and
    Z2 = sum_{st} (1+gamma_mu)_st b(x)_t a(x+mu)_s^dag.  Re tr(U Z1) has gradient
    Z1^dag and Re tr(U^dag Z2) has gradient Z2, so G = -kappa s (Z1^dag + Z2).
    """
    g = np.zeros(a.shape[:4] + (4, 3, 3), dtype=np.complex128)
    for mu in range(4):
        a_f = shift(a, mu, +1)
        b_f = shift(b, mu, +1)
        pm = ONE4 - GAMMA[mu]
        pp = ONE4 + GAMMA[mu]
        z1 = np.einsum("st,...ti,...sj->...ij", pm, b_f, np.conj(a))
        z2 = np.einsum("st,...ti,...sj->...ij", pp, b, np.conj(a_f))
        gm = -kappa * (dag(z1) + z2)
        if mu == 3:
            gm[-1] *= bc
        g[..., mu, :, :] = gm
    return g


def fermion_grad_from_solution(u, chi, eta, kappa, bc=-1):
    """G_f = -2 * grad Re[eta^dag D(U) chi] (eq. S3.12)."""
    return -2.0 * bilinear_grad(u, eta, chi, kappa, bc)


def fermion_grad(u, phi, kappa, bc=-1, tol=1e-12):
    chi, eta, it, res = solve_ddag_d(u, phi, kappa, bc, tol)
    return fermion_grad_from_solution(u, chi, eta, kappa, bc)


def fermion_force(u, phi, kappa, bc=-1, tol=1e-12):
    return force_from_grad(u, fermion_grad(u, phi, kappa, bc, tol))


def fermion_force_from_solution(u, chi, eta, kappa, bc=-1):
    return force_from_grad(u, fermion_grad_from_solution(u, chi, eta, kappa, bc))


# ---------------------------------------------------------------------------
# Finite-difference statements of the same derivatives (for pins)
# ---------------------------------------------------------------------------

def lie_fd(action_fn, u: np.ndarray, site: tuple, mu: int, a: int, h: float = 1e-5) -> float:
    """Central difference of d_a S = d/ds S(exp(i s T_a) U_mu(x))|_0 on one link."""
    up = u.copy()
    um = u.copy()
    idx = tuple(site) + (mu,)
    gen = 1j * T[a]
    up[idx] = expm_antihermitian(h * gen) @ u[idx]
    um[idx] = expm_antihermitian(-h * gen) @ u[idx]
    return (action_fn(up) - action_fn(um)) / (2 * h)


def component_fd(action_fn, u: np.ndarray, site: tuple, mu: int, i: int, j: int,
                 imag: bool, h: float = 1e-6) -> float:
    """Central difference of dS/dRe U_ij (or dS/dIm U_ij) on one link (off the group)."""
    up = u.copy()
    um = u.copy()
    idx = tuple(site) + (mu, i, j)
    step = 1j * h if imag else h
    up[idx] += step
    um[idx] -= step
    return (action_fn(up) - action_fn(um)) / (2 * h)


def lie_derivatives(f: np.ndarray) -> np.ndarray:
    """d_a S from a force F = i sum_a (d_a S) T_a:  d_a S = 2 Im tr(T_a F)."""
    return 2.0 * np.imag(np.einsum("aij,...ji->...a", T, f))


__all__ = [
    "force_from_grad", "gauge_grad", "gauge_force", "bilinear_grad",
    "fermion_grad_from_solution", "fermion_grad", "fermion_force",
    "fermion_force_from_solution", "lie_fd", "component_fd", "lie_derivatives",
    "gauge_action", "fermion_action",
]
