"""Actions and Hamiltonian for the oracle (test infrastructure only).

* Wilson plaquette gauge action (the paper's ``calc_action`` of the gauge-force
  listing, whose body it does not show):
      S_G = beta * sum_x sum_{mu<nu} (1 - Re tr P_mu,nu(x) / 3),
      P_mu,nu(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag,
  so that S_G = 0 at U = 1.  The gauge action uses the plain (periodic) links.
* Pseudofermion action S_f = phi^dag (D^dag D)^-1 phi (eq. S3.1) = Re phi^dag chi.
* Kinetic energy of the traceless anti-Hermitian momenta Pi = i sum_a p_a T_a:
  K = 1/2 sum p_a^2 = -sum tr Pi^2.
"""
from __future__ import annotations

import numpy as np

from .lattice import shift
from .solver import solve_ddag_d
from .su3 import dag, trace


def plaquette_field(u: np.ndarray, mu: int, nu: int) -> np.ndarray:
    """P_mu,nu(x) at every site."""
    a = u[..., mu, :, :]
    b = shift(u[..., nu, :, :], mu, +1)
    c = shift(u[..., mu, :, :], nu, +1)
    d = u[..., nu, :, :]
    return a @ b @ dag(c) @ dag(d)


def plaquette_sum(u: np.ndarray) -> float:
    """sum_x sum_{mu<nu} Re tr P_mu,nu(x) / 3."""
    s = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            s += float(np.sum(np.real(trace(plaquette_field(u, mu, nu))))) / 3.0
    return s


def mean_plaquette(u: np.ndarray) -> float:
    nsite = int(np.prod(u.shape[:4]))
    return plaquette_sum(u) / (6 * nsite)


def gauge_action(u: np.ndarray, beta: float) -> float:
    nsite = int(np.prod(u.shape[:4]))
    return beta * (6 * nsite - plaquette_sum(u))


def fermion_action(u: np.ndarray, phi: np.ndarray, kappa: float, bc: int = -1,
                   tol: float = 1e-12):
    """S_f = Re phi^dag chi; returns (S_f, chi, eta, iterations, true residual)."""
    chi, eta, it, res = solve_ddag_d(u, phi, kappa, bc, tol)
    s = float(np.real(np.vdot(phi.ravel(), chi.ravel())))
    return s, chi, eta, it, res


def kinetic(p: np.ndarray) -> float:
    """K = -sum tr Pi^2 = 1/2 sum_a p_a^2."""
    return float(-np.sum(np.real(trace(p @ p))))
