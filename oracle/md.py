"""Leapfrog molecular dynamics for the oracle (test infrastructure only).

Equations of motion (left-invariant form, eqs. S2.1-S2.2 with P = -i Pi):
  dU/dtau = Pi U,   dPi/dtau = -F(U),   F = F_G + F_f,
with H = K + S_G + S_f, K = -sum tr Pi^2.  The integrator is the second-order
reversible, symplectic leapfrog named in Sec. III B, in its
momentum-position-momentum form:

  Pi <- Pi - dt/2 F(U)
  repeat nsteps times:  U <- reunitarize(exp(dt Pi) U);  Pi <- Pi - dt F(U)
  (the final kick uses dt/2 instead of dt)

The pseudofermion field phi is held fixed along the trajectory and each force
evaluation solves (D^dag D) chi = phi from a zero guess.

The Sexton-Weingarten multiple time-scale integrator (the one Sec. III B uses
with 10 inner steps) nests a leapfrog of the cheap gauge force inside the
leapfrog of the expensive fermion force: each outer step of size dt is

  Pi <- Pi - dt/2 F_f(U)
  n_inner leapfrog steps of size h = dt / n_inner on the gauge force alone:
      Pi <- Pi - h/2 F_G(U);  U <- reunitarize(exp(h Pi) U);  Pi <- Pi - h/2 F_G(U)
  Pi <- Pi - dt/2 F_f(U)

written here without merging adjacent kicks.  The fermion part may be the
plain action or the stout-smeared one (stout.py).
"""
from __future__ import annotations

from .action import gauge_action, fermion_action, kinetic
from .force import force_from_grad, gauge_force, fermion_force_from_solution
from .solver import solve_ddag_d
from .su3 import expm_antihermitian, reunitarize


def total_force(u, phi, beta, kappa, bc=-1, tol=1e-12, with_fermion=True):
    f = gauge_force(u, beta)
    if with_fermion:
        chi, eta, _, _ = solve_ddag_d(u, phi, kappa, bc, tol)
        f = f + fermion_force_from_solution(u, chi, eta, kappa, bc)
    return f


def hamiltonian(u, p, phi, beta, kappa, bc=-1, tol=1e-12, with_fermion=True):
    h = kinetic(p) + gauge_action(u, beta)
    if with_fermion:
        h += fermion_action(u, phi, kappa, bc, tol)[0]
    return h


def link_update(u, p, dt):
    """U <- reunitarize(exp(dt Pi) U)  (eq. 5 / S2.1 with the reunitarization reading)."""
    return reunitarize(expm_antihermitian(dt * p) @ u)


def leapfrog(u, p, phi, beta, kappa, dt, nsteps, bc=-1, tol=1e-12, with_fermion=True):
    """Returns (U, Pi) after nsteps leapfrog steps of size dt."""
    def force(v):
        return total_force(v, phi, beta, kappa, bc, tol, with_fermion)

    p = p - 0.5 * dt * force(u)
    for k in range(nsteps):
        u = link_update(u, p, dt)
        step = dt if k < nsteps - 1 else 0.5 * dt
        p = p - step * force(u)
    return u, p


def trajectory_dh(u, p, phi, beta, kappa, dt, nsteps, bc=-1, tol=1e-12, with_fermion=True):
    """(U', Pi', Delta H) for one trajectory."""
    h0 = hamiltonian(u, p, phi, beta, kappa, bc, tol, with_fermion)
    u1, p1 = leapfrog(u, p, phi, beta, kappa, dt, nsteps, bc, tol, with_fermion)
    h1 = hamiltonian(u1, p1, phi, beta, kappa, bc, tol, with_fermion)
    return u1, p1, h1 - h0


def fermion_force_only(u, phi, kappa, bc=-1, tol=1e-12, rho=0.0, nlevels=0, eo=False):
    """F_f at U: of S_f(U), or of S_f(stout^n(U)) when nlevels > 0, or of the
    even/odd-preconditioned action S_eo(U; phi_o) when eo (eo.py)."""
    if eo:
        from .eo import eo_force
        return eo_force(u, phi, kappa, bc, tol)
    if nlevels > 0:
        from .stout import smeared_fermion_grad
        return force_from_grad(u, smeared_fermion_grad(u, phi, kappa, rho, nlevels, bc, tol))
    chi, eta, _, _ = solve_ddag_d(u, phi, kappa, bc, tol)
    return fermion_force_from_solution(u, chi, eta, kappa, bc)


def sexton_weingarten(u, p, phi, beta, kappa, dt, nsteps, n_inner, bc=-1, tol=1e-12, rho=0.0, nlevels=0,
                      eo=False):
    """Returns (U, Pi) after nsteps outer steps of size dt, each with n_inner
    gauge-force leapfrog steps of size dt / n_inner (module docstring)."""
    h = dt / n_inner
    for _ in range(nsteps):
        p = p - 0.5 * dt * fermion_force_only(u, phi, kappa, bc, tol, rho, nlevels, eo)
        for _ in range(n_inner):
            p = p - 0.5 * h * gauge_force(u, beta)
            u = link_update(u, p, h)
            p = p - 0.5 * h * gauge_force(u, beta)
        p = p - 0.5 * dt * fermion_force_only(u, phi, kappa, bc, tol, rho, nlevels, eo)
    return u, p


def hamiltonian_smeared(u, p, phi, beta, kappa, bc=-1, tol=1e-12, rho=0.0, nlevels=0, eo=False):
    if eo:
        from .eo import eo_action
        return kinetic(p) + gauge_action(u, beta) + eo_action(u, phi, kappa, bc, tol)
    if nlevels > 0:
        from .stout import total_action
        return kinetic(p) + total_action(u, phi, beta, kappa, rho, nlevels, bc, tol)
    return hamiltonian(u, p, phi, beta, kappa, bc, tol)


def sw_trajectory_dh(u, p, phi, beta, kappa, dt, nsteps, n_inner, bc=-1, tol=1e-12, rho=0.0, nlevels=0, eo=False):
    """(U', Pi', Delta H) for one Sexton-Weingarten trajectory (n_inner = 1: leapfrog)."""
    h0 = hamiltonian_smeared(u, p, phi, beta, kappa, bc, tol, rho, nlevels, eo)
    u1, p1 = sexton_weingarten(u, p, phi, beta, kappa, dt, nsteps, n_inner, bc, tol, rho, nlevels, eo)
    h1 = hamiltonian_smeared(u1, p1, phi, beta, kappa, bc, tol, rho, nlevels, eo)
    return u1, p1, h1 - h0
