"""Even/odd-preconditioned pseudofermion action, for the oracle (test
infrastructure only).

With the sites split by parity, D = [[1, -kappa H_eo], [-kappa H_oe, 1]]
(H_eo takes odd-site values to even sites), and since the even-even block
is the identity,

  det D = det(1 - kappa^2 H_oe H_eo) = det Dhat,   Dhat acting on odd sites.

The preconditioned action S_eo = phi_o^dag (Dhat^dag Dhat)^-1 phi_o gives the
same determinant weight with one solve per evaluation (the production
variant of the action of eq. S3.1).  Its heat bath is phi_o = Dhat^dag eta_o.

Fields are full-lattice arrays (as in dirac.py) whose even sites are zero.
Everything is built from dirac.hopping_term and masks: no even/odd storage.
"""
from __future__ import annotations

import numpy as np

from .dirac import hopping_term
from .force import bilinear_grad, force_from_grad
from .lattice import coords


def parity_mask(dims, parity: int) -> np.ndarray:
    """1 on the sites with (x + y + z + t) % 2 == parity, shaped to broadcast over [..., 4, 3]."""
    x, y, z, t = coords(dims)
    return (((x + y + z + t) % 2) == parity).astype(float)[..., None, None]


def hop_to(u, psi, to_parity, bc=-1, dagger=False):
    """H (or H^dag) restricted to output sites of to_parity (input: the other parity)."""
    dims = psi.shape[:4][::-1]
    src = parity_mask(dims, 1 - to_parity) * psi
    return parity_mask(dims, to_parity) * hopping_term(u, src, bc, +1 if dagger else -1)


def schur(u, psi_o, kappa, bc=-1):
    """Dhat psi_o = psi_o - kappa^2 H_oe H_eo psi_o (odd sites)."""
    return psi_o - kappa * kappa * hop_to(u, hop_to(u, psi_o, 0, bc), 1, bc)


def schur_dag(u, psi_o, kappa, bc=-1):
    """Dhat^dag psi_o = psi_o - kappa^2 (H_eo)^dag (H_oe)^dag psi_o; (H_oe)^dag takes odd
    sites to even ones and is the dagger hop restricted so."""
    return psi_o - kappa * kappa * hop_to(u, hop_to(u, psi_o, 0, bc, True), 1, bc, True)


def solve_normal(u, phi_o, kappa, bc=-1, tol=1e-14, max_iter=20000, shift=0.0):
    """X_o = (Dhat^dag Dhat + shift)^-1 phi_o by textbook CG on the odd sites
    (one system; the multi-shift solver's result for each shift, by definition)."""
    x = np.zeros_like(phi_o)
    r = phi_o.copy()
    p = r.copy()
    rr = float(np.vdot(r.ravel(), r.ravel()).real)
    bb = rr
    for _ in range(max_iter):
        if rr <= tol * tol * bb:
            break
        q = schur_dag(u, schur(u, p, kappa, bc), kappa, bc) + shift * p
        alpha = rr / float(np.vdot(p.ravel(), q.ravel()).real)
        x = x + alpha * p
        r = r - alpha * q
        rr_new = float(np.vdot(r.ravel(), r.ravel()).real)
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x


def eo_action(u, phi_o, kappa, bc=-1, tol=1e-14):
    """S_eo = phi_o^dag (Dhat^dag Dhat)^-1 phi_o."""
    x = solve_normal(u, phi_o, kappa, bc, tol)
    return float(np.vdot(phi_o.ravel(), x.ravel()).real)


def eo_grad(u, phi_o, kappa, bc=-1, tol=1e-14, shift=0.0):
    """G = dS_eo/dRe U + i dS_eo/dIm U (with shift: of phi_o^dag (Dhat^dag Dhat + shift)^-1 phi_o,
    whose variation is -X^dag d(Dhat^dag Dhat) X as well: the shift is constant).

    dS_eo = -2 Re[Y^dag dDhat X] with X = (Dhat^dag Dhat)^-1 phi_o, Y = Dhat X,
    and dDhat = -kappa^2 (dH_oe H_eo + H_oe dH_eo), so
    dS_eo = 2 kappa^2 Re[a^dag dH b] with the full-lattice fields
    a = (H_oe^dag Y on even sites, Y on odd), b = (H_eo X on even, X on odd):
    a^dag dH b = (H_oe^dag Y)^dag dH_eo X + Y^dag dH_oe (H_eo X).  With
    I = Re a^dag D b = Re a^dag (1 - kappa H) b, dI = -kappa Re a^dag dH b, so
    dS_eo = -2 kappa dI: the bilinear gradient with coefficient -2 kappa.
    """
    x = solve_normal(u, phi_o, kappa, bc, tol, shift=shift)
    y = schur(u, x, kappa, bc)
    a = hop_to(u, y, 0, bc, dagger=True) + y
    b = hop_to(u, x, 0, bc) + x
    return -2.0 * kappa * bilinear_grad(u, a, b, kappa, bc)


def eo_force(u, phi_o, kappa, bc=-1, tol=1e-14):
    return force_from_grad(u, eo_grad(u, phi_o, kappa, bc, tol))


# ---- rational (RHMC) pseudofermion action ------------------------------------
# A rational approximation in partial fractions, R(A) = a0 + sum_i a_i (A + sigma_i)^-1
# with A = Dhat^dag Dhat (RHMC is among the algorithms Sec. I names), gives the action
# S_R = phi_o^dag R(A) phi_o.  Its gradient is the residue-weighted sum of the shifted
# even/odd gradients; a0 contributes no force.

def rational_action(u, phi_o, kappa, a0, shifts, residues, bc=-1, tol=1e-14):
    """S_R = a0 |phi_o|^2 + sum_i a_i phi_o^dag (Dhat^dag Dhat + sigma_i)^-1 phi_o."""
    f = phi_o.ravel()
    s = a0 * float(np.vdot(f, f).real)
    for sig, a in zip(shifts, residues):
        x = solve_normal(u, phi_o, kappa, bc, tol, shift=sig)
        s += a * float(np.vdot(f, x.ravel()).real)
    return s


def rational_grad(u, phi_o, kappa, a0, shifts, residues, bc=-1, tol=1e-14):
    g = np.zeros(u.shape, dtype=complex)
    for sig, a in zip(shifts, residues):
        g = g + a * eo_grad(u, phi_o, kappa, bc, tol, shift=sig)
    return g


def rational_force(u, phi_o, kappa, a0, shifts, residues, bc=-1, tol=1e-14):
    return force_from_grad(u, rational_grad(u, phi_o, kappa, a0, shifts, residues, bc, tol))
