"""Conjugate gradient for the oracle (test infrastructure only).

The pseudofermion action and force need chi = A^-1 phi with A = D^dag D
(eq. S3.6); the paper names conjugate gradient as one way to solve it and does not
differentiate the solve.  This is the textbook CG (Hestenes-Stiefel) on the
Hermitian positive definite A, from a zero initial guess, stopping when the
recursively updated residual satisfies ||r|| <= tol * ||b||.  The true
residual ||b - A x|| / ||b|| is recomputed at exit and returned.
"""
from __future__ import annotations

import numpy as np

from .dirac import ddag_d, dslash


def vdot(a: np.ndarray, b: np.ndarray) -> complex:
    return complex(np.vdot(a.ravel(), b.ravel()))


def norm2(a: np.ndarray) -> float:
    return float(np.real(np.vdot(a.ravel(), a.ravel())))


class NotConverged(RuntimeError):
    pass


def cg(apply_a, b: np.ndarray, tol: float, max_iter: int = 20000):
    """Solve A x = b; returns (x, iterations, true relative residual)."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = norm2(r)
    bb = norm2(b)
    if bb == 0.0:
        return x, 0, 0.0
    k = 0
    while rr > tol * tol * bb:
        if k >= max_iter:
            raise NotConverged(f"CG did not reach {tol} in {max_iter} iterations")
        q = apply_a(p)
        alpha = rr / np.real(vdot(p, q))
        x = x + alpha * p
        r = r - alpha * q
        rr_new = norm2(r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        k += 1
    true_res = np.sqrt(norm2(b - apply_a(x)) / bb)
    return x, k, float(true_res)


def solve_ddag_d(u: np.ndarray, phi: np.ndarray, kappa: float, bc: int = -1,
                 tol: float = 1e-12, max_iter: int = 20000):
    """chi = (D^dag D)^-1 phi and eta = D chi (eq. S3.6 and the definition below S3.10).

    Returns (chi, eta, iterations, true relative residual).  The oracle calls
    the paper's eta "Y" to keep it apart from the Gaussian heat-bath field.
    """
    x, it, res = cg(lambda v: ddag_d(u, v, kappa, bc), phi, tol, max_iter)
    return x, dslash(u, x, kappa, bc), it, res
