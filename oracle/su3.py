"""SU(3) group and algebra helpers for the oracle (test infrastructure only).

* ``project_su`` is the su(N) projection P[A] = (A - A^dag)/2 - tr(A - A^dag)/(2N) * 1
  of eq. (7) / eq. (S2.9).
* ``expm_antihermitian`` is the matrix exponential of an anti-Hermitian matrix,
  as used by the left-multiplication update U -> exp(i eps H) U (eq. 5, S2.1).
  It is computed exactly through the Hermitian eigendecomposition.
* ``reunitarize`` re-projects a near-unitary 3x3 matrix onto SU(3) by row
  Gram-Schmidt with the third row conj(r1 x r2).
"""
from __future__ import annotations

import math

import numpy as np

NC = 3


def gell_mann() -> np.ndarray:
    """lambda_1..lambda_8, shape (8, 3, 3)."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = 1
    lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = 1
    lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = 1
    lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = 1 / math.sqrt(3)
    lam[7][1, 1] = 1 / math.sqrt(3)
    lam[7][2, 2] = -2 / math.sqrt(3)
    return lam


# Generators T_a = lambda_a / 2, tr(T_a T_b) = delta_ab / 2.
T = gell_mann() / 2


def dag(m: np.ndarray) -> np.ndarray:
    """Hermitian conjugate over the last two axes."""
    return np.conj(np.swapaxes(m, -1, -2))


def trace(m: np.ndarray) -> np.ndarray:
    return np.trace(m, axis1=-2, axis2=-1)


def identity_like(m: np.ndarray) -> np.ndarray:
    eye = np.zeros_like(m)
    n = m.shape[-1]
    for i in range(n):
        eye[..., i, i] = 1
    return eye


def project_su(a: np.ndarray) -> np.ndarray:
    """Traceless anti-Hermitian part, eq. (7): (A-A^dag)/2 - tr(A-A^dag)/(2N)."""
    d = a - dag(a)
    n = a.shape[-1]
    return 0.5 * d - (trace(d) / (2 * n))[..., None, None] * identity_like(a)


def expm_antihermitian(a: np.ndarray) -> np.ndarray:
    """exp(A) for anti-Hermitian A: with A = i*H, exp(A) = V diag(exp(i w)) V^dag."""
    h = -1j * a
    h = 0.5 * (h + dag(h))  # exactly Hermitian for eigh
    w, v = np.linalg.eigh(h)
    return np.einsum("...ij,...j,...kj->...ik", v, np.exp(1j * w), v.conj())


def reunitarize(u: np.ndarray) -> np.ndarray:
    """Row Gram-Schmidt on rows 1, 2; third row = conj(r1 x r2) (det = 1)."""
    r1 = u[..., 0, :]
    r1 = r1 / np.sqrt(np.sum(np.abs(r1) ** 2, axis=-1))[..., None]
    r2 = u[..., 1, :]
    r2 = r2 - np.sum(np.conj(r1) * r2, axis=-1)[..., None] * r1
    r2 = r2 / np.sqrt(np.sum(np.abs(r2) ** 2, axis=-1))[..., None]
    r3 = np.conj(np.cross(r1, r2))
    return np.stack([r1, r2, r3], axis=-2)


def algebra_coeffs(x: np.ndarray) -> np.ndarray:
    """Coefficients x_a of X = i*sum_a x_a T_a (traceless anti-Hermitian).

    tr(T_a X) = i x_a / 2, hence x_a = 2 Im tr(T_a X).
    """
    return 2.0 * np.imag(np.einsum("aij,...ji->...a", T, x))


def from_coeffs(x: np.ndarray) -> np.ndarray:
    """i * sum_a x_a T_a."""
    return 1j * np.einsum("...a,aij->...ij", x, T)


def unitarity_defect(u: np.ndarray) -> float:
    """max over the stack of ||U^dag U - 1||_F."""
    e = dag(u) @ u - identity_like(u)
    return float(np.max(np.sqrt(np.sum(np.abs(e) ** 2, axis=(-2, -1)))))
