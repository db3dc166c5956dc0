"""Seeded synthetic inputs for the Wilson-fermion HMC hot path.

This module is shared by the FP64 oracle (``oracle/``) and the HIP path
(``paper_2602_20516_amd``).  It draws random numbers and builds the fields
the workloads start from; it holds none of the method's arithmetic (no Dirac
operator, no solver, no action, no force, no update).

Field layouts (C order, lexicographic site = x + Lx*(y + Ly*(z + Lz*t))):

* gauge links / momenta: complex128 ``(Lt, Lz, Ly, Lx, 4, 3, 3)``; the
  direction index runs mu = 0,1,2,3 = x,y,z,t;
* spinors: complex128 ``(Lt, Lz, Ly, Lx, 4, 3)`` (spin, colour).

Recipes (the paper states none; these follow the workload descriptions the
paper's lattices are quoted with):

* links  U_mu(x) = exp(i*eps*sum_a c_a T_a), c_a ~ N(0,1) i.i.d., with
  T_a = lambda_a / 2 (Gell-Mann).  Drawn as ``standard_normal((Lt,Lz,Ly,Lx,4,8))``.
* eta    complex Gaussian with E|eta_i|^2 = 1: the real array is drawn first,
  then the imaginary array, from the same generator; both divided by sqrt(2).
* momenta Pi_mu(x) = i*sum_a p_a T_a, p_a ~ N(0,1): traceless anti-Hermitian.
* gauge transforms g(x) = exp(i*sum_a c_a T_a), c_a ~ N(0, scale^2).

Every generator is ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "CONFIGS",
    "config",
    "lattice_shape",
    "random_links",
    "unit_links",
    "gaussian_spinor",
    "random_momenta",
    "random_gauge_transform",
    "random_site_unitaries",
]


def _gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices lambda_a (a = 1..8), shape (8, 3, 3)."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0, 0, 1] = lam[0, 1, 0] = 1
    lam[1, 0, 1] = -1j
    lam[1, 1, 0] = 1j
    lam[2, 0, 0] = 1
    lam[2, 1, 1] = -1
    lam[3, 0, 2] = lam[3, 2, 0] = 1
    lam[4, 0, 2] = -1j
    lam[4, 2, 0] = 1j
    lam[5, 1, 2] = lam[5, 2, 1] = 1
    lam[6, 1, 2] = -1j
    lam[6, 2, 1] = 1j
    lam[7, 0, 0] = lam[7, 1, 1] = 1 / math.sqrt(3)
    lam[7, 2, 2] = -2 / math.sqrt(3)
    return lam


_T = _gell_mann() / 2.0


def lattice_shape(dims) -> tuple:
    """(Lx, Ly, Lz, Lt) -> array site shape (Lt, Lz, Ly, Lx)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    return (lt, lz, ly, lx)


def _exp_i_hermitian(h: np.ndarray, chunk: int = 1 << 20) -> np.ndarray:
    """exp(i*h) for a stack of Hermitian 3x3 matrices, by eigendecomposition."""
    flat = h.reshape(-1, 3, 3)
    out = np.empty_like(flat)
    for s in range(0, flat.shape[0], chunk):
        w, v = np.linalg.eigh(flat[s:s + chunk])
        out[s:s + chunk] = np.einsum("nij,nj,nkj->nik", v, np.exp(1j * w), v.conj())
    return out.reshape(h.shape)


def _coeffs_to_hermitian(c: np.ndarray) -> np.ndarray:
    return np.einsum("...a,aij->...ij", c, _T)


def random_links(dims, eps: float, seed: int) -> np.ndarray:
    """Seeded SU(3) link field U_mu(x) = exp(i*eps*sum_a c_a T_a)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.standard_normal(lattice_shape(dims) + (4, 8))
    return _exp_i_hermitian(eps * _coeffs_to_hermitian(c))


def unit_links(dims) -> np.ndarray:
    """The free (cold) configuration U_mu(x) = 1."""
    u = np.zeros(lattice_shape(dims) + (4, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1
    return u


def gaussian_spinor(dims, seed: int) -> np.ndarray:
    """Complex Gaussian spinor with E|eta_i|^2 = 1 (real part drawn first)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = lattice_shape(dims) + (4, 3)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) / math.sqrt(2.0)


def random_momenta(dims, seed: int) -> np.ndarray:
    """Traceless anti-Hermitian momenta Pi = i*sum_a p_a T_a, p_a ~ N(0,1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = rng.standard_normal(lattice_shape(dims) + (4, 8))
    return 1j * _coeffs_to_hermitian(p)


def random_site_unitaries(dims, seed: int, scale: float = 1.0) -> np.ndarray:
    """One SU(3) matrix per site (a gauge transformation), shape (Lt,Lz,Ly,Lx,3,3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.standard_normal(lattice_shape(dims) + (8,))
    return _exp_i_hermitian(scale * _coeffs_to_hermitian(c))


random_gauge_transform = random_site_unitaries


# ---------------------------------------------------------------------------
# Workload table.  dims are (Lx, Ly, Lz, Lt); seeds: links 100c+1, eta 100c+2,
# momenta 100c+3.  fermion_bc is the sign of the temporal boundary condition
# of the fermion field (-1: antiperiodic).
# ---------------------------------------------------------------------------
CONFIGS = {
    1: dict(name="c1-4^4-fp64", dims=(4, 4, 4, 4), eps=0.5, beta=5.7, kappa=0.12,
            tol=1e-12, dt=0.05, nsteps=1, precision="fp64",
            seeds=dict(links=101, eta=102, mom=103)),
    2: dict(name="c2-16^4-fp64", dims=(16, 16, 16, 16), eps=0.3, beta=6.0, kappa=0.125,
            tol=1e-10, precision="fp64",
            seeds=dict(links=201, eta=202, mom=203)),
    3: dict(name="c3-24^3x48-mixed", dims=(24, 24, 24, 48), eps=0.2, beta=6.0, kappa=0.13,
            tol=1e-10, precision="mixed_fp32",
            seeds=dict(links=301, eta=302, mom=303)),
    4: dict(name="c4-multi-rhs", dims_list=[(8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 16)],
            eps=0.3, beta=6.0, kappas=(0.10, 0.11, 0.12, 0.125, 0.13, 0.135), eta_seeds=(402, 403),
            tol=1e-10, precision="mixed_fp32", seeds=dict(links=401, mom=404)),
    5: dict(name="c5-32^3x64-stout", dims=(32, 32, 32, 64), eps=0.2, beta=6.0, kappa=0.135,
            rho=0.1, nstout=2, nsteps=10, tau=1.0, tol=1e-10, precision="mixed_fp32",
            seeds=dict(links=501, eta=502, mom=503)),
}

FERMION_BC = -1


def config(c: int) -> dict:
    d = dict(CONFIGS[c])
    d.setdefault("fermion_bc", FERMION_BC)
    return d
