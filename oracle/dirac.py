"""Wilson-Dirac operator for the oracle (test infrastructure only).

The paper uses "the Wilson-Dirac operator" D(U) inside the pseudofermion
action S_f = phi^dag (D^dag D)^-1 phi (eq. S3.1) without writing it out.  The
reading taken here is the hopping-parameter form

  (D psi)(x) = psi(x) - kappa * sum_mu [ (1 - gamma_mu) U~_mu(x) psi(x + mu)
                                       + (1 + gamma_mu) U~_mu(x - mu)^dag psi(x - mu) ]

with gamma matrices in the chiral basis

  gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] (k = 1, 2, 3),
  gamma_4 = [[0, 1], [1, 0]],  gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 = diag(1, 1, -1, -1),

periodic links in all directions, and the fermion's temporal boundary
condition folded into the links: U~_4(x) = bc * U_4(x) on the last time slice
(bc = -1 is antiperiodic), U~ = U elsewhere.

Everything is written with explicit 4x4 spin matrices on the full lattice;
there is no even/odd split and no spin projection.
"""
from __future__ import annotations

import numpy as np

from .lattice import shift
from .su3 import dag

_SIGMA = np.array([[[0, 1], [1, 0]],
                   [[0, -1j], [1j, 0]],
                   [[1, 0], [0, -1]]], dtype=np.complex128)


def _gammas():
    g = np.zeros((4, 4, 4), dtype=np.complex128)
    z = np.zeros((2, 2))
    for k in range(3):
        g[k] = np.block([[z, -1j * _SIGMA[k]], [1j * _SIGMA[k], z]])
    g[3] = np.block([[z, np.eye(2)], [np.eye(2), z]])
    return g


GAMMA = _gammas()
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
ONE4 = np.eye(4, dtype=np.complex128)


def fermion_links(u: np.ndarray, bc: int = -1) -> np.ndarray:
    """U~: the links with the temporal fermion boundary sign on the last t slice."""
    ut = u.copy()
    ut[-1, :, :, :, 3] *= bc
    return ut


def color_mul(u: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(U psi)_s,i = sum_j U_ij psi_s,j at every site."""
    return np.einsum("...ij,...sj->...si", u, psi)


def spin_mul(g: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(G psi)_s,i = sum_t G_st psi_t,i at every site."""
    return np.einsum("st,...ti->...si", g, psi)


def hopping_term(u: np.ndarray, psi: np.ndarray, bc: int = -1, sign: int = -1) -> np.ndarray:
    """sum_mu [(1 + sign*gamma_mu) U~_mu(x) psi(x+mu) + (1 - sign*gamma_mu) U~_mu(x-mu)^dag psi(x-mu)].

    sign = -1 is the hopping term of D, sign = +1 the one of D^dag.
    """
    ut = fermion_links(u, bc)
    out = np.zeros_like(psi)
    for mu in range(4):
        umu = ut[..., mu, :, :]
        fwd = color_mul(umu, shift(psi, mu, +1))
        bwd = color_mul(dag(shift(umu, mu, -1)), shift(psi, mu, -1))
        out += spin_mul(ONE4 + sign * GAMMA[mu], fwd)
        out += spin_mul(ONE4 - sign * GAMMA[mu], bwd)
    return out


def dslash(u: np.ndarray, psi: np.ndarray, kappa: float, bc: int = -1) -> np.ndarray:
    """D psi."""
    return psi - kappa * hopping_term(u, psi, bc, sign=-1)


def dslash_dag(u: np.ndarray, psi: np.ndarray, kappa: float, bc: int = -1) -> np.ndarray:
    """D^dag psi, written from the adjoint of each hopping block.

    The block of D coupling x to x+mu is -kappa (1 - gamma_mu) U~_mu(x); its
    adjoint couples x+mu to x with -kappa (1 - gamma_mu) U~_mu(x)^dag (gamma_mu
    is Hermitian).  Collecting terms by output site flips the sign of gamma_mu
    in both hops.
    """
    return psi - kappa * hopping_term(u, psi, bc, sign=+1)


def gamma5(psi: np.ndarray) -> np.ndarray:
    return spin_mul(GAMMA5, psi)


def ddag_d(u: np.ndarray, psi: np.ndarray, kappa: float, bc: int = -1) -> np.ndarray:
    """A psi = D^dag D psi (the operator of eq. S3.2)."""
    return dslash_dag(u, dslash(u, psi, kappa, bc), kappa, bc)


def site_index(dims, x, y, z, t) -> int:
    lx, ly, lz, lt = dims
    return x + lx * (y + ly * (z + lz * t))


def dense_dirac(u: np.ndarray, kappa: float, bc: int = -1) -> np.ndarray:
    """The 12V x 12V matrix of D, assembled block by block with Python loops.

    Row/column index = 12*site + 3*spin + colour, lexicographic site.  For
    tiny lattices only (it is an independent brute-force statement of D).
    """
    lt, lz, ly, lx = u.shape[:4]
    dims = (lx, ly, lz, lt)
    nsite = lx * ly * lz * lt
    d = np.zeros((12 * nsite, 12 * nsite), dtype=np.complex128)
    ext = (lx, ly, lz, lt)
    for t in range(lt):
        for z in range(lz):
            for y in range(ly):
                for x in range(lx):
                    s = site_index(dims, x, y, z, t)
                    d[12 * s:12 * s + 12, 12 * s:12 * s + 12] += np.eye(12)
                    c = [x, y, z, t]
                    for mu in range(4):
                        cf = list(c)
                        cf[mu] = (c[mu] + 1) % ext[mu]
                        cb = list(c)
                        cb[mu] = (c[mu] - 1) % ext[mu]
                        sf = site_index(dims, *cf)
                        sb = site_index(dims, *cb)
                        uf = u[t, z, y, x, mu].copy()
                        if mu == 3 and t == lt - 1:
                            uf = bc * uf
                        ub = u[cb[3], cb[2], cb[1], cb[0], mu].copy()
                        if mu == 3 and cb[3] == lt - 1:
                            ub = bc * ub
                        d[12 * s:12 * s + 12, 12 * sf:12 * sf + 12] += \
                            -kappa * np.kron(ONE4 - GAMMA[mu], uf)
                        d[12 * s:12 * s + 12, 12 * sb:12 * sb + 12] += \
                            -kappa * np.kron(ONE4 + GAMMA[mu], ub.conj().T)
    return d


def free_spectrum(dims, kappa: float, bc: int = -1) -> np.ndarray:
    """Eigenvalues of D at U = 1 in closed form (momentum space).

    D(p) = 1 - 2 kappa sum_mu cos p_mu + 2 i kappa sum_mu gamma_mu sin p_mu, whose
    eigenvalues are 1 - 2 kappa sum cos p_mu +- i 2 kappa sqrt(sum sin^2 p_mu), each twice
    (x3 colours).  p_mu = 2 pi n / L_mu, with n + 1/2 in time for bc = -1.
    """
    lx, ly, lz, lt = dims
    shift_t = 0.5 if bc == -1 else 0.0
    px = 2 * np.pi * np.arange(lx) / lx
    py = 2 * np.pi * np.arange(ly) / ly
    pz = 2 * np.pi * np.arange(lz) / lz
    pt = 2 * np.pi * (np.arange(lt) + shift_t) / lt
    P = np.meshgrid(px, py, pz, pt, indexing="ij")
    cos = sum(np.cos(p) for p in P)
    sin2 = sum(np.sin(p) ** 2 for p in P)
    re = 1 - 2 * kappa * cos
    im = 2 * kappa * np.sqrt(sin2)
    ev = np.concatenate([(re + 1j * im).ravel(), (re - 1j * im).ravel()])
    return np.repeat(ev, 6)
