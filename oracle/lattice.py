"""Periodic lattice shifts for the oracle (test infrastructure only).

Site fields have the leading shape (Lt, Lz, Ly, Lx); direction mu = 0, 1, 2, 3
is x, y, z, t.  ``shift(f, mu, +1)[x] = f[x + mu_hat]`` and
``shift(f, mu, -1)[x] = f[x - mu_hat]``, periodic in every direction.  The
fermion's temporal boundary condition is not applied here: it is folded into
the links by ``dirac.fermion_links``.
"""
from __future__ import annotations

import numpy as np

# array axis of direction mu in a (Lt, Lz, Ly, Lx, ...) field
AXIS = {0: 3, 1: 2, 2: 1, 3: 0}


def dims_of(field: np.ndarray) -> tuple:
    """(Lx, Ly, Lz, Lt) of a site field."""
    lt, lz, ly, lx = field.shape[:4]
    return (lx, ly, lz, lt)


def shift(f: np.ndarray, mu: int, sign: int) -> np.ndarray:
    """f(x + sign*mu_hat), periodic."""
    return np.roll(f, -sign, axis=AXIS[mu])


def coords(dims):
    """Integer coordinate arrays x, y, z, t, each of site shape (Lt, Lz, Ly, Lx)."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    return x, y, z, t
