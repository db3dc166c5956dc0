"""Pins of the oracle's Wilson-Dirac operator (CPU)."""
import numpy as np
import pytest

import lgt_inputs as li
from oracle import dirac
from oracle.lattice import shift
from oracle.su3 import dag

SMALL = (2, 2, 2, 4)


@pytest.fixture(scope="module")
def small():
    u = li.random_links(SMALL, 0.5, 1)
    psi = li.gaussian_spinor(SMALL, 2)
    return u, psi


@pytest.mark.parametrize("bc", [-1, 1])
def test_stencil_matches_dense_blocks(small, bc):
    u, psi = small
    d = dirac.dense_dirac(u, 0.12, bc)
    assert np.max(np.abs(d @ psi.ravel() - dirac.dslash(u, psi, 0.12, bc).ravel())) < 1e-14
    assert np.max(np.abs(d.conj().T @ psi.ravel()
                         - dirac.dslash_dag(u, psi, 0.12, bc).ravel())) < 1e-14


def test_stencil_matches_dense_4x4():
    dims = (4, 4, 4, 4)
    u = li.random_links(dims, 0.5, 101)
    psi = li.gaussian_spinor(dims, 102)
    d = dirac.dense_dirac(u, 0.12)
    assert np.max(np.abs(d @ psi.ravel() - dirac.dslash(u, psi, 0.12).ravel())) < 1e-13


def test_gamma5_hermiticity(small):
    u, psi = small
    lhs = dirac.dslash_dag(u, psi, 0.13)
    rhs = dirac.gamma5(dirac.dslash(u, dirac.gamma5(psi), 0.13))
    assert np.max(np.abs(lhs - rhs)) < 1e-14


def test_kappa_zero_is_identity(small):
    u, psi = small
    assert np.array_equal(dirac.dslash(u, psi, 0.0), psi)


@pytest.mark.parametrize("dims", [(2, 2, 2, 4), (4, 2, 2, 4)])
def test_free_spectrum_closed_form(dims):
    """Eigenvalues of D at U = 1 equal 1 - 2k sum cos p +- 2ik sqrt(sum sin^2 p), half-integer p_t."""
    k = 0.12
    ev = np.linalg.eigvals(dirac.dense_dirac(li.unit_links(dims), k))
    ref = dirac.free_spectrum(dims, k)
    assert np.max(np.abs(np.sort(ev.real) - np.sort(ref.real))) < 1e-12
    assert np.max(np.abs(np.sort(ev.imag) - np.sort(ref.imag))) < 1e-12
    assert max(np.min(np.abs(ref - e)) for e in ev) < 1e-12


def test_free_plane_wave_on_4x4x4x8():
    """A plane wave with antiperiodic p_t is an eigenvector of the free D(p)."""
    dims = (4, 4, 4, 8)
    lx, ly, lz, lt = dims
    k = 0.11
    n = (1, 3, 0, 2)
    p = [2 * np.pi * n[0] / lx, 2 * np.pi * n[1] / ly, 2 * np.pi * n[2] / lz,
         2 * np.pi * (n[3] + 0.5) / lt]
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    rng = np.random.default_rng(0)
    w = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    psi = phase[..., None, None] * w
    dp = (1 - 2 * k * sum(np.cos(q) for q in p)) * np.eye(4) \
        + 2j * k * sum(dirac.GAMMA[m] * np.sin(p[m]) for m in range(4))
    expect = phase[..., None, None] * (dp @ w)
    got = dirac.dslash(li.unit_links(dims), psi, k)
    assert np.max(np.abs(got - expect)) < 1e-13


def test_gauge_covariance(small):
    """D[U^g](g psi) = g D[U] psi with U^g_mu(x) = g(x) U_mu(x) g(x+mu)^dag."""
    u, psi = small
    g = li.random_site_unitaries(SMALL, 9)
    ug = np.empty_like(u)
    for mu in range(4):
        ug[..., mu, :, :] = g @ u[..., mu, :, :] @ dag(shift(g, mu, +1))
    gpsi = np.einsum("...ij,...sj->...si", g, psi)
    lhs = dirac.dslash(ug, gpsi, 0.12)
    rhs = np.einsum("...ij,...sj->...si", g, dirac.dslash(u, psi, 0.12))
    assert np.max(np.abs(lhs - rhs)) < 1e-14


def test_boundary_sign_only_on_last_time_slice(small):
    u, psi = small
    diff = dirac.dslash(u, psi, 0.12, -1) - dirac.dslash(u, psi, 0.12, +1)
    # only sites on t = 0 and t = Lt-1 feel the temporal boundary
    assert np.max(np.abs(diff[1:-1])) == 0
    assert np.max(np.abs(diff[0])) > 0 and np.max(np.abs(diff[-1])) > 0
