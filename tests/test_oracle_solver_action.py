"""Pins of the oracle's solver and actions (CPU)."""
import numpy as np
import pytest

import lgt_inputs as li
from oracle import action, dirac, solver
from oracle.lattice import shift
from oracle.su3 import dag

DIMS = (2, 2, 2, 4)


@pytest.fixture(scope="module")
def fields():
    u = li.random_links(DIMS, 0.5, 1)
    eta = li.gaussian_spinor(DIMS, 2)
    return u, eta


def test_cg_matches_dense_solve(fields):
    u, eta = fields
    k = 0.12
    d = dirac.dense_dirac(u, k)
    phi = dirac.dslash_dag(u, eta, k)
    x_dense = np.linalg.solve(d.conj().T @ d, phi.ravel())
    x, eta_cg, it, res = solver.solve_ddag_d(u, phi, k, tol=1e-13)
    assert res < 1e-13 * 10
    assert np.linalg.norm(x.ravel() - x_dense) / np.linalg.norm(x_dense) < 1e-11
    # eta = D chi solves D^dag eta = phi, i.e. eta = D^-dag phi
    assert np.linalg.norm(eta_cg.ravel() - np.linalg.solve(d.conj().T, phi.ravel())) < 1e-10


def test_fermion_action_heat_bath_identity():
    """S_f(phi = D^dag eta) = eta^dag eta exactly (eq. S3.1 at the heat-bath field)."""
    dims = (4, 4, 4, 4)
    u = li.random_links(dims, 0.5, 101)
    eta = li.gaussian_spinor(dims, 102)
    phi = dirac.dslash_dag(u, eta, 0.12)
    s, chi, y, it, res = action.fermion_action(u, phi, 0.12, tol=1e-12)
    ee = float(np.vdot(eta.ravel(), eta.ravel()).real)
    assert res <= 1e-12 * 1.5
    assert abs(s - ee) / ee < 1e-13
    # and eta itself is recovered: Y = D chi = D (D^dag D)^-1 D^dag eta = eta
    assert np.linalg.norm(y - eta) / np.linalg.norm(eta) < 1e-9


def test_cg_free_field_closed_form():
    """At U = 1, A = D^dag D is diagonal in momentum space: compare with an FFT solve."""
    dims = (4, 4, 4, 8)
    lx, ly, lz, lt = dims
    k = 0.12
    u = li.unit_links(dims)
    b = li.gaussian_spinor(dims, 5)
    x, it, res = solver.cg(lambda v: dirac.ddag_d(u, v, k), b, 1e-13)
    # half-integer p_t: untwist by exp(-i pi t / lt) to reach integer Fourier modes
    t = np.arange(lt)[:, None, None, None, None, None]
    tw = np.exp(-1j * np.pi * t / lt)
    bh = np.fft.fftn(b * tw, axes=(0, 1, 2, 3))
    # in the twisted frame plane wave index n corresponds to momentum p = 2 pi n / L (+ pi/L in t)
    pt = 2 * np.pi * (np.fft.fftfreq(lt) * lt + 0.5) / lt
    pz = 2 * np.pi * np.fft.fftfreq(lz)
    py = 2 * np.pi * np.fft.fftfreq(ly)
    px = 2 * np.pi * np.fft.fftfreq(lx)
    P = np.meshgrid(pt, pz, py, px, indexing="ij")
    # the fft sign convention: bh(n) = sum_x b(x) exp(-i p x); D acting on exp(+ipx) gives D(p)
    cos = sum(np.cos(q) for q in P)
    sin2 = sum(np.sin(q) ** 2 for q in P)
    a_p = (1 - 2 * k * cos) ** 2 + 4 * k * k * sin2     # D(p)^dag D(p) is a multiple of 1
    xh = bh / a_p[..., None, None]
    x_ref = np.fft.ifftn(xh, axes=(0, 1, 2, 3)) / tw
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-11


def test_plaquette_unit_field():
    u = li.unit_links((4, 4, 4, 4))
    assert action.mean_plaquette(u) == 1.0
    assert action.gauge_action(u, 6.0) == 0.0


def test_single_link_gauge_action_closed_form():
    """All links 1 except one: that link sits in 6 plaquettes, S_G = 6 beta (1 - Re tr U / 3)."""
    dims = (4, 4, 4, 4)
    u = li.unit_links(dims)
    v = li.random_links((1, 1, 1, 1), 0.9, 3)[0, 0, 0, 0, 2]
    u[1, 2, 3, 0, 2] = v
    beta = 5.7
    assert abs(action.gauge_action(u, beta) - 6 * beta * (1 - np.trace(v).real / 3)) < 1e-12


def test_gauge_invariance_of_actions(fields):
    u, eta = fields
    k = 0.12
    g = li.random_site_unitaries(DIMS, 9)
    ug = np.empty_like(u)
    for mu in range(4):
        ug[..., mu, :, :] = g @ u[..., mu, :, :] @ dag(shift(g, mu, +1))
    assert abs(action.gauge_action(ug, 5.7) - action.gauge_action(u, 5.7)) < 1e-11
    phi = dirac.dslash_dag(u, eta, k)
    gphi = np.einsum("...ij,...sj->...si", g, phi)
    s0 = action.fermion_action(u, phi, k, tol=1e-13)[0]
    s1 = action.fermion_action(ug, gphi, k, tol=1e-13)[0]
    assert abs(s0 - s1) / abs(s0) < 1e-12


def test_kinetic_normalisation():
    dims = (2, 2, 2, 2)
    p = li.random_momenta(dims, 33)
    coeff = np.random.Generator(np.random.PCG64(33)).standard_normal((2, 2, 2, 2, 4, 8))
    assert abs(action.kinetic(p) - 0.5 * np.sum(coeff ** 2)) < 1e-12
