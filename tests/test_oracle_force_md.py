"""Pins of the oracle's gradients, forces and leapfrog (CPU).

Every gradient is pinned by central finite differences of the action it
differentiates.  Re[a^dag D(U) b] and S_G are linear in the real components of
any single link, so their component differences are exact up to rounding;
derivatives through the solve use Lie-direction differences.
"""
import numpy as np
import pytest

import lgt_inputs as li
from oracle import action, dirac, force, md, su3
from oracle.lattice import shift
from oracle.su3 import dag

DIMS = (2, 2, 2, 4)
LINKS = [((0, 1, 0, 1), 2), ((3, 0, 1, 0), 3), ((1, 1, 1, 1), 0), ((0, 0, 0, 0), 1),
         ((3, 1, 1, 1), 3)]  # (t, z, y, x) site, mu; t = Lt-1 with mu = 3 crosses the t boundary


@pytest.fixture(scope="module")
def f():
    u = li.random_links(DIMS, 0.5, 1)
    eta = li.gaussian_spinor(DIMS, 2)
    k = 0.12
    phi = dirac.dslash_dag(u, eta, k)
    return u, eta, phi, k


def test_bilinear_grad_components_exact(f):
    u, _, _, k = f
    a = li.gaussian_spinor(DIMS, 21)
    b = li.gaussian_spinor(DIMS, 22)

    def re_i(v):
        return float(np.real(np.vdot(a.ravel(), dirac.dslash(v, b, k).ravel())))

    g = force.bilinear_grad(u, a, b, k)
    for site, mu in LINKS:
        for i in range(3):
            for j in range(3):
                gr = force.component_fd(re_i, u, site, mu, i, j, False, h=1e-3)
                gi = force.component_fd(re_i, u, site, mu, i, j, True, h=1e-3)
                assert abs(g[site + (mu, i, j)] - (gr + 1j * gi)) < 1e-11


def test_gauge_grad_components_exact(f):
    u = f[0]
    beta = 5.7
    g = force.gauge_grad(u, beta)
    for site, mu in LINKS:
        for i in range(3):
            for j in range(3):
                gr = force.component_fd(lambda v: action.gauge_action(v, beta), u, site, mu, i, j,
                                        False, h=1e-3)
                gi = force.component_fd(lambda v: action.gauge_action(v, beta), u, site, mu, i, j,
                                        True, h=1e-3)
                assert abs(g[site + (mu, i, j)] - (gr + 1j * gi)) < 1e-10


def test_gauge_force_lie_derivative(f):
    u = f[0]
    beta = 5.7
    d = force.lie_derivatives(force.gauge_force(u, beta))
    for site, mu in LINKS:
        for a in range(8):
            fd = force.lie_fd(lambda v: action.gauge_action(v, beta), u, site, mu, a, h=1e-4)
            assert abs(d[site + (mu, a)] - fd) < 1e-7 * max(1.0, abs(fd))


def test_fermion_force_lie_derivative(f):
    u, _, phi, k = f
    ff = force.fermion_force(u, phi, k, tol=1e-14)
    d = force.lie_derivatives(ff)
    for site, mu in LINKS[:3]:
        for a in (0, 3, 7):
            fd = force.lie_fd(lambda v: action.fermion_action(v, phi, k, tol=1e-14)[0], u, site,
                              mu, a, h=1e-4)
            assert abs(d[site + (mu, a)] - fd) < 1e-6 * max(1.0, abs(fd))


def test_force_is_traceless_antihermitian(f):
    u, _, phi, k = f
    for ff in (force.gauge_force(u, 5.7), force.fermion_force(u, phi, k)):
        assert np.allclose(ff, -dag(ff), atol=1e-14)
        assert np.allclose(su3.trace(ff), 0, atol=1e-14)


def test_single_link_gauge_force_closed_form():
    """All links 1 except U: F_G(U) = beta * P_su(3)[U] (six unit staples)."""
    dims = (4, 4, 4, 4)
    u = li.unit_links(dims)
    v = li.random_links((1, 1, 1, 1), 0.9, 3)[0, 0, 0, 0, 2]
    u[1, 2, 3, 0, 2] = v
    beta = 5.7
    ff = force.gauge_force(u, beta)
    assert np.max(np.abs(ff[1, 2, 3, 0, 2] - beta * su3.project_su(v))) < 1e-13


def test_gauge_covariance_of_forces(f):
    u, eta, phi, k = f
    g = li.random_site_unitaries(DIMS, 19)
    ug = np.empty_like(u)
    for mu in range(4):
        ug[..., mu, :, :] = g @ u[..., mu, :, :] @ dag(shift(g, mu, +1))
    gphi = np.einsum("...ij,...sj->...si", g, phi)
    gx = g[..., None, :, :]
    for f0, f1 in ((force.gauge_force(u, 5.7), force.gauge_force(ug, 5.7)),
                   (force.fermion_force(u, phi, k, tol=1e-14),
                    force.fermion_force(ug, gphi, k, tol=1e-14))):
        assert np.max(np.abs(f1 - gx @ f0 @ dag(gx))) < 1e-9 * np.max(np.abs(f0))


def test_kappa_zero_has_no_fermion_force(f):
    u, _, phi, _ = f
    assert np.max(np.abs(force.fermion_force(u, phi, 0.0))) == 0.0


def test_listing_momentum_step_equals_minus_dt_force(f):
    """P + (dt/2) P_su(3)[U G^dag] (gauge listing) equals P - dt F."""
    u = f[0]
    p = li.random_momenta(DIMS, 3)
    g = force.gauge_grad(u, 5.7)
    dt = 0.05
    assert np.allclose(p + 0.5 * dt * su3.project_su(u @ dag(g)),
                       p - dt * force.force_from_grad(u, g), atol=1e-15)


def test_leapfrog_reversibility(f):
    u, _, phi, k = f
    p = li.random_momenta(DIMS, 3)
    u1, p1 = md.leapfrog(u, p, phi, 5.7, k, 0.05, 3, tol=1e-14)
    u2, p2 = md.leapfrog(u1, -p1, phi, 5.7, k, 0.05, 3, tol=1e-14)
    assert np.max(np.abs(u2 - u)) < 1e-12
    assert np.max(np.abs(p2 + p)) < 1e-12
    assert su3.unitarity_defect(u1) < 1e-14


def test_delta_h_scales_as_dt_squared(f):
    """Single-trajectory |dH(dt)| / |dH(dt/2)| -> 4 for a second-order integrator (Sec. III B)."""
    u, _, phi, k = f
    p = li.random_momenta(DIMS, 3)
    dh = [md.trajectory_dh(u, p, phi, 5.7, k, 0.5 / n, n, tol=1e-13)[2] for n in (8, 16, 32)]
    r1, r2 = dh[0] / dh[1], dh[1] / dh[2]
    assert 3.5 < r1 < 4.5 and 3.8 < r2 < 4.2


def test_pure_gauge_delta_h_scaling():
    u = li.random_links(DIMS, 0.5, 1)
    p = li.random_momenta(DIMS, 3)
    dh = [md.trajectory_dh(u, p, None, 5.7, 0.0, 0.2 / n, n, with_fermion=False)[2]
          for n in (20, 40)]
    assert 3.8 < dh[0] / dh[1] < 4.2


# ---- Sexton-Weingarten multiple time-scale integrator -----------------------

def test_sw_with_one_inner_step_is_the_leapfrog(f):
    """With n_inner = 1 every kick acts at the same links as the leapfrog's,
    and kicks at equal links commute, so the two integrators coincide."""
    u, _, phi, k = f
    p = li.random_momenta(DIMS, 3)
    a = md.leapfrog(u, p, phi, 5.7, k, 0.05, 3, tol=1e-14)
    b = md.sexton_weingarten(u, p, phi, 5.7, k, 0.05, 3, 1, tol=1e-14)
    assert np.abs(a[0] - b[0]).max() < 1e-12
    assert np.abs(a[1] - b[1]).max() < 1e-11


def test_sw_without_fermions_is_a_fine_leapfrog(f):
    """kappa = 0: the outer kicks vanish and SW(dt, n, m) is the plain
    leapfrog with step dt/m and n*m steps, exactly."""
    u, _, phi, _ = f
    p = li.random_momenta(DIMS, 3)
    a = md.sexton_weingarten(u, p, phi, 5.7, 0.0, 0.1, 2, 4, tol=1e-14)
    b = md.leapfrog(u, p, phi, 5.7, 0.0, 0.025, 8, tol=1e-14, with_fermion=False)
    assert np.abs(a[0] - b[0]).max() < 1e-12
    assert np.abs(a[1] - b[1]).max() < 1e-11


def test_sw_reversibility(f):
    u, _, phi, k = f
    p = li.random_momenta(DIMS, 3)
    u1, p1 = md.sexton_weingarten(u, p, phi, 5.7, k, 0.1, 2, 5, tol=1e-14)
    u2, p2 = md.sexton_weingarten(u1, -p1, phi, 5.7, k, 0.1, 2, 5, tol=1e-14)
    assert np.abs(u2 - u).max() < 1e-11
    assert np.abs(-p2 - p).max() < 1e-10


def test_sw_delta_h_scales_as_dt_squared(f):
    u, _, phi, k = f
    p = li.random_momenta(DIMS, 3)
    dh = [md.sw_trajectory_dh(u, p, phi, 5.7, k, 0.5 / n, n, 10, tol=1e-13)[2] for n in (8, 16)]
    assert 3.5 < dh[0] / dh[1] < 4.5


def test_sw_smeared_reduces_to_leapfrog_of_smeared_action(f):
    """n_inner = 1 with one stout level: the same kicks as a leapfrog of the
    total smeared force (stout.total_force), applied by hand here."""
    from oracle import stout
    u, _, phi, k = f
    p = li.random_momenta(DIMS, 3)
    dt, n, rho = 0.05, 2, 0.3
    a = md.sexton_weingarten(u, p, phi, 5.7, k, dt, n, 1, tol=1e-14, rho=rho, nlevels=1)
    ub, pb = u, p - 0.5 * dt * stout.total_force(u, phi, 5.7, k, rho, 1, tol=1e-14)
    for j in range(n):
        ub = md.link_update(ub, pb, dt)
        pb = pb - (dt if j < n - 1 else 0.5 * dt) * stout.total_force(ub, phi, 5.7, k, rho, 1, tol=1e-14)
    assert np.abs(a[0] - ub).max() < 1e-12
    assert np.abs(a[1] - pb).max() < 1e-10
