"""Pins of the oracle's stout smearing and of the autograd gradient through it (CPU)."""
import numpy as np
import pytest

import lgt_inputs as li
from oracle import action, dirac, force, stout, su3
from oracle.lattice import shift
from oracle.su3 import dag

DIMS = (2, 2, 2, 4)


@pytest.fixture(scope="module")
def f():
    u = li.random_links(DIMS, 0.5, 1)
    eta = li.gaussian_spinor(DIMS, 2)
    return u, eta


def test_unit_field_is_a_fixed_point():
    u = li.unit_links((4, 4, 4, 4))
    assert np.max(np.abs(stout.stout(u, 0.1, 2) - u)) < 1e-15


def test_result_is_su3_and_smoother(f):
    u = li.random_links((4, 4, 4, 4), 0.5, 11)
    s1 = stout.stout(u, 0.1, 1)
    s2 = stout.stout(u, 0.1, 2)
    assert su3.unitarity_defect(s2) < 1e-13
    assert np.allclose(np.linalg.det(s2), 1.0, atol=1e-13)
    p0, p1, p2 = (action.mean_plaquette(v) for v in (u, s1, s2))
    assert p0 < p1 < p2


def test_gauge_covariance(f):
    u, _ = f
    g = li.random_site_unitaries(DIMS, 9)

    def gt(v):
        out = np.empty_like(v)
        for mu in range(4):
            out[..., mu, :, :] = g @ v[..., mu, :, :] @ dag(shift(g, mu, +1))
        return out

    assert np.max(np.abs(stout.stout(gt(u), 0.1, 2) - gt(stout.stout(u, 0.1, 2)))) < 1e-13


def test_equals_exponential_of_projected_plaquette_staple(f):
    """exp(iQ) U = exp(-rho P[U A]) U with A the plaquette staple sum of the gauge force."""
    u, _ = f
    rho, beta = 0.13, 6.0
    a = -(3.0 / beta) * dag(force.gauge_grad(u, beta))   # G_G = -(beta/3) A^dag
    alt = su3.expm_antihermitian(-rho * su3.project_su(u @ a)) @ u
    assert np.max(np.abs(stout.stout_level(u, rho) - alt)) < 1e-14


def test_numpy_and_torch_transcriptions_agree(f):
    import torch
    u, _ = f
    t = stout.stout_level_torch(torch.tensor(u), 0.1).numpy()
    assert np.max(np.abs(t - stout.stout_level(u, 0.1))) < 1e-14


def test_vjp_against_component_differences(f):
    u, _ = f
    g_top = li.random_links(DIMS, 1.0, 5)  # any cotangent
    rho = 0.1
    g0 = stout.stout_vjp(u, g_top, rho, 2)

    def loss(v):
        return float(np.sum(np.real(np.conj(g_top) * stout.stout(v, rho, 2))))

    for site, mu in [((0, 1, 0, 1), 2), ((3, 0, 1, 0), 3), ((1, 1, 1, 1), 0)]:
        for i, j in [(0, 0), (1, 2), (2, 1)]:
            fr = force.component_fd(loss, u, site, mu, i, j, False, h=1e-5)
            fi = force.component_fd(loss, u, site, mu, i, j, True, h=1e-5)
            assert abs(g0[site + (mu, i, j)] - (fr + 1j * fi)) < 1e-8


def test_smeared_force_against_lie_differences(f):
    u, eta = f
    k, beta, rho = 0.12, 5.7, 0.1
    phi = dirac.dslash_dag(u, eta, k)
    ff = stout.total_force(u, phi, beta, k, rho, 2, tol=1e-14)
    d = force.lie_derivatives(ff)
    for site, mu, a in [((0, 1, 0, 1), 2, 3), ((3, 0, 1, 0), 3, 0), ((1, 1, 1, 1), 0, 7)]:
        fd = force.lie_fd(lambda v: stout.total_action(v, phi, beta, k, rho, 2, tol=1e-14), u, site, mu, a,
                          h=1e-4)
        assert abs(d[site + (mu, a)] - fd) < 1e-6 * max(1.0, abs(fd))
