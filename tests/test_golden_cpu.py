"""Pins of the stored 16^4 and 24^3x48 oracle values (CPU): each file is
consistent with what the paper and the mathematics fix, independently of how
it was made."""
import json
import os

import numpy as np
import pytest

import lgt_inputs as li
from oracle import action, su3

HERE = os.path.join(os.path.dirname(__file__), "golden")
FILES = [f for f in ("c2_16x16x16x16.json", "c3_24x24x24x48.json") if os.path.exists(os.path.join(HERE, f))]


@pytest.fixture(params=FILES)
def g(request):
    with open(os.path.join(HERE, request.param)) as f:
        return json.load(f)


def test_stored_fermion_action_is_eta_norm(g):
    """S_f(phi = D^dag eta) = eta^dag eta (eq. S3.1 at the heat-bath field)."""
    eta = li.gaussian_spinor(tuple(g["dims"]), g["seeds"]["eta"])
    ee = float(np.vdot(eta.ravel(), eta.ravel()).real)
    assert abs(g["eta_norm2"] - ee) / ee < 1e-14  # BLAS summation order only
    assert abs(g["S_F"] - ee) / ee < 1e-12
    # the CG stops on its recursive residual; near 1e-15 the true residual
    # sits at the FP64 rounding floor of D^dag D X, a little above it
    assert g["oracle_true_residual"] <= max(g["oracle_tol"], 3e-15)


def test_stored_forces_are_in_the_algebra(g):
    for key in ("F_fermion", "F_gauge"):
        f = np.array([[complex(*v) for v in m] for m in g[key]]).reshape(-1, 3, 3)
        assert np.allclose(f, -su3.dag(f), atol=1e-14)
        assert np.allclose(su3.trace(f), 0, atol=1e-14)


def test_stored_gauge_action_recomputes(g):
    u = li.random_links(tuple(g["dims"]), g["eps"], g["seeds"]["links"])
    assert abs(action.gauge_action(u, g["beta"]) - g["S_G"]) / g["S_G"] < 1e-13
    # with T = lambda/2, 1 - Re tr P / 3 = (8/3) eps^2 to leading order (the
    # plaquette's exponent has generator variance 4 eps^2); the quartic
    # terms raise the plaquette a little (0.785 at eps = 0.3)
    e2 = g["eps"] ** 2
    assert 1 - 3 * e2 < g["mean_plaquette"] < 1 - 2 * e2


@pytest.mark.parametrize("name", ["c5_8x8x8x16_smeared_trajectory.json", "c5_8x8x8x8_periodic_trajectory.json"])
def test_stored_smeared_trajectory_is_consistent(name):
    """The stored smeared trajectories (8^3x16 antiperiodic, 8^4 periodic): the
    end links are SU(3), the end momenta traceless anti-Hermitian, and the
    trajectory's H at the start agrees with the heat-bath identity
    S_f(D(V)^dag eta) = |eta|^2 (the rest of H0 is K + S_G of the stored
    seeds)."""
    with open(os.path.join(HERE, name)) as f:
        g = json.load(f)
    dims = tuple(g["dims"])
    u = np.array([[complex(*v) for v in m] for m in g["U"]]).reshape(-1, 3, 3)
    p = np.array([[complex(*v) for v in m] for m in g["P"]]).reshape(-1, 3, 3)
    assert su3.unitarity_defect(u) < 1e-13
    assert np.allclose(np.linalg.det(u), 1.0, atol=1e-13)
    assert np.allclose(p, -su3.dag(p), atol=1e-14)
    assert np.allclose(su3.trace(p), 0, atol=1e-14)
    u0 = li.random_links(dims, g["eps"], g["seeds"]["links"])
    p0 = li.random_momenta(dims, g["seeds"]["mom"])
    eta = li.gaussian_spinor(dims, g["seeds"]["eta"])
    h0 = action.kinetic(p0) + action.gauge_action(u0, g["beta"]) + float(np.vdot(eta.ravel(), eta.ravel()).real)
    assert abs(g["H0"] - h0) / abs(h0) < 1e-12
