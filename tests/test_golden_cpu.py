"""Pins of the stored 16^4 oracle values (CPU): the file is consistent with
what the paper and the mathematics fix, independently of how it was made."""
import json
import os

import numpy as np

import lgt_inputs as li
from oracle import action, su3

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c2_16x16x16x16.json")


def load():
    with open(GOLDEN) as f:
        return json.load(f)


def test_stored_fermion_action_is_eta_norm():
    """S_f(phi = D^dag eta) = eta^dag eta (eq. S3.1 at the heat-bath field)."""
    g = load()
    eta = li.gaussian_spinor(tuple(g["dims"]), g["seeds"]["eta"])
    ee = float(np.vdot(eta.ravel(), eta.ravel()).real)
    assert abs(g["eta_norm2"] - ee) / ee < 1e-15
    assert abs(g["S_F"] - ee) / ee < 1e-12
    assert g["oracle_true_residual"] <= g["oracle_tol"]


def test_stored_forces_are_in_the_algebra():
    g = load()
    for key in ("F_fermion", "F_gauge"):
        f = np.array([[complex(*v) for v in m] for m in g[key]]).reshape(-1, 3, 3)
        assert np.allclose(f, -su3.dag(f), atol=1e-14)
        assert np.allclose(su3.trace(f), 0, atol=1e-14)


def test_stored_gauge_action_recomputes():
    g = load()
    u = li.random_links(tuple(g["dims"]), g["eps"], g["seeds"]["links"])
    assert abs(action.gauge_action(u, g["beta"]) - g["S_G"]) / g["S_G"] < 1e-13
    # with T = lambda/2 and eps = 0.3 the mean plaquette sits near 1 - 4 * 0.09 * 4/3 / 3
    assert 0.7 < g["mean_plaquette"] < 0.9
