"""The 32^3x64 smeared-trajectory workload on its 8^3x16 reduction against the
oracle: one leapfrog trajectory (2 steps, dt 0.05) of the action with two
stout levels (rho 0.1) before D, beta 6.0, kappa 0.135, from the seeded
inputs; U, P and Delta H against the stored oracle values
(tests/golden/c5_8x8x8x16_smeared_trajectory.json, oracle solves to 1e-14)."""
import json
import os
import sys

import numpy as np
import pytest

import lgt_inputs as li

from gpu_common import rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c5_8x8x8x16_smeared_trajectory.json")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("precision,tol,gate_u,gate_p,gate_dh", [
    ("fp64", 1e-14, 1e-12, 1e-12, 1e-9),
    ("mixed_fp32", 1e-11, 1e-10, 1e-9, 1e-7),
])
def test_smeared_trajectory_8x8x8x16_vs_oracle(precision, tol, gate_u, gate_p, gate_dh, margin):
    import paper_2602_20516_amd as lgt
    with open(GOLDEN) as f:
        g = json.load(f)
    dims = tuple(g["dims"])
    u = li.random_links(dims, g["eps"], g["seeds"]["links"])
    eta = li.gaussian_spinor(dims, g["seeds"]["eta"])
    p = li.random_momenta(dims, g["seeds"]["mom"])
    lat = lgt.Lattice(dims)
    U, P = to_dev(u), to_dev(p)
    phi = lat.dslash(lat.stout_smear(U, g["rho"], g["nstout"]), to_dev(eta), g["kappa"], dagger=True)
    dh, st = lat.md_step_smeared(U, P, phi, g["beta"], g["kappa"], g["rho"], g["nstout"], g["dt"], g["nsteps"],
                                 lgt.Params(precision=precision, tol=tol))
    say("c5 reduced", precision, dh, g["dH"], st)
    links = [tuple(l) for l in g["links"]]
    u_ref = np.array([[complex(*v) for v in m] for m in g["U"]]).reshape(-1, 3, 3)
    p_ref = np.array([[complex(*v) for v in m] for m in g["P"]]).reshape(-1, 3, 3)
    Uh, Ph = to_host(U), to_host(P)
    margin(f"8^3x16 smeared trajectory U vs oracle ({precision}, tol {tol:g})",
           rel_err(np.stack([Uh[l] for l in links]), u_ref), gate_u)
    margin(f"8^3x16 smeared trajectory P vs oracle ({precision}, tol {tol:g})",
           rel_err(np.stack([Ph[l] for l in links]), p_ref), gate_p)
    margin(f"8^3x16 smeared trajectory |P| vs oracle ({precision})",
           abs(np.linalg.norm(Ph.ravel()) - g["P_fro"]) / g["P_fro"], gate_p)
    margin(f"8^3x16 smeared trajectory dH vs oracle ({precision}, tol {tol:g})",
           abs(dh - g["dH"]) / max(1.0, abs(g["dH"])), gate_dh)
