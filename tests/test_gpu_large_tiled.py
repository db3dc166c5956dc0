"""GPU parity on the 32^3x64 lattice of the smeared-trajectory workload.

There both link fields exceed the size above which the hop streams its links
past the caches (FP64 1.2 GB, FP32 two-row 0.4 GB), and the hop takes its
64-site blocks t-fastest.  The oracle cannot handle the lattice itself, so the
links and the source are seeded 8^4 fields repeated with period 8, with a
periodic fermion boundary: the operator then commutes with translations by 8,
and D psi, X = (D^dag D)^-1 phi and Y = D X are the oracle's 8^4 results
repeated.  Gates as for the other sizes: 1e-13 for D, 1e-12 for the solves
with both sides far below it (GPU true residual 1e-14, oracle 1e-15).  The
smeared trajectory of the workload is checked the same way against stored
oracle values of its 8^4 periodic-boundary cell
(tests/golden/c5_8x8x8x8_periodic_trajectory.json), with the gates of its
8^3x16 reduction.
"""
import json
import os
import sys

import numpy as np
import pytest

import lgt_inputs as li
from oracle import dirac, solver

from gpu_common import rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

GOLDEN_C5P = os.path.join(os.path.dirname(__file__), "golden", "c5_8x8x8x8_periodic_trajectory.json")
DIMS = (32, 32, 32, 64)
SMALL = (8, 8, 8, 8)
REPS_S = (64 // 8, 32 // 8, 32 // 8, 32 // 8, 1, 1)
REPS_G = REPS_S + (1,)
KAPPA = 0.12


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def tiled():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2602_20516_amd as lgt
    u8 = li.random_links(SMALL, 0.2, 81)
    psi8 = li.gaussian_spinor(SMALL, 82)
    phi8 = dirac.dslash_dag(u8, psi8, KAPPA, bc=+1)
    x8, y8, it, res = solver.solve_ddag_d(u8, phi8, KAPPA, bc=+1, tol=1e-15)
    say("oracle 8^4 periodic solve", it, res)
    lat = lgt.Lattice(DIMS, fermion_bc=+1)
    U = to_dev(np.tile(u8, REPS_G))
    return dict(lgt=lgt, torch=torch, lat=lat, U=U, u8=u8, psi8=psi8, phi8=phi8, x8=x8, y8=y8)


def test_dslash_32x32x32x64(tiled, margin):
    t = tiled
    got = to_host(t["lat"].dslash(t["U"], to_dev(np.tile(t["psi8"], REPS_S)), KAPPA, dagger=False))
    ref = np.tile(dirac.dslash(t["u8"], t["psi8"], KAPPA, bc=+1), REPS_S)
    margin("32^3x64 D psi vs oracle", rel_err(got, ref), 1e-13)


@pytest.mark.parametrize("precision", ["fp64", "mixed_fp32"])
def test_solve_32x32x32x64(tiled, precision, margin):
    t = tiled
    X, Y, st = t["lat"].cg_solve(t["U"], to_dev(np.tile(t["phi8"], REPS_S)), KAPPA,
                                 t["lgt"].Params(precision=precision, tol=1e-14))
    say("32^3x64", precision, st)
    assert st["true_rel_residual"] <= 1e-14
    margin(f"32^3x64 X vs oracle ({precision}, tol 1e-14)", rel_err(to_host(X), np.tile(t["x8"], REPS_S)), 1e-12)
    margin(f"32^3x64 Y vs oracle ({precision}, tol 1e-14)", rel_err(to_host(Y), np.tile(t["y8"], REPS_S)), 1e-12)


# copies of a sampled 8^4 link on the 32^3x64 lattice: offsets (t, z, y, x) in units of 8
COPIES = [(0, 0, 0, 0), (7, 3, 3, 3), (3, 1, 2, 0), (5, 2, 0, 1)]


@pytest.mark.parametrize("precision,tol,gate_u,gate_p,gate_dh", [
    ("fp64", 1e-14, 1e-12, 1e-12, 1e-9),
    ("mixed_fp32", 1e-11, 1e-10, 1e-9, 1e-7),
])
def test_smeared_trajectory_32x32x32x64(tiled, precision, tol, gate_u, gate_p, gate_dh, margin):
    """The smeared-trajectory workload's physics (two stout levels of rho 0.1,
    beta 6.0, kappa 0.135, leapfrog, 2 steps of dt 0.05) on 32^3x64 with the
    fields of the stored 8^4 periodic-boundary trajectory repeated: U and P at
    the stored links in four of their copies, |P|, and Delta H = 512 times the
    oracle's."""
    t = tiled
    with open(GOLDEN_C5P) as f:
        g = json.load(f)
    small = tuple(g["dims"])
    assert g["fermion_bc"] == 1 and small == SMALL
    u8 = li.random_links(small, g["eps"], g["seeds"]["links"])
    eta8 = li.gaussian_spinor(small, g["seeds"]["eta"])
    p8 = li.random_momenta(small, g["seeds"]["mom"])
    lat = t["lat"]
    U, P = to_dev(np.tile(u8, REPS_G)), to_dev(np.tile(p8, REPS_G))
    phi = lat.dslash(lat.stout_smear(U, g["rho"], g["nstout"]), to_dev(np.tile(eta8, REPS_S)), g["kappa"],
                     dagger=True)
    dh, st = lat.md_step_smeared(U, P, phi, g["beta"], g["kappa"], g["rho"], g["nstout"], g["dt"], g["nsteps"],
                                 t["lgt"].Params(precision=precision, tol=tol))
    say("32^3x64 smeared trajectory", precision, dh, 512 * g["dH"], st)
    Uh, Ph = to_host(U), to_host(P)
    del U, P, phi
    links = [tuple(l) for l in g["links"]]
    at = [(l[0] + 8 * a, l[1] + 8 * b, l[2] + 8 * c, l[3] + 8 * d, l[4]) for (a, b, c, d) in COPIES for l in links]
    u_ref = np.array([[complex(*v) for v in m] for m in g["U"]]).reshape(-1, 3, 3)
    p_ref = np.array([[complex(*v) for v in m] for m in g["P"]]).reshape(-1, 3, 3)
    nc = len(COPIES)
    margin(f"32^3x64 smeared trajectory U vs oracle ({precision}, tol {tol:g})",
           rel_err(np.stack([Uh[l] for l in at]), np.concatenate([u_ref] * nc)), gate_u)
    margin(f"32^3x64 smeared trajectory P vs oracle ({precision}, tol {tol:g})",
           rel_err(np.stack([Ph[l] for l in at]), np.concatenate([p_ref] * nc)), gate_p)
    margin(f"32^3x64 smeared trajectory |P| vs oracle ({precision})",
           abs(np.linalg.norm(Ph.ravel()) - np.sqrt(512.0) * g["P_fro"]) / (np.sqrt(512.0) * g["P_fro"]), gate_p)
    margin(f"32^3x64 smeared trajectory dH vs 512 x oracle ({precision}, tol {tol:g})",
           abs(dh - 512 * g["dH"]) / max(1.0, abs(512 * g["dH"])), gate_dh)
