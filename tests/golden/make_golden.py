"""Write the stored expected values of a full-size workload, from the oracle only.

The 16^4 lattice (eps = 0.3 links, beta = 6.0, kappa = 0.125) and the
24^3x48 lattice (eps = 0.2, beta = 6.0, kappa = 0.13), each with the
pseudofermion phi = D^dag eta, are too slow for the NumPy oracle inside a
test (an unpreconditioned CG takes minutes to hours), so this script solves
each once, tightly, and stores: the actions, the fermion and gauge forces on
a seeded sample of links (random site classes plus boundary-crossing t-links
of one column), and norms of the full force fields.  Only ``oracle`` and the
input generator are used.

Usage:  python tests/golden/make_golden.py  [--config 2|3] [--tol 1e-15]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import lgt_inputs as li  # noqa: E402
from oracle import action, dirac, force, solver  # noqa: E402


def sample_links(dims, n=96, seed=7):
    lx, ly, lz, lt = dims
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = set()
    while len(pts) < n:
        pts.add((int(rng.integers(lt)), int(rng.integers(lz)), int(rng.integers(ly)), int(rng.integers(lx)),
                 int(rng.integers(4))))
    # t-links crossing the antiperiodic boundary, and links into it
    for x in range(0, lx, 5):
        pts.add((lt - 1, 1, 2, x, 3))
        pts.add((0, 1, 2, x, 3))
    return sorted(pts)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, default=2, choices=(2, 3))
    ap.add_argument("--tol", type=float, default=1e-15)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    c = li.config(args.config)
    dims, eps, beta, k = c["dims"], c["eps"], c["beta"], c["kappa"]
    t0 = time.time()
    u = li.random_links(dims, eps, c["seeds"]["links"])
    eta = li.gaussian_spinor(dims, c["seeds"]["eta"])
    phi = dirac.dslash_dag(u, eta, k)
    chi, y, iters, res = solver.solve_ddag_d(u, phi, k, tol=args.tol)
    print(f"solve: {iters} iterations, true residual {res:.3e}, {time.time() - t0:.0f} s", flush=True)
    ff = force.fermion_force_from_solution(u, chi, y, k)
    fg = force.gauge_force(u, beta)
    sf = float(np.real(np.vdot(phi.ravel(), chi.ravel())))
    sg = action.gauge_action(u, beta)
    links = sample_links(dims)
    name = "x".join(str(d) for d in dims)
    out = args.out or os.path.join(HERE, f"c{args.config}_{name}.json")
    rec = {
        "what": f"{name} workload (eps {eps} links seed {c['seeds']['links']}, eta seed {c['seeds']['eta']}, "
                f"beta {beta}, kappa {k}, antiperiodic t), oracle values",
        "writer": "tests/golden/make_golden.py (oracle only)",
        "dims": list(dims), "eps": eps, "beta": beta, "kappa": k, "fermion_bc": -1,
        "seeds": c["seeds"], "oracle_tol": args.tol, "oracle_iters": iters, "oracle_true_residual": res,
        "S_F": sf, "eta_norm2": float(np.vdot(eta.ravel(), eta.ravel()).real), "S_G": sg,
        "mean_plaquette": action.mean_plaquette(u),
        "F_fermion_fro": float(np.linalg.norm(ff.ravel())), "F_gauge_fro": float(np.linalg.norm(fg.ravel())),
        "links": [list(l) for l in links],
        "F_fermion": [[[float(v.real), float(v.imag)] for v in ff[l].ravel()] for l in links],
        "F_gauge": [[[float(v.real), float(v.imag)] for v in fg[l].ravel()] for l in links],
        "X_samples": [[[float(v.real), float(v.imag)] for v in chi[l[:4]].ravel()] for l in links[:16]],
    }
    with open(out, "w") as f:
        json.dump(rec, f, indent=0)
    print(f"wrote {out} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
