"""Write the stored expected values of a short smeared trajectory on the
8^3x16 reduction of the 32^3x64 workload, from the oracle only.

The 32^3x64 lattice is too large for the oracle, so its physics (beta 6.0,
kappa 0.135, two stout levels rho 0.1 before D, leapfrog, eps 0.2 links,
seeds 501/502/503) is checked on 8^3x16: one leapfrog trajectory of 2 steps
of dt 0.05 with the pseudofermion phi = D(V)^dag eta, V = stout^2(U).  The
oracle's solves run to 1e-14.  Stored: Delta H, H at the start, and U and P
at the end on a seeded sample of links, plus the full-field norms.

With --periodic-8x8x8x8 the same trajectory is taken on an 8^4 lattice with a
periodic fermion boundary (links, eta and momenta seeded as above on 8^4): the
32^3x64 lattice with these fields repeated has the same trajectory repeated,
and Delta H times 512, which the GPU test checks on the full-size lattice.

Usage:  python tests/golden/make_golden_c5.py [--periodic-8x8x8x8]
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
sys.path.insert(0, HERE)

import lgt_inputs as li  # noqa: E402
from make_golden import sample_links  # noqa: E402
from oracle import dirac, md, stout  # noqa: E402

DIMS = (8, 8, 8, 16)
DT, NSTEPS, TOL = 0.05, 2, 1e-14


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--periodic-8x8x8x8", dest="periodic", action="store_true")
    args = ap.parse_args()
    dims, bc = ((8, 8, 8, 8), +1) if args.periodic else (DIMS, -1)
    c = li.config(5)
    t0 = time.time()
    u = li.random_links(dims, c["eps"], c["seeds"]["links"])
    eta = li.gaussian_spinor(dims, c["seeds"]["eta"])
    p = li.random_momenta(dims, c["seeds"]["mom"])
    v = stout.stout(u, c["rho"], c["nstout"])
    phi = dirac.dslash_dag(v, eta, c["kappa"], bc=bc)
    h0 = md.hamiltonian_smeared(u, p, phi, c["beta"], c["kappa"], bc=bc, tol=TOL, rho=c["rho"],
                                nlevels=c["nstout"])
    u1, p1, dh = md.sw_trajectory_dh(u, p, phi, c["beta"], c["kappa"], DT, NSTEPS, 1, bc=bc, tol=TOL, rho=c["rho"],
                                     nlevels=c["nstout"])
    links = sample_links(dims, n=64, seed=11)
    name = "x".join(str(d) for d in dims)
    what = ("8^3x16 reduction of the 32^3x64 workload" if not args.periodic else
            "8^4 periodic-boundary cell of the 32^3x64 workload (its fields repeated give the full lattice)")
    rec = {
        "what": what + ": one smeared leapfrog trajectory (2 steps, dt 0.05, stout rho 0.1 x 2, beta 6.0, "
                "kappa 0.135, eps 0.2 links seed 501, eta 502, momenta 503), oracle values",
        "writer": "tests/golden/make_golden_c5.py (oracle only)",
        "dims": list(dims), "eps": c["eps"], "beta": c["beta"], "kappa": c["kappa"], "rho": c["rho"],
        "nstout": c["nstout"], "dt": DT, "nsteps": NSTEPS, "fermion_bc": bc, "seeds": c["seeds"],
        "oracle_tol": TOL, "H0": float(h0), "dH": float(dh),
        "U_fro": float(np.linalg.norm(u1.ravel())), "P_fro": float(np.linalg.norm(p1.ravel())),
        "links": [list(l) for l in links],
        "U": [[[float(z.real), float(z.imag)] for z in u1[l].ravel()] for l in links],
        "P": [[[float(z.real), float(z.imag)] for z in p1[l].ravel()] for l in links],
    }
    out = os.path.join(HERE, f"c5_{name}_{'periodic' if args.periodic else 'smeared'}_trajectory.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=0)
    print(f"dH {dh:.6e}; wrote {out} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
