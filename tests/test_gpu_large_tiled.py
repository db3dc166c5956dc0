"""GPU parity on the 32^3x64 lattice of the smeared-trajectory workload.

There both link fields exceed the size above which the hop streams its links
past the caches (FP64 1.2 GB, FP32 two-row 0.4 GB), and the hop takes its
64-site blocks t-fastest.  The oracle cannot handle the lattice itself, so the
links and the source are seeded 8^4 fields repeated with period 8, with a
periodic fermion boundary: the operator then commutes with translations by 8,
and D psi, X = (D^dag D)^-1 phi and Y = D X are the oracle's 8^4 results
repeated.  Gates as for the other sizes: 1e-13 for D, 1e-12 for the solves
with both sides far below it (GPU true residual 1e-14, oracle 1e-15).
"""
import sys

import numpy as np
import pytest

import lgt_inputs as li
from oracle import dirac, solver

from gpu_common import rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

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
