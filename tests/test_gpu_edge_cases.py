"""Degenerate inputs and error paths of the solver, force and trajectory calls,
for every solver precision: a zero source, kappa = 0 (D = 1), dt = 0,
non-finite links, iteration caps, and run-to-run determinism of the mixed
precision paths (whose reliable updates are decided on the device)."""
import numpy as np
import pytest

import lgt_inputs as li

from gpu_common import rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

DIMS = (4, 4, 4, 6)
PRECISIONS = ["fp64", "mixed_fp32", "mixed_bf16"]


@pytest.fixture(scope="module")
def lgt():
    import torch
    assert torch.cuda.is_available()
    import paper_2602_20516_amd as m
    return m


@pytest.fixture(scope="module")
def f(lgt):
    u, eta = li.random_links(DIMS, 0.5, 401), li.gaussian_spinor(DIMS, 402)
    return u, eta, lgt.Lattice(DIMS)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_zero_source(lgt, f, precision):
    u, eta, lat = f
    U, Z = to_dev(u), to_dev(np.zeros_like(eta))
    X, Y, st = lat.cg_solve(U, Z, 0.12, lgt.Params(precision=precision, tol=1e-10))
    assert np.abs(to_host(X)).max() == 0.0 and np.abs(to_host(Y)).max() == 0.0
    assert st["iters"] == 0
    F, st = lat.fermion_force(U, Z, 0.12, lgt.Params(precision=precision, tol=1e-10))
    assert np.abs(to_host(F)).max() == 0.0


@pytest.mark.parametrize("precision", PRECISIONS)
def test_kappa_zero(lgt, f, precision, margin):
    """D = 1: X = Y = phi, no fermion force."""
    u, eta, lat = f
    U, E = to_dev(u), to_dev(eta)
    X, Y, st = lat.cg_solve(U, E, 0.0, lgt.Params(precision=precision, tol=1e-12))
    margin("rel_err(to_host(X), eta) < 1e-12 and rel_err(to_host(Y), eta)", rel_err(to_host(X), eta) < 1e-12 and rel_err(to_host(Y), eta), 1e-12)
    F, _ = lat.fermion_force(U, E, 0.0, lgt.Params(precision=precision, tol=1e-12))
    assert np.abs(to_host(F)).max() < 1e-12


def test_dt_zero_trajectory(lgt, f, margin):
    """dt = 0 moves nothing: U and P unchanged to rounding, Delta H = 0."""
    u, eta, lat = f
    p = li.random_momenta(DIMS, 403)
    U, P = to_dev(u), to_dev(p)
    phi = lat.dslash(U, to_dev(eta), 0.12, dagger=True)
    dh, _ = lat.md_step(U, P, phi, 5.7, 0.12, 0.0, 3, lgt.Params(tol=1e-12))
    assert np.array_equal(to_host(P), p)
    margin("rel_err(to_host(U), u)", rel_err(to_host(U), u), 1e-15)
    assert abs(dh) < 1e-9


@pytest.mark.parametrize("precision", ["mixed_fp32", "mixed_bf16"])
def test_mixed_determinism(lgt, f, precision):
    """Fixed-order reductions and device-side decisions: the same bits twice."""
    u, eta, lat = f
    U, E = to_dev(u), to_dev(eta)
    prm = lgt.Params(precision=precision, tol=1e-10)
    a, sa = lat.fermion_force(U, E, 0.125, prm)
    b, sb = lat.fermion_force(U, E, 0.125, prm)
    assert np.array_equal(to_host(a), to_host(b))
    assert sa["iters"] == sb["iters"] and sa["reliable_updates"] == sb["reliable_updates"]


@pytest.mark.parametrize("precision", ["mixed_fp32", "mixed_bf16"])
def test_mixed_iteration_cap_and_recovery(lgt, f, precision):
    u, eta, lat = f
    U, E = to_dev(u), to_dev(eta)
    with pytest.raises(lgt.LGTNotConverged) as ei:
        lat.cg_solve(U, E, 0.125, lgt.Params(precision=precision, tol=1e-10, max_iter=3))
    assert ei.value.stats["iters"] >= 3
    X, _, st = lat.cg_solve(U, E, 0.125, lgt.Params(precision=precision, tol=1e-10))
    assert st["true_rel_residual"] <= 1e-10


def test_non_finite_links_and_bad_arguments(lgt, f):
    u, eta, lat = f
    bad = u.copy()
    bad[0, 1, 2, 3, 1, 0, 2] = np.inf
    with pytest.raises(lgt.LGTNonFinite):
        lat.fermion_force(to_dev(bad), to_dev(eta), 0.12, lgt.Params(precision="mixed_fp32"))
    U, E = to_dev(u), to_dev(eta)
    p = to_dev(li.random_momenta(DIMS, 404))
    with pytest.raises(lgt.LGTError):
        lat.md_step(U, p, E, 5.7, 0.12, 0.05, 0)  # nsteps >= 1
    with pytest.raises(lgt.LGTError):
        lat.cg_solve(U, E, 0.12, lgt.Params(tol=-1.0))
    with pytest.raises(lgt.LGTError):
        lat.fermion_force(U, E, float("nan"), lgt.Params())
    X, _, st = lat.cg_solve(U, E, 0.12, lgt.Params(tol=1e-10))  # still usable
    assert st["true_rel_residual"] <= 1e-10


@pytest.mark.parametrize("precision", ["mixed_fp32", "mixed_bf16"])
def test_mixed_solve_with_links_outside_su3(lgt, f, precision, margin):
    """Links scaled by 0.9 are not SU(3): the inner solver must read them in
    full (no third-row reconstruction) and still reach the FP64 answer."""
    u, eta, lat = f
    U, E = to_dev(0.9 * u), to_dev(eta)
    X, _, st = lat.cg_solve(U, E, 0.12, lgt.Params(precision=precision, tol=1e-11))
    X64, _, st64 = lat.cg_solve(U, E, 0.12, lgt.Params(precision="fp64", tol=1e-11))
    assert st["true_rel_residual"] <= 1e-11
    margin("rel_err(to_host(X), to_host(X64))", rel_err(to_host(X), to_host(X64)), 1e-9)
    # with the exact operator the inner recursion converges as the FP64 CG
    # does (a wrongly rebuilt third row would cost many more iterations)
    assert st["iters"] <= st64["iters"] + 5


def test_defect_correction_asks_only_for_the_missing_factor(lgt):
    """24^3x48 (the workload of the 24^3x48 force benchmark) with BF16-stored
    inner vectors and reliable_delta 1e-3: the first pass of the two Schur
    solves ends just short of the requested true residual, so an FP64
    defect-correction pass follows.  That pass only has to shrink the
    residual by tol / true_res; solved to the full relative tolerance it
    doubled the iteration count (892 against about 400)."""
    c = li.config(3)
    dims = c["dims"]
    lat = lgt.Lattice(dims)
    U = to_dev(li.random_links(dims, c["eps"], c["seeds"]["links"]))
    phi = lat.dslash(U, to_dev(li.gaussian_spinor(dims, c["seeds"]["eta"])), c["kappa"], dagger=True)
    _, st = lat.fermion_force(U, phi, c["kappa"], lgt.Params(precision="mixed_bf16", tol=c["tol"],
                                                              reliable_delta=1e-3))
    assert st["true_rel_residual"] <= c["tol"]
    assert st["iters"] < 600


@pytest.mark.parametrize("precision", PRECISIONS)
def test_one_correction_pass_after_a_large_miss(lgt, precision, margin):
    """The first pass is told to stop 30x above the target (first_pass_factor
    30), so it misses by far more than 3x.  The correction pass divides out
    the magnification that pass showed, and one pass is enough, for the
    chained solves of the force and for the single Schur solve of the
    even/odd action."""
    u, eta = li.random_links((6, 6, 6, 6), 0.4, 431), li.gaussian_spinor((6, 6, 6, 6), 432)
    lat = lgt.Lattice((6, 6, 6, 6))
    U = to_dev(u)
    phi = lat.dslash(U, to_dev(eta), 0.125, dagger=True)
    tol = 1e-10
    prm = lgt.Params(precision=precision, tol=tol, first_pass_factor=30.0)
    X, Y, st = lat.cg_solve(U, phi, 0.125, prm)
    X0, _, st0 = lat.cg_solve(U, phi, 0.125, lgt.Params(precision="fp64", tol=1e-13))
    assert st["true_rel_residual"] <= tol
    assert st["corrections"] == 1, st
    margin(f"one-pass correction: X vs tight solve ({precision})", rel_err(to_host(X), to_host(X0)), 1e-8)
    phi_o = lat.schur_dslash(U, to_dev(eta), 0.125, dagger=True)
    _, _, st_eo = lat.fermion_force_eo(U, phi_o, 0.125, prm)
    assert st_eo["true_rel_residual"] <= tol
    assert st_eo["corrections"] == 1, st_eo
