"""GPU parity of the multi-shift CG (lgt_cg_solve_multishift) against the
oracle's one-system-per-shift CG (eo.solve_normal with shift=), plus the
properties that hold at any size: the FP64 true residual of every shift,
recomputed on the CPU with the oracle's Schur operator, and the independence
of each shift's result from the other shifts in the call."""
import sys

import numpy as np
import pytest

import lgt_inputs as li
from oracle import eo

from gpu_common import rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def lgt():
    import torch
    assert torch.cuda.is_available()
    import paper_2602_20516_amd as m
    return m


def _setup(dims, k, seed):
    u, eta = li.random_links(dims, 0.5, seed), li.gaussian_spinor(dims, seed + 1)
    phi_o = eo.schur_dag(u, eo.parity_mask(dims, 1) * eta, k)
    return u, phi_o


def _true_residual(u, phi_o, x, k, sigma):
    r = phi_o - (eo.schur_dag(u, eo.schur(u, x, k), k) + sigma * x)
    return np.linalg.norm(r.ravel()) / np.linalg.norm(phi_o.ravel())


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 4, 8)])
def test_multishift_vs_oracle(lgt, dims):
    k = 0.125
    u, phi_o = _setup(dims, k, 201)
    shifts = [0.0, 0.003, 0.05, 0.4, 2.0, 25.0]
    lat = lgt.Lattice(dims)
    Xs, st = lat.cg_solve_multishift(to_dev(u), to_dev(phi_o), k, shifts, lgt.Params(tol=1e-13))
    say("multishift", dims, st)
    assert st["true_rel_residual"] <= 1e-13
    even = eo.parity_mask(dims, 0)
    for s, X in zip(shifts, Xs):
        x = to_host(X)
        assert np.abs(even * x).max() == 0.0
        ref = eo.solve_normal(u, phi_o, k, shift=s, tol=1e-15)
        e = rel_err(x, ref)
        say("  shift", s, "rel err", e)
        assert e < 1e-11
        assert _true_residual(u, phi_o, x, k, s) <= 1e-13


def test_multishift_iterations_set_by_smallest_shift(lgt):
    """The base recursion runs until the hardest (smallest) shift converges;
    larger shifts stop earlier and leave the count unchanged."""
    dims = (4, 4, 4, 4)
    k = 0.125
    u, phi_o = _setup(dims, k, 211)
    lat = lgt.Lattice(dims)
    U, P = to_dev(u), to_dev(phi_o)
    _, st1 = lat.cg_solve_multishift(U, P, k, [0.0], lgt.Params(tol=1e-12))
    _, st2 = lat.cg_solve_multishift(U, P, k, [0.0, 0.1, 1.0, 10.0], lgt.Params(tol=1e-12))
    _, st3 = lat.cg_solve_multishift(U, P, k, [1.0], lgt.Params(tol=1e-12))
    assert st1["iters"] == st2["iters"]
    assert st3["iters"] < st1["iters"]


def test_shift_result_independent_of_companions(lgt):
    """Each shift's scalars depend only on the base recursion and its own
    sigma, and a shift stops updating once converged: its result is the same
    bits whichever other shifts share the call."""
    dims = (4, 4, 4, 6)
    k = 0.12
    u, phi_o = _setup(dims, k, 221)
    lat = lgt.Lattice(dims)
    U, P = to_dev(u), to_dev(phi_o)
    p = lgt.Params(tol=1e-12)
    a, _ = lat.cg_solve_multishift(U, P, k, [0.2], p)
    b, _ = lat.cg_solve_multishift(U, P, k, [0.0, 0.2, 3.0], p)
    c, _ = lat.cg_solve_multishift(U, P, k, [0.2, 0.2], p)
    assert np.array_equal(to_host(a[0]), to_host(b[1]))
    assert np.array_equal(to_host(c[0]), to_host(c[1]))
    assert np.array_equal(to_host(a[0]), to_host(c[0]))


def test_zero_shift_matches_eo_solve(lgt, margin):
    """sigma = 0 is the even/odd normal solve of the e/o action: phi_o^dag X
    equals S_eo = |eta_o|^2 at the heat-bath phi_o."""
    dims = (4, 4, 4, 4)
    k = 0.12
    u, eta = li.random_links(dims, 0.5, 231), li.gaussian_spinor(dims, 232)
    eta_o = eo.parity_mask(dims, 1) * eta
    phi_o = eo.schur_dag(u, eta_o, k)
    lat = lgt.Lattice(dims)
    Xs, _ = lat.cg_solve_multishift(to_dev(u), to_dev(phi_o), k, [0.0], lgt.Params(tol=1e-13))
    s = float(np.vdot(phi_o.ravel(), to_host(Xs[0]).ravel()).real)
    ee = float(np.vdot(eta_o.ravel(), eta_o.ravel()).real)
    margin("abs(s - ee) / ee", abs(s - ee) / ee, 1e-12)


def test_multishift_max_shifts_and_repeat(lgt, margin):
    """32 shifts (the limit), then a smaller call on the same context."""
    dims = (4, 4, 4, 4)
    k = 0.12
    u, phi_o = _setup(dims, k, 241)
    lat = lgt.Lattice(dims)
    U, P = to_dev(u), to_dev(phi_o)
    shifts = list(np.geomspace(1e-4, 1e2, 32))
    Xs, st = lat.cg_solve_multishift(U, P, k, shifts, lgt.Params(tol=1e-12))
    assert st["true_rel_residual"] <= 1e-12
    for i in (0, 13, 31):
        margin("rel_err(to_host(Xs[i]), eo.solve_normal(u, phi_o, k, shift=shifts[i], tol=1e-15))", rel_err(to_host(Xs[i]), eo.solve_normal(u, phi_o, k, shift=shifts[i], tol=1e-15)), 1e-9)
    Ys, st2 = lat.cg_solve_multishift(U, P, k, shifts[5:8], lgt.Params(tol=1e-12))
    for j in range(3):
        assert np.array_equal(to_host(Ys[j]), to_host(Xs[5 + j]))


def test_multishift_zero_source_and_errors(lgt):
    dims = (4, 4, 4, 4)
    k = 0.12
    u, phi_o = _setup(dims, k, 251)
    lat = lgt.Lattice(dims)
    U, P = to_dev(u), to_dev(phi_o)
    Xs, st = lat.cg_solve_multishift(U, to_dev(np.zeros_like(phi_o)), k, [0.0, 1.0])
    assert all(np.abs(to_host(x)).max() == 0.0 for x in Xs)
    assert st["iters"] == 0
    with pytest.raises(lgt.LGTError):
        lat.cg_solve_multishift(U, P, k, [0.1, -0.5])
    with pytest.raises(lgt.LGTError):
        lat.cg_solve_multishift(U, P, k, [float("nan")])
    with pytest.raises(lgt.LGTError):
        lat.cg_solve_multishift(U, P, k, [0.1] * 33)
    with pytest.raises(lgt.LGTError):
        lat.cg_solve_multishift(U, P, k, [])
    with pytest.raises(lgt.LGTError):
        lat.cg_solve_multishift(U, P, k, [0.1], lgt.Params(precision="mixed_fp32"))
    with pytest.raises(lgt.LGTNotConverged) as ei:
        lat.cg_solve_multishift(U, P, k, [0.0, 0.1], lgt.Params(tol=1e-12, max_iter=5))
    assert ei.value.stats["iters"] == 5
    # the context still works after the errors
    Xs, st = lat.cg_solve_multishift(U, P, k, [0.1], lgt.Params(tol=1e-12))
    assert st["true_rel_residual"] <= 1e-12


def test_multishift_full_size(lgt):
    """16^4 (the headline lattice) with 8 shifts: the true residual of sampled
    shifts recomputed on the CPU with the oracle's operator."""
    dims = (16, 16, 16, 16)
    k = 0.1215
    u, eta = li.random_links(dims, 0.35, 261), li.gaussian_spinor(dims, 262)
    import torch
    lat = lgt.Lattice(dims)
    U = to_dev(u)
    phi = lat.schur_dslash(U, to_dev(eta), k, dagger=True)
    shifts = [0.0, 1e-3, 1e-2, 0.05, 0.2, 1.0, 5.0, 50.0]
    Xs, st = lat.cg_solve_multishift(U, phi, k, shifts, lgt.Params(tol=1e-10))
    say("multishift 16^4", st)
    assert st["true_rel_residual"] <= 1e-10
    torch.cuda.synchronize()
    phi_o = to_host(phi)
    for i in (0, 5):
        r = _true_residual(u, phi_o, to_host(Xs[i]), k, shifts[i])
        say("  shift", shifts[i], "cpu residual", r)
        assert r <= 1.05e-10


# ---- rational (RHMC) force ------------------------------------------------------

RAT = dict(a0=0.3, shifts=[0.0, 0.05, 0.6, 4.0], residues=[0.7, -0.2, 1.3, 2.1])


@pytest.mark.parametrize("mode", ["force", "grad", "momentum"])
def test_rational_force_vs_oracle(lgt, mode, margin):
    dims = (4, 4, 4, 4)
    k = 0.12
    u, phi_o = _setup(dims, k, 271)
    lat = lgt.Lattice(dims)
    U, P = to_dev(u), to_dev(phi_o)
    prm = lgt.Params(tol=1e-13)
    g_ref = eo.rational_grad(u, phi_o, k, RAT["a0"], RAT["shifts"], RAT["residues"])
    from oracle import force as oforce
    if mode == "grad":
        got, s_r, st = lat.rational_force_eo(U, P, k, RAT["shifts"], RAT["residues"], RAT["a0"], prm, "grad")
        ref = g_ref
    elif mode == "force":
        got, s_r, st = lat.rational_force_eo(U, P, k, RAT["shifts"], RAT["residues"], RAT["a0"], prm, "force")
        ref = oforce.force_from_grad(u, g_ref)
    else:
        p = li.random_momenta(dims, 272)
        dt = 0.05
        got, s_r, st = lat.rational_force_eo(U, P, k, RAT["shifts"], RAT["residues"], RAT["a0"], prm, "momentum",
                                             dt, out=to_dev(p))
        ref = p - dt * oforce.force_from_grad(u, g_ref)
    say("rational", mode, st, rel_err(to_host(got), ref))
    assert st["true_rel_residual"] <= 1e-13
    margin("rel_err(to_host(got), ref)", rel_err(to_host(got), ref), 1e-11)
    s_ref = eo.rational_action(u, phi_o, k, RAT["a0"], RAT["shifts"], RAT["residues"])
    assert abs(s_r - s_ref) < 1e-12 * abs(s_ref)


def test_rational_force_single_term_is_the_eo_force(lgt, margin):
    """One term, sigma = 0, residue 1, a0 = 0: the even/odd action and force."""
    dims = (4, 4, 4, 6)
    k = 0.12
    u, phi_o = _setup(dims, k, 281)
    lat = lgt.Lattice(dims)
    U, P = to_dev(u), to_dev(phi_o)
    prm = lgt.Params(tol=1e-13)
    f_rat, s_rat, _ = lat.rational_force_eo(U, P, k, [0.0], [1.0], 0.0, prm)
    f_eo, s_eo, _ = lat.fermion_force_eo(U, P, k, prm)
    margin("rel_err(to_host(f_rat), to_host(f_eo))", rel_err(to_host(f_rat), to_host(f_eo)), 1e-11)
    assert abs(s_rat - s_eo) < 1e-12 * abs(s_eo)


def test_rational_force_errors(lgt):
    dims = (4, 4, 4, 4)
    k = 0.12
    u, phi_o = _setup(dims, k, 291)
    lat = lgt.Lattice(dims)
    U, P = to_dev(u), to_dev(phi_o)
    with pytest.raises(lgt.LGTError):
        lat.rational_force_eo(U, P, k, [0.1, -1.0], [1.0, 1.0])
    with pytest.raises(lgt.LGTError):
        lat.rational_force_eo(U, P, k, [0.1], [float("inf")])
    with pytest.raises(lgt.LGTError):
        lat.rational_force_eo(U, P, k, [0.1] * 33, [1.0] * 33)
    with pytest.raises(lgt.LGTError):
        lat.rational_force_eo(U, P, k, [0.1], [1.0], 0.0, lgt.Params(precision="mixed_fp32"))
    f, s, st = lat.rational_force_eo(U, P, k, [0.1], [1.0], 0.0, lgt.Params(tol=1e-12))
    assert st["true_rel_residual"] <= 1e-12
