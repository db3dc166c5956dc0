"""GPU parity of the stout-smeared path (forward, hand-written adjoint,
smeared force, autograd Function, smeared leapfrog) against the oracle, whose
gradient through the smearing is PyTorch CPU autograd of the definition."""
import sys

import numpy as np
import pytest

import lgt_inputs as li
from oracle import dirac, force, md, stout, su3

from gpu_common import link_errors, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

RHO = 0.1


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def lgt():
    import torch
    assert torch.cuda.is_available()
    import paper_2602_20516_amd as m
    return m


@pytest.mark.parametrize("dims,nlev", [((4, 4, 4, 4), 1), ((4, 4, 4, 4), 2), ((6, 4, 4, 8), 3),
                                       ((2, 2, 2, 4), 2)])
def test_stout_forward(lgt, dims, nlev, margin):
    u = li.random_links(dims, 0.5, 3)
    lat = lgt.Lattice(dims)
    got = to_host(lat.stout_smear(to_dev(u), RHO, nlev))
    margin("rel_err(got, stout.stout(u, RHO, nlev))", rel_err(got, stout.stout(u, RHO, nlev)), 1e-13)


@pytest.mark.parametrize("dims,nlev", [((4, 4, 4, 4), 1), ((4, 4, 4, 4), 2), ((2, 2, 2, 4), 3)])
def test_stout_backprop_vs_autograd(lgt, dims, nlev, margin):
    u = li.random_links(dims, 0.5, 3)
    gt = li.random_links(dims, 1.0, 4) + 0.3 * li.random_links(dims, 1.0, 5)  # any cotangent
    lat = lgt.Lattice(dims)
    got = to_host(lat.stout_backprop(to_dev(u), to_dev(gt), RHO, nlev))
    ref = stout.stout_vjp(u, gt, RHO, nlev)
    say("backprop", dims, nlev, rel_err(got, ref))
    margin("rel_err(got, ref)", rel_err(got, ref), 1e-12)


def test_stout_tiled_16x16x32x64(lgt, margin):
    """Forward (2 levels) and backprop (1 level) on 16x16x32x64, the block
    order of large lattices, with links and cotangent of seeded 8^4 fields
    repeated periodically: every site equals the oracle's 8^4 result at the
    site modulo 8 (smearing has no boundary sign)."""
    small = (8, 8, 8, 8)
    u8 = li.random_links(small, 0.3, 61)
    g8 = li.random_links(small, 1.0, 62) + 0.3 * li.random_links(small, 1.0, 63)
    reps = (64 // 8, 32 // 8, 16 // 8, 16 // 8, 1, 1, 1)
    lat = lgt.Lattice((16, 16, 32, 64))
    U = to_dev(np.tile(u8, reps))
    got = to_host(lat.stout_smear(U, RHO, 2))
    ref = np.tile(stout.stout(u8, RHO, 2), reps)
    margin("forward rel_err(got, ref)", rel_err(got, ref), 1e-13)
    got = to_host(lat.stout_backprop(U, to_dev(np.tile(g8, reps)), RHO, 1))
    ref = np.tile(stout.stout_vjp(u8, g8, RHO, 1), reps)
    margin("backprop rel_err(got, ref)", rel_err(got, ref), 1e-12)


@pytest.mark.parametrize("case", ["unit_links", "rho_zero", "tiny_exponent"])
def test_stout_degenerate_cases(lgt, case, margin):
    """Unit links (every staple sum is 6, so the exponent X vanishes and exp,
    its Cayley-Hamilton coefficients and their derivatives sit at X = 0),
    rho = 0 (the identity map, whose adjoint is the identity), and links
    within 1e-6 of the identity (exponent of order 1e-7)."""
    dims = (4, 4, 4, 4)
    if case == "unit_links":
        u = np.zeros(li.random_links(dims, 0.1, 1).shape, dtype=np.complex128)
        u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1.0
    else:
        u = li.random_links(dims, 1e-6 if case == "tiny_exponent" else 0.5, 71)
    rho = 0.0 if case == "rho_zero" else RHO
    gt = li.random_links(dims, 1.0, 72) + 0.3 * li.random_links(dims, 1.0, 73)
    lat = lgt.Lattice(dims)
    got = to_host(lat.stout_smear(to_dev(u), rho, 2))
    ref = u if case != "tiny_exponent" else stout.stout(u, rho, 2)
    margin("forward rel_err(got, ref)", rel_err(got, ref), 1e-13)
    got = to_host(lat.stout_backprop(to_dev(u), to_dev(gt), rho, 2))
    ref = gt if case == "rho_zero" else stout.stout_vjp(u, gt, rho, 2)
    margin("backprop rel_err(got, ref)", rel_err(got, ref), 1e-12)


def test_stout_backprop_large_rho(lgt, margin):
    """rho = 0.3 (the paper's value in its smeared test) exercises the scaling of the exp adjoint."""
    dims = (4, 4, 4, 4)
    u = li.random_links(dims, 0.8, 13)
    gt = li.random_links(dims, 1.0, 14)
    lat = lgt.Lattice(dims)
    got = to_host(lat.stout_backprop(to_dev(u), to_dev(gt), 0.3, 2))
    margin("rel_err(got, stout.stout_vjp(u, gt, 0.3, 2))", rel_err(got, stout.stout_vjp(u, gt, 0.3, 2)), 1e-12)


@pytest.mark.parametrize("mode", ["force", "grad", "momentum"])
def test_smeared_force(lgt, mode, margin):
    dims = (4, 4, 4, 4)
    u = li.random_links(dims, 0.5, 101)
    eta = li.gaussian_spinor(dims, 102)
    k, beta, dt = 0.12, 6.0, 0.05
    phi = dirac.dslash_dag(stout.stout(u, RHO, 2), eta, k)
    g_ref = force.gauge_grad(u, beta) + stout.smeared_fermion_grad(u, phi, k, RHO, 2, tol=1e-14)
    lat = lgt.Lattice(dims)
    prm = lgt.Params(tol=1e-13)
    if mode == "grad":
        got, sf, st = lat.smeared_force(to_dev(u), to_dev(phi), beta, k, RHO, 2, prm, "grad")
        ref = g_ref
    elif mode == "force":
        got, sf, st = lat.smeared_force(to_dev(u), to_dev(phi), beta, k, RHO, 2, prm, "force")
        ref = force.force_from_grad(u, g_ref)
    else:
        p = li.random_momenta(dims, 7)
        P = to_dev(p)
        got, sf, st = lat.smeared_force(to_dev(u), to_dev(phi), beta, k, RHO, 2, prm, "momentum", dt, out=P)
        ref = p - dt * force.force_from_grad(u, g_ref)
    got = to_host(got)
    say("smeared force", mode, rel_err(got, ref), st)
    margin("rel_err(got, ref)", rel_err(got, ref), 1e-10)
    ee = float(np.vdot(eta.ravel(), eta.ravel()).real)
    margin("abs(sf - ee) / ee", abs(sf - ee) / ee, 1e-12)


def test_autograd_function_matches_oracle_gradient(lgt, margin):
    import torch
    dims = (4, 4, 4, 4)
    u = li.random_links(dims, 0.5, 101)
    eta = li.gaussian_spinor(dims, 102)
    k, beta = 0.12, 6.0
    phi = dirac.dslash_dag(stout.stout(u, RHO, 2), eta, k)
    lat = lgt.Lattice(dims)
    ur = torch.view_as_real(to_dev(u)).clone().requires_grad_(True)
    s = lgt.lattice_action(ur, to_dev(phi), lat, beta, k, RHO, 2, lgt.Params(tol=1e-13))
    s.backward()
    g = torch.view_as_complex(ur.grad.contiguous()).cpu().numpy()
    g_ref = force.gauge_grad(u, beta) + stout.smeared_fermion_grad(u, phi, k, RHO, 2, tol=1e-14)
    s_ref = stout.total_action(u, phi, beta, k, RHO, 2, tol=1e-14)
    margin("abs(float(s) - s_ref) / abs(s_ref)", abs(float(s) - s_ref) / abs(s_ref), 1e-12)
    margin("rel_err(g, g_ref)", rel_err(g, g_ref), 1e-10)


def test_autograd_gradcheck(lgt):
    """torch.autograd.gradcheck of the Function (finite differences off the group)."""
    import torch
    dims = (2, 2, 2, 4)
    u = li.random_links(dims, 0.5, 21)
    eta = li.gaussian_spinor(dims, 22)
    lat = lgt.Lattice(dims)
    phi = to_dev(eta)
    ur = torch.view_as_real(to_dev(u)).clone().requires_grad_(True)
    prm = lgt.Params(tol=1e-13, max_iter=5000)
    f = lambda x: lgt.LatticeAction.apply(x, phi, lat, 5.7, 0.12, RHO, 2, prm)  # noqa: E731
    assert torch.autograd.gradcheck(f, (ur,), eps=1e-6, atol=1e-6, rtol=1e-5, fast_mode=True)


def test_smeared_leapfrog_vs_oracle(lgt, margin):
    dims = (4, 4, 4, 4)
    u = li.random_links(dims, 0.4, 31)
    eta = li.gaussian_spinor(dims, 32)
    p = li.random_momenta(dims, 33)
    k, beta, dt, n = 0.12, 6.0, 0.05, 2
    phi = dirac.dslash_dag(stout.stout(u, RHO, 2), eta, k)

    def f_total(v):
        return stout.total_force(v, phi, beta, k, RHO, 2, tol=1e-14)

    def h(v, q):
        from oracle import action
        return action.kinetic(q) + stout.total_action(v, phi, beta, k, RHO, 2, tol=1e-14)

    h0 = h(u, p)
    pr = p - 0.5 * dt * f_total(u)
    ur = u
    for j in range(n):
        ur = md.link_update(ur, pr, dt)
        pr = pr - (dt if j < n - 1 else 0.5 * dt) * f_total(ur)
    dh_ref = h(ur, pr) - h0
    lat = lgt.Lattice(dims)
    U, P = to_dev(u), to_dev(p)
    dh, st = lat.md_step_smeared(U, P, to_dev(phi), beta, k, RHO, 2, dt, n, lgt.Params(tol=1e-13))
    say("smeared md", dh, dh_ref, st)
    margin("rel_err(to_host(U), ur)", rel_err(to_host(U), ur), 1e-12)
    margin("rel_err(to_host(P), pr)", rel_err(to_host(P), pr), 1e-10)
    assert abs(dh - dh_ref) < 1e-8


def test_smeared_trajectory_dt_squared_and_reversibility(lgt, margin):
    """Config-5 physics at a reduced 8^3x16 volume: kappa 0.135, rho 0.1, 2 levels, mixed CG."""
    dims = (8, 8, 8, 16)
    c = li.config(5)
    u = li.random_links(dims, c["eps"], c["seeds"]["links"])
    eta = li.gaussian_spinor(dims, c["seeds"]["eta"])
    p = li.random_momenta(dims, c["seeds"]["mom"])
    lat = lgt.Lattice(dims)
    U0 = to_dev(u)
    phi = lat.dslash(lat.stout_smear(U0, c["rho"], c["nstout"]), to_dev(eta), c["kappa"], dagger=True)
    prm = lgt.Params(precision="mixed_fp32", tol=1e-12)
    dhs = []
    for n in (4, 8):
        U, P = U0.clone(), to_dev(p)
        dh, st = lat.md_step_smeared(U, P, phi, c["beta"], c["kappa"], c["rho"], c["nstout"], 0.2 / n, n, prm)
        dhs.append(dh)
        say("dt", 0.2 / n, "dH", dh, st)
    assert 3.0 < dhs[0] / dhs[1] < 5.0
    U, P = U0.clone(), to_dev(p)
    lat.md_step_smeared(U, P, phi, c["beta"], c["kappa"], c["rho"], c["nstout"], 0.05, 4, prm)
    P.neg_()
    lat.md_step_smeared(U, P, phi, c["beta"], c["kappa"], c["rho"], c["nstout"], 0.05, 4, prm)
    margin("rel_err(to_host(U), u)", rel_err(to_host(U), u), 1e-10)
