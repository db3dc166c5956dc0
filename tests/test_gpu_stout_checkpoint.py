"""Deep stout chains on the GPU with checkpointed reverse passes: the
gradient is the same bits under every schedule (the recomputed levels are
the same deterministic forward kernels), matches the oracle's autograd VJP
and smeared force, and the reverse pass performs exactly the recomputation
count of its schedule."""
import sys

import numpy as np
import pytest

import lgt_inputs as li
from oracle import dirac, force, stout

from gpu_common import rel_err, to_dev, to_host

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


@pytest.mark.parametrize("dims,nlev", [((4, 4, 4, 4), 6), ((2, 2, 2, 4), 40)])
def test_backprop_every_schedule_same_bits(lgt, dims, nlev, margin):
    u = li.random_links(dims, 0.5, 31)
    gt = li.random_links(dims, 1.0, 32) + 0.3 * li.random_links(dims, 1.0, 33)
    lat = lgt.Lattice(dims)
    U, GT = to_dev(u), to_dev(gt)
    outs = {}
    for cap in (0, 1, 2, 3, nlev - 1, -1):
        lat.set_stout_checkpoints(cap)
        outs[cap] = to_host(lat.stout_backprop(U, GT, RHO, nlev))
        sch = lat.stout_last_schedule()
        slots = nlev - 1 if cap < 0 else min(cap, nlev - 1)
        assert sch["stored_levels"] == slots
        assert sch["recompute_passes"] == lgt.stout_schedule(nlev, slots)["recompute_passes"]
    for cap, g in outs.items():
        assert np.array_equal(g, outs[0]), cap
    ref = stout.stout_vjp(u, gt, RHO, nlev)
    say("deep backprop", dims, nlev, rel_err(outs[-1], ref))
    margin("rel_err(outs[-1], ref)", rel_err(outs[-1], ref), 1e-12)


def test_stout_at_full_block_size(lgt, margin):
    """8^4: 32 full 64-site blocks per parity (the small lattices fill one
    block partially); forward and reverse against the oracle."""
    dims = (8, 8, 8, 8)
    u = li.random_links(dims, 0.5, 71)
    gt = li.random_links(dims, 1.0, 72)
    lat = lgt.Lattice(dims)
    U = to_dev(u)
    margin("rel_err(to_host(lat.stout_smear(U, RHO, 2)), stout.stout(u, RHO, 2))", rel_err(to_host(lat.stout_smear(U, RHO, 2)), stout.stout(u, RHO, 2)), 1e-13)
    got = to_host(lat.stout_backprop(U, to_dev(gt), RHO, 2))
    margin("rel_err(got, stout.stout_vjp(u, gt, RHO, 2))", rel_err(got, stout.stout_vjp(u, gt, RHO, 2)), 1e-12)


def test_deep_smeared_force_vs_oracle(lgt, margin):
    dims = (4, 4, 4, 4)
    nlev = 6
    u, eta = li.random_links(dims, 0.5, 41), li.gaussian_spinor(dims, 42)
    k, beta = 0.12, 5.9
    phi = dirac.dslash_dag(stout.stout(u, RHO, nlev), eta, k)
    ref = force.force_from_grad(u, force.gauge_grad(u, beta)
                                + stout.smeared_fermion_grad(u, phi, k, RHO, nlev, tol=1e-14))
    lat = lgt.Lattice(dims)
    U, PHI = to_dev(u), to_dev(phi)
    outs = []
    for cap in (0, 2, -1):
        lat.set_stout_checkpoints(cap)
        got, sf, st = lat.smeared_force(U, PHI, beta, k, RHO, nlev, lgt.Params(tol=1e-13), "force")
        outs.append(to_host(got))
        assert lat.stout_last_schedule()["recompute_passes"] == \
            lgt.stout_schedule(nlev, nlev - 1 if cap < 0 else cap)["recompute_passes"]
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    say("deep smeared force", rel_err(outs[-1], ref))
    margin("rel_err(outs[-1], ref)", rel_err(outs[-1], ref), 1e-10)


def test_deep_trajectory_schedule_independent(lgt):
    """A 4-level smeared trajectory gives the same links, momenta and dH
    (same bits) with no checkpoints and with every level kept."""
    dims = (4, 4, 4, 4)
    u, eta, p = li.random_links(dims, 0.4, 51), li.gaussian_spinor(dims, 52), li.random_momenta(dims, 53)
    k, beta = 0.115, 5.8
    lat = lgt.Lattice(dims)
    phi = lat.dslash(lat.stout_smear(to_dev(u), RHO, 4), to_dev(eta), k, dagger=True)
    res = []
    for cap in (0, -1):
        lat.set_stout_checkpoints(cap)
        U, P = to_dev(u), to_dev(p)
        dh, st = lat.md_step_smeared(U, P, phi, beta, k, RHO, 4, 0.05, 3, lgt.Params(tol=1e-12))
        res.append((to_host(U), to_host(P), dh))
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    assert res[0][2] == res[1][2]


def test_checkpoint_arguments(lgt, margin):
    lat = lgt.Lattice((4, 4, 4, 4))
    with pytest.raises(lgt.LGTError):
        lat.set_stout_checkpoints(-2)
    U = to_dev(li.random_links((4, 4, 4, 4), 0.5, 61))
    with pytest.raises(lgt.LGTError):
        lat.stout_smear(U, RHO, 257)
    lat.set_stout_checkpoints(3)
    out = lat.stout_smear(U, RHO, 2)  # the context still works
    margin("rel_err(to_host(out), stout.stout(to_host(U), RHO, 2))", rel_err(to_host(out), stout.stout(to_host(U), RHO, 2)), 1e-13)
