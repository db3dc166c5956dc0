"""Both work shapes of the single-field hop kernel, and both orders of the
64-site blocks, against the oracle.

The hop runs with 64 sites per block (each wave both hops along one
direction) or 32 (each half-wave one hop), chosen by volume unless the
context fixes it (lgt_set_hop_block_sites); the 64-site blocks run in site
order or t-fastest in groups of t-slices (lgt_set_hop_block_order), again by
volume.  The lattices the oracle handles in a test are too small for the
automatic choice to take the larger shape's t-fastest order, so this file
forces each kernel configuration on the same inputs: D and D^dag (FP64, 1e-13 as the other
deterministic maps), the force in all three solver precisions (whose CG
launches the hop with every epilogue: Schur norm, CG update, residual), and
the multi-shift solve.  Shapes: a lattice smaller than one block, lattices
whose per-parity site count leaves a ragged last block for both shapes, and
an unragged one."""
import functools
import sys

import numpy as np
import pytest

import lgt_inputs as li
from oracle import dirac, eo, force

from gpu_common import max_rel_err, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

# (sites per block, order of the 64-site blocks)
SHAPES = [(32, 0), (64, 1), (64, 2)]
SITES = [32, 64]
# sites per parity: 16 (below one block), 432 (ragged for 32 and 64),
# 1080 (ragged for both), 384 (a whole number of blocks for both); then
# lattices whose t-slices hold whole 64-site blocks, where the 64-site
# kernel takes its blocks t-fastest in groups of 2, 8 and 4 slices
DIMS = [(2, 2, 2, 4), (6, 6, 6, 4), (10, 6, 6, 6), (8, 4, 6, 4), (8, 4, 8, 6), (16, 4, 4, 8), (8, 8, 8, 12)]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def lgt():
    import torch
    assert torch.cuda.is_available()
    import paper_2602_20516_amd as m
    return m


def _lattice(lgt, dims, sites, order=0):
    lat = lgt.Lattice(dims)
    lat.set_hop_block_sites(sites)
    lat.set_hop_block_order(order)
    return lat


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("dims", DIMS)
def test_dslash_both_shapes(lgt, dims, shape, margin):
    say("dslash", dims, "sites per block, order", shape)
    u, psi = li.random_links(dims, 0.5, 501), li.gaussian_spinor(dims, 502)
    lat = _lattice(lgt, dims, *shape)
    U, PSI = to_dev(u), to_dev(psi)
    for dag in (False, True):
        got = to_host(lat.dslash(U, PSI, 0.13, dag))
        ref = (dirac.dslash_dag if dag else dirac.dslash)(u, psi, 0.13)
        margin("rel_err(got, ref)", rel_err(got, ref), 1e-13)
        margin("max_rel_err(got, ref)", max_rel_err(got, ref), 1e-13)


@functools.lru_cache(maxsize=1)
def _force_case():
    dims = (6, 6, 6, 4)
    u, eta = li.random_links(dims, 0.5, 511), li.gaussian_spinor(dims, 512)
    phi = dirac.dslash_dag(u, eta, 0.12)
    return dims, u, phi, force.fermion_force(u, phi, 0.12, tol=1e-15)


CASES = [("fp64", 1e-14, 1e-12), ("mixed_fp32", 1e-11, 1e-9), ("mixed_bf16", 1e-11, 1e-9)]


@pytest.mark.parametrize("sites", SITES)
@pytest.mark.parametrize("precision,tol,gate", CASES)
def test_force_both_shapes(lgt, precision, tol, gate, sites, margin):
    dims, u, phi, ref = _force_case()
    k = 0.12
    lat = _lattice(lgt, dims, sites)
    got, st = lat.fermion_force(to_dev(u), to_dev(phi), k, lgt.Params(precision=precision, tol=tol))
    e = rel_err(to_host(got), ref)
    say("force", precision, "sites per block", sites, "iters", st["iters"], "rel err", e)
    assert st["true_rel_residual"] <= tol
    margin(f"force vs oracle, {sites}-site hop blocks ({precision}, tol {tol:g})", e, gate)


@functools.lru_cache(maxsize=1)
def _force_case_ordered():
    dims = (16, 4, 4, 8)
    u, eta = li.random_links(dims, 0.5, 541), li.gaussian_spinor(dims, 542)
    phi = dirac.dslash_dag(u, eta, 0.12)
    return dims, u, phi, force.fermion_force(u, phi, 0.12, tol=1e-15)


@pytest.mark.parametrize("precision,tol,gate", CASES[:2])
def test_force_t_fastest_block_order(lgt, precision, tol, gate, margin):
    """The force with the 64-site kernel on a lattice where it takes its
    blocks t-fastest (16 x 4 x 4 x 8: two blocks per t-slice, groups of 8
    slices), so every epilogue of the CG runs under that order."""
    dims, u, phi, ref = _force_case_ordered()
    lat = _lattice(lgt, dims, 64, 2)
    got, st = lat.fermion_force(to_dev(u), to_dev(phi), 0.12, lgt.Params(precision=precision, tol=tol))
    assert st["true_rel_residual"] <= tol
    margin(f"force vs oracle, t-fastest block order ({precision}, tol {tol:g})", rel_err(to_host(got), ref), gate)


@pytest.mark.parametrize("sites", SITES)
def test_multishift_both_shapes(lgt, sites, margin):
    dims = (6, 6, 6, 4)
    k = 0.125
    u, eta = li.random_links(dims, 0.5, 521), li.gaussian_spinor(dims, 522)
    phi_o = eo.schur_dag(u, eo.parity_mask(dims, 1) * eta, k)
    shifts = [0.0, 0.02, 1.5]
    lat = _lattice(lgt, dims, sites)
    Xs, st = lat.cg_solve_multishift(to_dev(u), to_dev(phi_o), k, shifts, lgt.Params(tol=1e-14))
    assert st["true_rel_residual"] <= 1e-14
    for s, X in zip(shifts, Xs):
        margin(f"multishift X vs oracle, shift {s}, {sites}-site blocks (FP64, tol 1e-14)",
               rel_err(to_host(X), eo.solve_normal(u, phi_o, k, shift=s, tol=1e-15)), 1e-12)


def test_shapes_agree_and_setting_is_checked(lgt, margin):
    """The two shapes sum the eight hop terms in different orders: FP64
    results agree to rounding, and each shape repeats its own bits."""
    dims = (10, 6, 6, 6)
    u, psi = li.random_links(dims, 0.5, 531), li.gaussian_spinor(dims, 532)
    lat = lgt.Lattice(dims)
    U, PSI = to_dev(u), to_dev(psi)
    out = {}
    for sites in (32, 64, 0):
        lat.set_hop_block_sites(sites)
        a = to_host(lat.dslash(U, PSI, 0.13))
        assert np.array_equal(a, to_host(lat.dslash(U, PSI, 0.13)))
        out[sites] = a
    margin("rel_err(out[32], out[64])", rel_err(out[32], out[64]), 1e-15)
    assert np.array_equal(out[0], out[32])  # 1080 sites per parity: automatic choice is 32
    for bad in (-1, 16, 48, 128):
        with pytest.raises(lgt.LGTError):
            lat.set_hop_block_sites(bad)
    for bad in (-1, 3):
        with pytest.raises(lgt.LGTError):
            lat.set_hop_block_order(bad)


def test_32_site_blocks_refused_above_4_gib_of_links(lgt):
    """The 32-site kernel reads both parities' links through one buffer
    resource with 32-bit offsets: a lattice whose FP64 gauge field reaches
    4 GiB (here 40^3 x 120, 4.4 GB of links) must refuse it, and keep the
    64-site kernel."""
    import torch
    lat = lgt.Lattice((40, 40, 40, 120))
    with pytest.raises(lgt.LGTError):
        lat.set_hop_block_sites(32)
    lat.set_hop_block_sites(64)
    lat.set_hop_block_sites(0)
    del lat
    torch.cuda.empty_cache()
