"""GPU parity of the batched multi-right-hand-side solve (12 pseudofermions:
6 kappa values x 2 Gaussian seeds on one lattice) against the oracle and
against the single-field solves."""
import sys

import numpy as np
import pytest

import lgt_inputs as li
from oracle import dirac, solver

from gpu_common import rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

KAPPAS = (0.10, 0.11, 0.12, 0.125, 0.13, 0.135)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def lgt():
    import torch
    assert torch.cuda.is_available()
    import paper_2602_20516_amd as m
    return m


def workload(dims, seeds=(402, 403)):
    u = li.random_links(dims, 0.3, 401)
    etas = [li.gaussian_spinor(dims, s) for s in seeds]
    items = [(k, eta) for k in KAPPAS for eta in etas]
    return u, items


@pytest.mark.parametrize("precision,tol,gate", [("fp64", 1e-14, 1e-12), ("mixed_fp32", 1e-14, 1e-12),
                                                ("mixed_fp32", 1e-11, 1e-9)])
def test_batch_vs_oracle_4x4(lgt, precision, tol, gate, margin):
    dims = (4, 4, 4, 4)
    u, items = workload(dims)
    phis = [dirac.dslash_dag(u, eta, k) for k, eta in items]
    lat = lgt.Lattice(dims)
    Xs, Ys, st = lat.cg_solve_batch(to_dev(u), [to_dev(p) for p in phis], [k for k, _ in items],
                                    lgt.Params(precision=precision, tol=tol))
    say("batch", precision, [s["iters"] for s in st], max(s["true_rel_residual"] for s in st))
    for (k, eta), phi, X, Y, s in zip(items, phis, Xs, Ys, st):
        assert s["true_rel_residual"] <= tol
        x_ref, y_ref, _, _ = solver.solve_ddag_d(u, phi, k, tol=1e-15)
        margin(f"batched X vs oracle, kappa {k} ({precision}, tol {tol:g})", rel_err(to_host(X), x_ref), gate)
        margin(f"batched Y vs eta, kappa {k} ({precision}, tol {tol:g})", rel_err(to_host(Y), eta), gate)


def test_batch_ragged_and_small(lgt, margin):
    """Ragged tail (V/2 * nr not a multiple of 64), a batch of one, and five items."""
    for dims, n in (((6, 6, 6, 6), 5), ((2, 2, 2, 4), 1), ((6, 4, 4, 8), 7)):
        u, items = workload(dims)
        items = items[:n]
        phis = [dirac.dslash_dag(u, eta, k) for k, eta in items]
        lat = lgt.Lattice(dims)
        Xs, Ys, st = lat.cg_solve_batch(to_dev(u), [to_dev(p) for p in phis], [k for k, _ in items],
                                        lgt.Params(tol=1e-12))
        for (k, eta), Y, s in zip(items, Ys, st):
            assert s["true_rel_residual"] <= 1e-12
            margin("rel_err(to_host(Y), eta)", rel_err(to_host(Y), eta), 1e-9)


@pytest.mark.parametrize("precision", ["fp64", "mixed_fp32"])
def test_batch_matches_single_solves_16(lgt, precision, margin):
    """16^4 with the 12 right-hand sides: each item equals its own single solve."""
    import torch
    dims = (16, 16, 16, 16)
    u, items = workload(dims)
    lat = lgt.Lattice(dims)
    U = to_dev(u)
    phis = [lat.dslash(U, to_dev(eta), k, dagger=True) for k, eta in items]
    prm = lgt.Params(precision=precision, tol=1e-10)
    torch.cuda.synchronize()
    Xs, Ys, st = lat.cg_solve_batch(U, phis, [k for k, _ in items], prm)
    say("batch16", precision, st[0]["ms"], [s["iters"] for s in st])
    for i in (0, 5, 11):
        k = items[i][0]
        X1, Y1, s1 = lat.cg_solve(U, phis[i], k, prm)
        assert st[i]["true_rel_residual"] <= 1e-10
        margin("rel_err(to_host(Xs[i]), to_host(X1))", rel_err(to_host(Xs[i]), to_host(X1)), 1e-8)
        margin("rel_err(to_host(Ys[i]), items[i][1])", rel_err(to_host(Ys[i]), items[i][1]), 1e-8)


def test_batch_rejects_bf16_storage(lgt):
    dims = (4, 4, 4, 4)
    u, items = workload(dims)
    lat = lgt.Lattice(dims)
    with pytest.raises(lgt.LGTError):
        lat.cg_solve_batch(to_dev(u), [to_dev(e) for _, e in items[:2]], [k for k, _ in items[:2]],
                           lgt.Params(precision="mixed_bf16"))


@pytest.mark.parametrize("precision", ["fp64", "mixed_fp32"])
def test_batch_with_systems_that_stop_at_once(lgt, precision, margin):
    """A zero right-hand side (stopped before the first iteration) and kappa = 0
    (D = 1: converged after one) in the same group as systems that run on: the
    batched hop skips the stopped ones, which keep their exact answers
    (X = Y = 0; X = Y = phi), and the others still match the oracle."""
    dims = (6, 4, 4, 8)
    u = li.random_links(dims, 0.3, 411)
    etas = [li.gaussian_spinor(dims, s) for s in (412, 413, 414)]
    kappas = [0.12, 0.0, 0.13, 0.125]
    phis = [dirac.dslash_dag(u, etas[0], kappas[0]), etas[1], np.zeros_like(etas[0]),
            dirac.dslash_dag(u, etas[2], kappas[3])]
    lat = lgt.Lattice(dims)
    Xs, Ys, st = lat.cg_solve_batch(to_dev(u), [to_dev(p) for p in phis], kappas,
                                    lgt.Params(precision=precision, tol=1e-12))
    say("batch stops", precision, [s["iters"] for s in st])
    assert np.abs(to_host(Xs[2])).max() == 0.0 and np.abs(to_host(Ys[2])).max() == 0.0
    assert st[2]["iters"] == 0
    # D = 1: the true residual is phi - X itself
    assert st[1]["true_rel_residual"] <= 1e-12
    margin("rel_err(to_host(Xs[1]), etas[1]) < 2e-12 and rel_err(to_host(Ys[1]), etas[1])", rel_err(to_host(Xs[1]), etas[1]) < 2e-12 and rel_err(to_host(Ys[1]), etas[1]), 2e-12)
    # a system's count is the iterations its own recursion ran (a stopped
    # one idles until the batch's reliable update without counting), summed
    # over the two Schur solves: with D = 1 one per solve in FP64; the FP32
    # recursion takes one per reliable-update cycle, and two cycles (about 7
    # digits each) reach 1e-12
    assert st[1]["iters"] <= (2 if precision == "fp64" else 4)
    for i, eta in ((0, etas[0]), (3, etas[2])):
        assert st[i]["true_rel_residual"] <= 1e-12
        x_ref, _, _, _ = solver.solve_ddag_d(u, phis[i], kappas[i], tol=1e-14)
        margin("rel_err(to_host(Xs[i]), x_ref)", rel_err(to_host(Xs[i]), x_ref), 1e-9)
        margin("rel_err(to_host(Ys[i]), eta)", rel_err(to_host(Ys[i]), eta), 1e-9)


@pytest.mark.parametrize("precision,tol,gate", [("fp64", 1e-14, 1e-12), ("mixed_fp32", 1e-11, 1e-9)])
def test_batch_over_several_lattices_vs_oracle(lgt, precision, tol, gate, margin):
    """One call over three lattices of different shapes (one of them ragged:
    its half volume is not a multiple of 64), each with its own kappas."""
    cases = [((4, 4, 4, 4), (0.10, 0.135)), ((6, 4, 4, 8), (0.12, 0.125, 0.13)), ((2, 2, 2, 4), (0.11,))]
    batch = lgt.Batch()
    items, refs = [], []
    for dims, kappas in cases:
        u = li.random_links(dims, 0.3, 451)
        lat = lgt.Lattice(dims)
        U = to_dev(u)
        for j, k in enumerate(kappas):
            eta = li.gaussian_spinor(dims, 452 + j)
            phi = dirac.dslash_dag(u, eta, k)
            items.append((lat, U, to_dev(phi), k))
            refs.append((dims, u, phi, eta, k))
    Xs, Ys, st = batch.cg_solve(items, lgt.Params(precision=precision, tol=tol))
    say("multi-lattice batch", precision, [s["iters"] for s in st])
    for (dims, u, phi, eta, k), X, Y, s in zip(refs, Xs, Ys, st):
        assert s["true_rel_residual"] <= tol
        x_ref, _, _, _ = solver.solve_ddag_d(u, phi, k, tol=1e-15)
        margin(f"multi-lattice batch X vs oracle {dims} kappa {k} ({precision}, tol {tol:g})",
               rel_err(to_host(X), x_ref), gate)
        margin(f"multi-lattice batch Y vs eta {dims} kappa {k} ({precision}, tol {tol:g})",
               rel_err(to_host(Y), eta), gate)


def test_batch_config4_one_call(lgt, margin):
    """The 36 solves of the batched workload (8^4, 12^4, 16^4; 6 kappa x 2 eta
    each) in one call: each item equals its own single solve and Y = eta."""
    import torch
    batch = lgt.Batch()
    items, meta = [], []
    for dims in ((8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 16)):
        u, its = workload(dims)
        lat = lgt.Lattice(dims)
        U = to_dev(u)
        for k, eta in its:
            items.append((lat, U, lat.dslash(U, to_dev(eta), k, dagger=True), k))
            meta.append((dims, eta))
    prm = lgt.Params(precision="mixed_fp32", tol=1e-10)
    torch.cuda.synchronize()
    Xs, Ys, st = batch.cg_solve(items, prm)
    say("c4 one call", st[0]["ms"], [s["iters"] for s in st])
    for i in range(len(items)):
        assert st[i]["true_rel_residual"] <= 1e-10
        margin(f"c4 one call Y vs eta {meta[i][0]} kappa {items[i][3]}", rel_err(to_host(Ys[i]), meta[i][1]), 1e-8)
    for i in (0, 11, 12, 23, 24, 35):
        lat, U, phi, k = items[i]
        X1, _, _ = lat.cg_solve(U, phi, k, prm)
        margin(f"c4 one call X vs single solve {meta[i][0]} kappa {k}", rel_err(to_host(Xs[i]), to_host(X1)), 1e-8)


def test_batch_rejects_bad_items(lgt):
    dims = (4, 4, 4, 4)
    u, its = workload(dims)
    lat = lgt.Lattice(dims)
    U1, U2 = to_dev(u), to_dev(u)
    batch = lgt.Batch()
    items = [(lat, U1, to_dev(its[0][1]), 0.1), (lat, U2, to_dev(its[1][1]), 0.1)]
    with pytest.raises(lgt.LGTError) as e:
        batch.cg_solve(items)
    assert "two gauge fields" in str(e.value)
    with pytest.raises(lgt.LGTError):
        batch.cg_solve([(lat, U1, to_dev(its[0][1]), 0.1)] * 17)


@pytest.mark.parametrize("kind", ["valu", "mfma"])
@pytest.mark.parametrize("dims,n", [((4, 4, 4, 4), 12), ((6, 4, 4, 8), 5), ((2, 2, 2, 4), 3), ((8, 6, 4, 6), 16)])
@pytest.mark.parametrize("dagger", [False, True])
def test_batched_dslash_kernels_vs_oracle(lgt, kind, dims, n, dagger, margin):
    """lgt_dslash_batch through each FP32 batched hop kernel (and FP64) against
    the oracle's D, field by field: groups of 4 and 8 (and a ragged last
    group), a half volume that is not a multiple of 16, the t boundary."""
    u = li.random_links(dims, 0.5, 461)
    psis = [li.gaussian_spinor(dims, 470 + j) for j in range(n)]
    kappas = [0.09 + 0.004 * j for j in range(n)]
    lat = lgt.Lattice(dims)
    lat.set_batch_hop_kernel(kind)
    U = to_dev(u)
    P = [to_dev(p) for p in psis]
    out32 = lat.dslash_batch(U, P, kappas, dagger, "mixed_fp32")
    out64 = lat.dslash_batch(U, P, kappas, dagger, "fp64")
    f = dirac.dslash_dag if dagger else dirac.dslash
    for j in range(n):
        ref = f(u, psis[j], kappas[j])
        margin(f"batched D FP32 ({kind}) {dims} field {j}/{n} dagger {dagger}", rel_err(to_host(out32[j]), ref), 1e-6)
        margin(f"batched D FP64 {dims} field {j}/{n} dagger {dagger}", rel_err(to_host(out64[j]), ref), 1e-13)


def test_batch_solve_with_each_kernel(lgt, margin):
    """The mixed batched solve with the FP32 hop forced to each kernel: both
    meet the oracle, and the MFMA run takes the iterations of the VALU run
    (a wrong inner operator would show as extra iterations, since the FP64
    reliable updates would still pull the solution to the right answer)."""
    dims = (6, 6, 6, 6)
    u, items = workload(dims)
    phis = [dirac.dslash_dag(u, eta, k) for k, eta in items]
    iters = {}
    for kind in ("valu", "mfma"):
        lat = lgt.Lattice(dims)
        lat.set_batch_hop_kernel(kind)
        Xs, Ys, st = lat.cg_solve_batch(to_dev(u), [to_dev(p) for p in phis], [k for k, _ in items],
                                        lgt.Params(precision="mixed_fp32", tol=1e-11))
        iters[kind] = [s["iters"] for s in st]
        say("batch kernel", kind, iters[kind])
        for (k, eta), phi, X, s in zip(items, phis, Xs, st):
            assert s["true_rel_residual"] <= 1e-11
            x_ref, _, _, _ = solver.solve_ddag_d(u, phi, k, tol=1e-15)
            margin(f"batched solve ({kind} FP32 hop) X vs oracle kappa {k}", rel_err(to_host(X), x_ref), 1e-9)
    for a, b in zip(iters["valu"], iters["mfma"]):
        assert abs(a - b) <= 3


def test_mixed_batch_with_links_outside_su3(lgt, margin):
    """Links scaled by 0.9 are not SU(3): the batched FP32 hop must read them
    in full (no third-row reconstruction) and still reach the oracle's
    answer, in about the iterations of the FP64 batch."""
    dims = (6, 6, 6, 6)
    u, items = workload(dims)
    u = 0.9 * u
    items = items[::3]
    phis = [dirac.dslash_dag(u, eta, k) for k, eta in items]
    lat = lgt.Lattice(dims)
    U, P, ks = to_dev(u), [to_dev(p) for p in phis], [k for k, _ in items]
    Xs, _, st = lat.cg_solve_batch(U, P, ks, lgt.Params(precision="mixed_fp32", tol=1e-12))
    _, _, st64 = lat.cg_solve_batch(U, P, ks, lgt.Params(precision="fp64", tol=1e-12))
    say("batch outside SU(3)", [s["iters"] for s in st], [s["iters"] for s in st64])
    for (k, eta), phi, X, s, s64 in zip(items, phis, Xs, st, st64):
        assert s["true_rel_residual"] <= 1e-12
        x_ref, _, _, _ = solver.solve_ddag_d(u, phi, k, tol=1e-15)
        margin(f"batched X vs oracle, links outside SU(3), kappa {k}", rel_err(to_host(X), x_ref), 1e-10)
        # a wrongly rebuilt third row would cost many more iterations
        assert s["iters"] <= s64["iters"] + 8
