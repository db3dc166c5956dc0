"""GPU parity of the even/odd-preconditioned pseudofermion action: Schur
operator, force (FP64, FP32 and BF16 inner solves) and trajectory, against
the oracle (eo.py)."""
import sys

import numpy as np
import pytest

import lgt_inputs as li
from oracle import eo, force, md

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


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 4, 8), (2, 2, 2, 4)])
@pytest.mark.parametrize("dagger", [False, True])
def test_schur_dslash(lgt, dims, dagger, margin):
    u, psi = li.random_links(dims, 0.5, 3), li.gaussian_spinor(dims, 4)
    k = 0.13
    psi_o = eo.parity_mask(dims, 1) * psi
    ref = (eo.schur_dag if dagger else eo.schur)(u, psi_o, k)
    lat = lgt.Lattice(dims)
    got = to_host(lat.schur_dslash(to_dev(u), to_dev(psi), k, dagger))  # even sites of psi are ignored
    margin("rel_err(got, ref)", rel_err(got, ref), 1e-14)


@pytest.mark.parametrize("precision", ["fp64", "mixed_fp32", "mixed_bf16"])
def test_eo_force_and_action(lgt, precision, margin):
    dims = (4, 4, 4, 4)
    u, eta = li.random_links(dims, 0.5, 101), li.gaussian_spinor(dims, 102)
    k = 0.12
    eta_o = eo.parity_mask(dims, 1) * eta
    phi_o = eo.schur_dag(u, eta_o, k)
    ref = eo.eo_force(u, phi_o, k, tol=1e-15)
    lat = lgt.Lattice(dims)
    got, s_eo, st = lat.fermion_force_eo(to_dev(u), to_dev(phi_o), k, lgt.Params(precision=precision, tol=1e-14))
    got = to_host(got)
    say("eo force", precision, st, rel_err(got, ref))
    assert st["true_rel_residual"] <= 1e-14
    margin(f"e/o force vs oracle ({precision}, tol 1e-14)", rel_err(got, ref), 1e-12)
    ee = float(np.vdot(eta_o.ravel(), eta_o.ravel()).real)
    margin("abs(s_eo - ee) / ee", abs(s_eo - ee) / ee, 1e-12)


def test_eo_grad_mode_and_heat_bath_on_gpu(lgt, margin):
    """Heat bath through lgt_schur_dslash, gradient output mode."""
    dims = (6, 4, 4, 8)
    u, eta = li.random_links(dims, 0.4, 111), li.gaussian_spinor(dims, 112)
    k = 0.125
    lat = lgt.Lattice(dims)
    U = to_dev(u)
    phi = lat.schur_dslash(U, to_dev(eta), k, dagger=True)
    g, s_eo, st = lat.fermion_force_eo(U, phi, k, lgt.Params(tol=1e-14), mode="grad")
    ref = eo.eo_grad(u, to_host(phi), k, tol=1e-15)
    margin("e/o gradient vs oracle (FP64, tol 1e-14)", rel_err(to_host(g), ref), 1e-12)
    eta_o = eo.parity_mask(dims, 1) * eta
    ee = float(np.vdot(eta_o.ravel(), eta_o.ravel()).real)
    margin("abs(s_eo - ee) / ee", abs(s_eo - ee) / ee, 1e-12)


@pytest.mark.parametrize("n_inner", [1, 3])
def test_eo_trajectory_vs_oracle(lgt, n_inner, margin):
    dims = (4, 4, 4, 4)
    u, eta, p = li.random_links(dims, 0.5, 121), li.gaussian_spinor(dims, 122), li.random_momenta(dims, 123)
    beta, k, dt, n = 5.7, 0.12, 0.1, 2
    phi_o = eo.schur_dag(u, eo.parity_mask(dims, 1) * eta, k)
    u1, p1, dh_ref = md.sw_trajectory_dh(u, p, phi_o, beta, k, dt, n, n_inner, tol=1e-15, eo=True)
    lat = lgt.Lattice(dims)
    U, P = to_dev(u), to_dev(p)
    dh, st = lat.md_step_eo(U, P, to_dev(phi_o), beta, k, dt, n, n_inner, lgt.Params(tol=1e-14))
    say("eo md", n_inner, dh, dh_ref, st)
    margin(f"e/o trajectory U vs oracle (n_inner {n_inner})", rel_err(to_host(U), u1), 1e-13)
    margin(f"e/o trajectory P vs oracle (n_inner {n_inner}, FP64, tol 1e-14)", rel_err(to_host(P), p1), 1e-12)
    assert abs(dh - dh_ref) < 1e-9 * max(1.0, abs(dh_ref))


def test_eo_force_full_size_mixed_matches_fp64(lgt, margin):
    """16^4: mixed and FP64 inner solves give the same force at the FP64 residual."""
    c = li.config(2)
    dims, k = c["dims"], c["kappa"]
    lat = lgt.Lattice(dims)
    U = to_dev(li.random_links(dims, c["eps"], c["seeds"]["links"]))
    phi = lat.schur_dslash(U, to_dev(li.gaussian_spinor(dims, c["seeds"]["eta"])), k, dagger=True)
    f64, s64, st64 = lat.fermion_force_eo(U, phi, k, lgt.Params(tol=1e-12))
    f32, s32, st32 = lat.fermion_force_eo(U, phi, k, lgt.Params(precision="mixed_fp32", tol=1e-12))
    say("eo 16^4", st64, st32)
    margin("rel_err(to_host(f32), to_host(f64))", rel_err(to_host(f32), to_host(f64)), 1e-9)
    margin("abs(s32 - s64) / abs(s64)", abs(s32 - s64) / abs(s64), 1e-12)
