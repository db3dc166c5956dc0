"""Dynamics on the GPU at the headline size, and the layout round trip.

* Canonical <-> packed layout: smearing zero levels and D at kappa = 0 give
  back their inputs bit for bit (ragged 6^4: 648 sites per parity).
* 16^4 (the headline workload's links, momenta and pseudofermion): the
  leapfrog is reversible to rounding, and the energy violation of one
  trajectory falls as dt^2 (second-order integrator, Sec. III B).
* A 4^4 HMC ensemble in equilibrium satisfies <exp(-Delta H)> = 1 (area
  preservation and reversibility of the integrator)."""
import math
import sys

import numpy as np
import pytest

import lgt_inputs as li

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


def test_layout_round_trip(lgt):
    dims = (6, 6, 6, 6)
    u, psi = li.random_links(dims, 0.7, 301), li.gaussian_spinor(dims, 302)
    lat = lgt.Lattice(dims)
    U, PSI = to_dev(u), to_dev(psi)
    assert np.array_equal(to_host(lat.stout_smear(U, 0.1, 0)), u)
    assert np.array_equal(to_host(lat.dslash(U, PSI, 0.0)), psi)


@pytest.fixture(scope="module")
def c2(lgt):
    c = li.config(2)
    dims = c["dims"]
    u = li.random_links(dims, c["eps"], c["seeds"]["links"])
    p = li.random_momenta(dims, c["seeds"]["mom"])
    lat = lgt.Lattice(dims)
    U = to_dev(u)
    phi = lat.dslash(U, to_dev(li.gaussian_spinor(dims, c["seeds"]["eta"])), c["kappa"], dagger=True)
    return dict(c=c, u=u, p=p, lat=lat, phi=phi)


def test_reversibility_16(lgt, c2):
    c, lat = c2["c"], c2["lat"]
    prm = lgt.Params(precision="fp64", tol=1e-12)
    U, P = to_dev(c2["u"]), to_dev(c2["p"])
    dh, _ = lat.md_step(U, P, c2["phi"], c["beta"], c["kappa"], 0.02, 5, prm)
    P.neg_()
    dh_back, _ = lat.md_step(U, P, c2["phi"], c["beta"], c["kappa"], 0.02, 5, prm)
    eu = rel_err(to_host(U), c2["u"])
    ep = rel_err(-to_host(P), c2["p"])
    say("16^4 reversibility", dh, dh_back, eu, ep)
    assert eu < 1e-12 and ep < 1e-11
    assert abs(dh + dh_back) < 1e-6 * max(1.0, abs(dh))


def test_delta_h_scales_as_dt_squared_16(lgt, c2):
    c, lat = c2["c"], c2["lat"]
    prm = lgt.Params(precision="fp64", tol=1e-12)
    tau = 0.1
    dh = []
    for n in (4, 8, 16):
        U, P = to_dev(c2["u"]), to_dev(c2["p"])
        d, _ = lat.md_step(U, P, c2["phi"], c["beta"], c["kappa"], tau / n, n, prm)
        dh.append(d)
    r1, r2 = dh[0] / dh[1], dh[1] / dh[2]
    say("16^4 dH", dh, r1, r2)
    assert 3.6 < r1 < 4.4 and 3.8 < r2 < 4.2


def test_exp_minus_delta_h_is_one_in_equilibrium(lgt):
    from paper_2602_20516_amd.hmc import HMC, HMCRecord
    dims = (4, 4, 4, 4)
    lat = lgt.Lattice(dims)
    hmc = HMC(lat, beta=5.7, kappa=0.12, dt=0.05, nsteps=20, params=lgt.Params(precision="mixed_fp32", tol=1e-11),
              seed=311)
    U = to_dev(li.random_links(dims, 0.5, 312))
    for _ in range(50):  # thermalisation: every trajectory kept, so the ordered start relaxes
        U = hmc.update(U, metropolis=False)
    rec = HMCRecord()
    for _ in range(200):
        U = hmc.update(U, rec)
    w = np.exp(-np.array(rec.dH))
    mean, err = float(w.mean()), float(w.std() / math.sqrt(len(w)))
    say("<exp(-dH)>", mean, "+-", err, "acceptance", rec.summary()["acceptance"])
    assert abs(mean - 1.0) < max(0.06, 4 * err)
