"""Pins of the oracle's even/odd-preconditioned pseudofermion action (CPU)."""
import numpy as np
import pytest

import lgt_inputs as li
from oracle import dirac, eo, force

DIMS = (2, 2, 2, 4)


@pytest.fixture(scope="module")
def f():
    u = li.random_links(DIMS, 0.5, 11)
    eta = li.gaussian_spinor(DIMS, 12)
    odd = eo.parity_mask(DIMS, 1)
    return u, odd * eta, odd


def _odd_indices():
    lx, ly, lz, lt = DIMS
    idx = []
    for t in range(lt):
        for z in range(lz):
            for y in range(ly):
                for x in range(lx):
                    if (x + y + z + t) % 2 == 1:
                        s = dirac.site_index(DIMS, x, y, z, t)
                        idx.extend(range(12 * s, 12 * s + 12))
    return np.array(idx)


def _schur_matrix(u, kappa):
    """Columns: Dhat applied to the odd-site unit vectors, in dense index order."""
    odd = _odd_indices()
    lx, ly, lz, lt = DIMS
    cols = []
    for j in odd:
        e = np.zeros(12 * lx * ly * lz * lt, dtype=np.complex128)
        e[j] = 1.0
        v = eo.schur(u, e.reshape((lt, lz, ly, lx, 4, 3)), kappa).ravel()
        cols.append(v[odd])
    return np.array(cols).T


def test_schur_is_the_schur_complement_of_the_dense_operator(f):
    """Dhat = D_oo - D_oe D_ee^-1 D_eo with D from the loop-built dense matrix."""
    u, _, _ = f
    k = 0.13
    d = dirac.dense_dirac(u, k)
    odd = _odd_indices()
    even = np.setdiff1d(np.arange(d.shape[0]), odd)
    ref = d[np.ix_(odd, odd)] - d[np.ix_(odd, even)] @ np.linalg.solve(d[np.ix_(even, even)], d[np.ix_(even, odd)])
    assert np.abs(_schur_matrix(u, k) - ref).max() < 1e-13


def test_same_determinant_as_the_unpreconditioned_operator(f):
    u, _, _ = f
    k = 0.13
    s_full, l_full = np.linalg.slogdet(dirac.dense_dirac(u, k))
    s_eo, l_eo = np.linalg.slogdet(_schur_matrix(u, k))
    assert abs(l_full - l_eo) < 1e-11
    assert abs(s_full - s_eo) < 1e-11


def test_schur_dagger_is_the_adjoint(f):
    u, eta_o, odd = f
    k = 0.12
    b = odd * li.gaussian_spinor(DIMS, 13)
    lhs = np.vdot(b.ravel(), eo.schur(u, eta_o, k).ravel())
    rhs = np.vdot(eo.schur_dag(u, b, k).ravel(), eta_o.ravel())
    assert abs(lhs - rhs) < 1e-13


def test_heat_bath_action_equals_eta_norm(f):
    u, eta_o, _ = f
    k = 0.12
    phi_o = eo.schur_dag(u, eta_o, k)
    s = eo.eo_action(u, phi_o, k)
    ee = float(np.vdot(eta_o.ravel(), eta_o.ravel()).real)
    assert abs(s - ee) / ee < 1e-12


def test_gradient_against_component_differences(f):
    u, _, odd = f
    k = 0.12
    phi_o = odd * li.gaussian_spinor(DIMS, 14)  # any odd-site field
    g = eo.eo_grad(u, phi_o, k)
    act = lambda v: eo.eo_action(v, phi_o, k)  # noqa: E731
    for site, mu, i, j in [((0, 0, 0, 0), 0, 0, 1), ((1, 1, 0, 1), 3, 2, 0), ((3, 0, 1, 0), 2, 1, 1)]:
        re = force.component_fd(act, u, site, mu, i, j, False)
        im = force.component_fd(act, u, site, mu, i, j, True)
        assert abs(g[site + (mu, i, j)] - (re + 1j * im)) < 1e-6 * max(1.0, abs(g[site + (mu, i, j)]))


def test_force_against_lie_differences(f):
    u, eta_o, _ = f
    k = 0.12
    phi_o = eo.schur_dag(u, eta_o, k)
    fo = eo.eo_force(u, phi_o, k)
    d = force.lie_derivatives(fo)
    act = lambda v: eo.eo_action(v, phi_o, k)  # noqa: E731
    for site, mu, a in [((0, 1, 0, 1), 1, 0), ((2, 0, 1, 1), 3, 5), ((1, 1, 1, 0), 0, 7)]:
        assert abs(d[site + (mu, a)] - force.lie_fd(act, u, site, mu, a)) < 1e-6


def test_eo_trajectory_reversible_and_second_order(f):
    from oracle import md
    u, eta_o, _ = f
    k = 0.12
    phi_o = eo.schur_dag(u, eta_o, k)
    p = li.random_momenta(DIMS, 15)
    u1, p1 = md.sexton_weingarten(u, p, phi_o, 5.7, k, 0.1, 3, 2, tol=1e-14, eo=True)
    u2, p2 = md.sexton_weingarten(u1, -p1, phi_o, 5.7, k, 0.1, 3, 2, tol=1e-14, eo=True)
    assert np.abs(u2 - u).max() < 1e-11 and np.abs(p2 + p).max() < 1e-10
    dh = [md.sw_trajectory_dh(u, p, phi_o, 5.7, k, 0.5 / n, n, 1, tol=1e-14, eo=True)[2] for n in (8, 16)]
    assert 3.5 < dh[0] / dh[1] < 4.5


@pytest.mark.parametrize("shift", [0.0, 0.05, 0.7])
def test_shifted_solve_against_dense(f, shift):
    """(Dhat^dag Dhat + shift) x = phi_o against numpy.linalg.solve of the dense Schur matrix."""
    u, eta_o, _ = f
    k = 0.13
    m = _schur_matrix(u, k)
    odd = _odd_indices()
    b = eta_o.ravel()[odd]
    ref = np.linalg.solve(m.conj().T @ m + shift * np.eye(m.shape[0]), b)
    x = eo.solve_normal(u, eta_o, k, shift=shift, tol=1e-14)
    assert np.abs(x.ravel()[odd] - ref).max() < 1e-11 * np.abs(ref).max()
    assert np.abs(np.delete(x.ravel(), odd)).max() == 0.0  # stays on the odd sites


def test_shifted_solve_large_shift_limit(f):
    """(A + s)^-1 phi = phi/s - A phi/s^2 + O(s^-3): at s = 1e6 the first two
    terms of the Neumann series fix x to ~1e-12 relative."""
    u, eta_o, _ = f
    k = 0.13
    s = 1e6
    x = eo.solve_normal(u, eta_o, k, shift=s, tol=1e-15)
    a_eta = eo.schur_dag(u, eo.schur(u, eta_o, k), k)
    approx = eta_o / s - a_eta / s**2
    assert np.abs(x - approx).max() < 1e-11 * np.abs(eta_o / s).max()


# ---- rational (RHMC) action ---------------------------------------------------

RAT = dict(a0=0.3, shifts=(0.0, 0.05, 0.6, 4.0), residues=(0.7, -0.2, 1.3, 2.1))


def _dense_schur(u, k):
    d = dirac.dense_dirac(u, k)
    odd = _odd_indices()
    even = np.setdiff1d(np.arange(d.shape[0]), odd)
    return d[np.ix_(odd, odd)] - d[np.ix_(odd, even)] @ np.linalg.solve(d[np.ix_(even, even)], d[np.ix_(even, odd)])


def test_rational_action_against_dense(f):
    """S_R = phi^dag [a0 + sum_i a_i (A + sigma_i)^-1] phi with A built from the
    Schur complement of the loop-built dense D (no oracle operator involved)."""
    u, eta_o, _ = f
    k = 0.125
    phi_o = eo.schur_dag(u, eta_o, k)
    m = _dense_schur(u, k)
    a = m.conj().T @ m
    b = phi_o.ravel()[_odd_indices()]
    ref = RAT["a0"] * np.vdot(b, b).real
    for sig, r in zip(RAT["shifts"], RAT["residues"]):
        ref += r * np.vdot(b, np.linalg.solve(a + sig * np.eye(a.shape[0]), b)).real
    got = eo.rational_action(u, phi_o, k, RAT["a0"], RAT["shifts"], RAT["residues"])
    assert abs(got - ref) < 1e-11 * abs(ref)


def test_rational_force_lie_derivative(f):
    u, eta_o, _ = f
    k = 0.125
    phi_o = eo.schur_dag(u, eta_o, k)
    fo = eo.rational_force(u, phi_o, k, RAT["a0"], RAT["shifts"], RAT["residues"])
    d = force.lie_derivatives(fo)
    act = lambda v: eo.rational_action(v, phi_o, k, RAT["a0"], RAT["shifts"], RAT["residues"])  # noqa: E731
    for site, mu, a in [((0, 1, 0, 1), 1, 0), ((3, 0, 1, 1), 3, 5), ((1, 1, 1, 0), 0, 7), ((2, 1, 0, 0), 2, 2)]:
        fd = force.lie_fd(act, u, site, mu, a)
        assert abs(d[site + (mu, a)] - fd) < 1e-6 * max(1.0, abs(fd))


def test_rational_force_of_a_large_shift_vanishes_as_its_square(f):
    """a (A + s)^-1 = a/s - a A/s^2 + ...: the force of one term falls off as
    1/s^2 (doubling s quarters it)."""
    u, eta_o, _ = f
    k = 0.125
    phi_o = eo.schur_dag(u, eta_o, k)
    f1 = eo.rational_force(u, phi_o, k, 0.0, (1e4,), (1.0,))
    f2 = eo.rational_force(u, phi_o, k, 0.0, (2e4,), (1.0,))
    ratio = np.linalg.norm(f1.ravel()) / np.linalg.norm(f2.ravel())
    assert abs(ratio - 4.0) < 2e-3
