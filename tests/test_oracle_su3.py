"""Pins of the oracle's group/algebra helpers and gamma matrices (CPU)."""
import numpy as np
import scipy.linalg

import lgt_inputs as li
from oracle import su3
from oracle.dirac import GAMMA, GAMMA5


def test_clifford_algebra():
    for m in range(4):
        assert np.allclose(GAMMA[m], GAMMA[m].conj().T)          # Hermitian
        for n in range(4):
            ac = GAMMA[m] @ GAMMA[n] + GAMMA[n] @ GAMMA[m]
            assert np.array_equal(ac, 2.0 * (m == n) * np.eye(4))
        assert np.allclose(GAMMA5 @ GAMMA[m] + GAMMA[m] @ GAMMA5, 0)


def test_gamma5_chiral_diagonal():
    assert np.array_equal(GAMMA5, np.diag([1, 1, -1, -1]).astype(complex))


def test_generators_normalisation_and_structure_constant():
    t = su3.T
    gram = np.einsum("aij,bji->ab", t, t)
    assert np.allclose(gram, 0.5 * np.eye(8), atol=1e-15)
    # [T1, T2] = i f_123 T3 with f_123 = 1
    assert np.allclose(t[0] @ t[1] - t[1] @ t[0], 1j * t[2])
    for a in range(8):
        assert abs(np.trace(t[a])) < 1e-15
        assert np.allclose(t[a], t[a].conj().T)


def test_projection_properties():
    rng = np.random.default_rng(7)
    a = rng.standard_normal((50, 3, 3)) + 1j * rng.standard_normal((50, 3, 3))
    p = su3.project_su(a)
    assert np.allclose(p, -su3.dag(p), atol=1e-15)             # anti-Hermitian
    assert np.allclose(su3.trace(p), 0, atol=1e-15)            # traceless
    assert np.allclose(su3.project_su(su3.dag(a)), -p)         # P[A^dag] = -P[A] (Sec. S2)
    assert np.allclose(su3.project_su(p), p)                   # idempotent on su(3)
    h = a + su3.dag(a)
    assert np.allclose(su3.project_su(h), 0, atol=1e-15)       # Hermitian part dropped
    # identity part dropped
    assert np.allclose(su3.project_su(a + 3.7j * np.eye(3)), p)


def test_expm_matches_library_and_diagonal_closed_form():
    rng = np.random.default_rng(3)
    c = rng.standard_normal((20, 8))
    x = su3.from_coeffs(0.7 * c)
    e = su3.expm_antihermitian(x)
    for k in range(20):
        assert np.allclose(e[k], scipy.linalg.expm(x[k]), atol=1e-14)
    d = np.diag([0.3j, -0.1j, -0.2j])
    assert np.allclose(su3.expm_antihermitian(d), np.diag(np.exp([0.3j, -0.1j, -0.2j])), atol=1e-15)
    assert su3.unitarity_defect(e) < 1e-14
    assert np.allclose(np.linalg.det(e), 1.0, atol=1e-14)


def test_coeff_round_trip():
    rng = np.random.default_rng(4)
    c = rng.standard_normal((10, 8))
    assert np.allclose(su3.algebra_coeffs(su3.from_coeffs(c)), c, atol=1e-14)


def test_reunitarize():
    u = li.random_links((2, 2, 2, 2), 0.8, 11)
    assert np.allclose(su3.reunitarize(u), u, atol=1e-14)          # fixed point on SU(3)
    rng = np.random.default_rng(5)
    noisy = u + 1e-6 * (rng.standard_normal(u.shape) + 1j * rng.standard_normal(u.shape))
    r = su3.reunitarize(noisy)
    assert su3.unitarity_defect(r) < 1e-14
    assert np.allclose(np.linalg.det(r), 1.0, atol=1e-14)
    assert np.max(np.abs(r - u)) < 1e-5


def test_input_links_are_su3_and_normalised():
    u = li.random_links((4, 4, 4, 4), 0.3, 201)
    assert su3.unitarity_defect(u) < 1e-14
    assert np.allclose(np.linalg.det(u), 1.0, atol=1e-14)
    # with T_a = lambda_a/2 and c_a ~ N(0,1): E[Re tr U / 3] = 1 - eps^2 * sum_a tr(T_a^2)/3 / 2 + ...
    m = np.mean(np.real(np.trace(u, axis1=-2, axis2=-1))) / 3
    assert abs(m - (1 - 0.3 ** 2 * 4 / 2 / 3)) < 5e-3
