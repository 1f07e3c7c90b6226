"""Pins of the oracle's B-spline layer (Sec. 2.1, App. A) against closed forms."""
from math import comb, factorial

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import bspline as bs


def cardinal(d, x):
    """Cardinal B-spline of degree d on [0, d+1] by the truncated-power
    formula N_d(x) = 1/d! sum_i (-1)^i C(d+1, i) (x - i)_+^d (independent of
    the Cox-de Boor recursion)."""
    return sum((-1) ** i * comb(d + 1, i) * max(x - i, 0.0) ** d for i in range(d + 2)) / factorial(d)


def cardinal_dd(d, x):
    """Second derivative of N_d."""
    return sum((-1) ** i * comb(d + 1, i) * max(x - i, 0.0) ** (d - 2) for i in range(d + 2)) / factorial(d - 2)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_partition_of_unity_including_right_end(p):
    kn = bs.open_knots(7, p)
    x = np.concatenate([np.linspace(0, 1, 301), [1.0]])
    B = bs.basis(kn, p, x)
    assert B.shape[1] == 7 + p
    np.testing.assert_allclose(B.sum(axis=1), 1.0, atol=1e-14)
    assert np.all(B >= -1e-15)


@pytest.mark.parametrize("p", [2, 3, 4])
def test_stiffness_annihilates_constants_and_mass_row_sums(p):
    n_el = 9
    kn = bs.open_knots(n_el, p)
    K = bs.matrix_full(n_el, p, "stiff")
    M = bs.matrix_full(n_el, p, "mass")
    np.testing.assert_allclose(K @ np.ones(K.shape[0]), 0.0, atol=1e-11)
    integrals = np.array([(kn[i + p + 1] - kn[i]) / (p + 1) for i in range(n_el + p)])
    np.testing.assert_allclose(M.sum(axis=1), integrals, rtol=1e-13)


@pytest.mark.parametrize("p", [2, 3, 4])
def test_interior_stencils_are_cardinal_autocorrelations(p):
    """Interior rows: M_{i,i+k} = h N_{2p+1}(p+1+k), K_{i,i+k} = -h^{-1} N''_{2p+1}(p+1+k)."""
    n_el = 4 * p + 6
    h = 1.0 / n_el
    M = bs.matrix_full(n_el, p, "mass")
    K = bs.matrix_full(n_el, p, "stiff")
    mid = (n_el + p) // 2
    ks = np.arange(-p, p + 1)
    m_ref = np.array([h * cardinal(2 * p + 1, p + 1 + k) for k in ks])
    k_ref = np.array([-cardinal_dd(2 * p + 1, p + 1 + k) / h for k in ks])
    np.testing.assert_allclose(M[mid, mid - p:mid + p + 1], m_ref, rtol=1e-12)
    np.testing.assert_allclose(K[mid, mid - p:mid + p + 1], k_ref, rtol=1e-11, atol=1e-11)
    # bandwidth p
    assert abs(M[mid, mid + p + 1]) == 0.0 and abs(K[mid, mid - p - 1]) == 0.0


def test_p2_stencil_values_as_fractions():
    n_el = 12
    h = 1.0 / n_el
    M = bs.matrix_full(n_el, 2, "mass")
    mid = 7
    np.testing.assert_allclose(M[mid, mid - 2:mid + 3] / h, np.array([1, 26, 66, 26, 1]) / 120.0, rtol=1e-13)


@pytest.mark.parametrize("p", [2, 3, 4])
def test_dirichlet_matrices_spd_and_smallest_eigenvalue(p):
    errs = []
    for n_el in (8, 16, 32):
        K = bs.matrix(n_el, p, "stiff")
        M = bs.matrix(n_el, p, "mass")
        assert K.shape == (n_el + p - 2,) * 2
        np.testing.assert_allclose(K, K.T, atol=1e-12)
        assert np.linalg.eigvalsh(M).min() > 0
        lam = sla.eigh(K, M, eigvals_only=True)
        errs.append(abs(lam[0] - np.pi ** 2))
    # Galerkin eigenvalue error decays like h^(2p)
    assert np.log2(errs[1] / errs[2]) > 2 * p - 0.5


def test_mixed_matrices_are_antisymmetric_pair():
    """int b_i' b_j + int b_i b_j' = [b_i b_j]_0^1 = 0 on the Dirichlet basis."""
    A = bs.matrix(10, 3, "mixed10")
    B = bs.matrix(10, 3, "mixed01")
    np.testing.assert_allclose(A, B.T, atol=1e-14)
    np.testing.assert_allclose(A + A.T, 0.0, atol=1e-13)


@pytest.mark.parametrize("kind", ["mass", "stiff"])
def test_weighted_quadrature_converged(kind):
    w = (1.0, 0.5, 1.7, 0.3)
    A = bs.matrix(32, 3, kind, w)
    B = bs.matrix(32, 3, kind, w, nq=2 * 3 + 8)
    assert np.abs(A - B).max() <= 1e-13 * np.abs(B).max()


def test_weighted_mass_of_affine_weight_closed_form():
    """With w = c0 + c1 cos(a x + b) and a -> 0 the weight is constant."""
    A = bs.matrix(10, 3, "mass", (2.0, 0.5, 0.0, 0.0))
    B = bs.matrix(10, 3, "mass")
    np.testing.assert_allclose(A, 2.5 * B, rtol=1e-14)


def test_load_vector_of_sine_integrates():
    """sum_i F_i * (coefficients of 1) = int sin(pi x) dx = 2/pi; the constant 1
    has all full-basis coefficients equal to 1."""
    n_el, p = 16, 3
    x, w = bs.gauss_points(n_el, p + 5)
    B = bs.basis(bs.open_knots(n_el, p), p, x)
    F_full = B.T @ (w * np.sin(np.pi * x))
    assert abs(F_full.sum() - 2.0 / np.pi) < 1e-14
    F = bs.load_vector(n_el, p, (0.0, 1.0, np.pi, -0.5 * np.pi))
    np.testing.assert_allclose(F, F_full[1:-1], rtol=1e-14)
