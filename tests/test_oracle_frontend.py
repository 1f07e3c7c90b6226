"""Pins of the oracle's Appendix A front end (oracle/frontend.py): the
Chebyshev interpolation, the separable approximations of Q and omega for
the thick quarter annulus, and the Tucker matrix and vector they induce.

* Chebyshev interpolation on t Lobatto points reproduces polynomials of
  degree < t; the coefficient tensor of a product of Chebyshev polynomials
  is a unit tensor;
* for the annulus map, Q = det(J) J^{-1} J^{-T} = diag(pi r / 2, 2 / (pi r),
  pi r / 2) with r = 1 + eta_1 (closed form): the approximation has the
  ranks the paper reports for this domain, (1, 1, 1) on the diagonal and
  none off it, and matches the closed form;
* the approximation of omega meets the paper's acceptance test (10 eps at
  Halton points);
* f = -Laplace u for the manufactured solution (finite differences);
* the Tucker matrix of eq. matrix_CP equals the stiffness matrix of the
  mapped Laplacian computed by brute-force 3D quadrature of
  grad B_i^T Q grad B_j with the exact Q (tiny size);
* the Galerkin solution with that matrix and rhs converges to the
  manufactured solution under refinement.
"""
import numpy as np
import pytest

from oracle import bspline, fullpcg
from oracle import frontend as fe
from oracle.tucker import Tucker


def test_chebyshev_interpolation_is_exact_for_polynomials():
    t = 9
    x = fe.cheb_points(t)
    E1, E2, E3 = np.meshgrid(x, x, x, indexing="ij")
    T = lambda m, e: np.cos(m * np.arccos(np.clip(2 * e - 1, -1, 1)))
    C = fe.cheb_coefficients(T(2, E1) * T(1, E2) * T(5, E3))
    ref = np.zeros((t, t, t))
    ref[2, 1, 5] = 1.0
    assert np.abs(C - ref).max() <= 1e-12
    rng = np.random.default_rng(1)
    c = rng.standard_normal(t)
    y = rng.uniform(0, 1, 20)
    vals = fe.cheb_eval(c, x)
    V = np.stack([fe.cheb_eval(np.eye(t)[m], x) for m in range(t)], axis=1)
    np.testing.assert_allclose(np.linalg.solve(V, vals), c, atol=1e-12)
    np.testing.assert_allclose(fe.cheb_eval(c, y), np.polynomial.chebyshev.chebval(2 * y - 1, c), atol=1e-13)


def test_annulus_q_has_the_papers_ranks_and_closed_form():
    op, ranks = fe.operator(4, 2, fe.annulus_jacobian, 17, 1e-10)
    for k in range(3):
        for l in range(3):
            assert ranks[(k, l)] == ((1, 1, 1) if k == l else (0, 0, 0)), (k, l, ranks[(k, l)])
    H = fe.halton(200)
    r = 1.0 + H[:, 0]
    closed = [0.5 * np.pi * r, 2.0 / (np.pi * r), 0.5 * np.pi * r]
    for k in range(3):
        g = fe.separable(fe.q_entry(fe.annulus_jacobian, k, k), 17, 1e-10)
        app = fe.evaluate(g, H[:, 0], H[:, 1], H[:, 2])
        assert np.abs(app - closed[k]).max() <= 1e-9 * np.abs(closed[k]).max(), k


@pytest.mark.parametrize("eps", [1e-4, 1e-6])
def test_omega_meets_the_halton_acceptance_test(eps):
    t = 48
    g = fe.separable(fe.annulus_omega, t, eps)
    scale = np.abs(fe.grid_values(fe.annulus_omega, t)).max()
    H = fe.halton(1000)
    err = np.abs(fe.evaluate(g, H[:, 0], H[:, 1], H[:, 2]) - fe.annulus_omega(H[:, 0], H[:, 1], H[:, 2])).max()
    assert err <= 10 * eps * scale, (err, scale)
    assert max(g.core.shape) < t   # a genuine compression


def test_load_is_minus_laplacian_of_the_solution():
    rng = np.random.default_rng(3)
    P = rng.uniform(-2, 2, (10, 3))
    h = 1e-4
    lap = 0.0
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        lap = lap + (fe.annulus_solution(*(P + e).T) - 2 * fe.annulus_solution(*P.T)
                     + fe.annulus_solution(*(P - e).T)) / h ** 2
    f = fe.annulus_load(*P.T)
    assert np.abs(f + lap).max() <= 1e-5 * np.abs(f).max()


def _brute_force_stiffness(n_el, p, nq=8, jacobian=fe.annulus_jacobian):
    """int grad B_i^T Q grad B_j over [0,1]^3 with the exact Q, tensor Gauss."""
    kn = bspline.open_knots(n_el, p)
    x, w = bspline.gauss_points(n_el, nq)
    B = [bspline.basis(kn, p, x, d)[:, 1:-1] for d in (0, 1)]   # (points, n)
    n = B[0].shape[1]
    E1, E2, E3 = np.meshgrid(x, x, x, indexing="ij")
    W = w[:, None, None] * w[None, :, None] * w[None, None, :]
    J = jacobian(E1, E2, E3)
    Ji = np.linalg.inv(J)
    Q = np.linalg.det(J)[..., None, None] * np.einsum("...ka,...la->...kl", Ji, Ji)
    A = np.zeros((n ** 3, n ** 3))
    for k in range(3):
        for l in range(3):
            # dB_i/d eta_l dB_j/d eta_k Q_kl: factors per direction
            Qw = Q[..., k, l] * W
            Fi = [B[int(s == l)] for s in range(3)]
            Fj = [B[int(s == k)] for s in range(3)]
            T = np.einsum("abc,ai,bj,ck,ax,by,cz->ijkxyz", Qw, Fi[0], Fi[1], Fi[2], Fj[0], Fj[1], Fj[2],
                          optimize=True)
            # vec order: index 1 fastest
            A += T.transpose(2, 1, 0, 5, 4, 3).reshape(n ** 3, n ** 3)
    return A


def test_operator_equals_brute_force_quadrature():
    n_el, p = 3, 2
    op, _ = fe.operator(n_el, p, fe.annulus_jacobian, 17, 1e-12)
    A = op.dense()
    Ab = _brute_force_stiffness(n_el, p)
    assert np.abs(A - Ab).max() <= 1e-9 * np.abs(Ab).max()
    assert np.abs(A - A.T).max() <= 1e-12 * np.abs(A).max()


def _solution_error(n_el, p):
    """Galerkin solution (sparse direct solve of the Tucker matrix assembled
    as a sum of Kronecker products) against the manufactured solution at
    9^3 interior points of the parametric cube, max-norm relative error."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    t, eps = 33, 1e-10
    op, _ = fe.operator(n_el, p, fe.annulus_jacobian, t, eps)
    f = fe.rhs(n_el, p, fe.annulus_omega, 64, eps)
    n = n_el + p - 2
    A = sum(c * sp.kron(sp.csr_matrix(op.mats[2][i3]), sp.kron(sp.csr_matrix(op.mats[1][i2]),
                                                                sp.csr_matrix(op.mats[0][i1])))
            for i1, i2, i3, c in op.nnz)
    X = spla.spsolve(A.tocsc(), f.full().reshape(-1, order="F")).reshape((n, n, n), order="F")
    e = np.linspace(0.05, 0.95, 9)
    E1, E2, E3 = np.meshgrid(e, e, e, indexing="ij")
    Bs = bspline.dirichlet_basis_at(n_el, p, e)
    uh = np.einsum("abc,ia,jb,kc->ijk", X, Bs, Bs, Bs)
    u = fe.annulus_solution(*fe.annulus_map(E1, E2, E3))
    return np.abs(uh - u).max() / np.abs(u).max()


def test_galerkin_solution_converges_to_the_manufactured_one():
    """p = 2: the error falls by more than 4 from n_el = 8 to 16 (measured
    0.59 -> 0.058; h^3 asymptotically) and is below 0.1 at n_el = 16."""
    e8, e16 = _solution_error(8, 2), _solution_error(16, 2)
    assert e16 < e8 / 4, (e8, e16)
    assert e16 < 0.1, e16


def test_annulus_samples_match_the_oracle():
    """The seeded-input module's closed-form samples of Q and omega (inputs of
    the library's front end) against the oracle's, computed from the map's
    Jacobian."""
    import workloads
    t = 9
    q, omega, u = workloads.annulus_samples(t)
    for k in range(3):
        for l in range(3):
            ref = fe.grid_values(fe.q_entry(fe.annulus_jacobian, k, l), t)
            assert np.abs(q[(k, l)] - ref).max() <= 1e-13 * 4.0, (k, l)
    ref = fe.grid_values(fe.annulus_omega, t)
    assert np.abs(omega - ref).max() <= 1e-12 * np.abs(ref).max()
    P = np.random.default_rng(0).uniform(-2, 2, (20, 3))
    np.testing.assert_allclose(u(*P.T), fe.annulus_solution(*P.T), rtol=0, atol=1e-14)


def test_front_end_chebyshev_transform_matches_the_vandermonde_inverse():
    """The library front end's values-to-coefficients map (a type-I cosine
    transform) against the inverse of the Chebyshev-Vandermonde matrix."""
    from numpy.polynomial import chebyshev
    from paper_2306_00632_amd import geometry
    for t in (2, 5, 16):
        V = chebyshev.chebvander(2.0 * fe.cheb_points(t) - 1.0, t - 1)
        np.testing.assert_allclose(geometry.cheb_transform(t), np.linalg.inv(V), atol=1e-12)
    np.testing.assert_allclose(geometry.cheb_points(7), fe.cheb_points(7), atol=0)


def test_shell_jacobian_matches_finite_differences():
    """The shell's analytic Jacobian against central differences of its map,
    and its image on the spheres of radii 1 and 2."""
    P = np.random.default_rng(5).uniform(0.05, 0.95, (12, 3))
    J = fe.shell_jacobian(*P.T)
    h = 1e-6
    for b in range(3):
        e = np.zeros(3)
        e[b] = h
        fd = (np.stack(fe.shell_map(*(P + e).T), -1) - np.stack(fe.shell_map(*(P - e).T), -1)) / (2 * h)
        assert np.abs(J[:, :, b] - fd).max() <= 1e-8, b
    for r0, e1 in ((1.0, 0.0), (2.0, 1.0)):
        X = np.stack(fe.shell_map(np.full(12, e1), P[:, 1], P[:, 2]), -1)
        np.testing.assert_allclose(np.linalg.norm(X, axis=1), r0, atol=1e-14)


def test_shell_operator_and_samples():
    """The shell's Tucker matrix equals brute-force quadrature of
    grad B_i^T Q grad B_j (a geometry that is not a tensor product and not
    orthogonal: Q_23 != 0 gets a nonzero rank, Q_1a none), and the seeded
    closed-form samples of Q and omega match the oracle's from the Jacobian."""
    import workloads
    op, ranks = fe.operator(3, 2, fe.shell_jacobian, 33, 1e-12)
    assert ranks[(0, 1)] == ranks[(1, 0)] == ranks[(0, 2)] == (0, 0, 0)
    assert ranks[(1, 2)][0] == 1 and min(ranks[(1, 2)][1:]) >= 2
    A = op.dense()
    Ab = _brute_force_stiffness(3, 2, nq=10, jacobian=fe.shell_jacobian)
    assert np.abs(A - Ab).max() <= 1e-9 * np.abs(Ab).max()
    t = 9
    q, omega = workloads.shell_samples(t)
    for k in range(3):
        for l in range(3):
            ref = fe.grid_values(fe.q_entry(fe.shell_jacobian, k, l), t)
            assert np.abs(q[(k, l)] - ref).max() <= 1e-13 * 4.0, (k, l)
    ref = fe.grid_values(fe.shell_omega, t)
    assert np.abs(omega - ref).max() <= 1e-13 * np.abs(ref).max()


def test_shell_operator_is_exactly_symmetric():
    """With the mirrored approximation of Q's lower triangle the Tucker
    matrix of a non-diagonal Q is symmetric to rounding even at a loose eps
    (separate approximations of Q_23 and Q_32 would differ at the eps
    level)."""
    op, _ = fe.operator(4, 3, fe.shell_jacobian, 17, 1e-4)
    A = op.dense()
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
