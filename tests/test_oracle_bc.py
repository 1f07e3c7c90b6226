"""Pins of the oracle's boundary-condition support (oracle/bc.py, the bc
flags of oracle/bspline.py and oracle/fd.py): Neumann ends of Appendix B
and the non-homogeneous Dirichlet system of the remark closing Sec. 3.

Each check is fixed by the mathematics, not by the oracle's own formulas:
* with Neumann at both ends the constants are in the space, so the
  stiffness matrix annihilates the vector of ones, and the mass matrix's
  row sums are the basis integrals (t_{i+p+1} - t_i)/(p+1);
* the low generalized eigenvalues of (K, M) converge to the continuous
  Laplacian's, ((j - k0/2 - k1/2) pi)^2 (the closed form Appendix B uses
  for its approximation), at the rate h^(2p) of spline eigenvalues;
* the Greville abscissae reproduce x;
* a linear function is in the spline space and harmonic, so the discrete
  solution with its Dirichlet data, homogeneous Neumann data where its
  normal derivative vanishes and f = 0 is the function itself, to
  rounding: u = 1 + 3z with Dirichlet at z = 0, 1 and Neumann on the other
  faces, and u = 1 with Dirichlet at z = 0 only;
* the exact FD of Algorithm 3 on the BC spaces inverts the Laplacian.
"""
import numpy as np
import pytest

import workloads as W
from oracle import bc as obc
from oracle import bspline, fd
from oracle.fullpcg import dense_solve
from oracle.tucker import Tucker

BCS = [(0, 0), (1, 1), (1, 0), (0, 1)]


@pytest.mark.parametrize("p", [2, 3, 4])
def test_neumann_stiffness_annihilates_constants(p):
    rng = np.random.default_rng(p)
    for _ in range(3):
        wgt = (1.0, 0.5, *rng.uniform(0, 2, 2))
        K = bspline.matrix(12, p, "stiff", wgt, bc=(1, 1))
        assert K.shape == (12 + p, 12 + p)
        assert np.abs(K @ np.ones(K.shape[0])).max() <= 1e-12 * np.abs(K).max()


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_neumann_mass_row_sums_are_basis_integrals(p):
    n_el = 9
    M = bspline.matrix(n_el, p, "mass", bc=(1, 1))
    t = bspline.open_knots(n_el, p)
    ref = np.array([(t[i + p + 1] - t[i]) / (p + 1) for i in range(n_el + p)])
    np.testing.assert_allclose(M.sum(axis=1), ref, rtol=1e-13, atol=0)


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("p", [2, 3])
def test_low_eigenvalues_match_the_continuous_laplacian(bc, p):
    n_el = 64
    K = bspline.matrix(n_el, p, "stiff", bc=bc)
    M = bspline.matrix(n_el, p, "mass", bc=bc)
    assert K.shape[0] == n_el + p - 2 + sum(bc)
    lam = np.sort(np.linalg.eigvals(np.linalg.solve(M, K)).real)
    shift = 0.5 * (bc[0] + bc[1])
    for j in range(1, 4):
        exact = ((j - shift) * np.pi) ** 2
        if exact == 0.0:
            assert abs(lam[j - 1]) <= 1e-9
            continue
        # spline eigenvalue error ~ (j pi h)^(2p) relative
        assert abs(lam[j - 1] - exact) <= 10 * (j * np.pi / n_el) ** (2 * p) * exact, (j, lam[j - 1], exact)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_greville_reproduces_x(p):
    n_el = 7
    x = np.linspace(0.0, 1.0, 23)
    B = bspline.basis(bspline.open_knots(n_el, p), p, x, 0)
    np.testing.assert_allclose(B @ bspline.greville(n_el, p), x, atol=1e-14)
    np.testing.assert_allclose(B.sum(axis=1), 1.0, atol=1e-14)


def _dense_bc_solve(w, bcs, g, f=None):
    op = obc.operator(w, bcs)
    rhs = obc.lifted_rhs(w, bcs, g, f)
    return dense_solve(op, rhs.full())


@pytest.mark.parametrize("p", [2, 3])
def test_linear_solution_dirichlet_top_bottom_neumann_sides(p):
    n_el = 5
    w = W.laplace_cube(n_el, p)
    bcs = ((1, 1), (1, 1), (0, 0))
    g = obc.linear_coefficients(n_el, p, (1.0, 0.0, 0.0, 3.0))
    x = _dense_bc_solve(w, bcs, g)
    ref = obc.restrict(g, n_el, p, bcs).full()
    assert x.shape == (n_el + p, n_el + p, n_el + p - 2)
    assert np.abs(x - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("p", [2, 3])
def test_constant_solution_dirichlet_at_one_face(p):
    n_el = 5
    w = W.laplace_cube(n_el, p)
    bcs = ((1, 1), (1, 1), (0, 1))
    g = obc.linear_coefficients(n_el, p, (1.0, 0.0, 0.0, 0.0))
    x = _dense_bc_solve(w, bcs, g)
    assert np.abs(x - 1.0).max() <= 1e-11


def test_lifting_vanishes_for_homogeneous_data_and_is_linear():
    n_el, p = 5, 2
    w = W.laplace_cube(n_el, p)
    bcs = ((1, 0), (0, 0), (0, 1))
    zero = Tucker(np.zeros((1, 1, 1)), [np.ones((n_el + p, 1))] * 3)
    assert np.abs(obc.lifted_rhs(w, bcs, zero).full()).max() == 0.0
    g1 = obc.linear_coefficients(n_el, p, (1.0, 2.0, 0.0, 0.0))
    g2 = obc.linear_coefficients(n_el, p, (0.0, 0.0, -1.0, 0.5))
    g12 = obc.linear_coefficients(n_el, p, (1.0, 2.0, -1.0, 0.5))
    r = [obc.lifted_rhs(w, bcs, g).full() for g in (g1, g2, g12)]
    np.testing.assert_allclose(r[0] + r[1], r[2], atol=1e-12 * np.abs(r[2]).max())


@pytest.mark.parametrize("bcs", [((1, 1), (1, 1), (0, 0)), ((1, 0), (0, 1), (0, 0)), ((0, 0), (1, 1), (0, 1))])
def test_exact_fd_inverts_the_laplacian_on_bc_spaces(bcs):
    n_el, p = 6, 3
    Ks = [bspline.matrix(n_el, p, "stiff", bc=b) for b in bcs]
    Ms = [bspline.matrix(n_el, p, "mass", bc=b) for b in bcs]
    P = fd.ExactFD(Ks, Ms)
    rng = np.random.default_rng(3)
    n = [k.shape[0] for k in Ks]
    X = rng.standard_normal(n)
    w = W.laplace_cube(n_el, p)
    AX = obc.operator(w, bcs).dense() @ X.reshape(-1, order="F")
    Y = P.apply_full(AX.reshape(n, order="F"))
    assert np.abs(Y - X).max() <= 1e-9 * np.abs(X).max()


def test_all_neumann_is_rejected():
    with pytest.raises(ValueError):
        fd.LowRankFD(6, 2, 0.1, exact=True, bcs=((1, 1),) * 3)


def test_workload_linear_data_matches_the_oracle():
    """The input generator of the manufactured runs (workloads) against the
    oracle's construction from its own knot vector and Greville abscissae."""
    for n_el, p in ((5, 2), (16, 3), (9, 5)):
        core, U = W.linear_dirichlet_data(n_el, p, (1.0, -2.0, 0.5, 3.0))
        ref = obc.linear_coefficients(n_el, p, (1.0, -2.0, 0.5, 3.0))
        np.testing.assert_allclose(Tucker(core, U).full(), ref.full(), rtol=0, atol=1e-14)


# --- Appendix B with Neumann ends ---------------------------------------------

@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_appendix_b_structure_with_flags(bc, p):
    """V_h1 has vanishing odd derivatives at Neumann ends and vanishing even
    ones at Dirichlet ends; its dimension equals the number of interpolation
    points (breakpoints without Dirichlet ends for odd p, midpoints for even
    p); the interpolants of sin((j - k0/2 - k1/2) pi x + k0 pi/2) have unit
    M-norm and Lambda1 = ((j - k0/2 - k1/2) pi)^2; V_h2 is M-orthogonal."""
    n_el = 12
    k0, k1 = bc
    Ut, lam, P = fd.approx_eig(n_el, p, bc)
    n, n1, n2 = fd.subspace_dims(n_el, p, bc)
    assert n == n_el + p - 2 + k0 + k1 and Ut.shape == (n, n)
    x = P["x"]
    assert len(x) == n1
    assert np.isclose(x[0], 0.0) == (p % 2 == 1 and k0 == 1)
    assert np.isclose(x[-1], 1.0) == (p % 2 == 1 and k1 == 1)
    kn = bspline.open_knots(n_el, p)
    lo, hi = bspline.dof_range(n_el, p, bc)
    W1 = Ut[:, :n1]
    for end, k in ((0.0, k0), (1.0, k1)):
        orders = range(1, p, 2) if k else range(2, p, 2)
        for d in orders:
            Dd = bspline.basis(kn, p, [end], d)[0, lo:hi]
            assert np.abs(Dd @ W1).max() <= 1e-9 * np.abs(Dd).max() * np.abs(W1).max(), (end, d)
    freq = np.arange(1, n1 + 1) - 0.5 * (k0 + k1)
    sines = np.sin(np.pi * np.outer(x, freq) + 0.5 * np.pi * k0)
    vals = bspline.basis(kn, p, x, 0)[:, lo:hi] @ W1
    # the interpolants reproduce the sines up to their normalisation
    ratio = vals / np.where(np.abs(sines) > 1e-8, sines, np.nan)
    for j in range(n1):
        r = ratio[:, j][~np.isnan(ratio[:, j])]
        assert np.ptp(r) <= 1e-9 * np.abs(r).max(), j
    M = bspline.matrix(n_el, p, "mass", bc=bc)
    np.testing.assert_allclose(np.einsum("ij,ij->j", W1, M @ W1), 1.0, rtol=1e-12)
    np.testing.assert_allclose(lam[:n1], (np.pi * freq) ** 2, rtol=1e-14)
    if n2:
        G = Ut.T @ M @ Ut
        assert np.abs(G[:n1, n1:]).max() < 1e-12
        np.testing.assert_allclose(G[n1:, n1:], np.eye(n2), atol=1e-12)


@pytest.mark.parametrize("p", [2, 3])
def test_appendix_b_flags_iterations_close_to_exact(p):
    """The remark of Sec. 5 with Neumann ends: TPCG with the Appendix B
    eigenpairs takes nearly as many iterations as with the exact ones
    (weighted operator, flags (N,N), (N,D), (D,D), n_el = 16)."""
    from oracle import tpcg as otpcg
    n_el = 16
    bcs = ((1, 1), (1, 0), (0, 0))
    w = W.weighted_cp(n_el, p, 6, 2, 41, 42)
    op = obc.operator(w, bcs)
    n = [n_el + p - 2 + sum(b) for b in bcs]
    f = Tucker(*W.random_tucker(n, (2, 2, 2), 43))
    its = [otpcg.tpcg(op, fd.LowRankFD(n_el, p, 0.1, exact=ex, bcs=bcs), f, tol=1e-6, eps_min=1e-8)[1].iters
           for ex in (False, True)]
    assert abs(its[0] - its[1]) <= max(2, 0.2 * its[1]), its
