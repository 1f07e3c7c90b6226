"""Pins of the oracle's TPCG (Algorithm 5) against dense solves, the exact
FD solution on the unit cube and a manufactured separable solution."""
import numpy as np
import pytest

import workloads as W
from oracle import bspline, fd, fullpcg, problem, tpcg
from oracle import tucker as T


def solve(w, **kw):
    op = problem.operator(w)
    f = problem.rhs(w)
    prec = fd.LowRankFD(w.n_el, w.p, 0.1)
    x, info = tpcg.tpcg(op, prec, f, tol=w.tol, eps_min=w.eps_min, **kw)
    return op, f, prec, x, info


def test_small_cube_matches_exact_solution():
    """Unit cube, p = 2, n_el = 16, sine load: A = P exactly and the sine
    moments are a discrete eigenvector, so TPCG stops after one step at the
    exact solution (rank 1)."""
    w = W.config_small()
    op, f, prec, x, info = solve(w)
    xr, it, res = fullpcg.pcg_exact_fd(w, op, f.full(), 1e-14)
    assert info.converged and info.iters <= 2
    assert x.ranks == (1, 1, 1)
    assert np.linalg.norm(x.full() - xr) <= 1e-10 * np.linalg.norm(xr)


@pytest.mark.parametrize("p", [2, 3])
def test_weighted_tiny_against_dense_solve(p):
    w = W.weighted_cp(6, p, 6, 2, 101, 102)
    w.tol = 1e-8
    op, f, prec, x, info = solve(w)
    xd = fullpcg.dense_solve(op, f.full())
    assert info.converged and not info.breakdown
    # solution error is bounded by cond(A) * relres; here it is far smaller
    assert np.linalg.norm(x.full() - xd) <= 1e-6 * np.linalg.norm(xd)
    # the returned residual is the true one up to the last truncation
    r = f.full() - op.dense().dot(T.vec(x.full())).reshape(f.full().shape, order="F")
    assert np.linalg.norm(r) <= 2 * w.tol * np.linalg.norm(f.full())


def test_manufactured_separable_solution_converges_at_order_p_plus_1():
    """-Lap(prod sin(pi x_i)) = 3 pi^2 prod sin(pi x_i): with f = prod sin(pi x_i)
    the Galerkin solution tends to prod sin(pi x_i)/(3 pi^2) with L2 error
    O(h^{p+1})."""
    p = 2
    errs = []
    for n_el in (4, 8, 16):
        w = W.laplace_cube(n_el, p)
        w.tol = 1e-12
        w.eps_min = 1e-13
        op, f, prec, x, info = solve(w)
        # L2 error by a tensor-product Gauss rule
        xq, wq = bspline.gauss_points(n_el, p + 4)
        B = bspline.dirichlet_basis_at(n_el, p, xq)
        vals = [B @ x.U[k] for k in range(3)]                # values of the factors
        uh = np.einsum("abc,ia,jb,kc->ijk", x.core, *vals)
        s = np.sin(np.pi * xq)
        u = np.einsum("i,j,k->ijk", s, s, s) / (3 * np.pi ** 2)
        W3 = np.einsum("i,j,k->ijk", wq, wq, wq)
        errs.append(np.sqrt(np.sum(W3 * (uh - u) ** 2)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > p + 1 - 0.3), rates


def test_iteration_count_flat_in_n_el_on_cube():
    """Table 2's qualitative claim for a tensor-product domain: the iteration
    count does not grow with n_el."""
    its = []
    for n_el in (8, 16, 32):
        w = W.laplace_cube(n_el, 3)
        w.rhs = W.random_rhs(w.n, 2, 7)
        # with the default floor 0.1*tol this rough random rhs stagnates just
        # above tol at n_el = 16; lowering eps_min is the remedy of Sec. 5.3
        w.eps_min = 1e-8
        op, f, prec, x, info = solve(w)
        assert info.converged
        its.append(info.iters)
    assert max(its) <= 1.5 * min(its), its


def test_zero_rhs_gives_zero():
    w = W.laplace_cube(6, 2)
    op = problem.operator(w)
    f = T.Tucker(np.zeros((1, 1, 1)), [np.zeros((w.n, 1))] * 3)
    x, info = tpcg.tpcg(op, fd.LowRankFD(6, 2), f)
    assert info.converged and T.norm(x) == 0.0
