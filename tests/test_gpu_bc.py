"""GPU parity of the boundary-condition support (Neumann ends of Appendix
B; non-homogeneous Dirichlet data by lifting, remark closing Sec. 3)
against the oracle (oracle/bc.py, pinned in test_oracle_bc.py):
* (the 1D matrices on the spaces with flags are checked on the host, in
  test_lib_host.py);
* tk_tucker_rows against slicing;
* the lifted right-hand side f - R A_full g_B against the oracle's, on the
  full tensor (1e-12) at a tiny size;
* the exact-eigenvector FD with flags against the oracle's LowRankFD with
  exact eigenpairs on the same spaces, factor columns at 1e-9 (independent
  eigensolvers and Remez solvers on both sides), and the Appendix B one
  (fd_setup_bc) against the oracle's approximate eigenpairs at 1e-8; with
  all flags Dirichlet the dense Appendix B path against the sine-transform
  path (1e-9);
* TPCG with that preconditioner and the lifted rhs: the manufactured linear
  solution u = 1 + 3z (Dirichlet at z = 0 and 1, Neumann on the other
  faces), which the discrete solution reproduces exactly, to the solver
  tolerance (relative error 1e-6 at tol 1e-8) at n_el = 8 and 64; a
  weighted operator with mixed flags and random data against the oracle's
  dense solve at n_el = 6.
"""
import numpy as np
import pytest

import workloads as W
from oracle import bc as obc
from oracle import fd as ofd
from oracle import tucker as T
from oracle.fullpcg import dense_solve

from gpu_helpers import context, rel, say, to_oracle, to_oracle_plain

pytestmark = pytest.mark.gpu

BCS = [(0, 0), (1, 1), (1, 0), (0, 1)]


@pytest.fixture(scope="module")
def ctx():
    return context()


def test_tucker_rows(ctx):
    from paper_2306_00632_amd import tk
    core, U = W.random_tucker((9, 7, 8), (3, 2, 4), 5)
    x = tk.Tucker.from_host(ctx, core, U)
    y = tk.axpby(ctx, 2.0, x, -1.0, x)   # a lazy sum: blocks are kept
    r = to_oracle(tk.tucker_rows(ctx, y, (1, 0, 2), (6, 7, 5)))
    ref = to_oracle(y)
    for k, (o, n) in enumerate(((1, 6), (0, 7), (2, 5))):
        np.testing.assert_array_equal(r.U[k], ref.U[k][o:o + n])
    assert [(c, off) for c, _, off in r.blocks] == [(c, off) for c, _, off in ref.blocks]
    with pytest.raises(tk.TkError):
        tk.tucker_rows(ctx, y, (4, 0, 0), (6, 7, 8))


@pytest.mark.parametrize("bcs", [((1, 1), (1, 1), (0, 0)), ((1, 0), (0, 1), (0, 0)), ((0, 1), (1, 1), (1, 0))])
def test_lifted_rhs(ctx, bcs):
    from paper_2306_00632_amd import problem
    say(f"lifted rhs {bcs}")
    w = W.weighted_cp(5, 3, 6, 2, 21, 22)
    g = T.Tucker(*W.random_tucker(w.n_el + w.p, (2, 3, 2), 9))
    got = to_oracle(problem.lifted_rhs(ctx, w, bcs, g.core, g.U)).full()
    ref = obc.lifted_rhs(w, bcs, g).full()
    assert got.shape == ref.shape
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("bcs,p", [(((1, 1), (1, 1), (0, 0)), 3), (((1, 0), (0, 1), (0, 0)), 2),
                                   (((0, 1), (1, 1), (1, 0)), 4)])
def test_exact_fd_bc(ctx, bcs, p):
    from paper_2306_00632_amd import tk
    n_el = 16
    say(f"exact fd with flags {bcs} p={p}")
    Pg = tk.Preconditioner.create(ctx, n_el, p, 0.1, exact=True, bcs=bcs)
    Po = ofd.LowRankFD(n_el, p, 0.1, exact=True, bcs=bcs)
    info = Pg.info()
    assert info["R_P"] == Po.R_P
    assert abs(info["lam_min"] - Po.lam_min) <= 1e-9 * Po.lam_min
    n = [n_el + p - 2 + sum(b) for b in bcs]
    core, U = W.random_tucker(n, (3, 2, 4), 91)
    got = to_oracle(tk.fd_precond(ctx, Pg, tk.Tucker.from_host(ctx, core, U)))
    ref = Po.apply(T.Tucker(core, U))
    for k in range(3):
        np.testing.assert_allclose(got.U[k], ref.U[k], rtol=1e-9, atol=1e-9 * np.abs(ref.U[k]).max())
    assert rel(got.full(), ref.full()) < 1e-9


@pytest.mark.parametrize("bcs,p", [(((1, 1), (1, 1), (0, 0)), 3), (((1, 0), (0, 1), (0, 0)), 2),
                                   (((0, 1), (1, 1), (1, 0)), 5)])
def test_appendix_b_fd_bc(ctx, bcs, p):
    """fd_setup_bc (Appendix B with Neumann flags, dense) against the oracle's
    LowRankFD with approximate eigenpairs on the same spaces (factor columns
    U~ D_j U~^T S, independent of eigenvector signs, 1e-8)."""
    from paper_2306_00632_amd import tk
    n_el = 16
    say(f"Appendix B fd with flags {bcs} p={p}")
    Pg = tk.Preconditioner.create(ctx, n_el, p, 0.1, bcs=bcs)
    Po = ofd.LowRankFD(n_el, p, 0.1, bcs=bcs)
    assert Pg.info()["R_P"] == Po.R_P
    n = [n_el + p - 2 + sum(b) for b in bcs]
    core, U = W.random_tucker(n, (3, 2, 4), 92)
    got = to_oracle(tk.fd_precond(ctx, Pg, tk.Tucker.from_host(ctx, core, U)))
    ref = Po.apply(T.Tucker(core, U))
    for k in range(3):
        np.testing.assert_allclose(got.U[k], ref.U[k], rtol=0, atol=1e-8 * np.abs(ref.U[k]).max())


@pytest.mark.parametrize("n_el,p", [(16, 3), (32, 2), (64, 5)])
def test_dense_appendix_b_equals_sine_transform_path(ctx, n_el, p):
    """With all flags Dirichlet the dense Appendix B preconditioner
    (fd_setup_bc) and the sine-transform one (fd_setup) apply the same
    operator: two independent constructions of Algorithm 4 (1e-9)."""
    from paper_2306_00632_amd import tk
    say(f"dense vs sine-transform Appendix B n_el={n_el} p={p}")
    Pd = tk.Preconditioner.create(ctx, n_el, p, 0.1, bcs=((0, 0),) * 3)
    Pf = tk.Preconditioner.create(ctx, n_el, p, 0.1)
    n = n_el + p - 2
    core, U = W.random_tucker(n, (2, 3, 2), 93)
    s = tk.Tucker.from_host(ctx, core, U)
    a, b = to_oracle(tk.fd_precond(ctx, Pd, s)), to_oracle(tk.fd_precond(ctx, Pf, s))
    for k in range(3):
        np.testing.assert_allclose(a.U[k], b.U[k], rtol=0, atol=1e-9 * np.abs(b.U[k]).max())


def test_all_neumann_rejected(ctx):
    from paper_2306_00632_amd import tk
    with pytest.raises(tk.TkError):
        tk.Preconditioner.create(ctx, 8, 2, 0.1, exact=True, bcs=((1, 1),) * 3)
    with pytest.raises(tk.TkError):
        tk.Preconditioner.create(ctx, 8, 2, 0.1, bcs=((1, 1),) * 3)


@pytest.mark.parametrize("exact", [False, True])
@pytest.mark.parametrize("n_el,p", [(8, 2), (8, 3), (64, 3)])
def test_tpcg_manufactured_linear_solution(ctx, n_el, p, exact):
    from paper_2306_00632_amd import problem, tk
    w = W.laplace_cube(n_el, p)
    bcs = ((1, 1), (1, 1), (0, 0))
    g = obc.linear_coefficients(n_el, p, (1.0, 0.0, 0.0, 3.0))
    say(f"tpcg manufactured u = 1 + 3z, n_el={n_el} p={p} exact={exact}")
    f = problem.lifted_rhs(ctx, w, bcs, g.core, g.U)
    x, info = tk.tpcg_solve(ctx, problem.operator_bc(ctx, w, bcs),
                            problem.preconditioner_bc(ctx, w, bcs, exact=exact), f, tol=1e-8)
    ref = obc.restrict(g, n_el, p, bcs)
    err = rel(to_oracle_plain(x).full(), ref.full())
    say(f"   iters={info['iters']} rank={info['rank']} rel_err={err:.2e}")
    assert info["converged"]
    assert err < 1e-6


def test_tpcg_weighted_mixed_flags_against_dense(ctx):
    from paper_2306_00632_amd import problem, tk
    n_el, p = 6, 3
    w = W.weighted_cp(n_el, p, 6, 2, 31, 32)
    bcs = ((1, 0), (1, 1), (0, 1))
    n = [n_el + p - 2 + sum(b) for b in bcs]
    fc, fU = W.random_tucker(n, (2, 2, 2), 33)
    g = T.Tucker(*W.random_tucker(n_el + p, (1, 2, 1), 34))
    say("tpcg weighted operator, mixed flags, random f and Dirichlet data")
    f = problem.lifted_rhs(ctx, w, bcs, g.core, g.U, f=tk.Tucker.from_host(ctx, fc, fU))
    x, info = tk.tpcg_solve(ctx, problem.operator_bc(ctx, w, bcs), problem.preconditioner_bc(ctx, w, bcs), f,
                            tol=1e-9)   # Appendix B with the flags
    rhs = obc.lifted_rhs(w, bcs, g, T.Tucker(fc, fU))
    xd = dense_solve(obc.operator(w, bcs), rhs.full())
    err = rel(to_oracle_plain(x).full(), xd)
    say(f"   iters={info['iters']} rel_err={err:.2e}")
    assert info["converged"]
    assert err < 1e-6
