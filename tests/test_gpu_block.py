"""GPU parity of the block (3-component) system of Sec. 5.3 (linear
elasticity stand-in) against the block oracle.

* tucker_apply_op_block: each component of (A x)_a = sum_b A_ab x_b against
  the oracle's blockwise eq. tt_product, as represented tensors, 1e-12;
* tpcg_solve_block on a tiny system against the dense solve of the assembled
  block matrix (tol 1e-10: relative error <= 1e-8, as the oracle itself);
* tpcg_solve_block at n_el = 16: the residual ||f - A x|| / ||f|| of the GPU
  solution recomputed by the oracle in Tucker arithmetic (cancellation free)
  is within 1.5 tol, and the iteration count matches the oracle's block TPCG
  within max(2, 10 %);
* the elasticity workload at full size (n_el = 256, 259 dofs/direction):
  the GPU solve converges and the oracle confirms its residual.
"""
import numpy as np
import pytest

import workloads as W
from oracle import block as B
from oracle import tucker as T

from gpu_helpers import context, say, to_oracle

pytestmark = pytest.mark.gpu
LAM, MU = 1.0, 0.5


@pytest.fixture(scope="module")
def ctx():
    return context()


def lib_modules():
    from paper_2306_00632_amd import problem, tk
    return tk, problem


def oracle_residual(bw, x):
    """||f - A x|| / ||f|| of block vector x (oracle Tucker arithmetic)."""
    A = B.operator(bw)
    f = B.rhs(bw)
    ax = B.apply(A, x)
    num = sum(T.rel_diff(ax[a], f[a]) ** 2 * T.norm(f[a]) ** 2 for a in range(3))
    return float(np.sqrt(num) / B.bnorm(f))


def test_apply_op_block(ctx):
    tk, prob = lib_modules()
    bw = W.elasticity(8, 3, LAM, MU, 2, 81, 82)
    say("apply_op_block n_el=8")
    ops = prob.block_operator(ctx, bw)
    xs = [W.random_tucker(bw.n, (3, 4, 2), 90 + a) for a in range(3)]
    xg = [tk.Tucker.from_host(ctx, c, U) for c, U in xs]
    yg = tk.tucker_apply_op_block(ctx, ops, xg)
    yo = B.apply(B.operator(bw), [T.Tucker(c, U) for c, U in xs])
    for a in range(3):
        got = to_oracle(yg[a])
        assert T.rel_diff(got, yo[a]) <= 1e-12


def test_tpcg_block_tiny_matches_dense_solve(ctx):
    tk, prob = lib_modules()
    bw = W.elasticity(4, 3, LAM, MU, 2, 75, 76)
    say("tpcg_block tiny n_el=4")
    ops = prob.block_operator(ctx, bw)
    precs = prob.block_preconditioner(ctx, bw)
    f = prob.block_rhs(ctx, bw)
    x, info = tk.tpcg_solve_block(ctx, ops, precs, f, tol=1e-10, eps_min=1e-13)
    assert info["converged"]
    xo = [T.Tucker(*xa.plain()) for xa in x]
    Ad = B.dense(B.operator(bw), bw.n)
    xd = np.linalg.solve(Ad, B.to_full(B.rhs(bw)))
    err = np.linalg.norm(B.to_full(xo) - xd) / np.linalg.norm(xd)
    assert err <= 1e-8, err


def test_tpcg_block_mid_size_matches_oracle(ctx):
    tk, prob = lib_modules()
    bw = W.elasticity(16, 3, LAM, MU, 3, 85, 86)
    bw.eps_min = 1e-8
    say("tpcg_block n_el=16")
    ops = prob.block_operator(ctx, bw)
    precs = prob.block_preconditioner(ctx, bw)
    f = prob.block_rhs(ctx, bw)
    x, info = tk.tpcg_solve_block(ctx, ops, precs, f, tol=bw.tol, eps_min=bw.eps_min)
    assert info["converged"]
    xo = [T.Tucker(*xa.plain()) for xa in x]
    res = oracle_residual(bw, xo)
    assert res <= 1.5 * bw.tol, res
    _, oinfo = B.tpcg(B.operator(bw), B.BlockFD(bw), B.rhs(bw), tol=bw.tol, eps_min=bw.eps_min)
    assert oinfo.converged
    assert abs(info["iters"] - oinfo.iters) <= max(2, int(0.1 * oinfo.iters)), (info["iters"], oinfo.iters)


@pytest.mark.timeout(600)
def test_tpcg_block_elasticity_full_size(ctx):
    """The elasticity workload as configured (p = 3, n_el = 256, lambda = 1,
    mu = 0.5, rank-4 rhs per component): converged GPU solve whose residual,
    recomputed by the oracle, is within 1.5 tol."""
    tk, prob = lib_modules()
    bw = W.config_elasticity()
    say("tpcg_block elasticity n_el=256")
    ops = prob.block_operator(ctx, bw)
    precs = prob.block_preconditioner(ctx, bw)
    f = prob.block_rhs(ctx, bw)
    x, info = tk.tpcg_solve_block(ctx, ops, precs, f, tol=bw.tol, eps_min=bw.eps_min)
    say(f"  iters {info['iters']} relres {info['relres']:.3e} rank {info['rank']}")
    assert info["converged"]
    xo = [T.Tucker(*xa.plain()) for xa in x]
    res = oracle_residual(bw, xo)
    say(f"  oracle residual {res:.3e}")
    assert res <= 1.5 * bw.tol, res
