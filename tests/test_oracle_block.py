"""Pins of the block (linear elasticity) oracle, Sec. 5.3, on the CPU.

What fixes the block operator without an implementation to compare with:
* rigid motions: the three translations and three infinitesimal rotations
  have eps(u) = 0 and div u = 0 pointwise, so the full (pre-Dirichlet)
  operator annihilates their B-spline interpolants exactly (the linear field
  x_d has the Greville abscissae as coefficients); a stretch is not
  annihilated;
* constant-strain energies: for u = x_1 e_1 (uniaxial), x_2 e_1 (simple
  shear), x_2 e_1 + x_1 e_2 (pure shear), x_1 e_1 + x_2 e_2 (biaxial,
  div u = 2) and x_1 e_1 - x_3 e_3 the energy u^T A u equals
  (lambda + 2 mu) int w, mu int w, 4 mu int w, 4 (lambda + mu) int w and
  4 mu int w, with int w from the closed form of the weights' integral; this
  catches a swapped lambda/mu, a missing or wrong off-diagonal term or a
  transposed mixed-derivative factor;
* the Dirichlet block matrix is symmetric and positive definite;
* block TPCG agrees with a dense solve of the assembled block system.
"""
import numpy as np
import pytest

import workloads as W
from oracle import block as B
from oracle import bspline

LAM, MU = 1.0, 0.5


def greville(n_el, p):
    kn = bspline.open_knots(n_el, p)
    m = n_el + p
    return np.array([kn[i + 1:i + p + 1].mean() for i in range(m)])


def field(bw, comps):
    """Full-basis coefficient vector of the displacement whose component a is
    coef * x_d (d given) or a constant (d = None), comps = {a: [(coef, d)]}."""
    m = bw.n_el + bw.p
    g = greville(bw.n_el, bw.p)
    one = np.ones(m)
    out = []
    for a in range(3):
        v = np.zeros(m ** 3)
        for coef, d in comps.get(a, []):
            c = [g if k == d else one for k in range(3)]
            v += coef * np.kron(c[2], np.kron(c[1], c[0]))
        out.append(v)
    return np.concatenate(out)


def int_w(bw):
    """int over the unit cube of w = sum_s prod_k (1 + amp cos(a x_k + b)),
    from int_0^1 cos(a x + b) dx = (sin(a + b) - sin b) / a."""
    modes, nnz = bw.blocks[(0, 0)]
    # the weights of the terms of block (0, 0): every term uses the same
    # weight triple within one s; collect the distinct triples
    triples = []
    for i1, i2, i3, c in nnz:
        wts = tuple(modes[k][[i1, i2, i3][k]][1] for k in range(3))
        if wts not in triples:
            triples.append(wts)
    total = 0.0
    for wts in triples:
        prod = 1.0
        for c0, c1, a, b in wts:
            prod *= c0 + c1 * (np.sin(a + b) - np.sin(b)) / a
        total += prod
    return total


@pytest.fixture(scope="module")
def small():
    bw = W.elasticity(3, 2, LAM, MU, 2, 71, 72)
    return bw, B.dense_full(bw)


def test_rigid_motions_in_kernel(small):
    bw, A = small
    scale = np.abs(A).max()
    motions = [{0: [(1.0, None)]}, {1: [(1.0, None)]}, {2: [(1.0, None)]},
               {0: [(1.0, 1)], 1: [(-1.0, 0)]}, {1: [(1.0, 2)], 2: [(-1.0, 1)]},
               {0: [(1.0, 2)], 2: [(-1.0, 0)]}]
    for mot in motions:
        u = field(bw, mot)
        assert np.abs(A @ u).max() <= 1e-12 * scale * np.abs(u).max(), mot
    stretch = field(bw, {0: [(1.0, 0)]})
    assert np.abs(A @ stretch).max() > 1e-3 * scale


def test_constant_strain_energies(small):
    bw, A = small
    iw = int_w(bw)
    cases = [({0: [(1.0, 0)]}, LAM + 2 * MU), ({0: [(1.0, 1)]}, MU),
             ({0: [(1.0, 1)], 1: [(1.0, 0)]}, 4 * MU), ({2: [(1.0, 2)]}, LAM + 2 * MU),
             ({1: [(1.0, 2)], 2: [(1.0, 1)]}, 4 * MU),
             ({0: [(1.0, 0)], 1: [(1.0, 1)]}, 4 * (LAM + MU)), ({0: [(1.0, 0)], 2: [(-1.0, 2)]}, 4 * MU)]
    for comps, factor in cases:
        u = field(bw, comps)
        energy = u @ (A @ u)
        assert abs(energy - factor * iw) <= 1e-10 * factor * iw, (comps, energy, factor * iw)


def test_dirichlet_block_matrix_symmetric_positive_definite():
    bw = W.elasticity(4, 3, LAM, MU, 2, 73, 74)
    A = B.dense(B.operator(bw), bw.n)
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    np.linalg.cholesky(A)   # raises unless SPD


def test_block_tpcg_matches_dense_solve():
    bw = W.elasticity(4, 3, LAM, MU, 2, 75, 76)
    A = B.operator(bw)
    f = B.rhs(bw)
    P = B.BlockFD(bw)
    x, info = B.tpcg(A, P, f, tol=1e-10, eps_min=1e-13)
    assert info.converged
    Ad = B.dense(A, bw.n)
    xd = np.linalg.solve(Ad, B.to_full(f))
    err = np.linalg.norm(B.to_full(x) - xd) / np.linalg.norm(xd)
    assert err <= 1e-8, err
    # the residual the iteration reports is the true one (up to truncation)
    res = np.linalg.norm(B.to_full(f) - Ad @ B.to_full(x)) / np.linalg.norm(B.to_full(f))
    assert res <= 2e-10, res
