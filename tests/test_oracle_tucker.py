"""Pins of the oracle's Tucker algebra and truncations (Sec. 2.3, Sec. 4.1)."""
import numpy as np
import pytest

import workloads as W
from oracle import problem
from oracle import tucker as T


def rnd_tucker(n, r, seed):
    core, U = W.random_tucker(n, r, seed)
    return T.Tucker(core, U)


def test_kronecker_vec_identity_brute_force():
    """(J3 x J2 x J1) vec(X) = vec(X x_3 J3 x_2 J2 x_1 J1)  (eq. kron_vec_multi),
    with rectangular J_i of size l_i x n_i."""
    rng = np.random.default_rng(1)
    X = rng.standard_normal((3, 4, 5))
    J = [rng.standard_normal((l, n)) for l, n in zip((2, 6, 3), (3, 4, 5))]
    lhs = np.kron(J[2], np.kron(J[1], J[0])) @ T.vec(X)
    Y = X
    for k in (2, 1, 0):
        Y = T.mode_product(Y, J[k], k)
    np.testing.assert_allclose(T.vec(Y), lhs, rtol=1e-13, atol=1e-13)
    # explicit entry of a single mode product
    Z = T.mode_product(X, J[1], 1)
    assert np.isclose(Z[1, 2, 3], sum(J[1][2, j] * X[1, j, 3] for j in range(4)))


def test_full_matches_explicit_sum():
    x = rnd_tucker((4, 3, 5), (2, 3, 2), 3)
    F = np.zeros((4, 3, 5))
    for a in range(2):
        for b in range(3):
            for c in range(2):
                F += x.core[a, b, c] * np.einsum("i,j,k->ijk", x.U[0][:, a], x.U[1][:, b], x.U[2][:, c])
    np.testing.assert_allclose(x.full(), F, atol=1e-12)


@pytest.mark.parametrize("wl", ["cube", "cp"])
def test_tucker_matrix_product_against_dense(wl):
    """eq. (tt_product) against the assembled Kronecker sum; rank R_k r_k."""
    w = W.laplace_cube(5, 2) if wl == "cube" else W.weighted_cp(5, 3, 4, 2, 7, 8)
    op = problem.operator(w)
    n = w.n
    x = rnd_tucker(n, (2, 3, 2), 5)
    y = T.apply_op(op, x)
    Rk = [len(op.mats[k]) for k in range(3)]
    assert y.m == tuple(Rk[k] * x.ranks[k] for k in range(3))
    ref = op.dense() @ T.vec(x.full())
    np.testing.assert_allclose(T.vec(y.full()), ref, rtol=1e-12, atol=1e-12)


def test_dot_and_sum():
    x = rnd_tucker((6, 5, 4), (2, 3, 2), 11)
    y = rnd_tucker((6, 5, 4), (3, 1, 2), 12)
    assert np.isclose(T.dot(x, y), np.sum(x.full() * y.full()), rtol=1e-13)
    s = T.tsum([(2.0, x), (-0.5, y)])
    assert s.m == (5, 4, 4)
    np.testing.assert_allclose(s.full(), 2.0 * x.full() - 0.5 * y.full(), atol=1e-12)
    assert np.isclose(T.dot(s, x), np.sum(s.full() * x.full()), rtol=1e-12)


@pytest.mark.parametrize("eps", [1e-1, 1e-3, 1e-6, 1e-10])
def test_trel_error_bound_and_orthonormal(eps):
    x = rnd_tucker((9, 8, 7), (4, 4, 3), 21)
    y = T.tsum([(1.0, x), (0.3, rnd_tucker((9, 8, 7), (3, 5, 3), 22))])
    yf = y.full()
    t = T.trel(y, eps)
    err = np.linalg.norm(t.full() - yf)
    assert err <= eps * np.linalg.norm(yf) * (1 + 1e-10) + 1e-14
    for U in t.U:
        np.testing.assert_allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-12)


def test_trel_reproduces_and_recovers_planted_rank():
    x = rnd_tucker((10, 9, 8), (3, 2, 4), 31)
    y = T.tsum([(1.0, x), (1.0, x), (-0.5, x)])        # represented rank stays (3,2,4)
    t = T.trel(y, 1e-12)
    assert t.ranks == (3, 2, 4)
    np.testing.assert_allclose(t.full(), 1.5 * x.full(), atol=1e-11)


def test_trel_equals_full_tensor_sthosvd():
    """Alg. 1 on the Tucker form = ST-HOSVD of the expanded tensor (the Q_k
    are orthonormal), same ranks and same represented tensor."""
    y = T.tsum([(1.0, rnd_tucker((7, 6, 5), (3, 3, 2), 41)), (1e-3, rnd_tucker((7, 6, 5), (2, 2, 2), 42))])
    eps = 1e-4
    t = T.trel(y, eps)
    core, S = T.sthosvd(y.full(), eps)
    assert t.ranks == core.shape
    np.testing.assert_allclose(t.full(), T.Tucker(core, S).full(), atol=1e-12)


def test_sthosvd_rank_rule_budget_split():
    """Superdiagonal core with sigma = 1, .1, .01, .001, 1e-4 in every
    unfolding.  eps is chosen so that eps^2 ||Z||^2 / 3 lies strictly between
    the tails of ranks 3 and 2: the rule must keep 3 per mode (a missing /3,
    or eps not squared, would keep 2)."""
    sig = np.array([1.0, 0.1, 0.01, 1e-3, 1e-4])
    Z = np.zeros((5, 5, 5))
    for i, s in enumerate(sig):
        Z[i, i, i] = s
    tail2 = np.sum(sig[2:] ** 2)
    budget = 0.5 * tail2
    eps = np.sqrt(3 * budget / np.sum(sig ** 2))
    core, S = T.sthosvd(Z, eps)
    assert core.shape == (3, 3, 3)
    # at a budget just above tail2 the rank drops to 2
    eps2 = np.sqrt(3 * 1.01 * tail2 / np.sum(sig ** 2))
    assert T.sthosvd(Z, eps2)[0].shape == (2, 2, 2)


def test_zero_tensor_truncates_to_rank_zero():
    z = T.Tucker.zero((4, 5, 6))
    t = T.trel(T.tsum([(1.0, z)]), 1e-3)
    assert t.ranks == (0, 0, 0)
    assert T.norm(t) == 0.0


def test_tdt_invariants():
    """Algorithm 2: eps_new <= eps, eps_new >= alpha * eps_min... and the exit
    condition |v - 1| < delta holds unless the floor was reached."""
    y0 = rnd_tucker((8, 8, 8), (3, 3, 3), 51)
    p = rnd_tucker((8, 8, 8), (4, 4, 4), 52)
    om = 1e-3
    yt = T.tsum([(1.0, y0), (om, p)])
    dyt = T.tsum([(om, p)])
    for eps, eps_min in [(0.1, 1e-7), (0.1, 1e-2)]:
        y1, eps_new, calls = T.tdt(y0, yt, dyt, eps, 0.5, eps_min, 1e-3)
        assert eps_new <= eps and eps_new > 0.5 * eps_min
        v = (T.dot(dyt, y1) - T.dot(dyt, y0)) / T.dot(dyt, dyt)
        if eps_new * 0.5 > eps_min:
            assert abs(v - 1) < 1e-3
        assert calls >= 1


def test_memory_compression_formula():
    x = rnd_tucker((10, 12, 14), (2, 3, 4), 3)
    assert np.isclose(T.memory_compression(x), (24 + 20 + 36 + 56) / (10 * 12 * 14) * 100)


def test_rel_diff_no_cancellation():
    x = rnd_tucker((6, 6, 6), (2, 2, 2), 61)
    d = rnd_tucker((6, 6, 6), (2, 2, 2), 62)
    y = T.tsum([(1.0, x), (1e-9, d)]).to_tucker()
    ref = 1e-9 * np.linalg.norm(d.full()) / np.linalg.norm(x.full())
    assert abs(T.rel_diff(y, x) - ref) < 1e-6 * ref
