"""Pins of the oracle's preconditioner pieces: exponential sums (Prop. 1,
Table 1), Appendix B eigenpairs, Algorithms 3 and 4."""
import os

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import bspline, expsum, fd, fullpcg, problem
from oracle import tucker as T

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1.txt")


def table1():
    rows = []
    for line in open(GOLD):
        if line.strip() and not line.startswith("#"):
            p, n_el, mp, rp = line.split()
            rows.append((int(p), int(n_el), float(mp), int(rp)))
    return rows


# --- exponential sums ---------------------------------------------------------

@pytest.mark.parametrize("M,R", [(50.0, 3), (1.6384e4, 11), (1.0e6, 17)])
def test_expsum_equioscillates_and_beats_bound(M, R):
    seq = {r: (a, b, E) for r, a, b, E in expsum.best_sequence(M, stop=lambda r, E: r >= R)}
    a, b, E = seq[R]
    assert np.all(np.isfinite(a)) and np.all(np.exp(b) > 0)      # omega_j > 0, alpha_j > 0
    x = np.exp(np.linspace(0, np.log(M), 200001))
    e = expsum.error(a, b, x)
    assert abs(np.max(np.abs(e)) - E) <= 1e-6 * E
    ext = expsum._extrema(a, b, M)
    assert len(ext) == 2 * R + 1
    ev = expsum.error(a, b, ext)
    np.testing.assert_allclose(np.abs(ev), E, rtol=1e-6)
    assert np.all(np.sign(ev[1:]) == -np.sign(ev[:-1]))          # alternation
    assert E <= expsum.bound_prop1(R, M)
    # E decreases with R
    Es = [seq[r][2] for r in sorted(seq)]
    assert all(Es[i + 1] < Es[i] for i in range(len(Es) - 1))


def test_expsum_R1_is_global_minimax_by_brute_force():
    """For R = 1 a brute-force search over (alpha, omega) cannot beat Remez."""
    M = 20.0
    (R, a, b, E), = list(expsum.best_sequence(M, stop=lambda r, E: True))
    x = np.exp(np.linspace(0, np.log(M), 3000))
    best = np.inf
    for al in np.exp(np.linspace(-4, 2, 241)):
        ex = np.exp(-al * x)
        # for fixed alpha, sweep omega
        for om in np.exp(np.linspace(-3, 3, 241)):
            best = min(best, np.max(np.abs(1 / x - om * ex)))
    assert E <= best * (1 + 1e-9)
    assert E > 0.9 * best


def test_exp_sum_gives_relative_diagonal_bound():
    """|1 - lambda s(lambda)| <= eps_prec on [1, M_P]  (the eigenvalues of
    D^{-1} D~ lie in [1 - eps, 1 + eps], Sec. 4.2)."""
    M = 2000.0
    R, al, om, E, Ep = expsum.exp_sum_for(M, 0.1)
    lam = np.exp(np.linspace(0, np.log(M), 100001))
    s = (om[None, :] * np.exp(-al[None, :] * lam[:, None])).sum(1)
    assert np.max(np.abs(1 - lam * s)) <= 0.1 * (1 + 1e-6)
    assert E <= 0.1 / M < Ep


# --- Appendix B -----------------------------------------------------------------

@pytest.mark.parametrize("p,n_el", [(2, 8), (3, 8), (3, 16), (4, 10), (5, 12)])
def test_appendix_b_structure(p, n_el):
    Ut, lam, P = fd.approx_eig(n_el, p)
    n, n1, n2 = fd.subspace_dims(n_el, p)
    assert Ut.shape == (n, n) and (P["n1"], P["n2"]) == (n1, n2)
    assert n1 == (n_el - 1 if p % 2 else n_el) and n2 == (p - 1 if p % 2 else p - 2)
    if n2:
        # V1 spans ker D; V_h1 and V_h2 are exactly M-orthogonal
        assert np.abs(P["D"] @ P["V1"]).max() <= 1e-9 * np.abs(P["D"]).max()
        G = Ut.T @ P["M"] @ Ut
        assert np.abs(G[:n1, n1:]).max() < 1e-12
        np.testing.assert_allclose(G[n1:, n1:], np.eye(n2), atol=1e-12)
        # Lambda2 are exact Rayleigh quotients of the V2 U2 columns
        V2U2 = Ut[:, n1:]
        np.testing.assert_allclose(np.diag(V2U2.T @ P["K"] @ V2U2), lam[n1:], rtol=1e-10)
    # columns of V1 U1 interpolate sqrt(2) sin(j pi x) at the points, up to
    # their normalization to unit L2 (M) norm
    vals = bspline.dirichlet_basis_at(n_el, p, P["x"]) @ Ut[:, :n1]
    np.testing.assert_allclose(vals / P["scale1"], P["Udft"], atol=1e-11)
    np.testing.assert_allclose(np.einsum("ij,ij->j", Ut[:, :n1], P["M"] @ Ut[:, :n1]), 1.0, rtol=1e-12)
    np.testing.assert_allclose(lam[:n1], (np.pi * np.arange(1, n1 + 1)) ** 2)
    # the smoothest sine's interpolant already has nearly unit L2 norm
    assert abs(P["scale1"][0] - 1.0) < 1e-3


def test_p2_sines_are_exact_eigenvectors():
    """For p = 2 the interpolated sines are exact generalized eigenvectors
    (the paper: eigenvectors known explicitly, no approximation needed)."""
    Ut, lam, P = fd.approx_eig(16, 2)
    A = np.linalg.solve(P["M"] @ Ut, P["K"] @ Ut)
    off = A - np.diag(np.diag(A))
    assert np.abs(off).max() < 1e-9 * np.abs(np.diag(A)).max()


@pytest.mark.slow
def test_table1_MP_and_RP():
    """Table 1: M_P to the printed two digits (the table rounds some entries,
    e.g. 65536 -> 6.6e4, and truncates others, e.g. 2.38e4 -> 2.3e4, so the
    value must lie within [-1/2, +1) unit of the last printed digit); R_P exactly, except where
    E_{R}(M_P) lies within 2% of eps_prec/M_P (the paper read tabulated
    coefficients at nearby M; there R_P may be one lower)."""
    for p, n_el, mp_tab, rp_tab in table1():
        _, lam, _ = fd.approx_eig(n_el, p)
        MP = lam.max() / lam.min()
        unit = 10.0 ** (np.floor(np.log10(mp_tab)) - 1)
        assert -0.5 * unit <= MP - mp_tab < 1.0 * unit, (p, n_el, MP)
        R, al, om, E, Ep = expsum.exp_sum_for(MP, 0.1)
        thr = 0.1 / MP
        assert E <= thr < Ep
        if R != rp_tab:
            assert R == rp_tab - 1 and E > 0.98 * thr, (p, n_el, R, rp_tab, E / thr)


# --- Algorithms 3 and 4 -----------------------------------------------------------

def test_exact_fd_factorizations_and_unit_cube_one_step():
    """U^T M U = I, K U = M U Lambda; on the unit cube A = P, so PCG with the
    exact FD preconditioner converges in one step to the dense solution."""
    w = W.laplace_cube(6, 3)
    K = bspline.matrix(6, 3, "stiff")
    M = bspline.matrix(6, 3, "mass")
    P = fd.ExactFD([K] * 3, [M] * 3)
    U, lam = P.U[0], P.lam[0]
    np.testing.assert_allclose(U.T @ M @ U, np.eye(len(lam)), atol=1e-12)
    np.testing.assert_allclose(K @ U, M @ U * lam[None, :], atol=1e-9)
    op = problem.operator(w)
    f = T.Tucker(*W.random_tucker(w.n, (2, 2, 2), 3))
    x_dense = fullpcg.dense_solve(op, f.full())
    x, it, res = fullpcg.pcg_exact_fd(w, op, f.full(), 1e-12)
    assert it == 1
    np.testing.assert_allclose(x, x_dense, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("p", [2, 3])
def test_lowrank_fd_apply_matches_dense_inverse(p):
    prec = fd.LowRankFD(6, p, 0.1)
    s = T.Tucker(*W.random_tucker(prec.Ut[0].shape[0], (2, 3, 2), 9))
    v = prec.apply(s)
    assert v.m == tuple(prec.R_P * r for r in s.ranks)
    ref = prec.dense_inverse() @ T.vec(s.full())
    np.testing.assert_allclose(T.vec(v.full()), ref, rtol=1e-11, atol=1e-12)
    # P~^{-1} is symmetric positive definite (omega_j > 0)
    Pinv = prec.dense_inverse()
    np.testing.assert_allclose(Pinv, Pinv.T, atol=1e-12 * np.abs(Pinv).max())
    assert np.linalg.eigvalsh(Pinv).min() > 0


def test_lowrank_fd_close_to_exact_fd_spectrally():
    """For p = 2 the normalized interpolated sines are the exact M-orthonormal
    eigenvectors, so P~^{-1} P is similar to diag(lambda_h s(lambda~)) over the
    Kronecker sums: each factor lambda_h / lambda~ lies between the extreme
    1D ratios r_j = lambda_h,j / (j pi)^2 (a ratio of sums lies between the
    ratios of its terms) and lambda~ s(lambda~) within 1 +- eps_prec (Prop. 1).
    Unnormalized sines (squared M-norms over about [0.6, 1.07]) fail it."""
    n_el, p, eps = 6, 2, 0.1
    prec = fd.LowRankFD(n_el, p, eps)
    K = bspline.matrix(n_el, p, "stiff")
    M = bspline.matrix(n_el, p, "mass")
    Pm = (np.kron(K, np.kron(M, M)) + np.kron(M, np.kron(K, M)) + np.kron(M, np.kron(M, K)))
    ev = np.linalg.eigvals(prec.dense_inverse() @ Pm).real
    lam_h = np.sort(sla.eigh(K, M, eigvals_only=True))
    r = lam_h / (np.pi * np.arange(1, len(lam_h) + 1)) ** 2
    assert ev.min() >= (1 - eps) * r.min() - 1e-9 and ev.max() <= (1 + eps) * r.max() + 1e-9, (ev.min(), ev.max())


def test_approximate_and_exact_eigenpairs_similar_iterations():
    """The remark of Sec. 5: TPCG with exact eigenpairs takes nearly the same
    number of iterations as with the Appendix B approximations (deformed
    workload's recipe at n_el = 32; unnormalized sines need twice as many)."""
    from oracle import problem as oprob, tpcg as otpcg
    for p in (2, 3):
        w = W.weighted_cp(32, p, 9, 5, 2002, 2003)
        op, f = oprob.operator(w), oprob.rhs(w)
        its = [otpcg.tpcg(op, fd.LowRankFD(32, p, 0.1, exact=ex), f, tol=1e-6, eps_min=1e-8)[1].iters
               for ex in (False, True)]
        assert abs(its[0] - its[1]) <= max(2, 0.2 * its[1]), (p, its)


@pytest.mark.parametrize("n_el,p", [(5, 2), (6, 3), (7, 4)])
def test_exact_eigenpair_lowrank_fd_within_prop1_bound(n_el, p):
    """Algorithm 4 with the exact factorizations (eq. factorizations): P~^{-1} P
    is similar to diag(lambda s(lambda)) over the Kronecker sums lambda of the
    1D eigenvalues, and Prop. 1 with R_P from eq. estimate_prec_rel bounds
    |1 - lambda s(lambda)| by eps_prec on [lambda_min, lambda_max]; the
    deviation is not zero (the sum approximates 1/lambda, it is not exact).
    A dropped 1/lambda_min, a wrong exponent or non-M-orthonormal
    eigenvectors break the bound."""
    eps = 0.1
    prec = fd.LowRankFD(n_el, p, eps, exact=True)
    K = bspline.matrix(n_el, p, "stiff")
    M = bspline.matrix(n_el, p, "mass")
    U = prec.Ut[0]
    np.testing.assert_allclose(U.T @ M @ U, np.eye(U.shape[0]), atol=1e-12)
    Pm = (np.kron(K, np.kron(M, M)) + np.kron(M, np.kron(K, M)) + np.kron(M, np.kron(M, K)))
    ev = np.linalg.eigvals(prec.dense_inverse() @ Pm).real
    assert ev.min() >= 1.0 - eps - 1e-9 and ev.max() <= 1.0 + eps + 1e-9, (ev.min(), ev.max())
    assert np.abs(ev - 1.0).max() > 1e-3
