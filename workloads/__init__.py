"""Seeded synthetic workloads for the low-rank isogeometric Poisson solver.

This module only draws random numbers and writes down recipes (which 1D
matrices make up each Kronecker term, which weights they carry, which seeds
feed the right-hand side).  It performs none of the method's arithmetic:
no B-spline evaluation, no quadrature, no tensor algebra.  Both the CPU
oracle and the GPU library build their matrices and vectors from these
recipes independently.

Recipe vocabulary
-----------------
A 1D matrix is ``(kind, weight)`` with ``kind`` in ``{"mass", "stiff",
"mixed10", "mixed01"}`` (``mixed10`` differentiates the test function,
``mixed01`` the trial function) and ``weight = (c0, c1, a, b)`` meaning
``w(x) = c0 + c1*cos(a*x + b)`` on the parametric interval [0, 1].

An operator is the Tucker matrix of eq. (tucker_matrix): per mode ``k`` a
list of distinct 1D matrices, plus the nonzeros ``(i1, i2, i3, c)`` of its
core.  A sum of R Kronecker terms is the superdiagonal-core special case.

A right-hand side is a Tucker vector: either ``{"kind": "random", "core",
"factors"}`` (values given) or ``{"kind": "load", "weight"}`` meaning the 1D
moments F_i = int b_i(x) w(x) dx in every mode with core [[[1]]] (the
separable load of Appendix A with a single term).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

UNIT = (1.0, 0.0, 0.0, 0.0)          # w(x) = 1
SIN_PI = (0.0, 1.0, math.pi, -0.5 * math.pi)   # w(x) = cos(pi x - pi/2) = sin(pi x)


@dataclass
class Workload:
    name: str
    n_el: int
    p: int
    modes: list            # modes[k] = list of (kind, weight)
    nnz: list              # list of (i1, i2, i3, coef)
    rhs: dict
    tol: float = 1e-6
    eps_min: float | None = None      # None: 0.1 * tol (paper, Sec. 5)
    params: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        """Interior dofs per direction, n = n_el + p - 2 (Dirichlet space)."""
        return self.n_el + self.p - 2


def laplace_cube(n_el: int, p: int, name: str | None = None) -> Workload:
    """-Laplace on the unit cube: K(x)M(x)M + M(x)K(x)M + M(x)M(x)K with the
    unweighted 1D stiffness K and mass M; rhs = moments of prod sin(pi x_i)."""
    modes = [[("stiff", UNIT), ("mass", UNIT)] for _ in range(3)]
    nnz = [(0, 1, 1, 1.0), (1, 0, 1, 1.0), (1, 1, 0, 1.0)]
    return Workload(name or f"laplace_cube_nel{n_el}_p{p}", n_el, p, modes, nnz,
                    {"kind": "load", "weight": SIN_PI})


def weighted_cp(n_el: int, p: int, R: int, rank: int, seed_op: int,
                seed_rhs: int, name: str | None = None,
                amp: float = 0.5) -> Workload:
    """Deformed-geometry stand-in: R Kronecker terms; term t has the stiffness
    matrix in direction t mod 3 and mass matrices in the other two; every 1D
    factor (k, t) carries its own weight 1 + amp*cos(a x + b) with a, b drawn
    i.i.d. from U[0, 2].  rhs: Tucker rank `rank`, core and factors N(0, 1)."""
    rng = np.random.default_rng(seed_op)
    ab = rng.uniform(0.0, 2.0, size=(R, 3, 2))
    modes = [[] for _ in range(3)]
    for t in range(R):
        for k in range(3):
            kind = "stiff" if k == t % 3 else "mass"
            a, b = float(ab[t, k, 0]), float(ab[t, k, 1])
            modes[k].append((kind, (1.0, amp, a, b)))
    nnz = [(t, t, t, 1.0) for t in range(R)]
    return Workload(name or f"weighted_cp_nel{n_el}_p{p}_R{R}_r{rank}", n_el, p,
                    modes, nnz, random_rhs(n_el + p - 2, rank, seed_rhs))


def linear_dirichlet_data(n_el: int, p: int, a) -> tuple:
    """(core, factors) of u(x, y, z) = a0 + a1 x + a2 y + a3 z on the full
    tensor-product B-spline basis (n_el + p functions per direction, open
    uniform knots): the constant has coefficients 1 and a coordinate the
    Greville abscissae (averages of p consecutive interior knots), so the
    tensor is exact; multilinear rank at most (2, 2, 2).  Input data of the
    manufactured-solution runs with non-homogeneous Dirichlet conditions."""
    knots = np.concatenate([np.zeros(p + 1), np.arange(1, n_el) / n_el, np.ones(p + 1)])
    xi = np.array([knots[i + 1:i + p + 1].sum() / p for i in range(n_el + p)])
    U = [np.stack([np.ones_like(xi), xi], axis=1) for _ in range(3)]
    core = np.zeros((2, 2, 2))
    core[0, 0, 0], core[1, 0, 0], core[0, 1, 0], core[0, 0, 1] = a
    return core, U


def random_rhs(n: int, rank: int, seed: int, ranks=None) -> dict:
    rng = np.random.default_rng(seed)
    r = tuple(ranks) if ranks is not None else (rank, rank, rank)
    core = rng.standard_normal(r)
    factors = [rng.standard_normal((n, r[k])) for k in range(3)]
    return {"kind": "random", "core": core, "factors": factors}


def random_tucker(n, ranks, seed):
    """A random Tucker tensor (core, [U1, U2, U3]) with N(0,1) entries; `n`
    may be an int or a 3-tuple."""
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    rng = np.random.default_rng(seed)
    core = rng.standard_normal(tuple(ranks))
    factors = [rng.standard_normal((nn[k], ranks[k])) for k in range(3)]
    return core, factors


# --- the benchmark configurations -------------------------------------------

def config_small() -> Workload:
    """3D Poisson on the unit cube, p = 2, n_el = 16 (16 dofs/direction),
    rhs = projected prod sin(pi x_i); tol 1e-6, truncation floor 1e-8."""
    w = laplace_cube(16, 2, name="poisson_cube_p2_nel16")
    w.eps_min = 1e-8
    return w


def config_deformed() -> Workload:
    """Deformed-geometry Poisson stand-in: p = 3, n_el = 128 (129 dofs),
    9 weighted Kronecker terms (seed 2002), rhs Tucker rank 5 (seed 2003).

    The rhs factors are white noise, so the solution is nearly full rank at
    tol = 1e-6; with the default floor eps_min = 0.1 tol the residual
    stagnates near 2.5e-6 (the stagnation reported for the elasticity column
    in Sec. 5.3), and the remedy given there, a lower eps_min, is applied:
    eps_min = 1e-8."""
    w = weighted_cp(128, 3, 9, 5, 2002, 2003, name="poisson_weighted9_p3_nel128_r5")
    w.eps_min = 1e-8
    return w


def config_large() -> Workload:
    """Large single solve: p = 3, n_el = 512 (515 dofs), 12 weighted terms
    (seed 3002), rhs Tucker rank 10 (seed 3003); eps_min as for the
    deformed workload."""
    w = weighted_cp(512, 3, 12, 10, 3002, 3003, name="poisson_weighted12_p3_nel512_r10")
    w.eps_min = 1e-8
    return w


# --- block (3-component) problems: linear elasticity -------------------------

@dataclass
class BlockWorkload:
    """A 3 x 3 block system (Sec. 5.3): ``blocks[(a, b)]`` is the operator
    recipe ``(modes, nnz)`` of block A_ab (test component a, trial component
    b; absent = zero block), ``rhs`` the three component recipes and
    ``prec_coef[a]`` the direction coefficients of component a's FD
    preconditioner (Algorithm 4 with c_1 L_1 + c_2 L_2 + c_3 L_3)."""
    name: str
    n_el: int
    p: int
    blocks: dict
    rhs: list
    prec_coef: list
    tol: float = 1e-6
    eps_min: float | None = None
    params: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.n_el + self.p - 2


def _add_term(modes, nnz, mats, coef):
    """Append the Kronecker term coef * mats[0] (x) mats[1] (x) mats[2] to a
    Tucker-matrix recipe, reusing 1D matrices already listed in a mode."""
    idx = []
    for k in range(3):
        if mats[k] not in modes[k]:
            modes[k].append(mats[k])
        idx.append(modes[k].index(mats[k]))
    nnz.append((idx[0], idx[1], idx[2], float(coef)))


def elasticity(n_el: int, p: int, lam: float, mu: float, rank: int, seed_op: int,
               seed_rhs: int, S: int = 2, amp: float = 0.5, name: str | None = None) -> BlockWorkload:
    """Compressible linear elasticity on a weighted ("deformed") cube, Dirichlet
    on all faces: b(u, v) = int w(x) [2 mu eps(u):eps(v) + lam div u div v]
    with w(x) = sum_{s<S} prod_k w_{s,k}(x_k), w_{s,k}(x) = 1 + amp cos(a x + b),
    a, b ~ U[0, 2] (seed_op).  Every w_s > 0, so the operator is SPD.

    Block (a, b) pairs test component a with trial component b:
      A_aa = sum_s [(lam + 2 mu) stiff_a + mu sum_{c != a} stiff_c]  (3 S terms)
      A_ab = sum_s [mu d_a(trial) d_b(test) + lam d_b(trial) d_a(test)]  (2 S terms)
    where stiff_c is the stiffness matrix in direction c with masses in the
    other directions, d_c(trial) the trial derivative in direction c
    ("mixed01") and d_c(test) the test derivative ("mixed10").  rhs: three
    Tucker vectors of rank `rank` with N(0, 1) core and factors
    (seeds seed_rhs + a).  Preconditioner of component a: direction
    coefficients lam + 2 mu in direction a and mu in the others."""
    rng = np.random.default_rng(seed_op)
    ab = rng.uniform(0.0, 2.0, size=(S, 3, 2))
    wt = [[(1.0, amp, float(ab[s, k, 0]), float(ab[s, k, 1])) for k in range(3)] for s in range(S)]
    blocks = {}
    for a in range(3):
        for b in range(3):
            modes, nnz = [[], [], []], []
            for s in range(S):
                if a == b:
                    for c in range(3):
                        mats = [("stiff" if k == c else "mass", wt[s][k]) for k in range(3)]
                        _add_term(modes, nnz, mats, (lam + 2.0 * mu) if c == a else mu)
                else:
                    third = 3 - a - b
                    m_mu, m_lam = [None] * 3, [None] * 3
                    m_mu[a], m_mu[b], m_mu[third] = ("mixed01", wt[s][a]), ("mixed10", wt[s][b]), ("mass", wt[s][third])
                    m_lam[a], m_lam[b], m_lam[third] = ("mixed10", wt[s][a]), ("mixed01", wt[s][b]), ("mass", wt[s][third])
                    _add_term(modes, nnz, m_mu, mu)
                    _add_term(modes, nnz, m_lam, lam)
            blocks[(a, b)] = (modes, nnz)
    n = n_el + p - 2
    rhs = [random_rhs(n, rank, seed_rhs + a) for a in range(3)]
    coef = [[(lam + 2.0 * mu) if k == a else mu for k in range(3)] for a in range(3)]
    return BlockWorkload(name or f"elasticity_nel{n_el}_p{p}_r{rank}", n_el, p, blocks, rhs, coef)


def config_elasticity() -> BlockWorkload:
    """3D linear elasticity stand-in: p = 3, n_el = 256 (259 dofs/direction),
    Lame lambda = 1, mu = 0.5, two separable weight terms (seed 5002): 6
    Kronecker terms in every diagonal block, 4 in every off-diagonal block;
    rhs of rank 4 per component (seeds 5003..5005); tol 1e-6, eps_min 1e-8
    (white-noise rhs, as for the deformed Poisson workload)."""
    w = elasticity(256, 3, 1.0, 0.5, 4, 5002, 5003, name="elasticity_p3_nel256_r4")
    w.eps_min = 1e-8
    return w


# --- Appendix A inputs: geometry coefficients sampled on a Chebyshev grid -----

def annulus_samples(t: int) -> tuple:
    """Samples, on the tensor grid of t Chebyshev-Lobatto points of [0, 1]^3
    (x_k = (1 + cos(pi k / (t - 1))) / 2), of the thick quarter annulus
    F(eta) = ((1 + eta_1) cos(pi eta_2 / 2), (1 + eta_1) sin(pi eta_2 / 2), eta_3):
    q[(k, l)] the entries of det(J) J^-1 J^-T, here diag(pi r / 2, 2 / (pi r),
    pi r / 2) with r = 1 + eta_1 (zero off the diagonal), and omega =
    det(J) f(F(eta)) for f = -Laplace u, u = (rho^2 - 1)(rho^2 - 4) sin(pi z)
    sin(7 x y), which vanishes on the boundary (the manufactured solution of
    Sec. 5.1).  Returns (q, omega, u) with u the solution as a function of
    physical coordinates."""
    x = 0.5 * (1.0 + np.cos(np.pi * np.arange(t) / (t - 1)))
    E1, E2, E3 = np.meshgrid(x, x, x, indexing="ij")
    r, th = 1.0 + E1, 0.5 * np.pi * E2
    q = {(k, l): np.zeros((t, t, t)) for k in range(3) for l in range(3)}
    q[(0, 0)] = 0.5 * np.pi * r
    q[(1, 1)] = 2.0 / (np.pi * r)
    q[(2, 2)] = 0.5 * np.pi * r
    X, Y, Z = r * np.cos(th), r * np.sin(th), E3
    rho2 = X * X + Y * Y
    g = (rho2 - 1.0) * (rho2 - 4.0)
    sn, cs, sz = np.sin(7.0 * X * Y), np.cos(7.0 * X * Y), np.sin(np.pi * Z)
    # Laplace of g * sin(7xy) in the plane: (16 rho^2 - 20) sn + 2 grad g . grad sn + g (-49 rho^2 sn)
    lap_xy = (16.0 * rho2 - 20.0) * sn + 28.0 * (4.0 * rho2 - 10.0) * X * Y * cs - 49.0 * rho2 * g * sn
    f = -(sz * lap_xy - np.pi ** 2 * g * sn * sz)
    omega = 0.5 * np.pi * r * f

    def u(X, Y, Z):
        rho2 = X * X + Y * Y
        return (rho2 - 1.0) * (rho2 - 4.0) * np.sin(np.pi * Z) * np.sin(7.0 * X * Y)
    return q, omega, u


def shell_samples(t: int) -> tuple:
    """Samples on the same grid for a piece of a spherical shell (radii 1 and
    2) over a gnomonic patch, F(eta) = rho w / |w|, rho = 1 + eta_1,
    w = (1, u, v), u = eta_2, v = eta_3: with D = 1 + u^2 + v^2 the metric
    of the patch gives det(J) = rho^2 D^{-3/2}, Q_11 = rho^2 D^{-3/2},
    Q_22 = (1 + u^2) D^{-1/2}, Q_33 = (1 + v^2) D^{-1/2},
    Q_23 = Q_32 = u v D^{-1/2} and Q_1a = 0; omega = det(J) (load f = 1).
    Returns (q, omega)."""
    x = 0.5 * (1.0 + np.cos(np.pi * np.arange(t) / (t - 1)))
    R, U, V = np.meshgrid(1.0 + x, x, x, indexing="ij")
    D = 1.0 + U * U + V * V
    q = {(k, l): np.zeros((t, t, t)) for k in range(3) for l in range(3)}
    q[(0, 0)] = R * R * D ** -1.5
    q[(1, 1)] = (1.0 + U * U) / np.sqrt(D)
    q[(2, 2)] = (1.0 + V * V) / np.sqrt(D)
    q[(1, 2)] = q[(2, 1)] = U * V / np.sqrt(D)
    return q, R * R * D ** -1.5
