"""Appendix A front end (oracle; test infrastructure only: the library never
imports it): separable approximations of the geometry coefficients Q(eta)
and omega(eta) (eqs. matrix_param, rhs_param) by Chebyshev interpolation on
a tensor grid and a Tucker truncation of the coefficient tensor, and the
Tucker matrix and vector they induce (eq. matrix_CP and the rhs factors
F~_t).

Readings of the paper taken here:
* the paper calls chebfun3f, which builds the Tucker form by cross
  approximation without the full evaluation tensor; here the full tensor of
  values on a Chebyshev-Lobatto grid of t points per direction is formed
  (t^3 evaluations, cheap for the t used) and its coefficient tensor is
  truncated by ST-HOSVD so that the discarded coefficients have Frobenius
  norm at most eps times the largest value on the grid (for Q, the largest
  over its entries, so that entries that vanish up to rounding are dropped,
  as the paper's zero ranks for the annulus' off-diagonal entries show), and
  Q being symmetric, the entries below the diagonal reuse the approximation
  of their mirror, so that the Tucker matrix is exactly symmetric (separate
  approximations differ at the eps level and make CG stagnate); the
  paper's acceptance test (error <= 10 eps at Halton points) is read relative
  to that scale and checked;
* Chebyshev polynomials are those of [0, 1]: T_m(2 eta - 1);
* stand-in geometries of the experiments (their maps are given as figures
  only): the thick quarter annulus F(eta) = ((1 + eta_1) cos(pi eta_2 / 2),
  (1 + eta_1) sin(pi eta_2 / 2), eta_3) (radii 1 and 2, height 1), and a
  piece of a spherical shell (radii 1 and 2) over a gnomonic patch,
  F(eta) = (1 + eta_1) w / |w| with w = (1, eta_2, eta_3), a map that is not
  orthogonal (Q_23 != 0) and not a tensor product, with the load f = 1.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import chebyshev

from . import bspline
from .tucker import Tucker, TuckerMatrix, mode_product, sthosvd


def cheb_points(t: int) -> np.ndarray:
    """Chebyshev-Lobatto points of [0, 1]."""
    return 0.5 * (1.0 + np.cos(np.pi * np.arange(t) / (t - 1)))


def cheb_eval(c, x):
    """sum_m c[m] T_m(2x - 1)."""
    return chebyshev.chebval(2.0 * np.asarray(x, dtype=float) - 1.0, c)


def cheb_coefficients(values: np.ndarray) -> np.ndarray:
    """Coefficient tensor C of the interpolant sum C_abc T_a T_b T_c of the
    values on the tensor Chebyshev-Lobatto grid (one Vandermonde solve per
    mode)."""
    C = values
    for k in range(3):
        t = values.shape[k]
        V = chebyshev.chebvander(2.0 * cheb_points(t) - 1.0, t - 1)   # V[i, m] = T_m(x_i)
        C = mode_product(C, np.linalg.inv(V), k)
    return C


def grid_values(fn, t: int) -> np.ndarray:
    x = cheb_points(t)
    E1, E2, E3 = np.meshgrid(x, x, x, indexing="ij")
    return fn(E1, E2, E3)


def separable(fn, t: int, eps: float, scale: float | None = None) -> Tucker:
    """Tucker approximation (core, factors of Chebyshev coefficients, t rows
    each) of fn(e1, e2, e3) on [0, 1]^3: the coefficient tensor truncated so
    that the discarded part has Frobenius norm <= eps * scale (scale: the
    largest |value| on the grid unless given, e.g. shared by the entries of
    Q, so that an entry that vanishes up to rounding gets rank 0)."""
    vals = grid_values(fn, t)
    C = cheb_coefficients(vals)
    scale = float(np.abs(vals).max()) if scale is None else scale
    nrm = float(np.linalg.norm(C))
    if nrm <= eps * scale:
        return Tucker(np.zeros((0, 0, 0)), [np.zeros((t, 0))] * 3)
    core, S = sthosvd(C, eps * scale / nrm)
    return Tucker(core, S)


def evaluate(g: Tucker, e1, e2, e3) -> np.ndarray:
    """The separable approximation at points (arrays of equal shape)."""
    B = [np.stack([cheb_eval(g.U[k][:, r], e) for r in range(g.U[k].shape[1])], axis=-1)
         for k, e in enumerate((e1, e2, e3))]
    return np.einsum("abc,...a,...b,...c->...", g.core, B[0], B[1], B[2])


def halton(count: int) -> np.ndarray:
    """The first `count` points of the Halton sequence in bases 2, 3, 5."""
    def radical(i, b):
        f, r = 1.0, 0.0
        while i > 0:
            f /= b
            r += f * (i % b)
            i //= b
        return r
    return np.array([[radical(i, b) for b in (2, 3, 5)] for i in range(1, count + 1)])


# ---------------------------------------------------------------------------
# the thick quarter annulus
# ---------------------------------------------------------------------------

def annulus_map(e1, e2, e3):
    r, th = 1.0 + e1, 0.5 * np.pi * e2
    return r * np.cos(th), r * np.sin(th), e3 + 0.0 * e1


def annulus_jacobian(e1, e2, e3):
    """J[..., a, b] = d F_a / d eta_b."""
    r, th = 1.0 + e1, 0.5 * np.pi * e2
    J = np.zeros(np.shape(e1) + (3, 3))
    J[..., 0, 0], J[..., 0, 1] = np.cos(th), -0.5 * np.pi * r * np.sin(th)
    J[..., 1, 0], J[..., 1, 1] = np.sin(th), 0.5 * np.pi * r * np.cos(th)
    J[..., 2, 2] = 1.0
    return J


def q_entry(jac, k, l):
    """eta -> [det(J) J^{-1} J^{-T}]_{kl} (Appendix A)."""
    def fn(e1, e2, e3):
        J = jac(e1, e2, e3)
        Ji = np.linalg.inv(J)
        return np.linalg.det(J) * np.einsum("...ka,...la->...kl", Ji, Ji)[..., k, l]
    return fn


def annulus_solution(x, y, z):
    """The manufactured solution of Sec. 5.1 (zero on the boundary)."""
    rho2 = x * x + y * y
    return (rho2 - 1.0) * (rho2 - 4.0) * np.sin(np.pi * z) * np.sin(7.0 * x * y)


def annulus_load(x, y, z):
    """f = -Laplace u for the manufactured solution: with g = (rho^2 - 1)(rho^2 - 4),
    grad g = (4 rho^2 - 10)(x, y), Laplace g = 16 rho^2 - 20, t = sin(7xy),
    grad t = 7 cos(7xy)(y, x), Laplace t = -49 rho^2 t and s = sin(pi z)."""
    rho2 = x * x + y * y
    g = (rho2 - 1.0) * (rho2 - 4.0)
    t, s = np.sin(7.0 * x * y), np.sin(np.pi * z)
    lap_xy = (16.0 * rho2 - 20.0) * t + 2.0 * (4.0 * rho2 - 10.0) * 14.0 * x * y * np.cos(7.0 * x * y) \
        - 49.0 * rho2 * g * t
    return -(s * lap_xy - np.pi ** 2 * g * t * s)


def annulus_omega(e1, e2, e3):
    """omega = det(J) f(F(eta))."""
    J = annulus_jacobian(e1, e2, e3)
    return np.linalg.det(J) * annulus_load(*annulus_map(e1, e2, e3))


# ---------------------------------------------------------------------------
# the spherical-shell piece (gnomonic patch)
# ---------------------------------------------------------------------------

def shell_map(e1, e2, e3):
    rho = 1.0 + e1
    nw = np.sqrt(1.0 + e2 * e2 + e3 * e3)
    return rho / nw, rho * e2 / nw, rho * e3 / nw


def shell_jacobian(e1, e2, e3):
    """J[..., a, b] = d F_a / d eta_b: the radial column is the unit vector
    S = w / |w|; d S / d eta_2 = (e_y - S S_y) / |w|, likewise for eta_3."""
    rho = 1.0 + e1
    nw = np.sqrt(1.0 + e2 * e2 + e3 * e3)
    S = np.stack([1.0 / nw, e2 / nw, e3 / nw], axis=-1)
    J = np.zeros(np.shape(e1) + (3, 3))
    J[..., :, 0] = S
    for b, comp in ((1, 1), (2, 2)):
        col = -S * S[..., comp:comp + 1]
        col[..., comp] += 1.0
        J[..., :, b] = rho[..., None] * col / nw[..., None]
    return J


def shell_omega(e1, e2, e3):
    """omega = det(J) for the load f = 1."""
    return np.linalg.det(shell_jacobian(e1, e2, e3))


# ---------------------------------------------------------------------------
# the induced Tucker matrix and vector
# ---------------------------------------------------------------------------

KIND = {(0, 0): "mass", (1, 1): "stiff", (1, 0): "mixed10", (0, 1): "mixed01"}


def exact_nq(p: int, t: int) -> int:
    """Gauss-Legendre points per span exact for a product of two degree-p
    basis functions and a weight of degree t - 1."""
    return p + 1 + (t + 1) // 2 + 2


def operator(n_el: int, p: int, jac, t: int, eps: float):
    """(TuckerMatrix, ranks) of eq. matrix_CP: for every entry (k, l) of Q
    with a nonzero approximation, its Tucker core as a diagonal block of the
    operator's core and, per mode s and factor column r, the 1D matrix
    int delta^(l,s)(b_i) delta^(k,s)(b_j) w_{s,r} (the test function
    differentiated when s = l, the trial function when s = k)."""
    mats = [[], [], []]
    nnz = []
    ranks = {}
    scale = max(float(np.abs(grid_values(q_entry(jac, k, l), t)).max()) for k in range(3) for l in range(3))
    seps = {}
    for k in range(3):
        for l in range(3):
            # Q = Q^T: below the diagonal, the mirror entry's approximation
            g = seps[(l, k)] if k > l else separable(q_entry(jac, k, l), t, eps, scale)
            seps[(k, l)] = g
            ranks[(k, l)] = tuple(g.core.shape)
            if g.core.size == 0:
                continue
            off = [len(mats[s]) for s in range(3)]
            for s in range(3):
                kind = KIND[(int(s == l), int(s == k))]
                for r in range(g.U[s].shape[1]):
                    c = g.U[s][:, r]
                    mats[s].append(bspline.matrix(n_el, p, kind, lambda x, c=c: cheb_eval(c, x), nq=exact_nq(p, t)))
            for (a, b, cc), v in np.ndenumerate(g.core):
                if v != 0.0:
                    nnz.append((off[0] + a, off[1] + b, off[2] + cc, float(v)))
    return TuckerMatrix(mats, nnz), ranks


def rhs(n_el: int, p: int, omega, t: int, eps: float) -> Tucker:
    """Tucker vector of the rhs factors F~_t[i, j] = int b_i w_{t, j}."""
    g = separable(omega, t, eps)
    U = [np.stack([bspline.load_vector(n_el, p, lambda x, c=g.U[s][:, j]: cheb_eval(c, x), nq=exact_nq(p, t))
                   for j in range(g.U[s].shape[1])], axis=1) for s in range(3)]
    return Tucker(g.core, U)
