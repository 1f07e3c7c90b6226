"""Univariate B-splines and 1D Galerkin matrices (oracle; test infrastructure).

Follows Sec. 2.1 (open uniform knot vectors, Cox-de Boor recursion with the
convention 0/0 = 0) and the univariate integrals of Appendix A
(int delta(b_i) delta(b_j) w, with delta either the identity or d/dx).

Readings of the paper taken here:
* the degree-0 rule of Sec. 2.1 is half-open, which would make the last
  basis function vanish at x = 1; the last non-empty knot span is closed at
  its right end so that the basis is a partition of unity on [0, 1];
* the paper does not state a quadrature for weighted integrals; Gauss-Legendre
  with p + 5 points per element is used (tests compare against 2p + 8).
"""
from __future__ import annotations

import numpy as np


def open_knots(n_el: int, p: int) -> np.ndarray:
    """Open uniform knot vector on [0, 1] with n_el spans (Sec. 2.1):
    p+1 zeros, the interior breakpoints i/n_el, p+1 ones.  m = n_el + p
    basis functions."""
    inner = np.arange(1, n_el) / n_el
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


def _degree0(knots: np.ndarray, x: np.ndarray) -> np.ndarray:
    """b_i^(0)(x) = 1 on [xi_i, xi_{i+1}), else 0; the last non-empty span is
    closed on the right (reading of the half-open rule at x = 1)."""
    nb = len(knots) - 1
    B = np.zeros((len(x), nb))
    last = max(i for i in range(nb) if knots[i] < knots[i + 1])
    for i in range(nb):
        lo, hi = knots[i], knots[i + 1]
        if lo < hi:
            inside = (x >= lo) & (x < hi)
            if i == last:
                inside |= (x == hi)
            B[inside, i] = 1.0
    return B


def _ratio(num, den):
    """num/den with 0/0 = 0 (Sec. 2.1)."""
    return 0.0 if den == 0.0 else num / den


def basis(knots: np.ndarray, p: int, x, der: int = 0) -> np.ndarray:
    """Values (der = 0) or der-th derivatives of all B-splines of degree p on
    `knots` at points x.  Shape (len(x), len(knots) - p - 1).

    Values follow the Cox-de Boor recursion of Sec. 2.1.  Derivatives use the
    standard differentiation of that recursion,
      D b_i^(p) = p [ b_i^(p-1)/(xi_{i+p}-xi_i) - b_{i+1}^(p-1)/(xi_{i+p+1}-xi_{i+1}) ],
    applied `der` times (again with 0/0 = 0)."""
    x = np.atleast_1d(np.asarray(x, dtype=float))
    if der > p:
        return np.zeros((len(x), len(knots) - p - 1))
    if p == 0:
        return _degree0(knots, x)
    low = basis(knots, p - 1, x, der - 1 if der > 0 else 0)
    nb = len(knots) - p - 1
    out = np.zeros((len(x), nb))
    for i in range(nb):
        d1 = knots[i + p] - knots[i]
        d2 = knots[i + p + 1] - knots[i + 1]
        if der == 0:
            a = (x - knots[i]) * _ratio(1.0, d1) if d1 != 0 else 0.0
            b = (knots[i + p + 1] - x) * _ratio(1.0, d2) if d2 != 0 else 0.0
            out[:, i] = a * low[:, i] + b * low[:, i + 1]
        else:
            out[:, i] = p * (_ratio(1.0, d1) * low[:, i] - _ratio(1.0, d2) * low[:, i + 1])
    return out


def weight_values(weight, x):
    """w(x) = c0 + c1*cos(a*x + b) (the weight family of the workloads), or
    weight(x) for a callable weight (the separable approximations of
    Appendix A)."""
    if callable(weight):
        return weight(np.asarray(x, dtype=float))
    c0, c1, a, b = weight
    return c0 + c1 * np.cos(a * x + b)


def gauss_points(n_el: int, nq: int):
    """Gauss-Legendre points/weights on every span [e/n_el, (e+1)/n_el]."""
    g, gw = np.polynomial.legendre.leggauss(nq)
    h = 1.0 / n_el
    xs = (np.arange(n_el)[:, None] + 0.5 * (g[None, :] + 1.0)) * h
    ws = np.broadcast_to(0.5 * h * gw[None, :], xs.shape)
    return xs.ravel(), np.array(ws).ravel()


_DER = {"mass": (0, 0), "stiff": (1, 1), "mixed10": (1, 0), "mixed01": (0, 1)}


def matrix_full(n_el: int, p: int, kind: str, weight=(1.0, 0.0, 0.0, 0.0),
                nq: int | None = None) -> np.ndarray:
    """[A]_{ij} = int_0^1 delta_a(b_i) delta_b(b_j) w dx over ALL m = n_el + p
    basis functions (App. A; kind selects the derivative orders (a, b))."""
    nq = p + 5 if nq is None else nq
    da, db = _DER[kind]
    kn = open_knots(n_el, p)
    x, w = gauss_points(n_el, nq)
    Ba = basis(kn, p, x, da)
    Bb = basis(kn, p, x, db)
    wx = w * weight_values(weight, x)
    return Ba.T @ (wx[:, None] * Bb)


def dof_range(n_el: int, p: int, bc=(0, 0)) -> tuple[int, int]:
    """[lo, hi) of the full basis kept by the space with boundary flags
    bc = (k0, k1) (Appendix B's notation: 1 = Neumann, 0 = Dirichlet at x = 0
    and x = 1): a Dirichlet end drops the one basis function that does not
    vanish there (Sec. 2.2), a Neumann end keeps it.  n = hi - lo =
    n_el + p - 2 + k0 + k1."""
    k0, k1 = bc
    return (0 if k0 else 1), n_el + p - (0 if k1 else 1)


def matrix(n_el: int, p: int, kind: str, weight=(1.0, 0.0, 0.0, 0.0),
           nq: int | None = None, bc=(0, 0)) -> np.ndarray:
    """The same integral restricted to the space with boundary flags bc; the
    default (0, 0) is the Dirichlet space of Sec. 2.2 (basis functions
    2..m-1), n = n_el + p - 2."""
    A = matrix_full(n_el, p, kind, weight, nq)
    lo, hi = dof_range(n_el, p, bc)
    return A[lo:hi, lo:hi]


def load_vector(n_el: int, p: int, weight, nq: int | None = None, bc=(0, 0)) -> np.ndarray:
    """F_i = int_0^1 b_i(x) g(x) dx for the basis of the space with boundary
    flags bc (App. A, the 1D moments forming the rhs factors), g from the
    weight family."""
    nq = p + 5 if nq is None else nq
    kn = open_knots(n_el, p)
    x, w = gauss_points(n_el, nq)
    B = basis(kn, p, x, 0)
    F = B.T @ (w * weight_values(weight, x))
    lo, hi = dof_range(n_el, p, bc)
    return F[lo:hi]


def dirichlet_basis_at(n_el: int, p: int, x, der: int = 0) -> np.ndarray:
    """Values/derivatives of the Dirichlet basis b_1..b_n at points x."""
    return basis(open_knots(n_el, p), p, x, der)[:, 1:-1]


def greville(n_el: int, p: int) -> np.ndarray:
    """Greville abscissae of the full basis, xi_i = (t_{i+1} + ... + t_{i+p})/p:
    sum_i xi_i b_i(x) = x on [0, 1] (B-splines of degree p >= 1 reproduce
    linear polynomials with these coefficients)."""
    kn = open_knots(n_el, p)
    m = n_el + p
    return np.array([kn[i + 1:i + p + 1].mean() for i in range(m)])
