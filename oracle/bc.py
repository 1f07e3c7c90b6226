"""Boundary conditions other than homogeneous Dirichlet (oracle; test
infrastructure only: the library never imports it).

* Neumann ends.  Appendix B describes the spaces with flags (k0, k1), 1 for
  a Neumann condition at x = 0 or x = 1: a Neumann end keeps the basis
  function that does not vanish there, a Dirichlet end drops it (Sec. 2.2),
  so direction k has n_k = n_el + p - 2 + k0 + k1 unknowns.  The operator's
  1D matrices are the same integrals on those spaces (bspline.matrix with
  bc) and the exact FD of Algorithm 3 uses their generalized eigenpairs
  (fd.exact_eig with bc).
* Non-homogeneous Dirichlet data (the remark closing Sec. 3, eq.
  nonhomog-dirichlet-system): with g~ the coefficients of (an extension of)
  the data on the full tensor-product basis, the unknowns solve
  A x = f - A_dOmega g~, where A_dOmega couples the test functions of the
  unknowns to the trial functions at prescribed dofs.  With the full-space
  operator A_full, R the restriction to the unknown dofs and g_B the part
  of g~ at prescribed dofs (g~ minus its restriction to the unknowns, put
  back by zero extension), A_dOmega g~ = R A_full g_B.  Everything stays in
  Tucker format: g_B is a sum of two Tucker tensors with the same core, R
  selects factor rows.
"""
from __future__ import annotations

import numpy as np

from . import bspline
from .tucker import Tucker, TuckerMatrix, TuckerSum, apply_op, tsum


def operator(w, bcs) -> TuckerMatrix:
    """The workload's Tucker matrix on the spaces with flags bcs[k]."""
    mats = [[bspline.matrix(w.n_el, w.p, kind, weight, bc=bcs[k]) for (kind, weight) in w.modes[k]]
            for k in range(3)]
    return TuckerMatrix(mats, w.nnz)


def operator_full(w) -> TuckerMatrix:
    """The workload's Tucker matrix on the full basis (m = n_el + p per mode)."""
    mats = [[bspline.matrix_full(w.n_el, w.p, kind, weight) for (kind, weight) in w.modes[k]]
            for k in range(3)]
    return TuckerMatrix(mats, w.nnz)


def unknown_mask(n_el: int, p: int, bc) -> np.ndarray:
    """1 on the full-basis indices that are unknowns of the space with flags bc."""
    lo, hi = bspline.dof_range(n_el, p, bc)
    m = np.zeros(n_el + p)
    m[lo:hi] = 1.0
    return m


def restrict(x, n_el: int, p: int, bcs):
    """Factor rows of a full-space tensor (Tucker or TuckerSum) restricted to
    the unknowns of the spaces with flags bcs."""
    rng = [bspline.dof_range(n_el, p, bcs[k]) for k in range(3)]
    if isinstance(x, Tucker):
        return Tucker(x.core, [x.U[k][rng[k][0]:rng[k][1]] for k in range(3)])
    return TuckerSum([x.U[k][rng[k][0]:rng[k][1]] for k in range(3)], x.blocks)


def boundary_part(g: Tucker, n_el: int, p: int, bcs) -> TuckerSum:
    """g_B = g~ - (g~ restricted to the unknowns, zero-extended): the same core
    with the factors and their masked copies, weights +1 and -1."""
    masked = Tucker(g.core, [unknown_mask(n_el, p, bcs[k])[:, None] * g.U[k] for k in range(3)])
    return tsum([(1.0, g), (-1.0, masked)])


def lifted_rhs(w, bcs, g: Tucker, f=None) -> TuckerSum:
    """f - R A_full g_B (eq. nonhomog-dirichlet-system); f (on the unknowns)
    may be None for f = 0."""
    lift = restrict(apply_op(operator_full(w), boundary_part(g, w.n_el, w.p, bcs)), w.n_el, w.p, bcs)
    if f is None:
        return tsum([(-1.0, lift)])
    return tsum([(1.0, f), (-1.0, lift)])


def linear_coefficients(n_el: int, p: int, a) -> Tucker:
    """Full-basis coefficients of u(x, y, z) = a0 + a1 x + a2 y + a3 z (exact:
    the constants have coefficients 1, the coordinates their Greville
    abscissae), a Tucker tensor of multilinear rank at most (2, 2, 2)."""
    xi = bspline.greville(n_el, p)
    one = np.ones_like(xi)
    U = [np.stack([one, xi], axis=1) for _ in range(3)]
    core = np.zeros((2, 2, 2))
    core[0, 0, 0] = a[0]
    core[1, 0, 0] = a[1]
    core[0, 1, 0] = a[2]
    core[0, 0, 1] = a[3]
    return Tucker(core, U)
