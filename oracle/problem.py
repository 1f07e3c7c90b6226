"""Operators and right-hand sides from the `workloads` recipes (oracle).

The operator is the Tucker matrix of eq. (tucker_matrix) whose 1D factors
are the weighted integrals of Appendix A; the right-hand side is a Tucker
vector (random data, or the 1D moments of a separable load, Appendix A).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import bspline
from .tucker import Tucker, TuckerMatrix


def operator(w) -> TuckerMatrix:
    mats = [[bspline.matrix(w.n_el, w.p, kind, weight) for (kind, weight) in w.modes[k]]
            for k in range(3)]
    return TuckerMatrix(mats, w.nnz)


def rhs(w) -> Tucker:
    spec = w.rhs
    if spec["kind"] == "random":
        return Tucker(spec["core"], spec["factors"])
    if spec["kind"] == "load":
        F = bspline.load_vector(w.n_el, w.p, spec["weight"])
        return Tucker(np.ones((1, 1, 1)), [F[:, None].copy() for _ in range(3)])
    raise ValueError(spec["kind"])


def sparse_mats(op: TuckerMatrix):
    return [[sp.csr_matrix(A) for A in op.mats[k]] for k in range(3)]


def apply_full(smats, nnz, X: np.ndarray) -> np.ndarray:
    """A vec(X) for the Tucker matrix, on a full tensor, with sparse 1D
    factors: sum_nz c * X x_1 A_(1,i1) x_2 A_(2,i2) x_3 A_(3,i3)."""
    n = X.shape
    out = np.zeros_like(X)
    cache = {}
    for i1, i2, i3, c in nnz:
        key1 = i1
        if ("1", key1) not in cache:
            cache[("1", key1)] = (smats[0][i1] @ X.reshape(n[0], -1, order="F")).reshape(n, order="F")
        T = cache[("1", key1)]
        T = np.moveaxis(T, 1, 0)
        T = (smats[1][i2] @ T.reshape(n[1], -1, order="F")).reshape((n[1], n[0], n[2]), order="F")
        T = np.moveaxis(T, 0, 1)
        T = np.moveaxis(T, 2, 0)
        T = (smats[2][i3] @ T.reshape(n[2], -1, order="F")).reshape((n[2], n[0], n[1]), order="F")
        T = np.moveaxis(T, 0, 2)
        out += c * T
    return out
