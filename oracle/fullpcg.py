"""Full-tensor reference solutions (oracle; test infrastructure).

* `dense_solve`: the assembled n^3 x n^3 system (eq. approx_ls) solved
  directly, for tiny n.
* `pcg_exact_fd`: textbook preconditioned CG on full tensors, with the exact
  Fast Diagonalization preconditioner of Algorithm 3 (eq. factorized_FD)
  built from the parametric 1D stiffness and mass matrices; stops at
  ||f - A x|| <= rtol ||f||.
"""
from __future__ import annotations

import numpy as np

from . import bspline, problem
from .fd import ExactFD
from .tucker import vec


def dense_solve(op, f_full: np.ndarray) -> np.ndarray:
    A = op.dense()
    x = np.linalg.solve(A, vec(f_full))
    return x.reshape(f_full.shape, order="F")


def pcg_exact_fd(w, op, f_full: np.ndarray, rtol: float = 1e-12, maxit: int = 2000,
                 fd_coef=(1.0, 1.0, 1.0)):
    K = [bspline.matrix(w.n_el, w.p, "stiff")] * 3
    M = [bspline.matrix(w.n_el, w.p, "mass")] * 3
    P = ExactFD(K, M, fd_coef)
    smats = problem.sparse_mats(op)
    A = lambda X: problem.apply_full(smats, op.nnz, X)
    x = np.zeros_like(f_full)
    r = f_full.copy()
    nf = np.linalg.norm(f_full)
    z = P.apply_full(r)
    p = z.copy()
    rz = np.sum(r * z)
    it = 0
    while np.linalg.norm(r) > rtol * nf and it < maxit:
        q = A(p)
        a = rz / np.sum(p * q)
        x += a * p
        r -= a * q
        z = P.apply_full(r)
        rz_new = np.sum(r * z)
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    # report the true residual
    res = np.linalg.norm(f_full - A(x)) / nf
    return x, it, res
