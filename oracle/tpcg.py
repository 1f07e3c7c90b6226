"""Truncated Preconditioned Conjugate Gradient, Algorithm 5 (oracle).

All vectors are Tucker vectors; products use eq. (tt_product), scalar
products Sec. 2.3, truncations Algorithms 1 and 2, the preconditioner
Algorithm 4.

Readings of the paper taken here:
* the rhs is normalised to ||f|| = 1 internally and the solution scaled back,
  so the absolute test ||r_k|| > tol of Algorithm 5 and the "relative
  tolerance" of Sec. 5 agree; eps_min = tol ||f~|| / 10 (Sec. 5) is taken
  with the norm of the given rhs (for IgA load vectors ||f~|| ~ n_el^{-3/2},
  so the floor tightens under refinement), capped at tol / 10 when
  ||f~|| > 1;
* eta_k follows eq. (rel_tol_iterates) as printed;
* x_0 = 0 (Sec. 5), so r_0 = f;
* when ||r_{k+1}|| <= tol the loop ends before z, p, q are formed (x is not
  affected);
* xi_k <= 0 or a non-finite scalar stops the iteration as a breakdown.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .tucker import Tucker, apply_op, dot, norm, tdt, trel, tsum


@dataclass
class TPCGInfo:
    iters: int = 0
    relres: float = 0.0
    converged: bool = False
    breakdown: bool = False
    ranks: list = field(default_factory=list)
    eps: list = field(default_factory=list)
    trel_calls: int = 0


def tpcg(op, prec, f: Tucker, tol=1e-6, beta=0.1, eps0=0.1, alpha=0.5,
         eps_min=None, delta=1e-3, maxit=1000):
    nf = norm(f)
    n = f.n
    if nf == 0.0:
        return Tucker.zero(n), TPCGInfo(converged=True)
    f = Tucker(f.core / nf, f.U)
    if eps_min is None:
        eps_min = 0.1 * tol * min(1.0, nf)    # tol ||f~|| 1e-1 (Sec. 5), at most tol / 10
    info = TPCGInfo()
    x = Tucker.zero(n)
    r = f                            # r_0 = f - A x_0 with x_0 = 0
    nr = 1.0
    eta = beta * tol / nr
    z = trel(prec.apply(r), eta)
    p = z
    q = trel(apply_op(op, p), eta)
    xi = dot(p, q)
    eps = eps0
    k = 0
    info.trel_calls = 2
    while nr > tol and k < maxit:
        if not np.isfinite(xi) or xi <= 0.0:
            info.breakdown = True
            break
        om = dot(r, p) / xi
        x_new, eps, calls = tdt(x, tsum([(1.0, x), (om, p)]), tsum([(om, p)]),
                                eps, alpha, eps_min, delta)
        info.trel_calls += calls
        x = x_new
        r = trel(tsum([(1.0, f), (-1.0, apply_op(op, x))]), eta)
        nr = norm(r)
        k += 1
        info.ranks.append(x.ranks)
        info.eps.append(eps)
        if nr <= tol:
            break
        eta = beta * tol / nr
        z = trel(prec.apply(r), eta)
        bk = -dot(z, q) / xi
        p = trel(tsum([(1.0, z), (bk, p)]), eta)
        q = trel(apply_op(op, p), eta)
        xi = dot(p, q)
        info.trel_calls += 4
    info.iters = k
    info.relres = nr
    info.converged = nr <= tol
    return Tucker(x.core * nf, x.U), info
