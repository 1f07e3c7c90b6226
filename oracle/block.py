"""Block (3-component) systems of Sec. 5.3, compressible linear elasticity
(oracle; test infrastructure).

The system matrix is a 3 x 3 block matrix whose blocks are Tucker matrices
and the unknown is a triple of Tucker vectors (eq. block-system-elasticity).
Following Sec. 5.3, matrix-vector products, scalar products, sums and
truncations act blockwise with the machinery of Secs. 2.3 and 4:

* (A x)_a = sum_b A_ab x_b, a Tucker sum per component (eq. tt_product per
  block);
* <x, y> = sum_a <x_a, y_a>;
* T^rel and T^dt truncate every component with the same relative tolerance
  (so the block vector meets the same bound);
* the preconditioner is block diagonal, one low-rank FD (Algorithm 4) per
  component, with the component's direction coefficients.

Readings of the paper taken here: the paper builds the blocks from a mapped
column by a Chebyshev/Tucker fit of the geometry coefficients (App. A);
here they come from the seeded recipe of ``workloads.elasticity`` (a
weighted cube, Dirichlet on all faces).
"""
from __future__ import annotations

import numpy as np

from . import bspline
from .fd import LowRankFD
from .tpcg import TPCGInfo
from .tucker import Tucker, TuckerMatrix, apply_op, dot, norm, trel, tsum


def operator(bw) -> dict:
    """{(a, b): TuckerMatrix} for the nonzero blocks of the block workload."""
    out = {}
    for (a, b), (modes, nnz) in bw.blocks.items():
        mats = [[bspline.matrix(bw.n_el, bw.p, kind, weight) for (kind, weight) in modes[k]]
                for k in range(3)]
        out[(a, b)] = TuckerMatrix(mats, nnz)
    return out


def rhs(bw) -> list:
    return [Tucker(spec["core"], spec["factors"]) for spec in bw.rhs]


def apply(A: dict, x: list) -> list:
    """(A x)_a = sum_b A_ab x_b, one Tucker sum per component."""
    out = []
    for a in range(3):
        terms = [(1.0, apply_op(A[(a, b)], x[b])) for b in range(3) if (a, b) in A]
        out.append(tsum(terms))
    return out


def bdot(x: list, y: list) -> float:
    return float(sum(dot(x[a], y[a]) for a in range(3)))


def bnorm(x: list) -> float:
    return float(np.sqrt(max(bdot(x, x), 0.0)))


def btrel(y: list, eps: float) -> list:
    return [trel(y[a], eps) for a in range(3)]


def bsum(terms) -> list:
    """sum_i c_i y_i for block vectors y_i, componentwise Tucker sums."""
    return [tsum([(c, y[a]) for c, y in terms]) for a in range(3)]


class BlockFD:
    """Block-diagonal preconditioner: component a gets Algorithm 4 with the
    direction coefficients prec_coef[a] (c_1 L~_1 + c_2 L~_2 + c_3 L~_3)."""

    def __init__(self, bw, eps_prec: float = 0.1):
        self.parts = [LowRankFD(bw.n_el, bw.p, eps_prec, coef=bw.prec_coef[a]) for a in range(3)]

    def apply(self, s: list) -> list:
        return [self.parts[a].apply(s[a]) for a in range(3)]


def btdt(y_k: list, y_tilde: list, dy_tilde: list, eps: float, alpha: float, eps_min: float,
         delta: float):
    """Algorithm 2 on block vectors: every component truncated at eps_new,
    v = dy.(y_{k+1} - y_k) / |dy|^2 with block scalar products."""
    eps_new = eps
    den = bdot(dy_tilde, dy_tilde)
    base = bdot(dy_tilde, y_k)
    calls = 0
    while True:
        y1 = btrel(y_tilde, eps_new)
        calls += 1
        if den == 0.0:
            break
        v = (bdot(dy_tilde, y1) - base) / den
        if abs(v - 1.0) < delta:
            break
        if alpha * eps_new > eps_min:
            eps_new *= alpha
        else:
            break
    return y1, eps_new, calls


def tpcg(A: dict, prec: BlockFD, f: list, tol=1e-6, beta=0.1, eps0=0.1, alpha=0.5, eps_min=None,
         delta=1e-3, maxit=1000):
    """Algorithm 5 on block vectors, with the readings of oracle.tpcg (rhs
    normalised to norm 1 and the solution scaled back, eps_min = tol / 10
    times min(1, ||f||), x_0 = 0, eta_k as
    printed, early exit when ||r_{k+1}|| <= tol, breakdown on xi <= 0)."""
    nf = bnorm(f)
    n = f[0].n
    if nf == 0.0:
        return [Tucker.zero(n) for _ in range(3)], TPCGInfo(converged=True)
    f = [Tucker(f[a].core / nf, f[a].U) for a in range(3)]
    if eps_min is None:
        eps_min = 0.1 * tol * min(1.0, nf)
    info = TPCGInfo()
    x = [Tucker.zero(n) for _ in range(3)]
    r = f
    nr = 1.0
    eta = beta * tol / nr
    z = btrel(prec.apply(r), eta)
    p = z
    q = btrel(apply(A, p), eta)
    xi = bdot(p, q)
    eps = eps0
    k = 0
    info.trel_calls = 2
    while nr > tol and k < maxit:
        if not np.isfinite(xi) or xi <= 0.0:
            info.breakdown = True
            break
        om = bdot(r, p) / xi
        x, eps, calls = btdt(x, bsum([(1.0, x), (om, p)]), bsum([(om, p)]), eps, alpha, eps_min, delta)
        info.trel_calls += calls
        r = btrel(bsum([(1.0, f), (-1.0, apply(A, x))]), eta)
        nr = bnorm(r)
        k += 1
        info.ranks.append([x[a].ranks for a in range(3)])
        info.eps.append(eps)
        if nr <= tol:
            break
        eta = beta * tol / nr
        z = btrel(prec.apply(r), eta)
        bk = -bdot(z, q) / xi
        p = btrel(bsum([(1.0, z), (bk, p)]), eta)
        q = btrel(apply(A, p), eta)
        xi = bdot(p, q)
        info.trel_calls += 4
    info.iters = k
    info.relres = nr
    info.converged = nr <= tol
    return [Tucker(x[a].core * nf, x[a].U) for a in range(3)], info


# ---------------------------------------------------------------------------
# assembled forms (tiny sizes; references and pins)
# ---------------------------------------------------------------------------

def dense(A: dict, n: int) -> np.ndarray:
    """The assembled 3N x 3N block matrix (Kronecker order of Sec. 2.3 per
    block), N = n^3."""
    N = n ** 3
    out = np.zeros((3 * N, 3 * N))
    for (a, b), op in A.items():
        out[a * N:(a + 1) * N, b * N:(b + 1) * N] = op.dense()
    return out


def dense_full(bw) -> np.ndarray:
    """The same block matrix over ALL m = n_el + p basis functions per
    direction (no boundary condition), for the rigid-motion pins."""
    m = bw.n_el + bw.p
    N = m ** 3
    out = np.zeros((3 * N, 3 * N))
    for (a, b), (modes, nnz) in bw.blocks.items():
        mats = [[bspline.matrix_full(bw.n_el, bw.p, kind, weight) for (kind, weight) in modes[k]]
                for k in range(3)]
        out[a * N:(a + 1) * N, b * N:(b + 1) * N] = TuckerMatrix(mats, nnz).dense()
    return out


def to_full(x: list) -> np.ndarray:
    """Concatenated vec of the three components."""
    return np.concatenate([x[a].full().ravel(order="F") for a in range(3)])
