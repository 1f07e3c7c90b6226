"""Appendix A front end: the Tucker matrix (eq. matrix_CP) and vector of a
problem on a mapped domain from separable approximations of Q(eta) =
det(J) J^{-1} J^{-T} and omega(eta) = det(J) f(F(eta)).

A coefficient function g sampled on the tensor grid of t Chebyshev-Lobatto
points of [0, 1] has the Chebyshev coefficient tensor G x_1 Phi x_2 Phi
x_3 Phi, Phi the values-to-coefficients map of one direction: the Tucker
tensor (values; Phi, Phi, Phi).  The library's relative truncation
(tucker_truncate, Algorithm 1 on the device) compresses it, the tolerance
set so that the discarded part has Frobenius norm eps * scale (scale: the
largest sampled value, shared by the entries of Q so that entries that
vanish up to rounding are dropped).  Every retained factor column is a
Chebyshev series in one variable; the 1D matrices and load vectors with
those weights come from tk_assemble_1d_cheb and tk_load_vector_1d_cheb.
The paper uses chebfun3f (cross approximation, never the full tensor) for
the same separable forms; here the t^3 samples are formed, which is cheap at
the t these coefficients need.
"""
from __future__ import annotations

import numpy as np

from . import tk

KIND = {(0, 0): "mass", (1, 1): "stiff", (1, 0): "mixed10", (0, 1): "mixed01"}


def cheb_points(t: int) -> np.ndarray:
    """Chebyshev-Lobatto points of [0, 1], x_k = (1 + cos(pi k / (t - 1))) / 2."""
    return 0.5 * (1.0 + np.cos(np.pi * np.arange(t) / (t - 1)))


def cheb_transform(t: int) -> np.ndarray:
    """Phi (t x t): values at the Lobatto points -> coefficients of
    sum_m c_m T_m(2x - 1) (the discrete cosine transform of type I:
    c_m = (2 / (t - 1)) sum''_k g_k cos(pi m k / (t - 1)), the sum halving
    the terms k = 0, t - 1, and c_0, c_{t-1} halved)."""
    k = np.arange(t)
    Phi = (2.0 / (t - 1)) * np.cos(np.pi * np.outer(k, k) / (t - 1))
    Phi[:, 0] *= 0.5
    Phi[:, -1] *= 0.5
    Phi[0, :] *= 0.5
    Phi[-1, :] *= 0.5
    return Phi


def separable(ctx, values: np.ndarray, eps: float, scale: float | None = None):
    """(core, [C1, C2, C3]) on the host: the truncated Tucker form of the
    Chebyshev coefficient tensor of the sampled values (t1 x t2 x t3), the
    factor columns being coefficient vectors; None when the whole tensor is
    below eps * scale."""
    scale = float(np.abs(values).max()) if scale is None else scale
    Phis = [cheb_transform(values.shape[k]) for k in range(3)]
    g = tk.Tucker.from_host(ctx, np.ascontiguousarray(values), Phis)
    nrm = float(np.sqrt(max(tk.dot(ctx, g, g), 0.0)))
    if nrm <= eps * scale:
        return None
    core, U = tk.tucker_truncate(ctx, g, eps * scale / nrm)[0].plain()
    if core.size == 0:
        return None
    return core, U


def operator(ctx, n_el: int, p: int, q_values, eps: float, bc=((0, 0),) * 3) -> tuple:
    """(Operator, ranks) of eq. matrix_CP from the sampled entries q_values[(k, l)]
    of Q (t x t x t arrays on the Lobatto grid; Q symmetric, the entries
    below the diagonal take their mirror's approximation): per entry with a nonzero
    approximation, its core as a diagonal block and, per mode s and factor
    column, the 1D matrix with the test function differentiated when s = l
    and the trial function when s = k."""
    scale = max(float(np.abs(v).max()) for v in q_values.values())
    bands = [[], [], []]
    nnz = []
    ranks = {}
    seps = {}
    for (k, l), vals in sorted(q_values.items()):
        # Q is symmetric: the entry below the diagonal reuses the approximation
        # of its mirror, which makes the (l, k) term the transpose of the
        # (k, l) one and the Tucker matrix exactly symmetric
        sep = seps[(l, k)] if k > l and (l, k) in seps else separable(ctx, vals, eps, scale)
        seps[(k, l)] = sep
        if sep is None:
            ranks[(k, l)] = (0, 0, 0)
            continue
        core, U = sep
        ranks[(k, l)] = core.shape
        off = [len(bands[s]) for s in range(3)]
        for s in range(3):
            kind = KIND[(int(s == l), int(s == k))]
            for r in range(U[s].shape[1]):
                bands[s].append(tk.assemble_1d_cheb(n_el, p, kind, U[s][:, r], bc[s]))
        for (a, b, c), v in np.ndenumerate(core):
            if v != 0.0:
                nnz.append((off[0] + a, off[1] + b, off[2] + c, float(v)))
    n = [n_el + p - 2 + bc[s][0] + bc[s][1] for s in range(3)]
    return tk.Operator.create(ctx, p, n, [np.stack(b) for b in bands], nnz), ranks


def rhs(ctx, n_el: int, p: int, omega_values: np.ndarray, eps: float, bc=((0, 0),) * 3) -> tk.Tucker:
    """Tucker vector with core W and factors F~_t[i, j] = int b_i w_{t, j}."""
    sep = separable(ctx, omega_values, eps)
    if sep is None:
        raise ValueError("the load vanishes")
    core, U = sep
    F = [np.stack([tk.load_vector_1d_cheb(n_el, p, U[s][:, j], bc[s]) for j in range(U[s].shape[1])], axis=1)
         for s in range(3)]
    return tk.Tucker.from_host(ctx, core, F)


def fd_coefficients(q_values) -> tuple:
    """Direction coefficients of the FD preconditioner (Algorithm 4 for
    c_1 K x M x M + ...): the mean over the samples of each diagonal entry
    of Q, i.e. the parametric Laplacian scaled to the geometry's average
    anisotropy."""
    return tuple(float(np.mean(q_values[(k, k)])) for k in range(3))


def evaluate(x: "tk.Tucker", n_el: int, p: int, e1, e2, e3, bc=((0, 0),) * 3) -> np.ndarray:
    """The spline function with Tucker coefficients x on the tensor grid
    e1 x e2 x e3 of parametric points: core x_k (B_k U_k), B_k the basis
    values from tk_basis_values_1d (host post-processing)."""
    core, U = x.plain()
    V = [tk.basis_values_1d(n_el, p, e, 0, bc[k]) @ U[k] for k, e in enumerate((e1, e2, e3))]
    return np.einsum("abc,ia,jb,kc->ijk", core, V[0], V[1], V[2])
