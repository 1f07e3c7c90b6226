"""Library objects from `workloads` recipes: 1D matrices are assembled by
the library (tk_assemble_1d / tk_load_vector_1d), then uploaded."""
from __future__ import annotations

import numpy as np

from . import tk


def operator(ctx, w) -> tk.Operator:
    bands = []
    for k in range(3):
        bands.append(np.stack([tk.assemble_1d(w.n_el, w.p, kind, weight) for kind, weight in w.modes[k]]))
    return tk.Operator.create(ctx, w.p, (w.n,) * 3, bands, w.nnz)


def rhs_arrays(w):
    """(core, factors) of the right-hand side as host arrays."""
    spec = w.rhs
    if spec["kind"] == "random":
        return np.asarray(spec["core"]), [np.asarray(u) for u in spec["factors"]]
    F = tk.load_vector_1d(w.n_el, w.p, spec["weight"])
    return np.ones((1, 1, 1)), [F[:, None].copy() for _ in range(3)]


def rhs(ctx, w) -> tk.Tucker:
    core, U = rhs_arrays(w)
    return tk.Tucker.from_host(ctx, core, U)


def preconditioner(ctx, w, eps_prec=0.1, coef=(1.0, 1.0, 1.0), exact=False) -> tk.Preconditioner:
    return tk.Preconditioner.create(ctx, w.n_el, w.p, eps_prec, coef, exact=exact)


# --- boundary conditions other than homogeneous Dirichlet ---------------------

def dof_range(n_el: int, p: int, bc) -> tuple:
    """[lo, hi) of the full spline basis (n_el + p functions) kept by the space
    with boundary flags bc = (k0, k1): 1 Neumann (kept end function), 0
    Dirichlet (dropped)."""
    return (0 if bc[0] else 1), n_el + p - (0 if bc[1] else 1)


def operator_bc(ctx, w, bcs) -> tk.Operator:
    """The workload's Tucker matrix on the spaces with flags bcs[k]
    (bcs = ((1, 1),) * 3: the full basis)."""
    bands = [np.stack([tk.assemble_1d_bc(w.n_el, w.p, kind, weight, bcs[k]) for kind, weight in w.modes[k]])
             for k in range(3)]
    n = [w.n_el + w.p - 2 + bcs[k][0] + bcs[k][1] for k in range(3)]
    return tk.Operator.create(ctx, w.p, n, bands, w.nnz)


def preconditioner_bc(ctx, w, bcs, eps_prec=0.1, coef=(1.0, 1.0, 1.0), exact=False) -> tk.Preconditioner:
    """FD (Algorithm 4) on the spaces with flags bcs[k]: the Appendix B
    eigen-approximations with Neumann ends (default) or the exact
    eigenpairs (Algorithm 3's factorizations), both applied densely."""
    return tk.Preconditioner.create(ctx, w.n_el, w.p, eps_prec, coef, exact=exact, bcs=bcs)


def lifted_rhs(ctx, w, bcs, g_core, g_factors, f=None, op_full=None) -> tk.Tucker:
    """f - A_dOmega g~ of the non-homogeneous Dirichlet system (remark closing
    Sec. 3): g~ (Tucker: g_core, full-basis factors g_factors, n_el + p rows)
    extends the Dirichlet data; g_B = g~ minus its restriction to the
    unknowns (zero-extended), and A_dOmega g~ = R A_full g_B with the
    full-basis operator and R the restriction of factor rows to the unknowns.
    f (a tensor on the unknowns) may be None for f = 0."""
    rng = [dof_range(w.n_el, w.p, bcs[k]) for k in range(3)]
    masked = []
    for k in range(3):
        u = np.array(g_factors[k], dtype=np.float64, copy=True)
        u[:rng[k][0]] = 0.0
        u[rng[k][1]:] = 0.0
        masked.append(u)
    g = tk.Tucker.from_host(ctx, g_core, g_factors)
    gm = tk.Tucker.from_host(ctx, g_core, masked)
    neg_gb = tk.axpby(ctx, -1.0, g, 1.0, gm)   # -g_B
    op_full = op_full or operator_bc(ctx, w, ((1, 1),) * 3)
    lift = tk.tucker_rows(ctx, tk.tucker_apply_op(ctx, op_full, neg_gb), [r[0] for r in rng],
                          [r[1] - r[0] for r in rng])   # -R A_full g_B
    return lift if f is None else tk.axpby(ctx, 1.0, f, 1.0, lift)


# --- block (3-component) systems --------------------------------------------

def block_operator(ctx, bw) -> list:
    """3 x 3 nested list of Operator (None for a zero block) of a BlockWorkload."""
    ops = [[None] * 3 for _ in range(3)]
    for (a, b), (modes, nnz) in bw.blocks.items():
        bands = [np.stack([tk.assemble_1d(bw.n_el, bw.p, kind, weight) for kind, weight in modes[k]])
                 for k in range(3)]
        ops[a][b] = tk.Operator.create(ctx, bw.p, (bw.n,) * 3, bands, nnz)
    return ops


def block_rhs(ctx, bw) -> list:
    return [tk.Tucker.from_host(ctx, np.asarray(spec["core"]), [np.asarray(u) for u in spec["factors"]])
            for spec in bw.rhs]


def block_preconditioner(ctx, bw, eps_prec=0.1) -> list:
    """Block-diagonal preconditioner: one FD per component with its direction
    coefficients."""
    return [tk.Preconditioner.create(ctx, bw.n_el, bw.p, eps_prec, bw.prec_coef[a]) for a in range(3)]
