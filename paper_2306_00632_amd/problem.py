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
