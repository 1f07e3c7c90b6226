"""GPU parity of the two HBM-bound mode-product kernels at the batched sizes
the benchmark times: one tall factor of m independent columns (tensor ranks
(m, 1, 1)), the banded operator of eq. (tt_product) at n_el = 1024, p = 2,
R = 9 with m = 40000, and the FD chain of Algorithm 4 at n_el = 1024, p = 3
with m = 25600.  The oracle cannot apply either to all columns in seconds, so
it checks a sample of columns that includes both ends of the range and the
first and last column of a column block; the one-column modes are checked
whole.  Tolerances as in the small parity tests: 1e-12 relative for the
banded sums, 1e-9 for the FD chain (independent Remez solvers)."""
import ctypes as C

import numpy as np
import pytest

import bench
from oracle import fd as ofd
from oracle import problem as oprob
from oracle import tucker as T

from gpu_helpers import context, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return context()


def factor_rows(ctx, t, k, cols=None):
    """Columns `cols` (all if None) of the stacked factor k of a library
    tensor, read on the device, as a host array (n, len(cols))."""
    import torch
    from paper_2306_00632_amd import tk
    n, m, _ = t.shape()
    buf = torch.empty(n[k] * m[k], dtype=torch.float64, device="cuda")
    ctx.check(tk.lib().tk_tucker_read(ctx.h, t.h, k, C.c_void_p(buf.data_ptr()), -1, None, 1),
              "tk_tucker_read")
    F = buf.view(m[k], n[k])   # row c holds column c of the column-major factor
    if cols is not None:
        F = F[torch.as_tensor(cols, device="cuda")]
    return F.cpu().numpy().T


def sample_columns(m, block, seed):
    rng = np.random.default_rng(seed)
    fixed = [0, 1, block - 1, block, m - block - 1, m - block, m - 2, m - 1]
    return np.unique(np.concatenate([fixed, rng.integers(0, m, 40)]))


def test_band_apply_batched(ctx):
    from paper_2306_00632_amd import problem, tk
    w, core, U = bench.k1_inputs()
    m = U[0].shape[1]
    say(f"band_apply batched n={w.n} p={w.p} R={len(w.nnz)} m={m}")
    y = tk.tucker_apply_op(ctx, problem.operator(ctx, w), tk.Tucker.from_host(ctx, core, U))
    n, mm, nb = y.shape()
    R = len(w.nnz)
    assert mm == (R * m, R, R) and nb == R
    op = oprob.operator(w)
    cols = sample_columns(m, 8, 31)
    got = factor_rows(ctx, y, 0, np.concatenate([t * m + cols for t in range(R)]))
    for t in range(R):
        ref = op.mats[0][t] @ U[0][:, cols]
        g = got[:, t * len(cols):(t + 1) * len(cols)]
        np.testing.assert_allclose(g, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    for k in (1, 2):
        ref = np.concatenate([A @ U[k] for A in op.mats[k]], axis=1)
        np.testing.assert_allclose(factor_rows(ctx, y, k), ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_fd_chain_batched(ctx):
    from paper_2306_00632_amd import tk
    core, U = bench.k2_inputs()
    sh = bench.K2_SHAPE
    m = U[0].shape[1]
    say(f"fd_precond batched n_el={sh['n_el']} p={sh['p']} m={m}")
    P = tk.Preconditioner.create(ctx, sh["n_el"], sh["p"], 0.1)
    z = tk.fd_precond(ctx, P, tk.Tucker.from_host(ctx, core, U))
    ref_P = ofd.LowRankFD(sh["n_el"], sh["p"], 0.1)
    Rp = ref_P.R_P
    assert P.info()["R_P"] == Rp
    cols = sample_columns(m, 1, 32)
    s = T.Tucker(core[cols], [U[0][:, cols], U[1], U[2]])
    ref = ref_P.apply(s)
    c = len(cols)
    got = factor_rows(ctx, z, 0, np.concatenate([j * m + cols for j in range(Rp)]))
    scale = np.abs(ref.U[0]).max()
    np.testing.assert_allclose(got, ref.U[0], rtol=1e-9, atol=1e-9 * scale)
    for k in (1, 2):
        np.testing.assert_allclose(factor_rows(ctx, z, k), ref.U[k], rtol=1e-9,
                                   atol=1e-9 * np.abs(ref.U[k]).max())
    # block structure: block j at offsets (j m, j, j) with coefficient omega_j / lambda_min
    blocks = z.blocks()
    assert [o for _, _, o in blocks] == [(j * m, j, j) for j in range(Rp)]
    assert c == ref.U[0].shape[1] // Rp
