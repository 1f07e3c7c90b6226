"""GPU checks of the library's FP64 matrix-core GEMM (tk_dgemm), the dense
contraction under the mode products of eq. tt_product and the Tucker scalar
products, against numpy's matmul on the same data.

Bound: |C - C_ref| <= 8 K u (|op(A)| |op(B)|) elementwise (+ the beta term),
the standard error bound of a length-K dot product with a few extra ulps for
reassociation (blocking over K, split-K partial sums)."""
import numpy as np
import pytest

from gpu_helpers import context, say

pytestmark = pytest.mark.gpu
U = np.finfo(float).eps


@pytest.fixture(scope="module")
def ctx():
    return context()


def dev(x):
    import torch
    return torch.tensor(np.asfortranarray(x).ravel(order="F"), dtype=torch.float64, device="cuda")


SHAPES = [
    (1, 1, 1), (7, 5, 3), (64, 16, 16), (65, 17, 17), (129, 129, 129),   # ragged tails of every tile
    (16641, 129, 5), (16641, 129, 130), (300, 33, 47), (129, 129, 16641),  # tall, split-K
    (140, 150, 2000), (33, 65, 97), (5, 200, 3),
]


@pytest.mark.parametrize("M,N,K", SHAPES)
@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
def test_dgemm_matches_numpy(ctx, M, N, K, ta, tb):
    from paper_2306_00632_amd import tk
    say(f"dgemm M={M} N={N} K={K} ta={ta} tb={tb}")
    rng = np.random.default_rng(M * 7 + N * 13 + K * 17 + 2 * ta + tb)
    opA = rng.standard_normal((M, K))
    opB = rng.standard_normal((K, N))
    C0 = rng.standard_normal((M + 3, N))  # ldc = M + 3
    A = opA.T.copy() if ta else opA
    B = opB.T.copy() if tb else opB
    alpha, beta = 0.75, (0.0 if (M + N) % 2 else -1.25)
    Ad, Bd, Cd = dev(A), dev(B), dev(C0)
    tk.dgemm(ctx, ta, tb, M, N, K, alpha, Ad, A.shape[0], Bd, B.shape[0], beta, Cd, M + 3)
    ctx.sync()
    got = Cd.cpu().numpy().reshape(N, M + 3).T
    ref = alpha * (opA @ opB) + beta * C0[:M]
    bound = 8 * K * U * abs(alpha) * (np.abs(opA) @ np.abs(opB)) + 4 * U * abs(beta) * np.abs(C0[:M])
    assert np.all(np.abs(got[:M] - ref) <= bound + 1e-300)
    assert np.array_equal(got[M:], C0[M:]), "rows beyond M must not be written"
