"""GPU checks of the symmetric eigensolver behind the ST-HOSVD (tk_sym_eig):
Householder tridiagonalisation, multisection, inverse iteration, two
Gram-Schmidt passes, back transformation.

Parity is stated against properties that pin an eigendecomposition at any
size, plus numpy's eigvalsh for the eigenvalues:
* orthonormality  max |V^T V - I| <= 50 a u;
* residual        max |G V - V diag(w)| <= 50 a u max |G|;
* eigenvalues     max |w - eigvalsh(G)| <= 50 a u max |G| (both descending).
The spectra cover the shapes the Gram matrices of the solver take: flat
(clustered), geometrically graded over 16 and 30 decades (below the rounding
level of G), low rank with an exactly zero tail, exactly repeated
eigenvalues, the zero matrix, and the orders 1, 2, 3, the largest order the
in-LDS path takes (136) and both sides of it, a = 300 (block Gram-Schmidt
with 32-column panels) and a = 700 (27-column panels, the LDS budget's
width)."""
import numpy as np
import pytest

from gpu_helpers import context, say

pytestmark = pytest.mark.gpu

U = np.finfo(float).eps


@pytest.fixture(scope="module")
def ctx():
    return context()


def spectrum(kind, a, rng):
    if kind == "flat":
        return 1.0 + rng.uniform(0, 1e-2, a)
    if kind == "graded16":
        return np.logspace(0, -16, a)
    if kind == "graded30":
        return np.logspace(0, -30, a)
    if kind == "lowrank":
        k = max(1, a // 4)
        return np.concatenate([np.logspace(0, -6, k), np.zeros(a - k)])
    if kind == "repeated":
        return np.repeat(np.logspace(0, -6, (a + 2) // 3), 3)[:a]
    if kind == "zero":
        return np.zeros(a)
    raise ValueError(kind)


def run_eig(ctx, G):
    import torch
    from paper_2306_00632_amd import tk
    a = G.shape[0]
    Gd = torch.tensor(np.asfortranarray(G).ravel(order="F"), dtype=torch.float64, device="cuda")
    V = torch.empty(a * a, dtype=torch.float64, device="cuda")
    w = torch.empty(a, dtype=torch.float64, device="cuda")
    tk.sym_eig(ctx, Gd, a, V, w)
    ctx.sync()
    Gback = Gd.cpu().numpy().reshape(a, a, order="F")
    assert np.array_equal(Gback, G), "G must not be modified"
    return V.cpu().numpy().reshape(a, a, order="F"), w.cpu().numpy()


@pytest.mark.parametrize("a", [1, 2, 3, 17, 64, 129, 135, 136, 137, 300, 700])
@pytest.mark.parametrize("kind", ["flat", "graded16", "graded30", "lowrank", "repeated", "zero"])
def test_sym_eig_properties(ctx, a, kind):
    say(f"sym_eig a={a} {kind}")
    rng = np.random.default_rng(1000 * a + len(kind))
    ev = spectrum(kind, a, rng)
    Q, _ = np.linalg.qr(rng.standard_normal((a, a)))
    Z = Q * np.sqrt(ev)
    G = Z @ Z.T
    G = 0.5 * (G + G.T)
    V, w = run_eig(ctx, G)
    gmax = max(np.abs(G).max(), np.finfo(float).tiny)
    tol = 50 * a * U
    assert np.all(np.isfinite(V)) and np.all(np.isfinite(w))
    assert np.abs(V.T @ V - np.eye(a)).max() <= tol
    if kind == "zero":
        assert np.abs(w).max() <= 1e-300
        return
    assert np.abs(G @ V - V * w).max() <= tol * gmax
    ref = np.sort(np.linalg.eigvalsh(G))[::-1]
    assert np.all(np.diff(w) <= 0)
    assert np.abs(w - ref).max() <= tol * gmax


def test_sym_eig_scale_invariance(ctx):
    """The power-of-two scaling makes the result independent of the scale of G."""
    rng = np.random.default_rng(7)
    a = 40
    Z = rng.standard_normal((a, 3 * a))
    G = Z @ Z.T
    V1, w1 = run_eig(ctx, G)
    V2, w2 = run_eig(ctx, G * 2.0 ** -700)
    V3, w3 = run_eig(ctx, G * 2.0 ** 600)
    assert np.array_equal(V1, V2) and np.array_equal(V1, V3)
    assert np.array_equal(w1 * 2.0 ** -700, w2) and np.array_equal(w1 * 2.0 ** 600, w3)


def test_sym_eig_deterministic(ctx):
    rng = np.random.default_rng(8)
    a = 129
    Z = rng.standard_normal((a, a)) * np.logspace(0, -8, a)
    G = Z @ Z.T
    V1, w1 = run_eig(ctx, G)
    V2, w2 = run_eig(ctx, G)
    assert np.array_equal(V1, V2) and np.array_equal(w1, w2)
