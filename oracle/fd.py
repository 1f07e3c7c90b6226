"""Fast Diagonalization preconditioners (oracle; test infrastructure).

Sec. 4.2:
* Algorithm 3 (exact FD): generalized eigendecompositions K_i U_i = M_i U_i
  Lambda_i with U_i^T M_i U_i = I (eq. factorizations) and
  P^{-1} = (U3 x U2 x U1) (I x I x L1 + I x L2 x I + L3 x I x I)^{-1} (U3 x U2 x U1)^T
  (eq. factorized_FD), applied here to full tensors.
* Algorithm 4 (low-rank FD): approximate eigenpairs (Appendix B), the
  exponential-sum approximation of the inverse diagonal (eqs.
  estimate_prec_rel, approx_diagonal, diag_factor) and the Tucker-format
  application with core P (x) S (eq. core_tens_prec).

Appendix B (Dirichlet at both ends) is built densely, as written:
  V_h = V_h1 (+) V_h2, V_h1 = {phi : phi^(2k)(0) = phi^(2k)(1) = 0, 2k <= p-1},
  basis Phi0 u Phi u Phi1 of V_h1 (columns of V1), interpolation points
  (breakpoints for odd p, span midpoints for even p), collocation matrix
  C_ij = v_i(x_j), U_dft = sqrt(2) sin(j pi x_i), Lambda1 = (j pi)^2,
  V_h2 = M-orthogonal complement of V_h1 with its exact small eigenproblem.
Readings of the paper taken here:
* "C^{-1} U_dft" is the interpolation in V_h1 of the sampled sines (the
  coefficients a with sum_i a_i v_i(x_j) = U_dft[j, :]);
* "normalized in the L^2 norm": every approximate eigenvector function (a
  column of V1 U1) is scaled to unit L^2 norm, i.e. unit M-norm, as the exact
  ones of eq. factorizations (U^T M U = I); the printed factors sqrt(2) then
  play no role.  With this reading exact and approximate eigenpairs give
  nearly the same TPCG iteration counts, as the remark in Sec. 5 states
  (25 against 12 iterations at n_el = 32, p = 2 without the scaling);
* the M-orthogonal complement of ker(D) is spanned by V2 = M^{-1} D^T, where
  D holds the even-derivative constraints;
* for p = 2 (n2 = 0) the same sine construction is used; it reproduces the
  p = 2 row of Table 1 (M_P = n_el^2).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import bspline, expsum
from .tucker import Tucker, TuckerSum, mode_product


# ---------------------------------------------------------------------------
# exact FD (Algorithm 3)
# ---------------------------------------------------------------------------

class ExactFD:
    """P = K3 x M2 x M1 + M3 x K2 x M1 + M3 x M2 x K1 (eq. FD_prec), with
    optional positive coefficients c_i scaling the stiffness of direction i."""

    def __init__(self, K, M, coef=(1.0, 1.0, 1.0)):
        self.U, self.lam = [], []
        for i in range(3):
            lam, U = sla.eigh(coef[i] * K[i], M[i])   # M-orthonormal eigenvectors
            self.U.append(U)
            self.lam.append(lam)

    def apply_full(self, S: np.ndarray) -> np.ndarray:
        """Steps 2-4 of Algorithm 3 on a full tensor."""
        T = S
        for k in range(3):
            T = mode_product(T, self.U[k].T, k)
        L = (self.lam[0][:, None, None] + self.lam[1][None, :, None] + self.lam[2][None, None, :])
        T = T / L
        for k in range(3):
            T = mode_product(T, self.U[k], k)
        return T


# ---------------------------------------------------------------------------
# Appendix B: approximate eigenpairs, Dirichlet at both ends
# ---------------------------------------------------------------------------

def subspace_dims(n_el: int, p: int, bc=(0, 0)):
    """n = n_el + p - 2 + k0 + k1; n1 = dim V_h1 and n2 = dim V_h2 (Appendix
    B): n1 = n_el - 1 + k0 + k1 for odd p, n_el for even p (the number of
    interpolation points), n2 = n - n1 (the end constraints)."""
    k0, k1 = bc
    n = n_el + p - 2 + k0 + k1
    n1 = n_el - 1 + k0 + k1 if p % 2 == 1 else n_el
    return n, n1, n - n1


def interpolation_points(n_el: int, p: int, bc=(0, 0)) -> np.ndarray:
    """Breakpoints for odd p (the ends only where the condition is Neumann),
    span midpoints for even p."""
    k0, k1 = bc
    if p % 2 == 1:
        return np.arange(1 - k0, n_el + k1) / n_el
    return (np.arange(1, n_el + 1) - 0.5) / n_el


def _constraint_orders(p: int, neumann: int):
    """Derivative orders fixed to zero at an end in V_h1 (Appendix B): the
    even ones 2k (k >= 1, 2k <= p - 1) at a Dirichlet end (the value is
    zero in the space already), the odd ones 2k + 1 <= p - 1 at a Neumann
    end."""
    if neumann:
        return list(range(1, p, 2))
    return list(range(2, p, 2))


def _constraints(n_el, p, at, bc=(0, 0)):
    """Rows phi -> phi^(d)(at) over the constrained orders d of that end, on
    the basis of the space with flags bc."""
    neumann = bc[0] if at == 0.0 else bc[1]
    lo, hi = bspline.dof_range(n_el, p, bc)
    kn = bspline.open_knots(n_el, p)
    rows = [bspline.basis(kn, p, [at], d)[0, lo:hi] for d in _constraint_orders(p, neumann)]
    return np.array(rows).reshape(-1, hi - lo)


def _end_block(p: int, neumann: int) -> int:
    """Number of leading (trailing) basis functions of the space that carry
    the constrained derivatives at x = 0 (x = 1): the derivative of order d
    there involves the first d + 1 functions of the full basis."""
    orders = _constraint_orders(p, neumann)
    return (max(orders) + 1 - (0 if neumann else 1)) if orders else 0


def exact_eig(n_el: int, p: int, bc=(0, 0)):
    """(U, Lambda) of eq. factorizations for one direction: K U = M U Lambda,
    U^T M U = I, with the parametric 1D stiffness and mass on the space with
    boundary flags bc (default: the Dirichlet space).  With Neumann at both
    ends the constants are in the space and the smallest eigenvalue is 0 in
    exact arithmetic; computed values below 1e-12 lambda_max (rounding: the
    smallest nonzero one is about pi^2) are set to 0."""
    K = bspline.matrix(n_el, p, "stiff", bc=bc)
    M = bspline.matrix(n_el, p, "mass", bc=bc)
    lam, U = sla.eigh(K, M)
    return U, np.where(lam < 1e-12 * lam.max(), 0.0, lam)


def approx_eig(n_el: int, p: int, bc=(0, 0)):
    """(U~, Lambda~, parts) of Appendix B for one direction, on the space
    with boundary flags bc = (k0, k1) (1 Neumann, 0 Dirichlet; the default is
    the Dirichlet case the appendix starts with).

    U~ = [V1 U1 | V2 U2] (n x n), Lambda~ = [Lambda1 ; Lambda2]; the sines
    are sin((j - k0/2 - k1/2) pi x + k0 pi/2) and Lambda1 = ((j - k0/2 -
    k1/2) pi)^2 (with Neumann at both ends j = 1 is the constant,
    eigenvalue 0)."""
    k0, k1 = bc
    n, n1, n2 = subspace_dims(n_el, p, bc)
    assert n_el > p, "Appendix B assumes n_el > p"
    K = bspline.matrix(n_el, p, "stiff", bc=bc)
    M = bspline.matrix(n_el, p, "mass", bc=bc)
    D0 = _constraints(n_el, p, 0.0, bc)
    D1 = _constraints(n_el, p, 1.0, bc)
    D = np.vstack([D0, D1]) if n2 > 0 else np.zeros((0, n))
    e0, e1 = _end_block(p, k0), _end_block(p, k1)

    # basis Phi0 u Phi u Phi1 of V_h1 (columns of V1)
    V1 = np.zeros((n, n1))
    col = 0
    if e0 > 0:
        N0 = sla.null_space(D0[:, :e0])              # Phi0 in the span of the first e0 functions
        V1[:e0, col:col + N0.shape[1]] = N0
        col += N0.shape[1]
    for j in range(e0, n - e1):                      # Phi: single basis functions
        V1[j, col] = 1.0
        col += 1
    if e1 > 0:
        N1 = sla.null_space(D1[:, n - e1:])          # Phi1 in the span of the last e1 functions
        V1[n - e1:, col:col + N1.shape[1]] = N1
        col += N1.shape[1]
    assert col == n1

    x = interpolation_points(n_el, p, bc)
    lo, hi = bspline.dof_range(n_el, p, bc)
    Bx = bspline.basis(bspline.open_knots(n_el, p), p, x, 0)[:, lo:hi]   # Bx[j, l] = b_l(x_j)
    C = (Bx @ V1).T                                  # C[i, j] = v_i(x_j)
    jj = np.arange(1, n1 + 1)
    freq = jj - 0.5 * (k0 + k1)
    Udft = np.sqrt(2.0) * np.sin(np.pi * np.outer(x, freq) + 0.5 * np.pi * k0)   # [U_dft]_{i,j}
    U1 = np.linalg.solve(C.T, Udft)                  # interpolation in V_h1
    # unit L^2 (= M) norm of every interpolated sine
    W1 = V1 @ U1
    scale1 = 1.0 / np.sqrt(np.einsum("ij,ij->j", W1, M @ W1))
    parts = {"V1": V1, "C": C, "Udft": Udft, "U1": U1, "D": D, "K": K, "M": M,
             "x": x, "n1": n1, "n2": n2, "scale1": scale1}
    lam1 = (np.pi * freq) ** 2
    if n2 > 0:
        V2 = np.linalg.solve(M, D.T)                 # M-orthogonal complement
        lam2, U2 = sla.eigh(V2.T @ K @ V2, V2.T @ M @ V2)
        parts.update(V2=V2, U2=U2, lam2=lam2)
        Ut = np.hstack([W1 * scale1, V2 @ U2])
        lam = np.concatenate([lam1, lam2])
    else:
        Ut = W1 * scale1
        lam = lam1
    return Ut, lam, parts


# ---------------------------------------------------------------------------
# Algorithm 4: low-rank FD
# ---------------------------------------------------------------------------

class LowRankFD:
    """P~^{-1} = (1/lambda_min) (U~3 x U~2 x U~1) (sum_j omega_j D3j x D2j x D1j)
    (U~3 x U~2 x U~1)^T (eq. prec); with exact=True the eigenpairs are the
    exact ones of eq. factorizations instead of Appendix B's.

    `coef` scales the approximate eigenvalues of each direction (block
    preconditioners with direction coefficients); `expsum_table` may hold
    precomputed (R_P, alpha, omega) for this M_P."""

    def __init__(self, n_el, p, eps_prec=0.1, coef=(1.0, 1.0, 1.0), expsum_table=None, exact=False,
                 bcs=((0, 0), (0, 0), (0, 0))):
        self.Ut, self.lam = [], []
        if np.isscalar(n_el):
            n_el = (n_el,) * 3
        for i in range(3):
            if exact:   # Algorithm 4 with the exact factorizations of Algorithm 3
                U, lam = exact_eig(n_el[i], p, bcs[i])
            else:
                U, lam, _ = approx_eig(n_el[i], p, tuple(bcs[i]))
            self.Ut.append(U)
            self.lam.append(coef[i] * lam)
        self.lam_min = sum(np.min(l) for l in self.lam)
        self.lam_max = sum(np.max(l) for l in self.lam)
        if not self.lam_min > 0:
            raise ValueError("the operator is singular (Neumann at every end of every direction)")
        self.M_P = self.lam_max / self.lam_min
        if expsum_table is None:
            R, al, om, E, Eprev = expsum.exp_sum_for(self.M_P, eps_prec)
        else:
            R, al, om = expsum_table[:3]
            E = Eprev = None
        self.R_P, self.alpha, self.omega = R, np.asarray(al), np.asarray(om)
        self.E, self.E_prev = E, Eprev

    def diag_factor(self, i, j):
        """[D_(i,j)]_mm = exp(-alpha_j/lambda_min [Lambda~_i]_mm)  (eq. diag_factor)."""
        return np.exp(-self.alpha[j] / self.lam_min * self.lam[i])

    def apply(self, s) -> TuckerSum:
        """Application steps of Algorithm 4: Z_i = U~_i^T S_i,
        W_(i,j) = D_(i,j) Z_i, Y_(i,j) = U~_i W_(i,j); core P (x) S, whose
        nonzero blocks are (omega_j / lambda_min) S at block (j, j, j)."""
        if not isinstance(s, Tucker):
            s = s.to_tucker()
        r = s.ranks
        U = []
        for i in range(3):
            Z = self.Ut[i].T @ s.U[i]
            Y = [self.Ut[i] @ (self.diag_factor(i, j)[:, None] * Z) for j in range(self.R_P)]
            U.append(np.concatenate(Y, axis=1) if Y else np.zeros((s.n[i], 0)))
        blocks = [(self.omega[j] / self.lam_min, s.core, (j * r[0], j * r[1], j * r[2]))
                  for j in range(self.R_P)]
        return TuckerSum(U, blocks)

    def dense_inverse(self) -> np.ndarray:
        """P~^{-1} assembled (tiny sizes only)."""
        N = np.prod([u.shape[0] for u in self.Ut])
        P = np.zeros((N, N))
        Ukron = np.kron(self.Ut[2], np.kron(self.Ut[1], self.Ut[0]))
        d = np.zeros(N)
        for j in range(self.R_P):
            d += self.omega[j] * np.kron(self.diag_factor(2, j),
                                         np.kron(self.diag_factor(1, j), self.diag_factor(0, j)))
        return Ukron @ np.diag(d / self.lam_min) @ Ukron.T
