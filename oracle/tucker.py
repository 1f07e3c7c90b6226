"""Tucker-format algebra and truncation (oracle; test infrastructure).

Sec. 2.3 of the paper: m-mode products, the Tucker format of a tensor and of
a vector, Tucker matrices (eq. tucker_matrix), the Tucker-matrix times
Tucker-vector product (eq. tt_product), scalar products and sums.
Sec. 4.1: relative truncation T^rel (Algorithm 1) and dynamic truncation
T^dt (Algorithm 2).

Memory layout follows the vec operator of Sec. 2.3 (first index fastest):
a tensor X of shape (n1, n2, n3) satisfies vec(X) = X.ravel(order="F").

A sum of Tucker vectors (eq. after tt_product) has a block-diagonal core and
the product with a Tucker matrix has the core C (x) X (eq. tt_product).  Both
are kept here as a `TuckerSum`: stacked factor matrices Y_k plus a list of
core blocks (coefficient, block core, column offset of the block in every
Y_k).  `dense_core()` writes out the full core; every operation below is the
corresponding operation on that core, evaluated block by block.
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------------------
# m-mode product and the Tucker format (Sec. 2.3)
# ---------------------------------------------------------------------------

def mode_product(X: np.ndarray, J: np.ndarray, m: int) -> np.ndarray:
    """[X x_m J]_{.., i_m, ..} = sum_j J[i_m, j] X[.., j, ..]  (Sec. 2.3).

    The printed index order of the sum is garbled ([J]_{j,i_m} with J of size
    l x n_m); the reading that makes eq. (kron_vec_multi) hold is used: J acts
    on mode m from the left.  m is 0-based here."""
    Xm = np.moveaxis(X, m, 0)
    Y = np.tensordot(J, Xm, axes=([1], [0]))
    return np.moveaxis(Y, 0, m)


def vec(X: np.ndarray) -> np.ndarray:
    """vec with the first index fastest (Sec. 2.3)."""
    return X.ravel(order="F")


class Tucker:
    """X = core x_3 U3 x_2 U2 x_1 U1 (eq. Tucker)."""

    def __init__(self, core, U):
        self.core = np.asarray(core, dtype=float)
        self.U = [np.asarray(u, dtype=float) for u in U]
        assert self.core.ndim == 3
        for k in range(3):
            assert self.U[k].shape[1] == self.core.shape[k]

    @property
    def n(self):
        return tuple(u.shape[0] for u in self.U)

    @property
    def ranks(self):
        return tuple(self.core.shape)

    def full(self) -> np.ndarray:
        X = self.core
        for k in range(3):
            X = mode_product(X, self.U[k], k)
        return X

    def as_sum(self) -> "TuckerSum":
        return TuckerSum([u.copy() for u in self.U], [(1.0, self.core, (0, 0, 0))])

    @staticmethod
    def zero(n) -> "Tucker":
        return Tucker(np.zeros((0, 0, 0)), [np.zeros((n[k], 0)) for k in range(3)])


class TuckerSum:
    """A Tucker vector whose core is block structured.

    U[k]   : stacked factor matrix Y_k, shape (n_k, m_k)
    blocks : list of (c, G, (o1, o2, o3)); the full core has c*G at rows
             o_k .. o_k + G.shape[k]-1 of every mode."""

    def __init__(self, U, blocks):
        self.U = [np.asarray(u, dtype=float) for u in U]
        self.blocks = [(float(c), np.asarray(G, dtype=float), tuple(int(o) for o in off))
                       for (c, G, off) in blocks]

    @property
    def n(self):
        return tuple(u.shape[0] for u in self.U)

    @property
    def m(self):
        return tuple(u.shape[1] for u in self.U)

    def dense_core(self) -> np.ndarray:
        C = np.zeros(self.m)
        for c, G, o in self.blocks:
            r = G.shape
            C[o[0]:o[0] + r[0], o[1]:o[1] + r[1], o[2]:o[2] + r[2]] += c * G
        return C

    def to_tucker(self) -> Tucker:
        return Tucker(self.dense_core(), self.U)

    def full(self) -> np.ndarray:
        return self.to_tucker().full()

    def block_factors(self, b):
        c, G, o = self.blocks[b]
        return [self.U[k][:, o[k]:o[k] + G.shape[k]] for k in range(3)]


def as_sum(x) -> TuckerSum:
    return x if isinstance(x, TuckerSum) else x.as_sum()


def tsum(terms) -> TuckerSum:
    """sum_i a_i x_i: factors concatenated, cores placed on the block
    diagonal (Sec. 2.3, sum of two Tucker vectors), scaled by a_i."""
    U = [[], [], []]
    blocks = []
    off = [0, 0, 0]
    for a, x in terms:
        s = as_sum(x)
        for c, G, o in s.blocks:
            blocks.append((a * c, G, tuple(o[k] + off[k] for k in range(3))))
        for k in range(3):
            U[k].append(s.U[k])
            off[k] += s.U[k].shape[1]
    n = as_sum(terms[0][1]).n
    U = [np.concatenate(U[k], axis=1) if U[k] else np.zeros((n[k], 0)) for k in range(3)]
    return TuckerSum(U, blocks)


# ---------------------------------------------------------------------------
# Tucker matrices and the product of eq. (tt_product)
# ---------------------------------------------------------------------------

class TuckerMatrix:
    """C = sum_{i1,i2,i3} [core]_{i1 i2 i3} C_(3,i3) (x) C_(2,i2) (x) C_(1,i1)
    (eq. tucker_matrix) with a sparse core given by its nonzeros."""

    def __init__(self, mats, nnz):
        self.mats = [[np.asarray(A, dtype=float) for A in mats[k]] for k in range(3)]
        self.nnz = [(int(a), int(b), int(c), float(v)) for (a, b, c, v) in nnz]

    def dense(self) -> np.ndarray:
        """The assembled matrix (tiny sizes only), Kronecker order of Sec. 2.3."""
        n = [self.mats[k][0].shape[0] for k in range(3)]
        A = np.zeros((n[0] * n[1] * n[2],) * 2)
        for i1, i2, i3, c in self.nnz:
            A += c * np.kron(self.mats[2][i3], np.kron(self.mats[1][i2], self.mats[0][i1]))
        return A


def apply_op(op: TuckerMatrix, x) -> TuckerSum:
    """C x via eq. (tt_product): the factor of mode k is
    [C_(k,1) Y_k, ..., C_(k,R_k) Y_k] and the core is core(C) (x) core(x);
    block (i1, i2, i3) of that Kronecker core is c_{i1 i2 i3} * core(x),
    placed at column block i_k of mode k."""
    s = as_sum(x)
    U = []
    for k in range(3):
        U.append(np.concatenate([A @ s.U[k] for A in op.mats[k]], axis=1))
    m = s.m
    blocks = []
    for i1, i2, i3, c in op.nnz:
        for cb, G, o in s.blocks:
            off = (i1 * m[0] + o[0], i2 * m[1] + o[1], i3 * m[2] + o[2])
            blocks.append((c * cb, G, off))
    return TuckerSum(U, blocks)


# ---------------------------------------------------------------------------
# scalar products (Sec. 2.3)
# ---------------------------------------------------------------------------

def _dot_single(Gx, Ux, Gy, Uy) -> float:
    """<X, Y> = vec(core_X)^T vec(core_Y x_3 X3^T Y3 x_2 X2^T Y2 x_1 X1^T Y1)."""
    T = Gy
    for k in range(3):
        T = mode_product(T, Ux[k].T @ Uy[k], k)
    return float(np.sum(Gx * T))


def dot(x, y) -> float:
    """Scalar product of Tucker vectors; sums are expanded bilinearly."""
    sx, sy = as_sum(x), as_sum(y)
    total = 0.0
    for bx in range(len(sx.blocks)):
        cx, Gx, _ = sx.blocks[bx]
        Fx = sx.block_factors(bx)
        for by in range(len(sy.blocks)):
            cy, Gy, _ = sy.blocks[by]
            total += cx * cy * _dot_single(Gx, Fx, Gy, sy.block_factors(by))
    return total


def norm(x) -> float:
    return float(np.sqrt(max(dot(x, x), 0.0)))


# ---------------------------------------------------------------------------
# ST-HOSVD and Algorithm 1 (relative truncation)
# ---------------------------------------------------------------------------

def unfold(Z: np.ndarray, k: int) -> np.ndarray:
    """Mode-k unfolding: rows indexed by i_k, columns by the remaining
    indices (first fastest)."""
    rest = int(np.prod([Z.shape[j] for j in range(3) if j != k]))
    return np.moveaxis(Z, k, 0).reshape(Z.shape[k], rest, order="F")


def sthosvd(Z: np.ndarray, eps: float):
    """Sequentially truncated HOSVD with ||Z - Z~||_F <= eps ||Z||_F (Sec. 2.3).

    Modes are processed in the order 1, 2, 3.  In mode k the singular values
    of the current core's unfolding (numpy SVD, never a Gram matrix) decide
    the rank: s_k is the smallest s whose discarded energy sum_{i>s} sigma_i^2
    is at most eps^2 ||Z||^2 / 3, which bounds the total error by eps ||Z||.
    Returns (core, [S1, S2, S3]) with orthonormal S_k of shape r_k x s_k."""
    budget = (eps ** 2) * float(np.sum(Z * Z)) / 3.0
    S = []
    core = Z
    for k in range(3):
        A = unfold(core, k)
        if A.size == 0 or not np.any(A):
            s = 0
            Uk = np.zeros((core.shape[k], 0))
        else:
            Uk, sig, _ = np.linalg.svd(A, full_matrices=False)
            tail = np.concatenate([np.cumsum((sig ** 2)[::-1])[::-1], [0.0]])
            s = int(np.argmax(tail <= budget))        # smallest s with tail[s] <= budget
            Uk = Uk[:, :s]
        S.append(Uk)
        core = mode_product(core, Uk.T, k)
    return core, S


def trel(y, eps: float) -> Tucker:
    """T^rel(y, eps), Algorithm 1.

    Step 1: QR of every stacked factor Y_k = Q_k R_k (economy size; when
            m_k > n_k the factor R_k is n_k x m_k).
    Step 2: Z = core x_3 R_3 x_2 R_2 x_1 R_1, evaluated block by block
            (Z = sum_b c_b G_b x_k R_k[:, cols of block b]).
    Step 3: (core~, S_k) = sthosvd(Z, eps).
    Step 4: Y~_k = Q_k S_k."""
    s = as_sum(y)
    Q, R = [], []
    for k in range(3):
        q, r = np.linalg.qr(s.U[k], mode="reduced")
        Q.append(q)
        R.append(r)
    Z = np.zeros(tuple(R[k].shape[0] for k in range(3)))
    for c, G, o in s.blocks:
        T = G
        for k in range(3):
            T = mode_product(T, R[k][:, o[k]:o[k] + G.shape[k]], k)
        Z += c * T
    core, S = sthosvd(Z, eps)
    return Tucker(core, [Q[k] @ S[k] for k in range(3)])


def tdt(y_k: Tucker, y_tilde, dy_tilde, eps: float, alpha: float,
        eps_min: float, delta: float):
    """Dynamic truncation T^dt, Algorithm 2.

    `dy_tilde` is the proposed step y_tilde - y_k (step 2).  In TPCG it equals
    omega_k p_k exactly, and the caller passes it in that form.
    Loop: y_{k+1} = T^rel(y_tilde, eps_new); v = dy_tilde.(y_{k+1}-y_k)/|dy_tilde|^2;
    stop if |v - 1| < delta; otherwise shrink eps_new by alpha while
    alpha*eps_new > eps_min (the printed test uses the loop-invariant eps,
    which cannot terminate; eps_new is read), else stop.
    Returns (y_{k+1}, eps_new, number of T^rel calls)."""
    eps_new = eps
    den = dot(dy_tilde, dy_tilde)
    base = dot(dy_tilde, y_k)
    calls = 0
    while True:
        y1 = trel(y_tilde, eps_new)
        calls += 1
        if den == 0.0:
            break
        v = (dot(dy_tilde, y1) - base) / den
        if abs(v - 1.0) < delta:
            break
        if alpha * eps_new > eps_min:
            eps_new *= alpha
        else:
            break
    return y1, eps_new, calls


def memory_compression(x: Tucker) -> float:
    """eq. (mem_comp): (r1 r2 r3 + sum_k r_k n_k) / (n1 n2 n3) * 100."""
    r, n = x.ranks, x.n
    return (r[0] * r[1] * r[2] + sum(r[k] * n[k] for k in range(3))) / (n[0] * n[1] * n[2]) * 100.0


def rel_diff(x, y) -> float:
    """||x - y|| / ||y|| for Tucker vectors, without forming full tensors and
    without cancellation: QR of the stacked factors, then the Frobenius norm
    of the small core of x - y."""
    d = tsum([(1.0, x), (-1.0, y)])
    Q, R = [], []
    for k in range(3):
        q, r = np.linalg.qr(d.U[k], mode="reduced")
        R.append(r)
    Z = np.zeros(tuple(R[k].shape[0] for k in range(3)))
    for c, G, o in d.blocks:
        T = G
        for k in range(3):
            T = mode_product(T, R[k][:, o[k]:o[k] + G.shape[k]], k)
        Z += c * T
    ny = norm(y)
    return float(np.linalg.norm(Z)) / ny if ny > 0 else float(np.linalg.norm(Z))
