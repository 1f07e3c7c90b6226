"""ctypes binding of libtk.so (include/tk.h).  Argument marshalling only:
every numerical step runs inside the library (HIP kernels on the GPU, host
C++ for the one-time setup).  The library must be built
(`paper_2306_00632_amd.build.build()`); nothing here falls back to Python or
CPU arithmetic."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtk.so")

TK_OK, TK_EINVAL, TK_ENOMEM, TK_EDEVICE, TK_ENOCONV, TK_EBREAKDOWN, TK_ENUMERIC = 0, -1, -2, -3, -4, -5, -6
KINDS = {"mass": 0, "stiff": 1, "mixed10": 2, "mixed01": 3}

_lib = None
vp = C.c_void_p
i64p = C.POINTER(C.c_int64)
i32p = C.POINTER(C.c_int32)
dp = C.POINTER(C.c_double)


class TkError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"tk status {status}: {msg}")
        self.status = status


class CoreNz(C.Structure):
    _fields_ = [("i1", C.c_int32), ("i2", C.c_int32), ("i3", C.c_int32), ("c", C.c_double)]


class TpcgParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("beta", C.c_double), ("eps0", C.c_double),
                ("alpha", C.c_double), ("eps_min", C.c_double), ("delta", C.c_double),
                ("maxit", C.c_int32), ("verbose", C.c_int32), ("arith", C.c_int32),
                ("refine_below", C.c_double), ("reuse_bases", C.c_int32)]


class TpcgInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("relres", C.c_double),
                ("rank", C.c_int64 * 3), ("eps_final", C.c_double), ("trel_calls", C.c_int32),
                ("f32_applications", C.c_int32)]


EXPORTS = {
    "tk_ctx_create": (C.c_int32, [C.c_int, vp, C.POINTER(vp)]),
    "tk_ctx_destroy": (None, [vp]),
    "tk_last_error": (C.c_char_p, [vp]),
    "tk_ctx_sync": (C.c_int32, [vp]),
    "tk_ctx_trim": (C.c_int32, [vp]),
    "tk_assemble_1d": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32, dp, dp]),
    "tk_assemble_1d_bc": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32, dp, C.c_int32, C.c_int32, dp]),
    "tk_assemble_1d_cheb": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, dp, C.c_int32, C.c_int32, dp]),
    "tk_load_vector_1d_cheb": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32, dp, C.c_int32, C.c_int32, dp]),
    "tk_truncate_refinements": (C.c_int32, [vp, i64p]),
    "tk_basis_values_1d": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int64, dp, dp]),
    "tk_load_vector_1d": (C.c_int32, [C.c_int32, C.c_int32, dp, dp]),
    "tk_fd_direction_host": (C.c_int32, [C.c_int32, C.c_int32, C.c_double, i32p, i32p, i32p, dp, dp, dp, dp]),
    "tk_expsum_host": (C.c_int32, [C.c_double, C.c_double, i32p, dp, dp, dp, dp]),
    "tk_tucker_create": (C.c_int32, [vp, i64p, i64p, vp, C.POINTER(vp), C.c_int32, C.POINTER(vp)]),
    "tk_tucker_free": (None, [vp]),
    "tk_tucker_shape": (C.c_int32, [vp, i64p, i64p, i32p]),
    "tk_tucker_block": (C.c_int32, [vp, C.c_int32, dp, i64p, i64p]),
    "tk_tucker_read": (C.c_int32, [vp, vp, C.c_int32, vp, C.c_int32, vp, C.c_int32]),
    "tk_tucker_dot": (C.c_int32, [vp, vp, vp, dp]),
    "tk_tucker_axpby": (C.c_int32, [vp, C.c_double, vp, C.c_double, vp, C.POINTER(vp)]),
    "tk_tucker_rows": (C.c_int32, [vp, vp, i64p, i64p, C.POINTER(vp)]),
    "tk_op_create": (C.c_int32, [vp, C.c_int32, i64p, i32p, C.POINTER(dp), C.POINTER(CoreNz),
                                 C.c_int64, C.POINTER(vp)]),
    "tk_op_free": (None, [vp]),
    "tucker_apply_op": (C.c_int32, [vp, vp, vp, C.POINTER(vp)]),
    "tucker_apply_op_arith": (C.c_int32, [vp, vp, vp, C.c_int32, C.POINTER(vp)]),
    "fd_setup": (C.c_int32, [vp, i32p, C.c_int32, C.c_double, dp, C.POINTER(vp), i32p]),
    "fd_setup_exact": (C.c_int32, [vp, i32p, C.c_int32, C.c_double, dp, C.POINTER(vp), i32p]),
    "fd_setup_exact_bc": (C.c_int32, [vp, i32p, C.c_int32, C.c_double, dp, i32p, C.POINTER(vp), i32p]),
    "fd_setup_bc": (C.c_int32, [vp, i32p, C.c_int32, C.c_double, dp, i32p, C.POINTER(vp), i32p]),
    "tk_fd_direction_dense_host": (C.c_int32, [C.c_int32, C.c_int32, C.c_double, C.c_int32, C.c_int32, i32p, dp, dp]),
    "tk_prec_free": (None, [vp]),
    "tk_prec_info": (C.c_int32, [vp, i32p, dp, dp, dp, dp, dp]),
    "tk_prec_direction": (C.c_int32, [vp, C.c_int32, i32p, i32p, i32p, dp, dp, dp, dp]),
    "fd_precond": (C.c_int32, [vp, vp, vp, C.POINTER(vp)]),
    "fd_precond_arith": (C.c_int32, [vp, vp, vp, C.c_int32, C.POINTER(vp)]),
    "tucker_truncate": (C.c_int32, [vp, vp, C.c_double, C.POINTER(vp), dp]),
    "tk_tpcg_defaults": (None, [C.POINTER(TpcgParams)]),
    "tk_sym_eig": (C.c_int32, [vp, vp, C.c_int32, vp, vp]),
    "tucker_apply_op_block": (C.c_int32, [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp)]),
    "tpcg_solve_block": (C.c_int32, [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                                     C.POINTER(TpcgParams), C.POINTER(vp), C.POINTER(TpcgInfo)]),
    "tk_dgemm": (C.c_int32, [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                             vp, C.c_int32, vp, C.c_int32, C.c_double, vp, C.c_int32]),
    "tk_prof_enable": (C.c_int32, [vp, C.c_int32]),
    "tk_prof_reset": (C.c_int32, [vp]),
    "tk_prof_read": (C.c_int32, [vp, C.c_int32, i64p, dp, dp, dp]),
    "tpcg_solve": (C.c_int32, [vp, vp, vp, vp, C.POINTER(TpcgParams), C.POINTER(vp),
                               C.POINTER(TpcgInfo)]),
}


def lib():
    """Load libtk.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2306_00632_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(dp)


def _fortran(a) -> np.ndarray:
    return np.asfortranarray(np.asarray(a, dtype=np.float64))


# --- host-only 1D data ---------------------------------------------------------

def assemble_1d(n_el: int, p: int, kind: str, weight=(1.0, 0.0, 0.0, 0.0)) -> np.ndarray:
    """DIA band (2p+1, n): band[o+p, i] = A[i, i+o]."""
    n = n_el + p - 2
    band = np.zeros((2 * p + 1, n))
    w = np.asarray(weight, dtype=np.float64)
    st = lib().tk_assemble_1d(n_el, p, KINDS[kind], _ptr(w), _ptr(band))
    if st != TK_OK:
        raise TkError(st, "tk_assemble_1d")
    return band


def assemble_1d_bc(n_el: int, p: int, kind: str, weight=(1.0, 0.0, 0.0, 0.0), bc=(0, 0)) -> np.ndarray:
    """DIA band (2p+1, n) on the space with boundary flags bc = (k0, k1)
    (1 Neumann, 0 Dirichlet), n = n_el + p - 2 + k0 + k1."""
    n = n_el + p - 2 + bc[0] + bc[1]
    band = np.zeros((2 * p + 1, n))
    w = np.asarray(weight, dtype=np.float64)
    st = lib().tk_assemble_1d_bc(n_el, p, KINDS[kind], _ptr(w), int(bc[0]), int(bc[1]), _ptr(band))
    if st != TK_OK:
        raise TkError(st, "tk_assemble_1d_bc")
    return band


def assemble_1d_cheb(n_el: int, p: int, kind: str, c, bc=(0, 0)) -> np.ndarray:
    """DIA band (2p+1, n) with the weight sum_m c[m] T_m(2x - 1)."""
    n = n_el + p - 2 + bc[0] + bc[1]
    band = np.zeros((2 * p + 1, n))
    cc = np.ascontiguousarray(c, dtype=np.float64)
    st = lib().tk_assemble_1d_cheb(n_el, p, KINDS[kind], len(cc), _ptr(cc), int(bc[0]), int(bc[1]), _ptr(band))
    if st != TK_OK:
        raise TkError(st, "tk_assemble_1d_cheb")
    return band


def load_vector_1d_cheb(n_el: int, p: int, c, bc=(0, 0)) -> np.ndarray:
    """F_i = int b_i(x) sum_m c[m] T_m(2x - 1) dx."""
    F = np.zeros(n_el + p - 2 + bc[0] + bc[1])
    cc = np.ascontiguousarray(c, dtype=np.float64)
    st = lib().tk_load_vector_1d_cheb(n_el, p, len(cc), _ptr(cc), int(bc[0]), int(bc[1]), _ptr(F))
    if st != TK_OK:
        raise TkError(st, "tk_load_vector_1d_cheb")
    return F


def basis_values_1d(n_el: int, p: int, x, der: int = 0, bc=(0, 0)) -> np.ndarray:
    """(len(x), n) values (or derivatives) of the basis of the space with flags bc."""
    xx = np.ascontiguousarray(x, dtype=np.float64).ravel()
    n = n_el + p - 2 + bc[0] + bc[1]
    out = np.zeros((xx.size, n), order="F")
    st = lib().tk_basis_values_1d(n_el, p, int(bc[0]), int(bc[1]), der, xx.size, _ptr(xx),
                                  out.ctypes.data_as(dp))
    if st != TK_OK:
        raise TkError(st, "tk_basis_values_1d")
    return out


def fd_direction_dense_host(n_el: int, p: int, coef: float = 1.0, bc=(0, 0)):
    """(U~, lam) of fd_setup_bc for one direction (host only)."""
    n = n_el + p - 2 + bc[0] + bc[1]
    lam = np.zeros(n)
    Ut = np.zeros(n * n)
    nn = C.c_int32()
    st = lib().tk_fd_direction_dense_host(n_el, p, coef, int(bc[0]), int(bc[1]), C.byref(nn), _ptr(lam), _ptr(Ut))
    if st != TK_OK:
        raise TkError(st, "tk_fd_direction_dense_host")
    return Ut.reshape(n, n, order="F"), lam


def load_vector_1d(n_el: int, p: int, weight) -> np.ndarray:
    F = np.zeros(n_el + p - 2)
    w = np.asarray(weight, dtype=np.float64)
    st = lib().tk_load_vector_1d(n_el, p, _ptr(w), _ptr(F))
    if st != TK_OK:
        raise TkError(st, "tk_load_vector_1d")
    return F


def fd_direction_host(n_el: int, p: int, coef: float = 1.0) -> dict:
    """Appendix B data of one direction (host setup of the FD transform)."""
    n, n1, n2 = C.c_int32(), C.c_int32(), C.c_int32()
    st = lib().tk_fd_direction_host(n_el, p, coef, C.byref(n), C.byref(n1), C.byref(n2), None, None, None, None)
    if st != TK_OK:
        raise TkError(st, "tk_fd_direction_host")
    lam = np.zeros(n.value)
    g = np.zeros(n1.value)
    E = np.zeros((n.value, n1.value), order="F")
    V = np.zeros((n.value, n2.value), order="F")
    lib().tk_fd_direction_host(n_el, p, coef, None, None, None, _ptr(lam), _ptr(g),
                               E.ctypes.data_as(dp), V.ctypes.data_as(dp))
    return {"n": n.value, "n1": n1.value, "n2": n2.value, "lam": lam, "g": g, "E": E, "v2u2": V}


def expsum_host(M: float, eps: float) -> dict:
    R = C.c_int32()
    al = np.zeros(64)
    om = np.zeros(64)
    err, errp = C.c_double(), C.c_double()
    st = lib().tk_expsum_host(M, eps, C.byref(R), _ptr(al), _ptr(om), C.byref(err), C.byref(errp))
    if st != TK_OK:
        raise TkError(st, "tk_expsum_host")
    return {"R": R.value, "alpha": al[:R.value].copy(), "omega": om[:R.value].copy(),
            "err": err.value, "err_prev": errp.value}


def band_to_dense(band: np.ndarray) -> np.ndarray:
    nb, n = band.shape
    p = (nb - 1) // 2
    A = np.zeros((n, n))
    for o in range(-p, p + 1):
        for i in range(n):
            j = i + o
            if 0 <= j < n:
                A[i, j] = band[o + p, i]
    return A


# --- context and objects -----------------------------------------------------------

class Context:
    """A library context bound to a HIP device and stream (default: torch's
    current stream on that device)."""

    def __init__(self, device: int = 0, stream=None):
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        h = vp()
        st = lib().tk_ctx_create(device, vp(stream), C.byref(h))
        if st != TK_OK:
            raise TkError(st, "tk_ctx_create")
        self.h = h
        self.device = device

    def check(self, st, what):
        if st not in (TK_OK,):
            msg = lib().tk_last_error(self.h)
            raise TkError(st, f"{what}: {msg.decode() if msg else ''}")

    def sync(self):
        self.check(lib().tk_ctx_sync(self.h), "sync")

    def truncate_refinements(self) -> int:
        """ST-HOSVD modes refined by a second eigendecomposition of their tail."""
        c = C.c_int64()
        self.check(lib().tk_truncate_refinements(self.h, C.byref(c)), "tk_truncate_refinements")
        return c.value

    PROF_KINDS = ["band_apply", "dgemm", "householder_qr", "sym_eig", "select_rank",
                  "fd_forward", "fd_backward", "misc"]

    def prof(self, on: bool = True, reset: bool = True):
        if reset:
            self.check(lib().tk_prof_reset(self.h), "tk_prof_reset")
        self.check(lib().tk_prof_enable(self.h, 1 if on else 0), "tk_prof_enable")

    def prof_read(self) -> dict:
        out = {}
        for k, name in enumerate(self.PROF_KINDS):
            n = C.c_int64()
            ms, by, fl = C.c_double(), C.c_double(), C.c_double()
            self.check(lib().tk_prof_read(self.h, k, C.byref(n), C.byref(ms), C.byref(by), C.byref(fl)),
                       "tk_prof_read")
            out[name] = {"launches": n.value, "ms": ms.value, "bytes": by.value, "flops": fl.value}
        return out

    def close(self):
        if getattr(self, "h", None):
            lib().tk_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Handle:
    _free = None

    def __init__(self, ctx: Context, h):
        self.ctx = ctx
        self.h = h

    def free(self):
        if getattr(self, "h", None) and self.ctx.h:
            getattr(lib(), self._free)(self.h)
        self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Tucker(_Handle):
    _free = "tk_tucker_free"

    @classmethod
    def from_host(cls, ctx, core, U) -> "Tucker":
        core = _fortran(core)
        U = [_fortran(u) for u in U]
        n = (C.c_int64 * 3)(*[u.shape[0] for u in U])
        r = (C.c_int64 * 3)(*core.shape)
        ptrs = (vp * 3)(*[u.ctypes.data for u in U])
        h = vp()
        ctx.check(lib().tk_tucker_create(ctx.h, n, r, vp(core.ctypes.data), ptrs, 0, C.byref(h)),
                  "tk_tucker_create")
        return cls(ctx, h)

    @classmethod
    def from_device(cls, ctx, n, r, core_t, U_t) -> "Tucker":
        """core_t, U_t: device tensors holding column-major data."""
        nn = (C.c_int64 * 3)(*n)
        rr = (C.c_int64 * 3)(*r)
        ptrs = (vp * 3)(*[u.data_ptr() for u in U_t])
        h = vp()
        ctx.check(lib().tk_tucker_create(ctx.h, nn, rr, vp(core_t.data_ptr()), ptrs, 1, C.byref(h)),
                  "tk_tucker_create")
        return cls(ctx, h)

    def shape(self):
        n = (C.c_int64 * 3)()
        m = (C.c_int64 * 3)()
        nb = C.c_int32()
        lib().tk_tucker_shape(self.h, n, m, C.byref(nb))
        return tuple(n), tuple(m), nb.value

    def blocks(self):
        _, _, nb = self.shape()
        out = []
        for b in range(nb):
            c = C.c_double()
            r = (C.c_int64 * 3)()
            o = (C.c_int64 * 3)()
            lib().tk_tucker_block(self.h, b, C.byref(c), r, o)
            out.append((c.value, tuple(r), tuple(o)))
        return out

    def factors(self):
        n, m, _ = self.shape()
        out = []
        for k in range(3):
            U = np.zeros((n[k], m[k]), order="F")
            if U.size:
                self.ctx.check(lib().tk_tucker_read(self.ctx.h, self.h, k, vp(U.ctypes.data), -1, None, 0),
                               "tk_tucker_read")
            out.append(U)
        return out

    def core(self, b=0):
        c, r, o = self.blocks()[b]
        G = np.zeros(r, order="F")
        if G.size:
            self.ctx.check(lib().tk_tucker_read(self.ctx.h, self.h, -1, None, b, vp(G.ctypes.data), 0),
                           "tk_tucker_read")
        return G

    def to_host(self):
        """(factors, [(coef, core, offsets)]) - the block representation."""
        U = self.factors()
        blocks = [(c, self.core(b), o) for b, (c, r, o) in enumerate(self.blocks())]
        return U, blocks

    def plain(self):
        """(core, factors) of a plain tensor (coefficient folded into the core)."""
        U, blocks = self.to_host()
        assert len(blocks) == 1, "lazy tensor: truncate first"
        c, G, _ = blocks[0]
        return c * G, U


class Operator(_Handle):
    _free = "tk_op_free"

    @classmethod
    def create(cls, ctx, p, n, bands, nnz) -> "Operator":
        """bands[k]: array (nmat_k, 2p+1, n_k) of DIA bands; nnz: (i1,i2,i3,c)."""
        arrs = [np.ascontiguousarray(np.asarray(b, dtype=np.float64)) for b in bands]
        nn = (C.c_int64 * 3)(*n)
        nm = (C.c_int32 * 3)(*[a.shape[0] for a in arrs])
        bp = (dp * 3)(*[_ptr(a) for a in arrs])
        nz = (CoreNz * max(len(nnz), 1))(*[CoreNz(int(a), int(b), int(c), float(v)) for a, b, c, v in nnz])
        h = vp()
        ctx.check(lib().tk_op_create(ctx.h, p, nn, nm, bp, nz, len(nnz), C.byref(h)), "tk_op_create")
        return cls(ctx, h)


class Preconditioner(_Handle):
    _free = "tk_prec_free"

    @classmethod
    def create(cls, ctx, n_el, p, eps_prec=0.1, coef=(1.0, 1.0, 1.0), exact=False, bcs=None) -> "Preconditioner":
        """Appendix B eigen-approximations (fd_setup), or with exact=True the
        exact generalized eigenpairs applied as dense GEMMs (fd_setup_exact);
        with boundary flags bcs = ((k0, k1),) * 3 both are built densely on
        those spaces (fd_setup_bc, fd_setup_exact_bc)."""
        ne = (C.c_int32 * 3)(*((n_el,) * 3 if np.isscalar(n_el) else n_el))
        cf = np.asarray(coef, dtype=np.float64)
        h = vp()
        R = C.c_int32()
        if bcs is not None:
            # Appendix B (fd_setup_bc) or exact eigenpairs (fd_setup_exact_bc), dense, on the flagged spaces
            flags = (C.c_int32 * 6)(*[int(f) for b in bcs for f in b])
            name = "fd_setup_exact_bc" if exact else "fd_setup_bc"
            ctx.check(getattr(lib(), name)(ctx.h, ne, p, eps_prec, _ptr(cf), flags, C.byref(h), C.byref(R)), name)
            return cls(ctx, h)
        name = "fd_setup_exact" if exact else "fd_setup"
        ctx.check(getattr(lib(), name)(ctx.h, ne, p, eps_prec, _ptr(cf), C.byref(h), C.byref(R)), name)
        return cls(ctx, h)

    def info(self):
        R = C.c_int32()
        lmin, lmax, err = C.c_double(), C.c_double(), C.c_double()
        lib().tk_prec_info(self.h, C.byref(R), C.byref(lmin), C.byref(lmax), C.byref(err), None, None)
        al = np.zeros(R.value)
        om = np.zeros(R.value)
        lib().tk_prec_info(self.h, None, None, None, None, _ptr(al), _ptr(om))
        return {"R_P": R.value, "lam_min": lmin.value, "lam_max": lmax.value, "err": err.value,
                "alpha": al, "omega": om}

    def direction(self, k):
        n, n1, n2 = C.c_int32(), C.c_int32(), C.c_int32()
        lib().tk_prec_direction(self.h, k, C.byref(n), C.byref(n1), C.byref(n2), None, None, None, None)
        lam = np.zeros(n.value)
        g = np.zeros(n1.value)
        E = np.zeros((n.value, n1.value), order="F")
        V = np.zeros((n.value, n2.value), order="F")
        lib().tk_prec_direction(self.h, k, None, None, None, _ptr(lam), _ptr(g),
                                E.ctypes.data_as(dp), V.ctypes.data_as(dp))
        return {"lam": lam, "g": g, "E": E, "v2u2": V, "n1": n1.value, "n2": n2.value}


# --- the hot-path calls ----------------------------------------------------------------

ARITH = {"f64": 0, "f32": 1}   # TK_ARITH_F64, TK_ARITH_F32
ARITH_MIXED = 2                 # TK_ARITH_MIXED (tpcg_solve's precision rule)


def tucker_apply_op(ctx, op: Operator, x: Tucker, arith: str = "f64") -> Tucker:
    h = vp()
    if arith == "f64":
        ctx.check(lib().tucker_apply_op(ctx.h, op.h, x.h, C.byref(h)), "tucker_apply_op")
    else:
        ctx.check(lib().tucker_apply_op_arith(ctx.h, op.h, x.h, ARITH[arith], C.byref(h)), "tucker_apply_op_arith")
    return Tucker(ctx, h)


def fd_precond(ctx, P: Preconditioner, s: Tucker, arith: str = "f64") -> Tucker:
    h = vp()
    if arith == "f64":
        ctx.check(lib().fd_precond(ctx.h, P.h, s.h, C.byref(h)), "fd_precond")
    else:
        ctx.check(lib().fd_precond_arith(ctx.h, P.h, s.h, ARITH[arith], C.byref(h)), "fd_precond_arith")
    return Tucker(ctx, h)


def tucker_truncate(ctx, y: Tucker, eps: float):
    h = vp()
    d = C.c_double()
    ctx.check(lib().tucker_truncate(ctx.h, y.h, eps, C.byref(h), C.byref(d)), "tucker_truncate")
    return Tucker(ctx, h), d.value


def dot(ctx, x: Tucker, y: Tucker) -> float:
    out = C.c_double()
    ctx.check(lib().tk_tucker_dot(ctx.h, x.h, y.h, C.byref(out)), "tk_tucker_dot")
    return out.value


def tucker_rows(ctx, t: Tucker, off, n) -> Tucker:
    """Rows [off[k], off[k] + n[k]) of every mode-k factor (cores shared)."""
    h = vp()
    ctx.check(lib().tk_tucker_rows(ctx.h, t.h, (C.c_int64 * 3)(*off), (C.c_int64 * 3)(*n), C.byref(h)),
              "tk_tucker_rows")
    return Tucker(ctx, h)


def axpby(ctx, a, x: Tucker, b, y: Tucker) -> Tucker:
    h = vp()
    ctx.check(lib().tk_tucker_axpby(ctx.h, a, x.h, b, y.h, C.byref(h)), "tk_tucker_axpby")
    return Tucker(ctx, h)


def sym_eig(ctx, G_dev, a: int, V_dev, w_dev) -> None:
    """Eigendecomposition G = V diag(w) V^T of a device a x a matrix
    (column-major) into device V (a x a) and w (a), descending order.
    Asynchronous on the context's stream."""
    import torch
    for t, n in ((G_dev, a * a), (V_dev, a * a), (w_dev, a)):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() < n:
            raise ValueError("sym_eig needs contiguous float64 device tensors of the right size")
    ctx.check(lib().tk_sym_eig(ctx.h, vp(G_dev.data_ptr()), a, vp(V_dev.data_ptr()),
                               vp(w_dev.data_ptr())), "tk_sym_eig")


def _block_ops(ops):
    """3 x 3 nested list of Operator (or None for a zero block) -> void*[9]."""
    return (vp * 9)(*[(ops[a][b].h if ops[a][b] is not None else None) for a in range(3) for b in range(3)])


def tucker_apply_op_block(ctx, ops, x) -> list:
    """y_a = sum_b A_ab x_b; ops is a 3 x 3 nested list (None = zero block)."""
    out = (vp * 3)()
    ctx.check(lib().tucker_apply_op_block(ctx.h, _block_ops(ops), (vp * 3)(*[t.h for t in x]), out),
              "tucker_apply_op_block")
    return [Tucker(ctx, out[a]) for a in range(3)]


def tpcg_solve_block(ctx, ops, precs, f, allow_noconv=False, **params):
    """Algorithm 5 on a 3-component block system (Sec. 5.3); returns
    ([x_1, x_2, x_3], info)."""
    prm = tpcg_params(**params)
    info = TpcgInfo()
    out = (vp * 3)()
    st = lib().tpcg_solve_block(ctx.h, _block_ops(ops), (vp * 3)(*[P.h for P in precs]),
                                (vp * 3)(*[t.h for t in f]), C.byref(prm), out, C.byref(info))
    x = [Tucker(ctx, out[a]) if out[a] else None for a in range(3)]
    if st != TK_OK and not (allow_noconv and st == TK_ENOCONV):
        msg = lib().tk_last_error(ctx.h)
        raise TkError(st, f"tpcg_solve_block: {msg.decode() if msg else ''}")
    return x, {"iters": info.iters, "converged": bool(info.converged), "relres": info.relres,
               "rank": tuple(info.rank), "eps_final": info.eps_final, "trel_calls": info.trel_calls,
               "f32_applications": info.f32_applications, "status": st}


def dgemm(ctx, ta: bool, tb: bool, M: int, N: int, K: int, alpha: float, A_dev, lda: int,
          B_dev, ldb: int, beta: float, C_dev, ldc: int) -> None:
    """C = alpha op(A) op(B) + beta C on device float64 tensors (column-major
    storage, leading dimensions as in BLAS).  Asynchronous."""
    import torch
    for t in (A_dev, B_dev, C_dev):
        if t.dtype != torch.float64 or not t.is_cuda:
            raise ValueError("dgemm needs float64 device tensors")
    ctx.check(lib().tk_dgemm(ctx.h, int(ta), int(tb), M, N, K, alpha, vp(A_dev.data_ptr()), lda,
                             vp(B_dev.data_ptr()), ldb, beta, vp(C_dev.data_ptr()), ldc), "tk_dgemm")


def tpcg_params(**kw) -> TpcgParams:
    """Parameters of tpcg_solve; arith="mixed" selects the precision rule of
    TK_ARITH_MIXED ("f64", the default, keeps every step in FP64)."""
    prm = TpcgParams()
    lib().tk_tpcg_defaults(C.byref(prm))
    for k, v in kw.items():
        if v is None:
            continue
        if k == "arith":
            v = {"f64": ARITH["f64"], "mixed": ARITH_MIXED}[v] if isinstance(v, str) else v
        setattr(prm, k, v)
    return prm


def tpcg_solve(ctx, op: Operator, P: Preconditioner, f: Tucker, allow_noconv=False, **params):
    prm = tpcg_params(**params)
    info = TpcgInfo()
    h = vp()
    st = lib().tpcg_solve(ctx.h, op.h, P.h, f.h, C.byref(prm), C.byref(h), C.byref(info))
    x = Tucker(ctx, h) if h.value else None
    if st != TK_OK and not (allow_noconv and st == TK_ENOCONV):
        msg = lib().tk_last_error(ctx.h)
        raise TkError(st, f"tpcg_solve: {msg.decode() if msg else ''}")
    return x, {"iters": info.iters, "converged": bool(info.converged), "relres": info.relres,
               "rank": tuple(info.rank), "eps_final": info.eps_final, "trel_calls": info.trel_calls,
               "f32_applications": info.f32_applications, "status": st}
