/*
 * tk.h - C ABI of the MI355X (gfx950) Tucker-format TPCG library.
 *
 * The library solves  A~ x~ = f~  (eq. approx_ls) for a Galerkin operator
 * given as a Tucker matrix of banded 1D B-spline matrices (eq. tuck_matrix)
 * and a Tucker right-hand side, with the Truncated Preconditioned Conjugate
 * Gradient method (Algorithm 5), the low-rank Fast Diagonalization
 * preconditioner (Algorithm 4, Appendix B) and relative/dynamic Tucker
 * truncation (Algorithms 1-2).  Everything that touches tensor data runs as
 * HIP kernels on the GPU of the context; host code does bookkeeping, the
 * once-per-problem setup (1D B-spline matrices, Appendix B data,
 * exponential sums) and reads back the scalars that steer the iteration.
 *
 * Conventions
 *  - d = 3 throughout.  Tensors are column-major with mode 1 fastest, the
 *    vec ordering of Sec. 2.3: element (i1,i2,i3) of an n1 x n2 x n3 array
 *    is at i1 + n1*(i2 + n2*i3).  Factor matrices are n_k x r_k column-major
 *    with leading dimension n_k.  All floating point data are double.
 *  - Every call returns tk_status (0 = TK_OK, negative = error) and never
 *    throws; tk_last_error(ctx) returns a message for the last failure on
 *    that context.  Functions taking `tk_ctx*` enqueue their GPU work on the
 *    context's stream; calls that return host scalars or ranks synchronise
 *    that stream.
 *  - Objects (tk_tucker, tk_op, tk_prec) are owned by the library and must
 *    be released with their _free function before tk_ctx_destroy.  A
 *    tk_tucker may be "lazy": a sum of core blocks over stacked factor
 *    matrices (the result of a sum, an operator or a preconditioner
 *    application, see Sec. 2.3); tucker_truncate turns it into a plain
 *    Tucker tensor with orthonormal factors.
 *  - One context per host thread; a context is not thread safe.
 */
#ifndef TK_H
#define TK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tk_status;
enum {
  TK_OK = 0,
  TK_EINVAL = -1,      /* invalid argument or shape */
  TK_ENOMEM = -2,      /* device or host allocation failed */
  TK_EDEVICE = -3,     /* HIP runtime error */
  TK_ENOCONV = -4,     /* maxit reached (result holds the last iterate) */
  TK_EBREAKDOWN = -5,  /* xi_k <= 0 or a non-finite scalar in TPCG */
  TK_ENUMERIC = -6     /* setup failed numerically (Remez, factorization) */
};

/* 1D matrix kinds for tk_assemble_1d: int delta_a(b_i) delta_b(b_j) w dx (App. A) */
enum { TK_MASS = 0, TK_STIFF = 1, TK_MIXED_TEST = 2, TK_MIXED_TRIAL = 3 };

typedef struct tk_ctx tk_ctx;
typedef struct tk_tucker tk_tucker;
typedef struct tk_op tk_op;
typedef struct tk_prec tk_prec;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device` using `hip_stream` (a hipStream_t;
 * NULL = the null stream).  The stream is borrowed, not destroyed. */
tk_status tk_ctx_create(int device, void* hip_stream, tk_ctx** out);
void tk_ctx_destroy(tk_ctx* ctx);
const char* tk_last_error(const tk_ctx* ctx);
/* Wait for all work of the context's stream. */
tk_status tk_ctx_sync(tk_ctx* ctx);
/* Release cached device memory that no live object uses. */
tk_status tk_ctx_trim(tk_ctx* ctx);

/* ---- 1D B-spline data (host only; Sec. 2.1, App. A) --------------------- */

/* Banded n x n matrix (n = n_el + p - 2, Dirichlet space of Sec. 2.2) of
 * int delta_a(b_i) delta_b(b_j) w(x) dx with w(x) = weight[0] +
 * weight[1]*cos(weight[2]*x + weight[3]), Gauss-Legendre with p+5 points per
 * span.  Output `band` (host, caller-owned, (2p+1)*n doubles) in DIA layout:
 * band[(o+p)*n + i] = A[i, i+o], zero outside the matrix.
 * EINVAL if p < 1, n_el < 1 or kind is unknown. */
tk_status tk_assemble_1d(int32_t n_el, int32_t p, int32_t kind, const double weight[4], double* band);

/* tk_assemble_1d on the space with boundary flags (k0, k1) of Appendix B:
 * 1 = Neumann (the basis function that does not vanish at that end is
 * kept), 0 = Dirichlet (it is dropped, Sec. 2.2); n = n_el + p - 2 + k0 + k1
 * and (0, 0) is tk_assemble_1d.  With (1, 1) (every basis function) the
 * matrices of the full space, used for the lifting of non-homogeneous
 * Dirichlet data (remark closing Sec. 3, eq. nonhomog-dirichlet-system).
 * EINVAL as tk_assemble_1d or if a flag is not 0 or 1. */
tk_status tk_assemble_1d_bc(int32_t n_el, int32_t p, int32_t kind, const double weight[4], int32_t k0,
                            int32_t k1, double* band);

/* tk_assemble_1d_bc with the weight given as a Chebyshev series on [0, 1],
 * w(x) = sum_{m < nc} c[m] T_m(2x - 1): the univariate integrals of
 * Appendix A (eq. matrix_CP, a factor column of the separable approximation
 * of an entry of Q), Gauss-Legendre exact for the polynomial integrand.
 * EINVAL as tk_assemble_1d_bc or if nc is not in [1, 4096]. */
tk_status tk_assemble_1d_cheb(int32_t n_el, int32_t p, int32_t kind, int32_t nc, const double* c, int32_t k0,
                              int32_t k1, double* band);

/* F_i = int b_i(x) w(x) dx on the space with flags (k0, k1), w a Chebyshev
 * series as above (the rhs factors of Appendix A, F~_t). */
tk_status tk_load_vector_1d_cheb(int32_t n_el, int32_t p, int32_t nc, const double* c, int32_t k0, int32_t k1,
                                 double* F);

/* Values (der = 0) or derivatives (der <= p) of the n = n_el + p - 2 + k0 + k1
 * B-splines of the space with flags (k0, k1) (Sec. 2.1-2.2) at npts points
 * x in [0, 1]: out (npts x n, column-major, caller-owned; host).  A solution
 * with Tucker factors U_k is evaluated at a tensor grid of points as its
 * core times (B_k U_k) in each mode.  EINVAL on bad flags, der > p or a
 * point outside [0, 1]. */
tk_status tk_basis_values_1d(int32_t n_el, int32_t p, int32_t k0, int32_t k1, int32_t der, int64_t npts,
                             const double* x, double* out);

/* Load vector F_i = int b_i(x) w(x) dx (host, caller-owned, n doubles). */
tk_status tk_load_vector_1d(int32_t n_el, int32_t p, const double weight[4], double* F);

/* Appendix B data of one direction computed on the host without a context
 * (for inspection and tests): sizes, approximate eigenvalues lam (n, scaled
 * by coef), g_j = sqrt(2)/sigma(j pi/n_el) (n1), the boundary map E (n x n1,
 * column-major) and V2 U2 (n x n2, column-major).  Call once with the array
 * pointers NULL to get the sizes.  EINVAL for unsupported (n_el, p). */
tk_status tk_fd_direction_host(int32_t n_el, int32_t p, double coef, int32_t* n, int32_t* n1,
                               int32_t* n2, double* lam, double* g, double* E, double* v2u2);

/* Minimax exponential sum for 1/x on [1, M] with the smallest R such that
 * E_R(M) <= eps/M (Prop. 1, eq. estimate_prec_rel), computed on the host by
 * the Remez exchange.  alpha/omega (ascending alpha) need room for 64
 * entries; err_prev = E_{R-1}(M).  ENUMERIC if the exchange fails. */
tk_status tk_expsum_host(double M, double eps, int32_t* R, double* alpha, double* omega, double* err,
                         double* err_prev);

/* ---- Tucker tensors (Sec. 2.3, eq. Tucker) -------------------------------- */

/* Copy a Tucker tensor (core r1 x r2 x r3, factors n_k x r_k) from caller
 * memory into a new library object.  `on_device` = 1: pointers are device
 * memory on the context's device (the copy is enqueued on the stream and
 * the caller must keep the memory valid until the stream reaches it);
 * 0: host memory (copied before return).  A rank may be 0 (zero tensor). */
tk_status tk_tucker_create(tk_ctx* ctx, const int64_t n[3], const int64_t r[3],
                           const double* core, const double* const U[3], int32_t on_device,
                           tk_tucker** out);
void tk_tucker_free(tk_tucker* t);

/* Sizes: n_k, total stacked factor columns m_k and the number of core
 * blocks (1 for a plain Tucker tensor; ranks are then m_k). */
tk_status tk_tucker_shape(const tk_tucker* t, int64_t n[3], int64_t m[3], int32_t* nblocks);

/* Block b of a lazy tensor: coefficient, block ranks and the column offsets
 * of the block inside the stacked factors. */
tk_status tk_tucker_block(const tk_tucker* t, int32_t b, double* coef, int64_t r[3], int64_t off[3]);

/* Copy the stacked factor k (n_k x m_k) and the core of block b (r1*r2*r3)
 * to caller memory (`on_device` as above; synchronises).  Either pointer
 * may be NULL. */
tk_status tk_tucker_read(tk_ctx* ctx, const tk_tucker* t, int32_t k, double* U, int32_t b,
                         double* core, int32_t on_device);

/* <x, y> (Sec. 2.3 scalar product; lazy sums expanded bilinearly). Syncs. */
tk_status tk_tucker_dot(tk_ctx* ctx, const tk_tucker* x, const tk_tucker* y, double* out);

/* Rows [off[k], off[k] + n[k]) of every mode-k factor of t (device copies;
 * the cores are shared): the restriction of a tensor on a larger basis to a
 * contiguous index range per direction, e.g. from the full spline basis to
 * the unknowns of the spaces of tk_assemble_1d_bc.  EINVAL on a range outside
 * t or an empty one.  Asynchronous. */
tk_status tk_tucker_rows(tk_ctx* ctx, const tk_tucker* t, const int64_t off[3], const int64_t n[3],
                         tk_tucker** out);

/* Lazy a*x + b*y (Sec. 2.3 sum: factors concatenated, block-diagonal core). */
tk_status tk_tucker_axpby(tk_ctx* ctx, double a, const tk_tucker* x, double b,
                          const tk_tucker* y, tk_tucker** out);

/* ---- operator (eq. tuck_matrix, eq. tt_product) --------------------------- */

typedef struct { int32_t i1, i2, i3; double c; } tk_core_nz;

/* Tucker matrix sum_nz c * A_(3,i3) x A_(2,i2) x A_(1,i1).  bands[k] (host)
 * holds nmat[k] banded n[k] x n[k] matrices of half-bandwidth p in the DIA
 * layout of tk_assemble_1d, matrix t at bands[k] + t*(2p+1)*n[k].  The data
 * are copied to the device.  EINVAL on out-of-range indices or p outside
 * [0, 6] (the banded kernels hold a row's 2p + 1 entries in registers). */
tk_status tk_op_create(tk_ctx* ctx, int32_t p, const int64_t n[3], const int32_t nmat[3],
                       const double* const bands[3], const tk_core_nz* nz, int64_t nnz,
                       tk_op** out);
void tk_op_free(tk_op* op);

/* y = A x (eq. tt_product), untruncated: mode-k factor [A_(k,1) X_k, ...,
 * A_(k,R_k) X_k] computed by banded mode-product kernels, core C (x) X kept
 * as one block per nonzero of C.  Asynchronous. */
tk_status tucker_apply_op(tk_ctx* ctx, const tk_op* op, const tk_tucker* x, tk_tucker** y);

/* Arithmetic of the mode products (the factors stay FP64 in memory). */
enum { TK_ARITH_F64 = 0, TK_ARITH_F32 = 1 };

/* tucker_apply_op with the arithmetic chosen: TK_ARITH_F32 rounds the bands
 * (an FP32 copy made by tk_op_create) and the staged factor rows to FP32,
 * accumulates in FP32 and widens the sums to FP64 on the store (relative
 * error of order (2p+1) 2^-24 per entry); TK_ARITH_F64 is tucker_apply_op.
 * The FP32 arithmetic of the growth direction on precision of the mode
 * products (eq. tt_product).  EINVAL on another value.  Asynchronous. */
tk_status tucker_apply_op_arith(tk_ctx* ctx, const tk_op* op, const tk_tucker* x, int32_t arith,
                                tk_tucker** y);

/* ---- low-rank FD preconditioner (Algorithm 4, Appendix B) ----------------- */

/* Setup from the parametric 1D stiffness and mass (Dirichlet at both ends)
 * of each direction: Appendix B eigen-approximations (scaled by coef[k]),
 * M_P = lambda_max/lambda_min, R_P = min{R : E_R(M_P) <= eps_prec/M_P} with
 * minimax exponential sums (Prop. 1, eq. estimate_prec_rel).  n_el[k] must
 * be a power of two in [4, 1024] with n_el[k] > p.  `R_P` may be NULL. */
tk_status fd_setup(tk_ctx* ctx, const int32_t n_el[3], int32_t p, double eps_prec,
                   const double coef[3], tk_prec** out, int32_t* R_P);

/* Exact-eigenvector variant (Algorithm 4 with the factorizations of
 * Algorithm 3, eq. factorizations; the check of Sec. 5's remark on exact
 * eigenpairs): the generalized eigenpairs of (coef[k] K, M) of each direction
 * are computed at setup (C = L^{-1} K L^{-T} with M = L L^T, diagonalized by
 * the library's symmetric eigensolver, U = L^{-T} Q), kept on the device as
 * dense M-orthonormal n x n matrices, and applied by fd_precond as two
 * matrix-core GEMMs per mode (U^T S, then U [D_1 Z, ..., D_R Z]).  The
 * exponential sum and everything else as fd_setup.  n_el[k] in (p, 4096];
 * no power-of-two restriction.  Setup costs O(n^3) per direction on the
 * device; the dense U take 8 n^2 bytes per direction.  EINVAL on bad
 * arguments, ENUMERIC if an eigenvalue is not positive. */
tk_status fd_setup_exact(tk_ctx* ctx, const int32_t n_el[3], int32_t p, double eps_prec,
                         const double coef[3], tk_prec** out, int32_t* R_P);

/* fd_setup_exact on the spaces with boundary flags bc[2k] (x = 0) and
 * bc[2k+1] (x = 1) of direction k (Appendix B's k0, k1: 1 Neumann, 0
 * Dirichlet; n_k = n_el[k] + p - 2 + k0 + k1).  A direction with Neumann at
 * both ends has the eigenvalue 0 (the constants; computed values below
 * 1e-12 lambda_max are set to 0); the operator stays SPD as long as one
 * direction has a Dirichlet end, else EINVAL.  EINVAL also for flags other
 * than 0 and 1; the rest as fd_setup_exact. */
tk_status fd_setup_exact_bc(tk_ctx* ctx, const int32_t n_el[3], int32_t p, double eps_prec,
                            const double coef[3], const int32_t bc[6], tk_prec** out, int32_t* R_P);

/* The Appendix B eigen-approximations on the spaces with boundary flags
 * bc[2k], bc[2k+1] (Neumann ends: V_h1 with vanishing odd derivatives there,
 * the sines sin((j - k0/2 - k1/2) pi x + k0 pi/2) interpolated at the
 * breakpoints or span midpoints, Lambda1 = ((j - k0/2 - k1/2) pi)^2; V_h2 its
 * M-orthogonal complement with exact eigenpairs), built densely on the host
 * (O(n^3) per direction) and applied by fd_precond like fd_setup_exact's
 * (two matrix-core GEMMs per mode).  With all flags 0 it is fd_setup's
 * approximation without the sine transforms.  p >= 2, p < n_el <= 4096;
 * EINVAL on bad arguments or a singular operator. */
tk_status fd_setup_bc(tk_ctx* ctx, const int32_t n_el[3], int32_t p, double eps_prec, const double coef[3],
                      const int32_t bc[6], tk_prec** out, int32_t* R_P);
void tk_prec_free(tk_prec* P);

/* R_P, lambda_min, lambda_max, E_{R_P}(M_P); alpha/omega (R_P doubles each,
 * host) may be NULL. */
tk_status tk_prec_info(const tk_prec* P, int32_t* R_P, double* lam_min, double* lam_max,
                       double* err, double* alpha, double* omega);

/* v = P~^{-1} s (eq. prec), untruncated: factors [U~ D_(k,1) U~^T S_k, ...],
 * core P (x) S as R_P blocks with weights omega_j/lambda_min.  For a
 * preconditioner from fd_setup U~ is applied by sine transforms (no dense
 * eigenvector matrix); from fd_setup_exact by GEMMs with the dense exact U.
 * Asynchronous. */
tk_status fd_precond(tk_ctx* ctx, const tk_prec* P, const tk_tucker* s, tk_tucker** v);

/* fd_precond with the arithmetic chosen (Algorithm 4, steps 5-9):
 * TK_ARITH_F32 runs the boundary maps, sine transforms, exponential scalings
 * and V_2 products in FP32 with tables rounded at fd_setup, reading and
 * writing FP64 factors (relative error of order log2(n) 2^-24 per factor
 * entry); TK_ARITH_F64 is fd_precond.  A preconditioner from fd_setup_exact
 * runs in FP64 either way.  EINVAL on another value.  Asynchronous. */
tk_status fd_precond_arith(tk_ctx* ctx, const tk_prec* P, const tk_tucker* s, int32_t arith,
                           tk_tucker** v);

/* Appendix B data of direction k for inspection (host, caller-owned):
 * lam (n), g (n1), E (n x n1 dense, column-major), v2u2 (n x n2). Any may be NULL.
 * For a preconditioner from fd_setup_exact: n, n1 = n, n2 = 0 and lam (the
 * exact eigenvalues, in the eigensolver's descending order); g, E and v2u2
 * are left untouched. */
tk_status tk_prec_direction(const tk_prec* P, int32_t k, int32_t* n, int32_t* n1, int32_t* n2,
                            double* lam, double* g, double* E, double* v2u2);

/* Host-only inspection of fd_setup_bc's direction data: n, lam (n) and the
 * dense U~ (n x n, column-major, caller-owned; either may be NULL) for the
 * space with flags (k0, k1).  EINVAL on bad arguments. */
tk_status tk_fd_direction_dense_host(int32_t n_el, int32_t p, double coef, int32_t k0, int32_t k1, int32_t* n,
                                     double* lam, double* Ut);

/* ---- truncation (Algorithm 1) --------------------------------------------- */

/* out = T^rel(y, eps): QR of the stacked factors (Householder, FP64),
 * core Z = sum_b c_b G_b x_k R_k, ST-HOSVD of Z (modes 1,2,3; rank s_k the
 * smallest whose discarded energy is <= eps^2 ||Z||^2 / 3), factors Q_k S_k.
 * The result has orthonormal factors and ||y - out|| <= eps ||y||.
 * `discarded` (may be NULL) receives the total discarded energy / ||Z||^2.
 * Synchronises (ranks are data dependent). */
tk_status tucker_truncate(tk_ctx* ctx, const tk_tucker* y, double eps, tk_tucker** out,
                          double* discarded);

/* Symmetric eigendecomposition G = V diag(w) V^T of an a x a matrix,
 * 1 <= a <= 2048: the building block of the ST-HOSVD in tucker_truncate
 * (Sec. 2.3; the left singular vectors of a mode unfolding A are the
 * eigenvectors of its Gram matrix A A^T).  Householder tridiagonalisation,
 * Sturm-count multisection for the eigenvalues, inverse iteration and two
 * Gram-Schmidt passes for the vectors.  G, V (a x a, column-major) and w (a)
 * are device memory owned by the caller; G is not modified.  V has
 * orthonormal columns ordered by descending eigenvalue, w is descending.
 * Asynchronous on the context's stream. */
tk_status tk_sym_eig(tk_ctx* ctx, const double* G, int32_t a, double* V, double* w);

/* C = alpha op(A) op(B) + beta C (op = transpose when ta / tb is nonzero),
 * column-major, FP64: the dense contraction behind the mode products of
 * eq. tt_product and the Tucker scalar products, on the library's matrix-core
 * GEMM (K split over workgroups when the output has few tiles).  A, B, C are
 * device memory owned by the caller; lda >= rows of A as stored (M, or K
 * when transposed), likewise ldb, and ldc >= M.  With beta = 0, C is not
 * read.  Asynchronous on the context's stream. */
tk_status tk_dgemm(tk_ctx* ctx, int32_t ta, int32_t tb, int32_t M, int32_t N, int32_t K, double alpha,
                   const double* A, int32_t lda, const double* B, int32_t ldb, double beta, double* C,
                   int32_t ldc);

/* ---- solver (Algorithm 5) -------------------------------------------------- */

typedef struct {
  double tol;      /* stop when ||r_k|| <= tol ||f|| (default 1e-6) */
  double beta;     /* eta_k = beta tol ||f|| / ||r_k||, eq. rel_tol_iterates (0.1) */
  double eps0;     /* initial dynamic-truncation tolerance (0.1) */
  double alpha;    /* reduction factor of Algorithm 2 (0.5) */
  double eps_min;  /* floor of Algorithm 2; <= 0 means tol ||f|| / 10 with the
                      given rhs' norm (Sec. 5), at most tol / 10 */
  double delta;    /* update-ratio threshold of Algorithm 2 (1e-3) */
  int32_t maxit;   /* iteration cap (1000) */
  int32_t verbose; /* 1: print one line per iteration to stderr */
  int32_t arith;   /* TK_ARITH_F64 (default) or TK_ARITH_MIXED: the preconditioner
                      application z = P(r) and the operator application q = A p
                      run in FP32 arithmetic whenever the relative tolerance
                      eta_k of the truncation that follows is >= 10 * 2^-24;
                      the x update, the residual f - A x, scalar products and
                      truncations stay FP64 (the residual is recomputed from x,
                      so the FP32 steps change the search directions only) */
  double refine_below; /* truncations with a relative tolerance below this refine
                          the unresolved tail of each ST-HOSVD mode by a second
                          eigendecomposition (tk_truncate_refinements); above
                          it the Gram eigenvectors alone decide the ranks, which
                          may then exceed the SVD-based ones (1e-8) */
  int32_t reuse_bases; /* 1 (default): in every truncation of the solver, the
                          mode-2 and mode-3 bases are the eigenvectors of the
                          untruncated core's Gram matrices, computed on side
                          streams while mode 1 runs, also after mode 1 was
                          truncated; the discarded energies are measured on the
                          sequentially truncated core, so ||y - T(y)|| <= eps ||y||
                          holds exactly and the ranks are at least those of the
                          exact ST-HOSVD (equal unless a cut is borderline).
                          0: exact ST-HOSVD of Algorithm 1 (a fresh Gram matrix
                          per truncated mode), as tucker_truncate does */
} tk_tpcg_params;

enum { TK_ARITH_MIXED = 2 };

typedef struct {
  int32_t iters;
  int32_t converged;
  double relres;         /* ||r_k|| / ||f|| at exit */
  int64_t rank[3];       /* multilinear rank of the solution */
  double eps_final;      /* last dynamic-truncation tolerance */
  int32_t trel_calls;    /* number of relative truncations performed */
  int32_t f32_applications; /* preconditioner and operator applications run in FP32 */
} tk_tpcg_info;

/* ---- instrumentation ----------------------------------------------------- */

/* Kernel families timed with HIP events on the context's stream when
 * instrumentation is on (off by default; it adds two events per launch). */
enum { TK_PROF_BAND = 0, TK_PROF_GEMM = 1, TK_PROF_QR = 2, TK_PROF_EIG = 3, TK_PROF_SELECT = 4,
       TK_PROF_FD_FORWARD = 5, TK_PROF_FD_BACKWARD = 6, TK_PROF_MISC = 7 };
tk_status tk_prof_enable(tk_ctx* ctx, int32_t on);
tk_status tk_prof_reset(tk_ctx* ctx);
/* Accumulated launches, kernel milliseconds, algorithmic bytes and flops of
 * one family since the last reset (synchronises). */
tk_status tk_prof_read(tk_ctx* ctx, int32_t kind, int64_t* launches, double* ms, double* bytes,
                       double* flops);

/* Number of ST-HOSVD modes, over the context's life, whose rank cut fell
 * among directions that the mode's Gram matrix does not resolve (energies
 * below about 64 a eps_mach times the mode's energy) and that were refined by
 * a second eigendecomposition of the remaining coordinates (tucker_truncate
 * and every truncation inside the solvers).  Host only. */
tk_status tk_truncate_refinements(const tk_ctx* ctx, int64_t* count);

/* Fill `p` with the defaults of Sec. 5. */
void tk_tpcg_defaults(tk_tpcg_params* p);

/* Solve A x = f by TPCG (x_0 = 0).  The rhs is normalised internally and
 * the solution scaled back.  *x receives a plain Tucker tensor (orthonormal
 * factors).  Returns TK_ENOCONV (with *x set) if maxit is reached and
 * TK_EBREAKDOWN if xi_k <= 0 or a scalar is not finite. */
tk_status tpcg_solve(tk_ctx* ctx, const tk_op* op, const tk_prec* P, const tk_tucker* f,
                     const tk_tpcg_params* params, tk_tucker** x, tk_tpcg_info* info);

/* ---- block (3-component) systems, Sec. 5.3 (eq. block-system-elasticity) -- */

/* y_a = sum_b A_ab x_b for a 3 x 3 block operator.  A is row-major (A[3a+b]
 * is block (a, b): test component a, trial component b); a null entry is a
 * zero block, at least one must be set.  x[3] are the components (one shape
 * for all, matching every block); y[3] receive new lazy tensors (caller frees
 * each with tk_tucker_free).  TK_EINVAL on null or mismatched arguments. */
tk_status tucker_apply_op_block(tk_ctx* ctx, const tk_op* const A[9], tk_tucker* const x[3],
                                tk_tucker* y[3]);

/* Algorithm 5 on block vectors: products, sums, scalar products
 * (<x, y> = sum_a <x_a, y_a>) and truncations (every component with the same
 * relative tolerance, also inside Algorithm 2) act blockwise; P[a] is the
 * preconditioner of component a (block-diagonal preconditioner, Sec. 5.3).
 * A as for tucker_apply_op_block; f[3] the right-hand side components.  x[3]
 * receive plain Tucker tensors; info->rank holds, per mode, the largest rank
 * over the components.  Status as for tpcg_solve. */
tk_status tpcg_solve_block(tk_ctx* ctx, const tk_op* const A[9], const tk_prec* const P[3],
                           tk_tucker* const f[3], const tk_tpcg_params* params, tk_tucker* x[3],
                           tk_tpcg_info* info);

#ifdef __cplusplus
}
#endif
#endif /* TK_H */
