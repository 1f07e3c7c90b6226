// Launch wrappers of the HIP kernels (internal).  All take the stream to
// launch on; none synchronises.  Matrices are column-major.
#pragma once

#include <hip/hip_runtime.h>

namespace tk {
namespace gpu {

// W[:, t*m + c] = A_t Y[:, c] for the nmat banded matrices (DIA, half-bandwidth p);
// Y and W FP64, the arithmetic FP32 with the bands band_f when band_f is given
void band_apply(hipStream_t s, int n, int m, int nmat, int p, const double* band, const float* band_f,
                const double* Y, int ldy, double* W, int ldw);

// C = alpha op(A) op(B) + beta C, batched with element strides.  With
// `part` (nsplit * M * N doubles) and nsplit > 1 (batch 1), K is split over
// nsplit workgroup layers whose partial products are summed by a second
// kernel in a fixed order (deterministic).
int dgemm_split_count(int M, int N, int K);
void dgemm(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha,
           const double* A, int lda, long long sA, const double* B, int ldb, long long sB,
           double beta, double* C, int ldc, long long sC, int batch = 1, double* part = nullptr,
           int nsplit = 1);
// C = sum_z part[z] (+ beta C) over nsplit M x N partial products (leading dimension M)
void splitk_reduce(hipStream_t s, int M, int N, int nsplit, const double* part, double beta, double* C, int ldc);

// Householder QR of up to 3 independent tall matrices (m <= n), one
// workgroup each.  A (n x m, ld n) is overwritten by the reflectors; R (m x m)
// and Q (n x m) are written explicitly; tau is scratch of m doubles.
struct QrJob {
  double* A;
  double* R;
  double* Q;
  double* tau;
  int n, m;
};
void householder_qr(hipStream_t s, const QrJob* jobs, int njobs);

// Symmetric eigendecomposition G = V diag(w) V^T of an a x a matrix
// (a <= 2048): Householder tridiagonalisation, multisection for the
// eigenvalues, inverse iteration, two Gram-Schmidt passes and the back
// transformation on stream s (five launches up to order 136; beyond, the
// Gram-Schmidt step runs by column panels with matrix-core GEMMs).  V is column-major with the
// eigenvectors in descending eigenvalue order, w descending.  `work` holds
// sym_eig_work(a) doubles.  G is not modified.
size_t sym_eig_work(int a);
void sym_eig(hipStream_t s, const double* G, int a, double* V, double* w, double* work);

// Several device-to-device copies (dst[0..n) = src[0..n) each) in one launch.
constexpr int kMaxSegs = 6;
struct CopySeg {
  double* dst;
  const double* src;
  long long n;
};
struct CopySegs {
  CopySeg s[kMaxSegs];
  int n = 0;
};
void copy_segments(hipStream_t s, const CopySegs& cs);

// Energies e[j] = sum_i P[i, j]^2 of the a columns of P (rows x a, ld rows)
// as S = column_energy_parts(rows) partial sums per column: part[j * S + s]
int column_energy_parts(int rows);
void column_energy(hipStream_t s, const double* P, int rows, int a, double* part);

// Rank choice of one ST-HOSVD mode from the partial energies (e[j] = sum of
// the S partials of column j): sort energies descending, keep the smallest
// s whose discarded tail is <= budget, where budget = eps^2 * norm2 / 3 and
// norm2 = *norm2_io (if set_norm, norm2 is first set to sum(e)).  Writes
// sel[0] = s, sel[1..a] = the columns in descending energy order; tail energy
// to disc[0], s (as a double) to disc[1], k1 to disc[2] and sum(e) to
// disc[3], where k1 counts the columns whose energy e is at least
// max(64 a eps_mach sum(e), 10 (a eps_mach e_max)^2 / budget): directions a
// Gram matrix of this mode resolves, with eigenvectors whose rounding leaks
// less than a tenth of the budget into the other directions.
void select_rank(hipStream_t s, const double* part, int S, int a, double eps, double* norm2_io,
                 int set_norm, int* sel, double* disc);

// out[:, j] = in[:, idx[j]] for j < s (rows x ., ld rows); idx read from device
void gather_columns(hipStream_t s, const double* in, int rows, const int* idx, int count,
                    double* out);

// out = sum over the whole array of x*y (device scalar, accumulated with coef)
void dot_accumulate(hipStream_t s, const double* x, const double* y, long long n, double coef,
                    double* out);
void fill(hipStream_t s, double* x, long long n, double v);
void scale_copy(hipStream_t s, const double* x, long long n, double a, double* y);

// Low-rank FD transform of one direction (see setup_fd.cpp).
// the transform's real tables in one arithmetic type (complex ones as
// interleaved (re, im) pairs)
template <class T>
struct FdTab {
  const T* g = nullptr;       // n1
  const T* e_val = nullptr;   // n * ke
  const T* et_val = nullptr;  // n1 * ket
  const T* v2u2 = nullptr;    // n x n2
  const T* ge = nullptr;      // R x n: exp(-alpha_j lam_m / lam_min), times g_m for m < n1
  const T* cs = nullptr;      // N complex: exp(-2 pi i x / N)
  const T* sn = nullptr;      // N: sin(pi x / N)
  const T* tq = nullptr;      // N/2 + 1 complex: exp(-i pi x / (2N))
};
struct FdDev {
  int n, n1, n2, N, odd, ke, ket, R;
  // rows [e_lo, e_hi) of E hold a single 1 at column row + e_sh; rows
  // [et_lo, et_hi) of E^T a single 1 at column row + et_sh; the others use
  // the ELL tables
  int e_lo, e_hi, e_sh, et_lo, et_hi, et_sh;
  const int* e_idx;      // n * ke
  const int* et_idx;     // n1 * ket
  FdTab<double> t64;     // FP64 arithmetic
  FdTab<float> t32;      // FP32 arithmetic (the same values rounded)
};
// Z (n x r) = U~^T S (n x r, ld lds); S and Z FP64, the arithmetic FP32 when f32
void fd_forward(hipStream_t s, const FdDev& d, const double* S, int lds, int r, double* Z, bool f32);
// Y[:, j*r + c] = U~ D_j Z[:, c] for j < R, c < r  (Y ld = n); FP64 data,
// the arithmetic FP32 when f32
void fd_backward(hipStream_t s, const FdDev& d, const double* Z, int r, double* Y, bool f32);
// exact-eigenvector variant: W[:, j r + c] = E[j, :] .* Z[:, c] (E: R x n, row j
// at E + j n; Z: n x r; W: n x R r)
void fd_exact_scale(hipStream_t s, int n, int r, int R, const double* E, const double* Z, double* W);

}  // namespace gpu
}  // namespace tk
