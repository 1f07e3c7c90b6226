// HIP kernels for gfx950 (CDNA4, wave64) of the Tucker TPCG library.
//
//  band_apply     banded mode products A_(k,t) X_k of eq. (tt_product): one
//                 workgroup stages a 256-row window of a factor column in LDS
//                 and applies every 1D matrix of the mode to it (coalesced
//                 along n, the factor column is read from HBM once).
//  dgemm          FP64 tiled GEMM (64x64x16 tiles in LDS, 4x4 outputs per
//                 thread) for the dense core and factor contractions.
//  householder_qr QR of stacked factors (Algorithm 1, step 1), one workgroup
//                 per mode, one wavefront per trailing column.
//  jacobi_eig     parallel cyclic Jacobi (round-robin pairing, two-sided 2x2
//                 block updates) of the ST-HOSVD Gram matrices, LDS resident.
//  column_energy, select_rank, gather_columns
//                 the rank choice of each ST-HOSVD mode from directly
//                 measured energies ||A^T v_j||^2.
//  fd_forward / fd_backward
//                 the low-rank FD transform U~^T and U~ D_j (Algorithm 4,
//                 Appendix B) as sparse boundary maps and radix-2 Stockham
//                 FFTs of length 2N in LDS (DST-I for odd p, DST-II/III for
//                 even p).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <string>

#include "kernels.h"

namespace tk {
namespace gpu {

static void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// block-wide sum; `red` is LDS of >= blockDim.x/64 doubles; result to all threads
__device__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += red[i];
  return t;
}

// ---------------------------------------------------------------------------
// banded mode products
// ---------------------------------------------------------------------------

constexpr int kBandRows = 256;

__global__ __launch_bounds__(kBandRows) void k_band_apply(int n, int m, int nmat, int p,
                                                          const double* __restrict__ band,
                                                          const double* __restrict__ Y, int ldy,
                                                          double* __restrict__ W, int ldw) {
  extern __shared__ double ys[];
  const int i0 = blockIdx.x * kBandRows;
  const int c = blockIdx.y;
  for (int t = threadIdx.x; t < kBandRows + 2 * p; t += kBandRows) {
    const int i = i0 - p + t;
    ys[t] = (i >= 0 && i < n) ? Y[i + (long long)c * ldy] : 0.0;
  }
  __syncthreads();
  const int i = i0 + threadIdx.x;
  if (i >= n) return;
  const int nb = 2 * p + 1;
  for (int t = 0; t < nmat; ++t) {
    const double* bt = band + (long long)t * nb * n;
    double acc = 0.0;
    for (int o = 0; o < nb; ++o) acc += bt[(long long)o * n + i] * ys[threadIdx.x + o];
    W[i + (long long)(t * m + c) * ldw] = acc;
  }
}

void band_apply(hipStream_t s, int n, int m, int nmat, int p, const double* band,
                const double* Y, int ldy, double* W, int ldw) {
  if (n <= 0 || m <= 0 || nmat <= 0) return;
  dim3 grid((n + kBandRows - 1) / kBandRows, m);
  const size_t lds = sizeof(double) * (kBandRows + 2 * p);
  hipLaunchKernelGGL(k_band_apply, grid, dim3(kBandRows), lds, s, n, m, nmat, p, band, Y, ldy, W, ldw);
  check_launch("band_apply");
}

// ---------------------------------------------------------------------------
// FP64 GEMM
// ---------------------------------------------------------------------------

// FP64 GEMM on the matrix cores (v_mfma_f64_16x16x4f64).  A workgroup of WM
// wavefronts computes a (16 WM) x (16 NT) tile of C; wavefront w owns rows
// [16w, 16w+16) and NT column tiles of 16, i.e. NT 16x16 accumulators.  K is
// staged through LDS in steps of BK = 16 (double buffered: the next step's
// global loads are in flight while the current step is multiplied).  The
// tile leaves through LDS, 48 columns at a time, so every column of C is
// written (and, with beta != 0, read) as one contiguous run of rows.
// Operand layout of the instruction (lane l, element v): A[l%16][l/16],
// B[l/16][l%16], D[l/16 + 4v][l%16].
constexpr int BK = 16;

typedef double dbl4 __attribute__((ext_vector_type(4)));

template <int WM, int NT>
struct GemmLds {
  static constexpr int BM = 16 * WM, BN = 16 * NT;
  static constexpr int kAPad = BM + 1, kBPad = BN + 1;  // odd strides: conflict-free transposing stores
  static constexpr int kOps = 2 * BK * (kAPad + kBPad);  // double-buffered A and B tiles
  static constexpr int kOut = 48 * kAPad;                // 48 output columns staged at a time
  static constexpr int kSize = kOps > kOut ? kOps : kOut;
};

// With `part` set, blockIdx.z selects the K range [z*kchunk, (z+1)*kchunk)
// and alpha*op(A)op(B) over that range is written to part + z*M*N (ld M);
// otherwise blockIdx.z is the batch index.
template <bool TA, bool TB, int WM, int NT>
__global__ __launch_bounds__(64 * WM) void k_dgemm(int M, int N, int K, double alpha,
                                                   const double* __restrict__ A, int lda, long long sA,
                                                   const double* __restrict__ B, int ldb, long long sB,
                                                   double beta, double* __restrict__ C, int ldc,
                                                   long long sC, int kchunk, double* __restrict__ part) {
  using Lds = GemmLds<WM, NT>;
  constexpr int NTH = 64 * WM;
  constexpr int BM = Lds::BM, BN = Lds::BN, kAPad = Lds::kAPad, kBPad = Lds::kBPad;
  constexpr int kALoads = BM * BK / NTH;  // 4
  constexpr int kBLoads = (BN * BK + NTH - 1) / NTH;
  constexpr bool kBTail = BN * BK % NTH != 0;  // last B load round only partly used
  static_assert(BM * BK % NTH == 0, "A tile loads must divide evenly");
  __shared__ double smem[Lds::kSize];
  double(*As)[BK][kAPad] = reinterpret_cast<double(*)[BK][kAPad]>(smem);
  double(*Bs)[BK][kBPad] = reinterpret_cast<double(*)[BK][kBPad]>(smem + 2 * BK * kAPad);
  int kbeg = 0, kend = K;
  if (part) {
    kbeg = blockIdx.z * kchunk;
    kend = min(K, kbeg + kchunk);
    C = part + (long long)blockIdx.z * M * N;
    ldc = M;
    beta = 0.0;
  } else {
    A += sA * blockIdx.z;
    B += sB * blockIdx.z;
    C += sC * blockIdx.z;
  }
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int row0 = blockIdx.x * BM, col0 = blockIdx.y * BN;
  double ra[kALoads], rb[kBLoads];
  auto load = [&](int k0) {
#pragma unroll
    for (int l = 0; l < kALoads; ++l) {
      const int e = t + NTH * l;
      const int i = TA ? e / BK : e % BM, kk = TA ? e % BK : e / BM;
      const int gr = row0 + i, gk = k0 + kk;
      ra[l] = (gr < M && gk < kend) ? (TA ? A[gk + (long long)gr * lda] : A[gr + (long long)gk * lda]) : 0.0;
    }
#pragma unroll
    for (int l = 0; l < kBLoads; ++l) {
      const int e = t + NTH * l;
      const int j = TB ? e % BN : e / BK, kk = TB ? e / BN : e % BK;
      const int gc = col0 + j, gk = k0 + kk;
      const bool in = !kBTail || e < BN * BK;
      rb[l] = (in && gc < N && gk < kend) ? (TB ? B[gc + (long long)gk * ldb] : B[gk + (long long)gc * ldb]) : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int l = 0; l < kALoads; ++l) {
      const int e = t + NTH * l;
      const int i = TA ? e / BK : e % BM, kk = TA ? e % BK : e / BM;
      As[buf][kk][i] = ra[l];
    }
#pragma unroll
    for (int l = 0; l < kBLoads; ++l) {
      const int e = t + NTH * l;
      const int j = TB ? e % BN : e / BK, kk = TB ? e / BN : e % BK;
      if (!kBTail || e < BN * BK) Bs[buf][kk][j] = rb[l];
    }
  };
  dbl4 acc[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) acc[j] = dbl4{0.0, 0.0, 0.0, 0.0};
  const int fr = 16 * wv + (lane & 15);  // A fragment row within the tile
  const int fk = lane >> 4;              // fragment k within a step of 4
  const int fc = lane & 15;              // B fragment column within a 16-wide tile
  int buf = 0;
  if (kbeg < kend) {
    load(kbeg);
    store(0);
  }
  __syncthreads();
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) load(k0 + BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const double af = As[buf][ks + fk][fr];
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const double bf = Bs[buf][ks + fk][16 * j + fc];
        acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, bf, acc[j], 0, 0, 0);
      }
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // epilogue through LDS (the operand tiles are free after the last barrier)
  double(*Cs)[kAPad] = reinterpret_cast<double(*)[kAPad]>(smem);
#pragma unroll
  for (int j0 = 0; j0 < NT; j0 += 3) {
#pragma unroll
    for (int j = j0; j < j0 + 3 && j < NT; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) Cs[16 * (j - j0) + fc][16 * wv + (lane >> 4) + 4 * v] = acc[j][v];
    __syncthreads();
    const int ncol = min(48, BN - 16 * j0);
    for (int e = t; e < ncol * BM; e += NTH) {
      const int i = e % BM, jc = e / BM;
      const int gr = row0 + i, gc = col0 + 16 * j0 + jc;
      if (gr < M && gc < N) {
        double* cp = C + gr + (long long)gc * ldc;
        const double val = alpha * Cs[jc][i];
        *cp = (beta == 0.0) ? val : val + beta * (*cp);
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_splitk_reduce(int M, int N, int nsplit, const double* __restrict__ part,
                                                       double beta, double* __restrict__ C, int ldc) {
  const long long MN = (long long)M * N;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < MN; e += 256LL * gridDim.x) {
    // partial sums added in split order; the loads of eight splits are issued together
    double acc = 0.0;
    int z = 0;
    for (; z + 8 <= nsplit; z += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[(z + u) * MN + e];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; z < nsplit; ++z) acc += part[z * MN + e];
    const int i = int(e % M), j = int(e / M);
    double* cp = C + i + (long long)j * ldc;
    *cp = (beta == 0.0) ? acc : acc + beta * (*cp);
  }
}

// row tiles of 16 per workgroup: 3 for short products where 48-row tiles pad
// M less than 64-row tiles, 4 otherwise
static int dgemm_wm(int M) {
  const long long p64 = (M + 63) / 64 * 64LL, p48 = (M + 47) / 48 * 48LL;
  return (M <= 144 && p48 < p64) ? 3 : 4;
}
// column tiles of 16 per workgroup for an N-wide product; 48-column tiles
// (same padding for N in (96, 144]) when the wide tile would leave fewer than
// two workgroups per compute unit to hide the global-load latency
static int dgemm_nt(int M, int N, int batch) {
  const int nt = N <= 32 ? 2 : N <= 64 ? 4 : N <= 96 ? 6 : 9;
  if (nt == 9) {
    const int bm = 16 * dgemm_wm(M);
    const long long blocks = (long long)((M + bm - 1) / bm) * ((N + 143) / 144) * batch;
    const long long p144 = (N + 143) / 144 * 144LL, p48 = (N + 47) / 48 * 48LL;
    if (blocks < 512 && p48 <= p144) return 3;
  }
  return nt;
}

int dgemm_split_count(int M, int N, int K) {
  const int bn = 16 * dgemm_nt(M, N, 1), bm = 16 * dgemm_wm(M);
  const long long tiles = (long long)((M + bm - 1) / bm) * ((N + bn - 1) / bn);
  if (tiles >= 128 || K < 1024) return 1;
  long long ns = std::min<long long>(K / 256, 256 / std::max<long long>(tiles, 1));
  return (int)std::max<long long>(1, std::min<long long>(ns, 64));
}

template <int WM, int NT>
static void launch_dgemm(hipStream_t s, bool ta, bool tb, dim3 grid, int M, int N, int K, double alpha,
                         const double* A, int lda, long long sA, const double* B, int ldb, long long sB,
                         double beta, double* C, int ldc, long long sC, int kchunk, double* part) {
  const dim3 blk(64 * WM);
  if (!ta && !tb) hipLaunchKernelGGL((k_dgemm<false, false, WM, NT>), grid, blk, 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, kchunk, part);
  else if (ta && !tb) hipLaunchKernelGGL((k_dgemm<true, false, WM, NT>), grid, blk, 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, kchunk, part);
  else if (!ta && tb) hipLaunchKernelGGL((k_dgemm<false, true, WM, NT>), grid, blk, 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, kchunk, part);
  else hipLaunchKernelGGL((k_dgemm<true, true, WM, NT>), grid, blk, 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, kchunk, part);
}

template <int WM>
static void launch_dgemm_nt(hipStream_t s, int nt, bool ta, bool tb, dim3 grid, int M, int N, int K, double alpha,
                            const double* A, int lda, long long sA, const double* B, int ldb, long long sB,
                            double beta, double* C, int ldc, long long sC, int kchunk, double* part) {
  switch (nt) {
    case 2: launch_dgemm<WM, 2>(s, ta, tb, grid, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, kchunk, part); break;
    case 3: launch_dgemm<WM, 3>(s, ta, tb, grid, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, kchunk, part); break;
    case 4: launch_dgemm<WM, 4>(s, ta, tb, grid, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, kchunk, part); break;
    case 6: launch_dgemm<WM, 6>(s, ta, tb, grid, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, kchunk, part); break;
    default: launch_dgemm<WM, 9>(s, ta, tb, grid, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, kchunk, part); break;
  }
}

void dgemm(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha,
           const double* A, int lda, long long sA, const double* B, int ldb, long long sB,
           double beta, double* C, int ldc, long long sC, int batch, double* part, int nsplit) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  if (K <= 0) {
    if (beta == 1.0) return;
    // C = beta C
    for (int b = 0; b < batch; ++b)
      for (int j = 0; j < N; ++j) scale_copy(s, C + sC * b + (long long)j * ldc, M, beta, C + sC * b + (long long)j * ldc);
    return;
  }
  int kchunk = K;
  int gz = batch;
  if (part && nsplit > 1 && batch == 1) {
    kchunk = ((K + nsplit - 1) / nsplit + BK - 1) / BK * BK;
    gz = (K + kchunk - 1) / kchunk;
  } else {
    part = nullptr;
  }
  const int nt = dgemm_nt(M, N, gz), wm = dgemm_wm(M);
  dim3 grid((M + 16 * wm - 1) / (16 * wm), (N + 16 * nt - 1) / (16 * nt), gz);
  if (wm == 3) launch_dgemm_nt<3>(s, nt, ta, tb, grid, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, kchunk, part);
  else launch_dgemm_nt<4>(s, nt, ta, tb, grid, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, kchunk, part);
  check_launch("dgemm");
  if (part) {
    const long long MN = (long long)M * N;
    const int nb = (int)std::min<long long>(1024, (MN + 255) / 256);
    hipLaunchKernelGGL(k_splitk_reduce, dim3(nb), dim3(256), 0, s, M, N, gz, part, beta, C, ldc);
    check_launch("splitk_reduce");
  }
}

// ---------------------------------------------------------------------------
// Householder QR
// ---------------------------------------------------------------------------

struct QrJobs {
  QrJob j[3];
};

constexpr int kQrThreads = 512;

__global__ __launch_bounds__(kQrThreads) void k_householder_qr(QrJobs jobs) {
  const QrJob job = jobs.j[blockIdx.x];
  double* A = job.A;
  const int n = job.n, m = job.m;
  __shared__ double red[kQrThreads / 64];
  __shared__ double s_tau;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = kQrThreads / 64;
  for (int e = threadIdx.x; e < m * m; e += kQrThreads) job.R[e] = 0.0;
  for (int j = 0; j < m; ++j) {
    double part = 0.0;
    for (int i = j + threadIdx.x; i < n; i += kQrThreads) {
      const double v = A[i + (long long)j * n];
      part += v * v;
    }
    const double s2 = block_sum(part, red);
    if (threadIdx.x == 0) {
      const double x0 = A[j + (long long)j * n];
      const double nrm = sqrt(s2);
      double tau = 0.0, alpha = 0.0;
      if (nrm > 0.0) {
        alpha = (x0 >= 0.0) ? -nrm : nrm;
        const double v0 = x0 - alpha;
        A[j + (long long)j * n] = v0;
        const double vtv = s2 - x0 * x0 + v0 * v0;
        tau = (vtv > 0.0) ? 2.0 / vtv : 0.0;
      }
      job.R[j + (long long)j * m] = alpha;
      job.tau[j] = tau;
      s_tau = tau;
    }
    __syncthreads();
    const double tau = s_tau;
    for (int c = j + 1 + wid; c < m; c += nw) {
      double d = 0.0;
      if (tau != 0.0)
        for (int i = j + lane; i < n; i += 64) d += A[i + (long long)j * n] * A[i + (long long)c * n];
      d = wave_sum(d) * tau;
      if (tau != 0.0)
        for (int i = j + lane; i < n; i += 64) A[i + (long long)c * n] -= d * A[i + (long long)j * n];
      if (lane == 0) job.R[j + (long long)c * m] = A[j + (long long)c * n];
    }
    __syncthreads();
  }
  // Q = H_0 ... H_{m-1} [I; 0]
  for (long long e = threadIdx.x; e < (long long)n * m; e += kQrThreads) {
    const int i = int(e % n), c = int(e / n);
    job.Q[e] = (i == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = m - 1; j >= 0; --j) {
    const double tau = job.tau[j];
    if (tau != 0.0) {
      for (int c = j + wid; c < m; c += nw) {
        double d = 0.0;
        for (int i = j + lane; i < n; i += 64) d += A[i + (long long)j * n] * job.Q[i + (long long)c * n];
        d = wave_sum(d) * tau;
        for (int i = j + lane; i < n; i += 64) job.Q[i + (long long)c * n] -= d * A[i + (long long)j * n];
      }
    }
    __syncthreads();
  }
}

void householder_qr(hipStream_t s, const QrJob* jobs, int njobs) {
  if (njobs <= 0) return;
  QrJobs js;
  for (int i = 0; i < njobs; ++i) js.j[i] = jobs[i];
  hipLaunchKernelGGL(k_householder_qr, dim3(njobs), dim3(kQrThreads), 0, s, js);
  check_launch("householder_qr");
}

// ---------------------------------------------------------------------------
// rank selection
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_column_energy(const double* __restrict__ P, int rows,
                                                       double* __restrict__ e) {
  __shared__ double red[4];
  const double* col = P + (long long)blockIdx.x * rows;
  double s = 0.0;
  for (int i = threadIdx.x; i < rows; i += 256) s += col[i] * col[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) e[blockIdx.x] = s;
}

void column_energy(hipStream_t s, const double* P, int rows, int a, double* e) {
  if (a <= 0) return;
  hipLaunchKernelGGL(k_column_energy, dim3(a), dim3(256), 0, s, P, rows, e);
  check_launch("column_energy");
}

constexpr int kSelMax = 2048;

__global__ __launch_bounds__(1024) void k_select(const double* __restrict__ e, int a, double eps,
                                                 double* norm2_io, int set_norm, int* sel,
                                                 double* disc) {
  __shared__ double key[kSelMax];
  __shared__ int idx[kSelMax];
  __shared__ double red[16];
  int P2 = 1;
  while (P2 < a) P2 <<= 1;
  double part = 0.0;
  for (int i = threadIdx.x; i < P2; i += 1024) {
    key[i] = (i < a) ? e[i] : -1.0;
    idx[i] = i;
    if (i < a) part += e[i];
  }
  const double tot = block_sum(part, red);
  __syncthreads();
  // bitonic sort, descending by key (ties: ascending index)
  for (int k = 2; k <= P2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P2; i += 1024) {
        const int l = i ^ j;
        if (l > i) {
          const bool desc = ((i & k) == 0);
          const double ki = key[i], kl = key[l];
          const int ii = idx[i], il = idx[l];
          const bool i_first = (ki > kl) || (ki == kl && ii < il);
          const bool swap = desc ? !i_first : i_first;
          if (swap) {
            key[i] = kl; key[l] = ki;
            idx[i] = il; idx[l] = ii;
          }
        }
      }
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    double norm2 = set_norm ? tot : *norm2_io;
    if (set_norm) *norm2_io = norm2;
    const double budget = eps * eps * norm2 / 3.0;
    double tail = 0.0;
    int s = a;
    for (int i = a - 1; i >= 0; --i) {
      const double v = key[i] > 0.0 ? key[i] : 0.0;
      if (tail + v <= budget) { tail += v; s = i; }
      else break;
    }
    sel[0] = s;
    disc[0] = tail;
    disc[1] = (double)s;  // the rank again, beside the tail, for a single readback
  }
  __syncthreads();
  const int s = sel[0];
  for (int i = threadIdx.x; i < s; i += 1024) sel[1 + i] = idx[i];
}

void select_rank(hipStream_t s, const double* e, int a, double eps, double* norm2_io,
                 int set_norm, int* sel, double* disc) {
  if (a > kSelMax) throw std::runtime_error("select_rank: more than 2048 columns");
  hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, s, e, a, eps, norm2_io, set_norm, sel, disc);
  check_launch("select_rank");
}

__global__ __launch_bounds__(256) void k_gather_columns(const double* __restrict__ in, int rows,
                                                        const int* __restrict__ idx,
                                                        double* __restrict__ out) {
  const int j = blockIdx.y;
  const int src = idx[j];
  const double* col = in + (long long)src * rows;
  double* dst = out + (long long)j * rows;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < rows; i += 256 * gridDim.x) dst[i] = col[i];
}

void gather_columns(hipStream_t s, const double* in, int rows, const int* idx, int count,
                    double* out) {
  if (count <= 0 || rows <= 0) return;
  const int bx = std::min((rows + 255) / 256, 64);
  hipLaunchKernelGGL(k_gather_columns, dim3(bx, count), dim3(256), 0, s, in, rows, idx, out);
  check_launch("gather_columns");
}

// ---------------------------------------------------------------------------
// reductions and elementwise helpers
// ---------------------------------------------------------------------------

constexpr int kRedBlocks = 256;

__global__ __launch_bounds__(256) void k_dot_partial(const double* __restrict__ x,
                                                     const double* __restrict__ y, long long n,
                                                     double* __restrict__ part) {
  __shared__ double red[4];
  double s = 0.0;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) s += x[i] * y[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_dot_final(const double* __restrict__ part, int np,
                                                   double coef, double* out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) s += part[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) *out += coef * s;
}

void dot_accumulate(hipStream_t s, const double* x, const double* y, long long n, double coef,
                    double* out) {
  // out is followed by kRedBlocks doubles of scratch (see runtime)
  if (n <= 0) return;
  const int nb = (int)std::min<long long>(kRedBlocks, (n + 255) / 256);
  double* part = out + 1;
  hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(256), 0, s, x, y, n, part);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, s, part, nb, coef, out);
  check_launch("dot_accumulate");
}

// up to kMaxSegs independent device copies in one launch
__global__ __launch_bounds__(256) void k_copy_segments(CopySegs cs) {
  for (int i = 0; i < cs.n; ++i) {
    const CopySeg g = cs.s[i];
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < g.n; e += 256LL * gridDim.x) g.dst[e] = g.src[e];
  }
}

void copy_segments(hipStream_t s, const CopySegs& cs) {
  long long mx = 0;
  for (int i = 0; i < cs.n; ++i) mx = std::max(mx, cs.s[i].n);
  if (mx == 0) return;
  const int nb = (int)std::min<long long>(1024, (mx + 255) / 256);
  hipLaunchKernelGGL(k_copy_segments, dim3(nb), dim3(256), 0, s, cs);
  check_launch("copy_segments");
}

__global__ void k_fill(double* x, long long n, double v) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) x[i] = v;
}

void fill(hipStream_t s, double* x, long long n, double v) {
  if (n <= 0) return;
  const int nb = (int)std::min<long long>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(k_fill, dim3(nb), dim3(256), 0, s, x, n, v);
  check_launch("fill");
}

__global__ void k_scale_copy(const double* x, long long n, double a, double* y) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) y[i] = a * x[i];
}

void scale_copy(hipStream_t s, const double* x, long long n, double a, double* y) {
  if (n <= 0) return;
  const int nb = (int)std::min<long long>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(k_scale_copy, dim3(nb), dim3(256), 0, s, x, n, a, y);
  check_launch("scale_copy");
}

// ---------------------------------------------------------------------------
// low-rank FD transform: FFT-based DSTs in LDS
// ---------------------------------------------------------------------------

constexpr int kFdThreads = 256;

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Radix-2 Stockham FFT of length L (power of two) in LDS; `sign` = -1 forward
// (exp(-2 pi i)), +1 inverse (unnormalised).  Returns the buffer holding
// the result.
__device__ double2* fft_lds(double2* in, double2* out, const double2* tw, int L, int sign) {
  const int half = L >> 1;
  for (int Ns = 1; Ns < L; Ns <<= 1) {
    const int step = half / Ns;
    for (int j = threadIdx.x; j < half; j += blockDim.x) {
      const int k = j & (Ns - 1);
      double2 w = tw[k * step];
      if (sign > 0) w.y = -w.y;
      const double2 a = in[j];
      const double2 b = cmul(in[j + half], w);
      const int idx = 2 * (j - k) + k;
      out[idx] = make_double2(a.x + b.x, a.y + b.y);
      out[idx + Ns] = make_double2(a.x - b.x, a.y - b.y);
    }
    __syncthreads();
    double2* t = in;
    in = out;
    out = t;
  }
  return in;
}

__global__ __launch_bounds__(kFdThreads) void k_fd_forward(FdDev d, const double* __restrict__ S,
                                                           int lds_, double* __restrict__ Z) {
  extern __shared__ double2 sm2[];
  const int N = d.N, L = 2 * N;
  double2* b0 = sm2;
  double2* b1 = b0 + L;
  double2* tw = b1 + L;
  double* sv = reinterpret_cast<double*>(tw + N);
  double* red = sv + d.n;
  const int c = blockIdx.x;
  const double* col = S + (long long)c * lds_;
  for (int i = threadIdx.x; i < d.n; i += kFdThreads) sv[i] = col[i];
  for (int i = threadIdx.x; i < N; i += kFdThreads) tw[i] = d.tw[i];
  for (int i = threadIdx.x; i < L; i += kFdThreads) b0[i] = make_double2(0.0, 0.0);
  __syncthreads();
  // t = E^T s, laid out as the odd extension of the DST input
  for (int mm = threadIdx.x; mm < d.n1; mm += kFdThreads) {
    double t = 0.0;
    for (int k = 0; k < d.ket; ++k) {
      const int src = d.et_idx[mm * d.ket + k];
      if (src >= 0) t += d.et_val[mm * d.ket + k] * sv[src];
    }
    if (d.odd) {            // y[m+1] = t, y[2N-m-1] = -t   (DST-I)
      b0[mm + 1].x = t;
      b0[L - mm - 1].x = -t;
    } else {                // y[m] = t, y[2N-1-m] = -t      (DST-II)
      b0[mm].x = t;
      b0[L - 1 - mm].x = -t;
    }
  }
  __syncthreads();
  double2* Y = fft_lds(b0, b1, tw, L, -1);
  double* zc = Z + (long long)c * d.n;
  for (int mm = threadIdx.x; mm < d.n1; mm += kFdThreads) {
    const int k = mm + 1;
    double u;
    if (d.odd) {
      u = -0.5 * Y[k].y;
    } else {
      const double ang = -3.14159265358979323846 * k / (2.0 * N);
      double sa, ca;
      sincos(ang, &sa, &ca);
      // Im(e^{i ang} Y[k])
      u = -0.5 * (ca * Y[k].y + sa * Y[k].x);
    }
    zc[mm] = d.g[mm] * u;
  }
  for (int a = 0; a < d.n2; ++a) {
    double part = 0.0;
    for (int i = threadIdx.x; i < d.n; i += kFdThreads) part += d.v2u2[i + (long long)a * d.n] * sv[i];
    const double t = block_sum(part, red);
    if (threadIdx.x == 0) zc[d.n1 + a] = t;
  }
}

__global__ __launch_bounds__(kFdThreads) void k_fd_backward(FdDev d, const double* __restrict__ Z,
                                                            int r, double* __restrict__ Yout) {
  extern __shared__ double2 sm2[];
  const int N = d.N, L = 2 * N;
  double2* b0 = sm2;
  double2* b1 = b0 + L;
  double2* tw = b1 + L;
  double* cv = reinterpret_cast<double*>(tw + N);
  double* w2 = cv + d.n1;
  const int c = blockIdx.x, j = blockIdx.y;
  const double* zc = Z + (long long)c * d.n;
  const double* ej = d.expD + (long long)j * d.n;
  for (int i = threadIdx.x; i < N; i += kFdThreads) tw[i] = d.tw[i];
  for (int i = threadIdx.x; i < L; i += kFdThreads) b0[i] = make_double2(0.0, 0.0);
  for (int a = threadIdx.x; a < d.n2; a += kFdThreads) w2[a] = ej[d.n1 + a] * zc[d.n1 + a];
  __syncthreads();
  for (int mm = threadIdx.x; mm < d.n1; mm += kFdThreads) {
    const double wv = ej[mm] * d.g[mm] * zc[mm];
    if (d.odd) {
      b0[mm + 1].x = wv;
      b0[L - mm - 1].x = -wv;
    } else {                // c[k] = w_{k-1} e^{i pi k / 2N}, k = 1..N
      const int k = mm + 1;
      double sa, ca;
      sincos(3.14159265358979323846 * k / (2.0 * N), &sa, &ca);
      b0[k] = make_double2(wv * ca, wv * sa);
    }
  }
  __syncthreads();
  double2* F = fft_lds(b0, b1, tw, L, d.odd ? -1 : +1);
  for (int mm = threadIdx.x; mm < d.n1; mm += kFdThreads)
    cv[mm] = d.odd ? -0.5 * F[mm + 1].y : F[mm].y;
  __syncthreads();
  double* yc = Yout + (long long)(j * r + c) * d.n;
  for (int l = threadIdx.x; l < d.n; l += kFdThreads) {
    double acc = 0.0;
    for (int k = 0; k < d.ke; ++k) {
      const int src = d.e_idx[l * d.ke + k];
      if (src >= 0) acc += d.e_val[l * d.ke + k] * cv[src];
    }
    for (int a = 0; a < d.n2; ++a) acc += d.v2u2[l + (long long)a * d.n] * w2[a];
    yc[l] = acc;
  }
}

static size_t fd_lds_bytes(const FdDev& d) {
  return sizeof(double2) * (4 * d.N + d.N) + sizeof(double) * (d.n + d.n1 + d.n2 + 16);
}

void fd_forward(hipStream_t s, const FdDev& d, const double* S, int lds_, int r, double* Z) {
  if (r <= 0) return;
  hipLaunchKernelGGL(k_fd_forward, dim3(r), dim3(kFdThreads), fd_lds_bytes(d), s, d, S, lds_, Z);
  check_launch("fd_forward");
}

void fd_backward(hipStream_t s, const FdDev& d, const double* Z, int r, double* Y) {
  if (r <= 0 || d.R <= 0) return;
  hipLaunchKernelGGL(k_fd_backward, dim3(r, d.R), dim3(kFdThreads), fd_lds_bytes(d), s, d, Z, r, Y);
  check_launch("fd_backward");
}

}  // namespace gpu
}  // namespace tk
