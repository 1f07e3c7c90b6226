// FP64 GEMM for gfx950 on the matrix cores (v_mfma_f64_16x16x4f64 tiles,
// LDS double buffering, deterministic split-K): the dense contractions of
// the truncation (core formation, Gram matrices, projections, factor
// updates) and of the Tucker dots.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <string>

#include "device_common.h"
#include "kernels.h"

namespace tk {
namespace gpu {

// ---------------------------------------------------------------------------
// FP64 GEMM
// ---------------------------------------------------------------------------

// FP64 GEMM on the matrix cores (v_mfma_f64_16x16x4f64).  A workgroup of WM
// wavefronts computes a (16 WM) x (16 NT) tile of C; wavefront w owns rows
// [16w, 16w+16) and NT column tiles of 16, i.e. NT 16x16 accumulators.  K is
// staged through LDS in steps of BK = 16 (double buffered: the next step's
// global loads are in flight while the current step is multiplied; sub-steps
// of 4 wholly past the end of K, all zero padding, are skipped).  The
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
      if (k0 + ks >= kend) break;  // the rest of the step is zero padding (uniform)
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

// C = sum_z part[z] (+ beta C): the sum of nsplit M x N partial products
// (part[z] column-major with leading dimension M), e.g. of a batched GEMM
void splitk_reduce(hipStream_t s, int M, int N, int nsplit, const double* part, double beta, double* C, int ldc) {
  if (M <= 0 || N <= 0) return;
  const long long MN = (long long)M * N;
  const int nb = (int)std::min<long long>(1024, (MN + 255) / 256);
  hipLaunchKernelGGL(k_splitk_reduce, dim3(nb), dim3(256), 0, s, M, N, nsplit, part, beta, C, ldc);
  check_launch("splitk_reduce");
}

}  // namespace gpu
}  // namespace tk
