// HIP kernels for gfx950 (CDNA4, wave64) of the Tucker TPCG library: the
// pieces of the truncation (Algorithm 1) and the vector arithmetic.
//
//  householder_qr QR of stacked factors (Algorithm 1, step 1), one workgroup
//                 per mode, one wavefront per trailing column.
//  column_energy, select_rank, gather_columns
//                 the rank choice of each ST-HOSVD mode from directly
//                 measured energies ||A^T v_j||^2.
//  dot_accumulate, copy_segments, fill, scale_copy
//                 reductions and copies of Tucker data.
// The mode products are in modeprod.hip, the FP64 GEMM in gemm.hip and the
// symmetric eigensolver in eig.hip.
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

// Partial energies of the columns of P (rows x a): segment s of column j
// (kEnergySeg rows) into part[j * S + s]; k_select adds the S partials of a
// column in a fixed order.
constexpr int kEnergySeg = 2048;  // 256 threads x 8 rows
int column_energy_parts(int rows) { return std::max(1, (rows + kEnergySeg - 1) / kEnergySeg); }

__global__ __launch_bounds__(256) void k_column_energy(const double* __restrict__ P, int rows,
                                                       double* __restrict__ part) {
  __shared__ double red[4];
  const int j = blockIdx.y, sg = blockIdx.x;
  const double* col = P + (long long)j * rows;
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < kEnergySeg / 256; ++u) {
    const int i = sg * kEnergySeg + u * 256 + threadIdx.x;
    const double v = col[min(i, rows - 1)];  // unconditional load, masked below
    s += i < rows ? v * v : 0.0;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[(long long)j * gridDim.x + sg] = s;
}

void column_energy(hipStream_t s, const double* P, int rows, int a, double* part) {
  if (a <= 0 || rows <= 0) return;
  hipLaunchKernelGGL(k_column_energy, dim3(column_energy_parts(rows), a), dim3(256), 0, s, P, rows, part);
  check_launch("column_energy");
}

constexpr int kSelMax = 2048;
constexpr double kGramNoise = 64.0;

__global__ __launch_bounds__(1024) void k_select(const double* __restrict__ part, int S, int a, double eps,
                                                 double* norm2_io, int set_norm, int* sel,
                                                 double* disc) {
  __shared__ double key[kSelMax];
  __shared__ int idx[kSelMax];
  __shared__ double red[16];
  int P2 = 1;
  while (P2 < a) P2 <<= 1;
  double psum = 0.0;
  for (int i = threadIdx.x; i < P2; i += 1024) {
    double ei = 0.0;
    if (i < a)
      for (int sg = 0; sg < S; ++sg) ei += part[(long long)i * S + sg];
    key[i] = (i < a) ? ei : -1.0;
    idx[i] = i;
    if (i < a) psum += ei;
  }
  const double tot = block_sum(psum, red);
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
  const double norm2 = set_norm ? tot : *norm2_io;
  const double budget = eps * eps * norm2 / 3.0;
  // directions resolved by the Gram matrix: rounding in G = A A^T (about
  // a eps_mach ||A||^2) mixes the eigenvectors of smaller energies, and an
  // eigenvector of energy e leaks about (a eps_mach e_max)^2 / e of energy
  // into the others, which must stay a tenth of the budget; the keys are
  // sorted, so their count is the number of leading resolved columns
  const double ua = a * 2.220446049250313e-16;
  const double thr = budget > 0.0 ? fmax(kGramNoise * ua * tot, 10.0 * (ua * key[0]) * (ua * key[0]) / budget)
                                  : 2.0 * key[0] + 1.0;
  double cnt = 0.0;
  for (int i = threadIdx.x; i < a; i += 1024) cnt += key[i] >= thr ? 1.0 : 0.0;
  const double k1 = block_sum(cnt, red);
  if (threadIdx.x == 0) {
    if (set_norm) *norm2_io = norm2;
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
    disc[2] = k1;
    disc[3] = tot;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < a; i += 1024) sel[1 + i] = idx[i];
}

void select_rank(hipStream_t s, const double* part, int S, int a, double eps, double* norm2_io,
                 int set_norm, int* sel, double* disc) {
  if (a > kSelMax) throw std::runtime_error("select_rank: more than 2048 columns");
  hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, s, part, S, a, eps, norm2_io, set_norm, sel, disc);
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

}  // namespace gpu
}  // namespace tk
