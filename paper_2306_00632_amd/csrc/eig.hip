// Symmetric eigendecomposition G = V diag(w) V^T of the Gram matrices of the
// ST-HOSVD (Sec. 2.3, step 3 of Algorithm 1) on one device.
//
// Pipeline (five launches for a <= kTriLdsMax, a few more per column panel
// beyond; no host synchronisation):
//   tridiag        Householder reduction Q^T G Q = T (tridiagonal), one
//                  workgroup; the matrix lives in registers for
//                  a <= kTriLdsMax, in global memory beyond
//   bisect         eigenvalues of T by Sturm-count multisection, one
//                  wavefront per eigenvalue, 63 trial points per step
//   invit          two steps of inverse iteration per eigenvalue (one
//                  thread each, tridiagonal LU with partial pivoting, seeded
//                  pseudo-random start vectors)
//   mgs            modified Gram-Schmidt in descending eigenvalue order, a
//                  second pass when the first met nearly parallel columns
//                  (clusters of close eigenvalues), so the columns are
//                  orthonormal to rounding level (beyond kTriLdsMax: block
//                  Gram-Schmidt, panels projected twice by GEMMs)
//   backtransform  V = Q X, one wavefront per column
// The matrix is scaled by a power of two so that max |G_ij| is in [1, 2);
// w is returned unscaled, in descending order.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <stdexcept>
#include <string>

#include "kernels.h"

namespace tk {
namespace gpu {

namespace {

constexpr int kTriThreads = 1024;
constexpr int kTriLdsMax = 136;  // a^2 + 10 a doubles fit in the 160 KB of LDS
constexpr int kBisWaves = 4;
constexpr int kInvThreads = 64;
constexpr int kBackWaves = 16;

void check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

// Cross-lane moves of a double through DPP on its two 32-bit halves.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ double lane_value(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Reductions over the 64 lanes of a wavefront (all lanes active), returned
// to every lane: quad swaps (quad_perm 1,0,3,2 and 2,3,0,1), half-row and
// row mirrors leave each 16-lane row holding its total in every lane; the
// four row totals are then combined in a fixed order, so the result is the
// same in every lane and from run to run.
#define TK_WAVE_REDUCE(NAME, OP)                                                              \
  __device__ __forceinline__ double NAME(double v) {                                          \
    v = OP(v, dpp_move<0xB1>(v));                                                              \
    v = OP(v, dpp_move<0x4E>(v));                                                              \
    v = OP(v, dpp_move<0x141>(v));                                                             \
    v = OP(v, dpp_move<0x140>(v));                                                             \
    return OP(OP(lane_value(v, 0), lane_value(v, 16)), OP(lane_value(v, 32), lane_value(v, 48))); \
  }

__device__ __forceinline__ double op_add(double x, double y) { return x + y; }
__device__ __forceinline__ double op_max(double x, double y) { return fmax(x, y); }
__device__ __forceinline__ double op_min(double x, double y) { return fmin(x, y); }
TK_WAVE_REDUCE(wave_sum, op_add)
TK_WAVE_REDUCE(wave_max, op_max)
TK_WAVE_REDUCE(wave_min, op_min)
#undef TK_WAVE_REDUCE

// 1/q to full double precision: hardware reciprocal and two Newton steps
// (|q| is a normal number here)
__device__ __forceinline__ double recip(double q) {
  double r = __builtin_amdgcn_rcp(q);
  double e = fma(-q, r, 1.0);
  r = fma(r, e, r);
  e = fma(-q, r, 1.0);
  return fma(r, e, r);
}

// Register-resident layout of an a x a matrix (a <= kTriLdsMax) in one
// workgroup of kRegThreads threads: the four lanes of a quad hold one column,
// lane b of the quad the kRegRows rows [b kRegRows, (b+1) kRegRows); wavefront
// w holds columns [16w, 16w+16).  Reductions over a column are two DPP quad
// permutes, with no LDS and no barrier.  Rows at or beyond a are zero padding
// (in registers and in the LDS vectors they meet), so the per-row loops have
// compile-time bounds and no tests.
constexpr int kRegBlocks = 4;
constexpr int kRegRows = 34;  // kRegBlocks * kRegRows >= kTriLdsMax
constexpr int kRegThreads = 576;  // 9 wavefronts x 16 columns >= kTriLdsMax
constexpr int kPadRows = kRegBlocks * kRegRows;
static_assert(kPadRows >= kTriLdsMax, "row blocks must cover kTriLdsMax rows");
static_assert(kRegThreads / 4 >= kTriLdsMax, "one quad per column");

struct RegLayout {
  int c, b, r0;
  bool act;
  __device__ RegLayout(int a, int t) {
    c = t >> 2;
    b = t & 3;
    act = c < a;
    r0 = b * kRegRows;
  }
};

// sum over the four lanes of a quad (all four hold the result, bitwise equal)
__device__ __forceinline__ double quad_sum(double v) {
  v += dpp_move<0xB1>(v);
  v += dpp_move<0x4E>(v);
  return v;
}

// SplitMix64 finaliser (Steele, Lea, Flood 2014) mapped to [-1, 1)
__device__ inline double unit_rand(unsigned long long key) {
  key += 0x9e3779b97f4a7c15ULL;
  key = (key ^ (key >> 30)) * 0xbf58476d1ce4e5b9ULL;
  key = (key ^ (key >> 27)) * 0x94d049bb133111ebULL;
  key ^= key >> 31;
  return (double)(key >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Householder tridiagonalisation.  Step j maps column j below the diagonal
// to alpha e_1 with H_j = I - tau_j v_j v_j^T (v_j stored in column j of R,
// rows j+1..a-1) and updates the trailing block as
// S <- S - v w^T - w v^T, w = p - (tau/2)(p.v) v, p = tau S v.  This
// version (a > kTriLdsMax) keeps S in global memory and runs the steps
// j < jstop; k_tridiag_reg below holds the matrix in registers and takes
// over the trailing block of order kTriLdsMax (its steps cost about the same
// whatever the trailing order, so the hand-off saves a - 2 - jstop of them).
__global__ __launch_bounds__(kTriThreads) void k_tridiag(const double* __restrict__ G, int a,
                                                         double* Sg, double* __restrict__ R,
                                                         double* __restrict__ tau_out,
                                                         double* __restrict__ d,
                                                         double* __restrict__ e,
                                                         double* __restrict__ misc, int jstop) {
  extern __shared__ double sm[];
  constexpr int ng = 4;
  double* S = Sg;
  double* v = sm;
  double* w = v + a;
  double* part = w + a;  // ng x a partial products
  __shared__ double red[kTriThreads / 64];
  __shared__ double scale_s, tau_s;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int aa = a * a;

  double mx = 0.0;
  for (int i = tid; i < aa; i += kTriThreads) mx = fmax(mx, fabs(G[i]));
  mx = wave_max(mx);
  if (lane == 0) red[wv] = mx;
  __syncthreads();
  if (tid == 0) {
    double m = 0.0;
    for (int i = 0; i < kTriThreads / 64; ++i) m = fmax(m, red[i]);
    scale_s = (m > 0.0 && m <= DBL_MAX) ? ldexp(1.0, -ilogb(m)) : 1.0;
    misc[0] = scale_s;
  }
  __syncthreads();
  const double sc = scale_s;
  for (int i = tid; i < aa; i += kTriThreads) S[i] = G[i] * sc;
  __syncthreads();

  for (int j = 0; j + 2 < a && j < jstop; ++j) {
    const int m = a - 1 - j;  // trailing order, >= 2
    const int o = j + 1;      // first trailing index
    const double* xj = S + (size_t)j * a + o;
    if (wv == 0) {
      double xx = 0.0;
      for (int r = 1 + lane; r < m; r += 64) xx += xj[r] * xj[r];
      xx = wave_sum(xx);
      const double x0 = xj[0];
      double alpha, tau, v0;
      if (xx == 0.0) {
        alpha = x0;
        tau = 0.0;
        v0 = 0.0;
      } else {
        const double nx = sqrt(x0 * x0 + xx);
        alpha = x0 >= 0.0 ? -nx : nx;
        v0 = x0 - alpha;
        tau = 2.0 / (v0 * v0 + xx);
      }
      for (int r = lane; r < m; r += 64) {
        const double vr = tau == 0.0 ? 0.0 : (r == 0 ? v0 : xj[r]);
        v[r] = vr;
        R[(size_t)j * a + o + r] = vr;
      }
      if (lane == 0) {
        tau_s = tau;
        tau_out[j] = tau;
        e[j] = alpha;
        d[j] = S[(size_t)j * a + j];
      }
    }
    __syncthreads();
    const double tau = tau_s;
    if (tau != 0.0) {
      for (int idx = tid; idx < m * ng; idx += kTriThreads) {
        const int r = idx % m, g = idx / m;
        const double* col = S + (size_t)o * a + o + r;
        double acc = 0.0;
        for (int c = g; c < m; c += ng) acc += col[(size_t)c * a] * v[c];
        part[g * a + r] = acc;
      }
      __syncthreads();
      if (wv == 0) {
        double pv = 0.0;
        for (int r = lane; r < m; r += 64) {
          double p = 0.0;
          for (int g = 0; g < ng; ++g) p += part[g * a + r];
          p *= tau;
          w[r] = p;
          pv += p * v[r];
        }
        pv = wave_sum(pv);
        const double K = 0.5 * tau * pv;
        for (int r = lane; r < m; r += 64) w[r] -= K * v[r];
      }
      __syncthreads();
      for (int idx = tid; idx < m * m; idx += kTriThreads) {
        const int r = idx % m, c = idx / m;
        S[(size_t)(o + c) * a + o + r] -= v[r] * w[c] + w[r] * v[c];
      }
    }
    __syncthreads();
  }
  if (tid == 0 && jstop + 2 >= a) {
    if (a >= 2) {
      d[a - 2] = S[(size_t)(a - 2) * a + a - 2];
      e[a - 2] = S[(size_t)(a - 2) * a + a - 1];
    }
    d[a - 1] = S[(size_t)(a - 1) * a + a - 1];
    e[a - 1] = 0.0;
  }
}

// Sum of n <= 16 LDS values in index order; the loads are issued together.
__device__ __forceinline__ double lds_sum16(const double* p, int n) {
  double v[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = i < n ? p[i] : 0.0;
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += v[i];
  return s;
}

__device__ __forceinline__ double lds_sum16_strided(const double* p, int stride, int n) {
  double v[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = i < n ? p[i * stride] : 0.0;
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += v[i];
  return s;
}

// The same reduction for a <= kTriLdsMax with the matrix in registers
// (RegLayout; S symmetric, so a column slice is also a row slice).  Only the
// trailing rows of a column are updated, so rows above the subdiagonal hold
// stale values; they are masked where a column is read.  Step j, two
// barriers:
//   P  p_c = tau (S v)_c for the trailing columns (quad reduction), p to
//      LDS, wavefront partials of p.v
//   U  K = tau/2 p.v, S <- S - v w^T - w v^T with w = p - K v, i.e.
//      x_r -= v_r (p_c - 2 K v_c) + p_r v_c; then the wavefront owning
//      column j+1 derives the next reflector from its registers and
//      publishes it (v, tau double buffered by step parity)
// d, e and tau are staged in LDS and written, with the reflectors, at the end.
__global__ __launch_bounds__(kRegThreads) void k_tridiag_reg(const double* __restrict__ G, int a,
                                                             double* __restrict__ R,
                                                             double* __restrict__ tau_out,
                                                             double* __restrict__ d,
                                                             double* __restrict__ e,
                                                             double* __restrict__ misc, int ld,
                                                             int noscale) {
  constexpr int nw = kRegThreads / 64;
  __shared__ double vbuf[2][kPadRows], pbuf[kPadRows], colbuf[kPadRows];
  __shared__ double dl[kTriLdsMax], el[kTriLdsMax], tl[kTriLdsMax];
  __shared__ double red[nw], tau_s[2];
  __shared__ double sc_s;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const RegLayout L(a, t);
  const int c = L.c, b = L.b, r0 = L.r0;
  const bool act = L.act;

  for (int i = t; i < kPadRows; i += kRegThreads) {
    vbuf[0][i] = 0.0;
    vbuf[1][i] = 0.0;
    pbuf[i] = 0.0;
    colbuf[i] = 0.0;
  }
  // G and R have leading dimension ld; with noscale the matrix is the
  // trailing block of one already scaled (misc[0] is left as it is)
  double mx = 0.0;
  if (!noscale)
    for (int i = t; i < a * a; i += kRegThreads) mx = fmax(mx, fabs(G[(size_t)(i / a) * ld + i % a]));
  mx = wave_max(mx);
  if (lane == 0) red[wv] = mx;
  __syncthreads();
  if (t == 0) {
    double m = 0.0;
    for (int i = 0; i < nw; ++i) m = fmax(m, red[i]);
    sc_s = noscale ? 1.0 : (m > 0.0 && m <= DBL_MAX) ? ldexp(1.0, -ilogb(m)) : 1.0;
    if (!noscale) misc[0] = sc_s;
  }
  __syncthreads();
  const double sc = sc_s;
  double x[kRegRows];
#pragma unroll
  for (int k = 0; k < kRegRows; ++k) x[k] = (act && r0 + k < a) ? G[(size_t)c * ld + r0 + k] * sc : 0.0;
  const double* prow = pbuf + r0;

  // Reflector of column jj, run by the whole wavefront that owns it: the
  // owner quad writes the column to LDS, then all 64 lanes take three rows
  // each (masked norm below the subdiagonal, v, the stored reflector).
  auto reflector = [&](int jj) {
    if (act && c == jj) {
#pragma unroll
      for (int k = 0; k < kRegRows; ++k) colbuf[r0 + k] = x[k];
    }
    double col[3], sq = 0.0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const int r = lane + 64 * m;
      col[m] = r < kPadRows ? colbuf[r] : 0.0;
      if (r > jj + 1) sq += col[m] * col[m];
    }
    const double xx = wave_sum(sq);
    const double x0 = colbuf[jj + 1];
    double alpha, tau, v0;
    if (xx == 0.0) {
      alpha = x0;
      tau = 0.0;
      v0 = 0.0;
    } else {
      const double nx = sqrt(x0 * x0 + xx);
      alpha = x0 >= 0.0 ? -nx : nx;
      v0 = x0 - alpha;
      tau = 2.0 / (v0 * v0 + xx);
    }
    double* vb = vbuf[jj & 1];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const int r = lane + 64 * m;
      const double vr = (tau == 0.0 || r <= jj) ? 0.0 : (r == jj + 1 ? v0 : col[m]);
      if (r < kPadRows) vb[r] = vr;
      if (r > jj && r < a) R[(size_t)jj * ld + r] = vr;
    }
    if (lane == 0) {
      tau_s[jj & 1] = tau;
      tl[jj] = tau;
      el[jj] = alpha;
      dl[jj] = colbuf[jj];
    }
  };
  if (a > 2 && wv == 0) reflector(0);
  __syncthreads();

  for (int j = 0; j + 2 < a; ++j) {
    const double tau = tau_s[j & 1];
    const double* v = vbuf[j & 1];
    const double* vrow = v + r0;
    const bool live = act && c > j;
    double pc = 0.0, vc = 0.0;
    if (tau != 0.0) {
      // finished columns (c <= j; quads are uniform in c) skip the product
      if (live) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int k = 0; k < kRegRows; k += 2) {
          s0 += x[k] * vrow[k];
          s1 += x[k + 1] * vrow[k + 1];
        }
        pc = tau * quad_sum(s0 + s1);
        vc = v[c];
      }
      if (act && b == 0) pbuf[c] = pc;
      const double contrib = wave_sum((live && b == 0) ? pc * vc : 0.0);
      if (lane == 0) red[wv] = contrib;
      __syncthreads();
      if (live) {
        double kk = 0.0;
#pragma unroll
        for (int i = 0; i < nw; ++i) kk += red[i];
        const double K = 0.5 * tau * kk;
        const double g = pc - 2.0 * K * vc;
#pragma unroll
        for (int k = 0; k < kRegRows; ++k) x[k] = fma(-vrow[k], g, fma(-prow[k], vc, x[k]));
      }
    }
    if (j + 3 < a && wv == ((j + 1) >> 4)) reflector(j + 1);
    __syncthreads();
  }
  // the last 2 x 2 block
  if (act && c == a - 1) {
#pragma unroll
    for (int k = 0; k < kRegRows; ++k) colbuf[r0 + k] = x[k];
  }
  if (a >= 2 && act && c == a - 2) {
#pragma unroll
    for (int k = 0; k < kRegRows; ++k) pbuf[r0 + k] = x[k];
  }
  __syncthreads();
  if (t == 0) {
    if (a >= 2) {
      d[a - 2] = pbuf[a - 2];
      e[a - 2] = pbuf[a - 1];
    }
    d[a - 1] = colbuf[a - 1];
    e[a - 1] = 0.0;
  }
  for (int i = t; i + 2 < a; i += kRegThreads) {
    tau_out[i] = tl[i];
    e[i] = el[i];
    d[i] = dl[i];
  }
}

// Number of eigenvalues of T below x (Sturm sequence of the LDL^T pivots);
// pivots smaller than pivmin in magnitude are replaced by -pivmin.
__device__ inline int sturm_count(const double* dd, const double* e2, int a, double x, double pivmin) {
  double q = dd[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int c = q < 0.0;
  for (int i = 1; i < a; ++i) {
    q = (dd[i] - x) - e2[i - 1] * recip(q);
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
  }
  return c;
}

// Eigenvalue k (k-th smallest) of T: the interval [L, H] with
// count(L) <= k < count(H) is cut at 63 interior points per step (one per
// lane) and replaced by the sub-interval where the count passes k.
__global__ __launch_bounds__(64 * kBisWaves) void k_bisect(int a, const double* __restrict__ d,
                                                           const double* __restrict__ e,
                                                           const double* __restrict__ misc,
                                                           double* __restrict__ lam,
                                                           double* __restrict__ w_out) {
  extern __shared__ double bs[];
  double* dd = bs;
  double* e2 = bs + a;
  __shared__ double rlo[kBisWaves], rhi[kBisWaves], re2[kBisWaves];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double lo = INFINITY, hi = -INFINITY, em = 0.0;
  for (int i = tid; i < a; i += 64 * kBisWaves) {
    const double di = d[i];
    const double el = i > 0 ? fabs(e[i - 1]) : 0.0;
    const double er = i + 1 < a ? fabs(e[i]) : 0.0;
    dd[i] = di;
    e2[i] = er * er;
    lo = fmin(lo, di - el - er);
    hi = fmax(hi, di + el + er);
    em = fmax(em, er * er);
  }
  lo = wave_min(lo);
  hi = wave_max(hi);
  em = wave_max(em);
  if (lane == 0) {
    rlo[wv] = lo;
    rhi[wv] = hi;
    re2[wv] = em;
  }
  __syncthreads();
  lo = rlo[0];
  hi = rhi[0];
  em = re2[0];
  for (int i = 1; i < kBisWaves; ++i) {
    lo = fmin(lo, rlo[i]);
    hi = fmax(hi, rhi[i]);
    em = fmax(em, re2[i]);
  }
  const int k = blockIdx.x * kBisWaves + wv;
  if (k >= a) return;  // no barrier follows
  const double tn = fmax(fabs(lo), fabs(hi));
  const double pivmin = DBL_MIN * fmax(1.0, em);
  const double margin = 2.0 * DBL_EPSILON * tn * a + 2.0 * pivmin;
  double L = lo - margin, H = hi + margin;
  // below 1e-3 u ||T|| the eigenvalues of the rounded Gram matrix carry no
  // information; bisecting further only costs time
  const double abstol = 1e-3 * DBL_EPSILON * tn;
  for (int it = 0; it < 24; ++it) {
    const double x = L + (H - L) * (double)(lane + 1) * (1.0 / 64.0);
    const bool above = lane < 63 && sturm_count(dd, e2, a, x, pivmin) > k;
    const unsigned long long mask = __ballot(above);
    const int first = mask ? __ffsll((long long)mask) - 1 : 63;
    const double xf = __shfl(x, first, 64);
    const double xp = __shfl(x, first > 0 ? first - 1 : 0, 64);
    const double nH = first == 63 ? H : xf;
    const double nL = first == 0 ? L : xp;
    if (!(nL > L || nH < H)) break;
    L = nL;
    H = nH;
    if (H - L <= fmax(2.0 * DBL_EPSILON * fmax(fabs(L), fabs(H)), abstol)) break;
  }
  if (lane == 0) {
    const double l = 0.5 * (L + H);
    lam[a - 1 - k] = l;
    w_out[a - 1 - k] = l / misc[0];
  }
}

// Inverse iteration for one eigenvalue l of T (one thread): T - l I = P L U
// with partial pivoting (multiplier, pivot flag and the three rows of U per
// row), then two solves, the first from a pseudo-random start, the second
// from its normalised result.  Pivots smaller than u ||T|| are replaced by
// +-u ||T|| and right-hand sides have norm <= sqrt(a), so a row of the back
// substitution stays finite; the column is rescaled whenever a value exceeds
// 1e100.  Row r of the work arrays and of the vector x is at [r * stride].
__device__ void invit_one(int a, const double* dd, const double* ee, double tn, double l,
                          unsigned long long seed, double* Mu, double* Ui, double* U1, double* U2,
                          double* Pv, double* x, int stride) {
  // ||T|| >= max |G_ij| >= 1 after the scaling unless G = 0, where any
  // nonzero floor gives the same direction
  const double pert = tn > 0.0 ? DBL_EPSILON * tn : 1.0;
  auto floor_pivot = [pert](double u) { return fabs(u) < pert ? (u >= 0.0 ? pert : -pert) : u; };
  // factorisation, eliminating the random right-hand side on the fly; Ui
  // holds the reciprocals of the pivots
  double cd = dd[0] - l, cu = a > 1 ? ee[0] : 0.0, cb = unit_rand(seed);
#pragma unroll 4
  for (int r = 0; r + 1 < a; ++r) {
    const double sub = ee[r];
    const double nd = dd[r + 1] - l;
    const double nu = r + 2 < a ? ee[r + 1] : 0.0;
    const double nb = unit_rand(seed + r + 1);
    double ui, u1, u2, mlt, pv, br;
    if (fabs(cd) >= fabs(sub)) {
      ui = 1.0 / floor_pivot(cd);
      mlt = sub * ui;
      u1 = cu;
      u2 = 0.0;
      pv = 0.0;
      br = cb;
      cb = nb - mlt * cb;
      cd = nd - mlt * cu;
      cu = nu;
    } else {
      ui = 1.0 / sub;
      mlt = cd * ui;
      u1 = nd;
      u2 = nu;
      pv = 1.0;
      br = nb;
      cb = cb - mlt * nb;
      cd = cu - mlt * nd;
      cu = -mlt * nu;
    }
    const int o = r * stride;
    Mu[o] = mlt;
    Ui[o] = ui;
    U1[o] = u1;
    U2[o] = u2;
    Pv[o] = pv;
    x[o] = br;
  }
  Ui[(a - 1) * stride] = 1.0 / floor_pivot(cd);
  x[(a - 1) * stride] = cb;

  for (int step = 0; step < 2; ++step) {
    if (step == 1) {
      double cbf = x[0];
#pragma unroll 4
      for (int r = 0; r + 1 < a; ++r) {
        const int o = r * stride;
        const double nb = x[o + stride];
        const double mlt = Mu[o];
        double br;
        if (Pv[o] != 0.0) {
          br = nb;
          cbf = cbf - mlt * nb;
        } else {
          br = cbf;
          cbf = nb - mlt * cbf;
        }
        x[o] = br;
      }
      x[(a - 1) * stride] = cbf;
    }
    double x1 = 0.0, x2 = 0.0, nrm = 0.0;
#pragma unroll 4
    for (int r = a - 1; r >= 0; --r) {
      const int o = r * stride;
      const double u1 = r + 1 < a ? U1[o] : 0.0;
      const double u2 = r + 2 < a ? U2[o] : 0.0;
      double xr = (x[o] - u1 * x1 - u2 * x2) * Ui[o];
      while (fabs(xr) > 1e100) {
        // growth through several floored pivots: the system is linear, so
        // rescale the whole column (solved rows and pending right-hand side)
        for (int q = 0; q < a; ++q) x[q * stride] *= 1e-100;
        xr *= 1e-100;
        x1 *= 1e-100;
        x2 *= 1e-100;
        nrm *= 1e-200;
      }
      x[o] = xr;
      nrm += xr * xr;
      x2 = x1;
      x1 = xr;
    }
    if (step == 0) {
      const double sn = nrm > 0.0 ? 1.0 / sqrt(nrm) : 1.0;
      for (int r = 0; r < a; ++r) x[r * stride] *= sn;
    }
  }
}

__device__ inline double tri_norm(int a, const double* dd, const double* ee) {
  double t = 0.0;
  for (int r = threadIdx.x & 63; r < a; r += 64)
    t = fmax(t, fabs(dd[r]) + fabs(ee[r]) + (r > 0 ? fabs(ee[r - 1]) : 0.0));
  return wave_max(t);
}

__device__ inline unsigned long long invit_seed(int i) {
  return 0x5851f42d4c957f2dULL * (unsigned long long)(i + 1);
}

// a <= kTriLdsMax: kInvLds threads (eigenvalues) per workgroup, work arrays
// and vectors in LDS as [row][thread]; X (global, [row][eigenvalue])
// receives the unnormalised vectors.
constexpr int kInvLds = 16;

__global__ __launch_bounds__(64) void k_invit_lds(int a, const double* __restrict__ d,
                                                  const double* __restrict__ e,
                                                  const double* __restrict__ lam,
                                                  double* __restrict__ X) {
  __shared__ double dd[kTriLdsMax], ee[kTriLdsMax];
  __shared__ double wk[6 * kTriLdsMax * kInvLds];
  __shared__ double tnr;
  for (int r = threadIdx.x; r < a; r += 64) {
    dd[r] = d[r];
    ee[r] = e[r];
  }
  __syncthreads();
  const double tn = tri_norm(a, dd, ee);
  if (threadIdx.x == 0) tnr = tn;
  __syncthreads();
  const int tl = threadIdx.x;
  const int i = blockIdx.x * kInvLds + tl;
  if (tl >= kInvLds || i >= a) return;  // no barrier follows
  const int plane = kTriLdsMax * kInvLds;
  double* base = wk + tl;
  invit_one(a, dd, ee, tnr, lam[i], invit_seed(i), base, base + plane, base + 2 * plane,
            base + 3 * plane, base + 4 * plane, base + 5 * plane, kInvLds);
  for (int r = 0; r < a; ++r) X[(size_t)r * a + i] = base[5 * plane + r * kInvLds];
}

// a > kTriLdsMax: one thread per eigenvalue, work arrays in global memory
// ([row][eigenvalue], contiguous across a wavefront).
__global__ __launch_bounds__(kInvThreads) void k_invit(int a, const double* __restrict__ d,
                                                       const double* __restrict__ e,
                                                       const double* __restrict__ lam,
                                                       double* __restrict__ LU,
                                                       double* __restrict__ X) {
  extern __shared__ double ts[];
  double* dd = ts;
  double* ee = ts + a;
  __shared__ double tnr;
  for (int r = threadIdx.x; r < a; r += kInvThreads) {
    dd[r] = d[r];
    ee[r] = e[r];
  }
  __syncthreads();
  const double tn = tri_norm(a, dd, ee);
  if (threadIdx.x == 0) tnr = tn;
  __syncthreads();
  const int i = blockIdx.x * kInvThreads + threadIdx.x;
  if (i >= a) return;  // no barrier follows
  const size_t aa = (size_t)a * a;
  invit_one(a, dd, ee, tnr, lam[i], invit_seed(i), LU + i, LU + aa + i, LU + 2 * aa + i,
            LU + 3 * aa + i, LU + 4 * aa + i, X + i, a);
}

// Block Gram-Schmidt for a > kTriLdsMax (left-looking, two projections per
// panel, BCGS2): the columns, in eigenvalue order, are taken in panels of
// panel_width(a) (kPanel, fewer where a x kPanel doubles exceed the LDS
// budget); each panel is projected twice against all finished
// columns by two GEMMs on the matrix cores (W = Q_done^T P, P -= Q_done W),
// then orthonormalised within itself by two passes of modified Gram-Schmidt
// in LDS (k_mgs_panel).  The triangular structure is that of Gram-Schmidt,
// so the result equals the column-by-column version up to rounding; the
// O(a^3) projection work runs on many compute units instead of streaming
// the whole matrix through one.
constexpr int kPanel = 32;
constexpr int kPanelLds = 19200;  // doubles of LDS for one panel (150 KB)
inline int panel_width(int a) { return std::max(1, std::min(kPanel, kPanelLds / a)); }

// out (column-major) = transpose of in ([row][column]), a x a
__global__ __launch_bounds__(256) void k_transpose_sq(int a, const double* __restrict__ in,
                                                      double* __restrict__ out) {
  __shared__ double tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int r = by + k, c = bx + tx;
    tile[k][tx] = (r < a && c < a) ? in[(size_t)r * a + c] : 0.0;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int c = bx + k, r = by + tx;  // out[r + c a] = in[r][c]
    if (r < a && c < a) out[(size_t)c * a + r] = tile[tx][k];
  }
}

// Two passes of modified Gram-Schmidt on the nb <= kPanel columns of the
// panel P (a rows, ld a, in place), each followed by normalisation; one
// wavefront per column update, the panel held in LDS.
__global__ __launch_bounds__(kTriThreads) void k_mgs_panel(int a, int nb, double* __restrict__ P) {
  extern __shared__ double pl[];  // a * nb
  __shared__ double nrm_s[kPanel];
  constexpr int nw = kTriThreads / 64;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int tot = a * nb;
  for (int i = tid; i < tot; i += kTriThreads) pl[i] = P[i];
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    for (int j = 0; j < nb; ++j) {
      const double* qj = pl + (size_t)j * a;
      if (wv == 0) {
        double s = 0.0;
        for (int r = lane; r < a; r += 64) s += qj[r] * qj[r];
        s = wave_sum(s);
        if (lane == 0) nrm_s[j] = s;
      }
      __syncthreads();
      const double nj = nrm_s[j];
      for (int c = j + 1 + wv; c < nb; c += nw) {
        double* qc = pl + (size_t)c * a;
        double dp = 0.0;
        for (int r = lane; r < a; r += 64) dp += qj[r] * qc[r];
        dp = wave_sum(dp);
        const double coef = nj > 0.0 ? dp / nj : 0.0;
        for (int r = lane; r < a; r += 64) qc[r] -= coef * qj[r];
      }
      __syncthreads();
    }
    for (int i = tid; i < tot; i += kTriThreads) {
      const double n2 = nrm_s[i / a];
      if (n2 > 0.0) pl[i] *= 1.0 / sqrt(n2);
    }
    __syncthreads();
  }
  for (int i = tid; i < tot; i += kTriThreads) P[i] = pl[i];
}

// Modified Gram-Schmidt for a <= kTriLdsMax with the columns in registers
// (RegLayout), one barrier per step: every column c > j takes its product
// with the published column j (quad reduction) and is updated; the wavefront
// owning column j+1 then publishes it with its squared norm (double buffered
// by step parity).  A second pass runs only when some pair of columns of the
// first pass had |cos| > 1e-3 (below that one pass already leaves them
// orthogonal to rounding level).  Xin is [row][column], Xo column-major.
__global__ __launch_bounds__(kRegThreads) void k_mgs_reg(int a, const double* __restrict__ Xin,
                                                         double* __restrict__ Xo) {
  constexpr int nw = kRegThreads / 64;
  __shared__ double qbuf[2][kPadRows];
  __shared__ double nrm_s[2];
  __shared__ double red[nw];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const RegLayout L(a, t);
  const int c = L.c, r0 = L.r0;
  const bool act = L.act;
  double x[kRegRows];
#pragma unroll
  for (int k = 0; k < kRegRows; ++k) x[k] = (act && r0 + k < a) ? Xin[(size_t)(r0 + k) * a + c] : 0.0;
  // publish column jj (by its whole wavefront: the quad reduction needs every
  // lane active) and return its squared norm in the owner quad
  auto publish = [&](int jj) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kRegRows; ++k) s += x[k] * x[k];
    s = quad_sum(s);
    if (act && c == jj) {
      double* qn = qbuf[jj & 1] + r0;
#pragma unroll
      for (int k = 0; k < kRegRows; ++k) qn[k] = x[k];
      if (L.b == 0) nrm_s[jj & 1] = s;
    }
    return s;
  };
  for (int pass = 0; pass < 2; ++pass) {
    double cmax = 0.0;  // largest |cos| between column c and an earlier column
    double cur = 0.0;   // squared norm of column c, tracked through the updates
#pragma unroll
    for (int k = 0; k < kRegRows; ++k) cur += x[k] * x[k];
    cur = quad_sum(cur);
    double mynorm = 0.0;
    if (wv == 0) publish(0);
    __syncthreads();
    for (int j = 0; j + 1 < a; ++j) {
      const double nj = nrm_s[j & 1];
      if (c == j) mynorm = nj;
      const double* q = qbuf[j & 1] + r0;
      // columns c <= j are finished: their quads (uniform in c) skip the step
      double dot = 0.0;
      if (act && c > j) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int k = 0; k < kRegRows; k += 2) {
          s0 += q[k] * x[k];
          s1 += q[k + 1] * x[k + 1];
        }
        dot = quad_sum(s0 + s1);
      }
      // reload q for the update instead of holding 34 more values in registers
      asm volatile("" ::: "memory");
      if (act && c > j) {
        const double coef = nj > 0.0 ? dot / nj : 0.0;
        if (pass == 0 && nj > 0.0 && cur > 0.0) cmax = fmax(cmax, fabs(dot) * rsqrt(nj) * rsqrt(cur));
#pragma unroll
        for (int k = 0; k < kRegRows; ++k) x[k] = fma(-coef, q[k], x[k]);
        cur = fmax(cur - dot * coef, 0.0);
      }
      if (wv == ((j + 1) >> 4)) publish(j + 1);
      __syncthreads();
    }
    if (c == a - 1) mynorm = nrm_s[(a - 1) & 1];
    const double sc = mynorm > 0.0 ? 1.0 / sqrt(mynorm) : 0.0;
#pragma unroll
    for (int k = 0; k < kRegRows; ++k) x[k] *= sc;
    // decide on the second pass (the same decision in every thread)
    cmax = wave_max(cmax);
    if (lane == 0) red[wv] = cmax;
    __syncthreads();
    double cm = 0.0;
#pragma unroll
    for (int i = 0; i < nw; ++i) cm = fmax(cm, red[i]);
    if (pass == 0 && cm <= 1e-3) break;
    __syncthreads();
  }
  if (act) {
#pragma unroll
    for (int k = 0; k < kRegRows; ++k)
      if (r0 + k < a) Xo[(size_t)c * a + r0 + k] = x[k];
  }
}

// V = H_0 H_1 ... H_{a-3} X, one wavefront per column of X.  For a <=
// kTriLdsMax the column lives in registers (three rows per lane) and the
// reflectors are staged once per workgroup in LDS; beyond, the column is in
// LDS and the reflectors are read from global memory.
__global__ __launch_bounds__(64 * kBackWaves) void k_backtransform(int a, const double* __restrict__ Rg,
                                                                   const double* __restrict__ tau_g,
                                                                   const double* __restrict__ X,
                                                                   double* __restrict__ V) {
  extern __shared__ double bt[];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nwv = blockDim.x >> 6;
  const int c = blockIdx.x * nwv + wv;
  if (a <= kTriLdsMax) {
    const int aa = a * a;
    for (int idx = tid; idx < aa; idx += blockDim.x) bt[idx] = Rg[idx];
    for (int idx = tid; idx < a; idx += blockDim.x) bt[aa + idx] = tau_g[idx];
    __syncthreads();
    if (c >= a) return;  // no barrier follows
    double x[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const int r = lane + 64 * m;
      x[m] = r < a ? X[(size_t)c * a + r] : 0.0;
    }
    for (int j = a - 3; j >= 0; --j) {
      const double t = bt[aa + j];
      if (t == 0.0) continue;
      const double* vj = bt + (size_t)j * a;
      double v[3], dp = 0.0;
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const int r = lane + 64 * m;
        v[m] = (r > j && r < a) ? vj[r] : 0.0;
        dp += v[m] * x[m];
      }
      dp = wave_sum(dp) * t;
#pragma unroll
      for (int m = 0; m < 3; ++m) x[m] -= dp * v[m];
    }
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const int r = lane + 64 * m;
      if (r < a) V[(size_t)c * a + r] = x[m];
    }
    return;
  }
  if (c >= a) return;
  double* x = bt + (size_t)wv * a;
  for (int r = lane; r < a; r += 64) x[r] = X[(size_t)c * a + r];
  for (int j = a - 3; j >= 0; --j) {
    const double t = tau_g[j];
    if (t == 0.0) continue;
    const double* vj = Rg + (size_t)j * a;
    double dp = 0.0;
    for (int r = j + 1 + lane; r < a; r += 64) dp += vj[r] * x[r];
    dp = wave_sum(dp) * t;
    for (int r = j + 1 + lane; r < a; r += 64) x[r] -= dp * vj[r];
  }
  for (int r = lane; r < a; r += 64) V[(size_t)c * a + r] = x[r];
}

}  // namespace

size_t sym_eig_work(int a) { return (size_t)10 * a * a + 8 * (size_t)a + 16; }

void sym_eig(hipStream_t s, const double* G, int a, double* V, double* w, double* work) {
  if (a <= 0) return;
  const size_t aa = (size_t)a * a;
  double* R = work;
  double* tau = R + aa;
  double* d = tau + a;
  double* e = d + a;
  double* lam = e + a;
  double* misc = lam + a;
  double* S = misc + 16;
  double* LU = S + aa;
  double* X = LU + 5 * aa;
  double* Xo = X + aa;
  if (a <= kTriLdsMax) {
    hipLaunchKernelGGL(k_tridiag_reg, dim3(1), dim3(kRegThreads), 0, s, G, a, R, tau, d, e, misc, a, 0);
  } else {
    // global-memory steps until the trailing order is kTriLdsMax, then the
    // register kernel on that block of S (already scaled)
    const int o0 = a - kTriLdsMax;
    hipLaunchKernelGGL(k_tridiag, dim3(1), dim3(kTriThreads), sizeof(double) * 6 * a, s, G, a, S, R, tau, d,
                       e, misc, o0);
    check("sym_eig tridiag (global steps)");
    const size_t off = (size_t)o0 * a + o0;
    hipLaunchKernelGGL(k_tridiag_reg, dim3(1), dim3(kRegThreads), 0, s, S + off, kTriLdsMax, R + off, tau + o0,
                       d + o0, e + o0, misc, a, 1);
  }
  check("sym_eig tridiag");
  hipLaunchKernelGGL(k_bisect, dim3((a + kBisWaves - 1) / kBisWaves), dim3(64 * kBisWaves),
                     sizeof(double) * 2 * a, s, a, d, e, misc, lam, w);
  check("sym_eig bisect");
  if (a <= kTriLdsMax) {
    hipLaunchKernelGGL(k_invit_lds, dim3((a + kInvLds - 1) / kInvLds), dim3(64), 0, s, a, d, e, lam, X);
  } else {
    hipLaunchKernelGGL(k_invit, dim3((a + kInvThreads - 1) / kInvThreads), dim3(kInvThreads),
                       sizeof(double) * 2 * a, s, a, d, e, lam, LU, X);
  }
  check("sym_eig invit");
  if (a <= kTriLdsMax) {
    hipLaunchKernelGGL(k_mgs_reg, dim3(1), dim3(kRegThreads), 0, s, a, X, Xo);
  } else {
    const int nt = (a + 31) / 32, pw = panel_width(a);
    hipLaunchKernelGGL(k_transpose_sq, dim3(nt, nt), dim3(256), 0, s, a, X, Xo);
    double* W = S;  // a x pw projection coefficients (S is free after the tridiagonalisation)
    for (int k0 = 0; k0 < a; k0 += pw) {
      const int nb = std::min(pw, a - k0);
      double* Pk = Xo + (size_t)k0 * a;
      for (int rep = 0; k0 > 0 && rep < 2; ++rep) {
        dgemm(s, true, false, k0, nb, a, 1.0, Xo, a, 0, Pk, a, 0, 0.0, W, k0, 0);
        dgemm(s, false, false, a, nb, k0, -1.0, Xo, a, 0, W, k0, 0, 1.0, Pk, a, 0);
      }
      hipLaunchKernelGGL(k_mgs_panel, dim3(1), dim3(kTriThreads), sizeof(double) * (size_t)a * nb, s, a, nb, Pk);
    }
  }
  check("sym_eig mgs");
  // one wavefront per column; 8 per workgroup when columns live in LDS
  const int bw = a <= kTriLdsMax ? kBackWaves : 8;
  const size_t bt_lds = sizeof(double) * (a <= kTriLdsMax ? aa + a : (size_t)bw * a);
  hipLaunchKernelGGL(k_backtransform, dim3((a + bw - 1) / bw), dim3(64 * bw), bt_lds, s, a, R, tau, Xo, V);
  check("sym_eig backtransform");
}

}  // namespace gpu
}  // namespace tk
