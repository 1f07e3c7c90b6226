// Mode-product kernels for gfx950 (CDNA4, wave64): the HBM-bound part of
// one TPCG iteration.
//
//  band_apply     banded mode products A_(k,t) X_k of eq. (tt_product): one
//                 workgroup stages 256-row windows of 8 factor columns in LDS
//                 and applies every 1D matrix of the mode to them, a row's
//                 band entries held in registers (coalesced along n, the
//                 factor is read from HBM once).
//  fd_forward / fd_backward
//                 the low-rank FD transform U~^T and U~ D_j (Algorithm 4,
//                 Appendix B): sparse boundary maps around sine transforms
//                 of length N, each one complex FFT of length N/2 held in the
//                 registers of one wavefront (DST-I for odd p, DST-II/III
//                 for even p).
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
// banded mode products
// ---------------------------------------------------------------------------

constexpr int kBandRows = 256;   // rows of a factor column per workgroup
constexpr int kBandCols = 8;     // factor columns per workgroup (band rows reused across them)

// W[:, t*m + c] = A_t Y[:, c]: a workgroup stages kBandCols windows of 256 + 2p
// rows of Y in LDS; each thread keeps the 2p + 1 band entries of its row of
// A_t in registers, loading those of A_{t+1} while it applies A_t to every
// staged column.  All loads are unconditional (clamped indices), only
// stores are guarded, so the loads of a step issue together.  Y and W are
// FP64; T is the arithmetic type (the bands are stored in T, the staged
// window is rounded to T, the sums are widened on the store).
template <int PD, class T>
__global__ __launch_bounds__(kBandRows) void k_band_apply(int n, int m, int nmat, const T* __restrict__ band,
                                                          const double* __restrict__ Y, int ldy,
                                                          double* __restrict__ W, int ldw) {
  constexpr int NB = 2 * PD + 1, WIN = kBandRows + 2 * PD;
  __shared__ T ys[kBandCols * WIN];
  const int i0 = blockIdx.x * kBandRows;
  const int c0 = blockIdx.y * kBandCols;
  const int nc = min(kBandCols, m - c0);
#pragma unroll
  for (int cc = 0; cc < kBandCols; ++cc) {
    const double* col = Y + (long long)(c0 + min(cc, nc - 1)) * ldy;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int t = min((int)threadIdx.x + h * kBandRows, WIN - 1);
      const int i = i0 - PD + t;
      const T v = T(col[min(max(i, 0), n - 1)]);
      ys[cc * WIN + t] = (i >= 0 && i < n) ? v : T(0);
    }
  }
  __syncthreads();
  const int i = i0 + threadIdx.x;
  if (i >= n) return;
  T bv[NB], bnext[NB];
#pragma unroll
  for (int o = 0; o < NB; ++o) bv[o] = band[(long long)o * n + i];
  for (int t = 0; t < nmat; ++t) {
    const T* bt = band + (long long)min(t + 1, nmat - 1) * NB * n + i;
#pragma unroll
    for (int o = 0; o < NB; ++o) bnext[o] = bt[(long long)o * n];
#pragma unroll
    for (int cc = 0; cc < kBandCols; ++cc) {
      const T* yw = ys + cc * WIN + threadIdx.x;
      T acc = T(0);
#pragma unroll
      for (int o = 0; o < NB; ++o) acc += bv[o] * yw[o];
      // streaming store: the R outputs are written once and read by later kernels
      if (cc < nc) __builtin_nontemporal_store(double(acc), W + i + (long long)(t * m + c0 + cc) * ldw);
    }
#pragma unroll
    for (int o = 0; o < NB; ++o) bv[o] = bnext[o];
  }
}

template <class T>
static void band_apply_t(hipStream_t s, int n, int m, int nmat, int p, const T* band, const double* Y, int ldy,
                         double* W, int ldw) {
  dim3 grid((n + kBandRows - 1) / kBandRows, (m + kBandCols - 1) / kBandCols);
  if (grid.y > 65535) throw std::runtime_error("band_apply: more than 524280 columns");
  switch (p) {
#define TK_BAND(PD) \
  case PD: hipLaunchKernelGGL((k_band_apply<PD, T>), grid, dim3(kBandRows), 0, s, n, m, nmat, band, Y, ldy, W, ldw); break;
    TK_BAND(0) TK_BAND(1) TK_BAND(2) TK_BAND(3) TK_BAND(4) TK_BAND(5) TK_BAND(6)
#undef TK_BAND
    default: throw std::runtime_error("band_apply: half-bandwidth above 6");
  }
}

void band_apply(hipStream_t s, int n, int m, int nmat, int p, const double* band, const float* band_f,
                const double* Y, int ldy, double* W, int ldw) {
  if (n <= 0 || m <= 0 || nmat <= 0) return;
  if (band_f)
    band_apply_t<float>(s, n, m, nmat, p, band_f, Y, ldy, W, ldw);
  else
    band_apply_t<double>(s, n, m, nmat, p, band, Y, ldy, W, ldw);
  check_launch("band_apply");
}

// ---------------------------------------------------------------------------
// low-rank FD transform (Algorithm 4): sine transforms of length N = n_el
// through one complex FFT of length M = N/2 per transform
// ---------------------------------------------------------------------------
//
// A workgroup is one wavefront.  Every lane holds RL = min(8, M) complex
// values of a transform, P = M / RL lanes share one transform and a wave
// runs B = 64 / P transforms side by side (slot b = lane / P), each in its
// own M-element LDS region.  The FFT is a Stockham sequence of radix-8 passes
// (a final radix-4 or radix-2 pass when log2 M is not a multiple of 3), the
// butterflies in registers and one LDS exchange per pass.
//
// Real transforms on top of it (x_0 = x_N = 0 where it applies):
//  * DST-I   F_k = sum_{j=1}^{N-1} x_j sin(pi j k / N): the real DFT of
//    y_j = sin(pi j/N)(x_j + x_{N-j}) + (x_j - x_{N-j})/2 gives F_{2k} = -Im Y_k
//    and F_{2k+1} - F_{2k-1} = Re Y_k (F_1 = Re Y_0 / 2), a prefix sum;
//  * DST-II  S_k = sum_{m<N} x_m sin(pi (2m+1) k / 2N): the DCT-II of
//    (-1)^m x_m read backwards, through the even/odd reordering of the
//    input and one real DFT of length N;
//  * DST-III T_m = sum_{k=1}^{N} w_{k-1} sin(pi k (2m+1) / 2N): DST-II
//    applied in reverse (its rows are orthogonal with squared norms N/2,
//    and N for the last one).
// A real DFT of length N is one complex FFT of length M of the even/odd
// samples packed as (re, im) plus an O(N) split.

// Raw buffer access: a resource covers `count` doubles from a base that is
// the same for the whole wave (so it lives in scalar registers); a lane that
// must not touch memory passes an offset past the range instead.  The
// hardware range check returns 0 for such loads and drops such stores, so
// the ragged ends of unrolled loops need no branches (a branch around a load
// lets the compiler sink the load next to its use and serialise the waits).
typedef unsigned int tk_u32x2 __attribute__((ext_vector_type(2)));
constexpr int kBufWord3 = 0x00020000;      // 32-bit data format, gfx9 family
constexpr unsigned kBufOff = 0xFFFFFFF8u;  // an offset past every range
constexpr unsigned long long kBufOffHost = 0xFFFFFFF0ull;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const double* p, long long count) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(p), (short)0, (int)(unsigned)(count * 8), kBufWord3);
}
__device__ __forceinline__ double buf_ld(__amdgpu_buffer_rsrc_t r, int i, bool ok) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, ok ? unsigned(i) * 8u : kBufOff, 0, 0));
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, int i, bool ok, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(tk_u32x2, v), r, ok ? unsigned(i) * 8u : kBufOff, 0, 0);
}

// Workgroup b of a grid of G is dispatched to XCD b mod 8 (round robin), as
// the local-th workgroup there (local = b / 8).  xcd_order(b, G) numbers the
// workgroups XCD by XCD, so consecutive logical indices share an XCD and its
// L2 (a bijection of [0, G)).
constexpr int kNumXcd = 8;
__device__ __forceinline__ int xcd_order(int b, int G) {
  const int q = G / kNumXcd, r = G % kNumXcd;
  const int x = b % kNumXcd, local = b / kNumXcd;
  return x < r ? x * (q + 1) + local : r * (q + 1) + (x - r) * q + local;
}

constexpr int kFdWave = 64;
constexpr int kFdMaxV2 = 4;  // V_2 columns: p - 1 or p - 2, at most 4 for p <= 6

// Single-precision loads for the float tables (same range rule as above).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const float* p, long long count) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p), (short)0, (int)(unsigned)(count * 4), kBufWord3);
}
template <class T>
__device__ __forceinline__ T buf_ldt(__amdgpu_buffer_rsrc_t r, int i, bool ok) {
  if constexpr (sizeof(T) == 8)
    return buf_ld(r, i, ok);
  else
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, ok ? unsigned(i) * 4u : kBufOff, 0, 0));
}

// The transform's tables in the arithmetic type T of the kernel
template <class T>
__device__ __forceinline__ const FdTab<T>& fd_tab(const FdDev& d) {
  if constexpr (sizeof(T) == 8)
    return d.t64;
  else
    return d.t32;
}

template <int M>
struct FdShape {
  static constexpr int RL = M < 8 ? M : 8;
  static constexpr int P = M / RL;
  static constexpr int B = kFdWave / P;
};

// complex value of the arithmetic type (16-byte aligned for double, 8 for float)
template <class T>
struct alignas(2 * sizeof(T)) Cx {
  T x, y;
};

// LDS views of a slot, padded against bank conflicts (lanes that touch 8
// consecutive complex or 16 consecutive real elements each): complex element
// i sits at i + i/8, real element i at i + i/16; the two views alias.
template <int M>
struct FdSlot {
  static constexpr int SIZE = M + M / 8;  // complex elements
};
template <class T>
struct CBuf {
  Cx<T>* p;
  __device__ __forceinline__ Cx<T>& operator[](int i) const { return p[i + (i >> 3)]; }
};
template <class T>
struct RBuf {
  T* p;
  __device__ __forceinline__ T& operator[](int i) const { return p[i + (i >> 4)]; }
};

template <class T>
__device__ __forceinline__ Cx<T> c_add(Cx<T> a, Cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <class T>
__device__ __forceinline__ Cx<T> c_sub(Cx<T> a, Cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <class T>
__device__ __forceinline__ Cx<T> c_mul(Cx<T> a, Cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class T>
__device__ __forceinline__ Cx<T> c_conj(Cx<T> a) { return {a.x, -a.y}; }
// multiply by SIGN * i
template <int SIGN, class T>
__device__ __forceinline__ Cx<T> c_rot(Cx<T> a) {
  return SIGN > 0 ? Cx<T>{-a.y, a.x} : Cx<T>{a.y, -a.x};
}

// in-register DFT of length R with kernel exp(SIGN 2 pi i t k / R)
template <int R, int SIGN, class T>
__device__ __forceinline__ void dft_reg(Cx<T>* v) {
  if constexpr (R == 2) {
    const Cx<T> t = v[1];
    v[1] = c_sub(v[0], t);
    v[0] = c_add(v[0], t);
  } else if constexpr (R == 4) {
    const Cx<T> t0 = c_add(v[0], v[2]), t1 = c_sub(v[0], v[2]);
    const Cx<T> t2 = c_add(v[1], v[3]), t3 = c_rot<SIGN>(c_sub(v[1], v[3]));
    v[0] = c_add(t0, t2);
    v[2] = c_sub(t0, t2);
    v[1] = c_add(t1, t3);
    v[3] = c_sub(t1, t3);
  } else {
    static_assert(R == 8, "radix");
    Cx<T> e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    dft_reg<4, SIGN>(e);
    dft_reg<4, SIGN>(o);
    constexpr T h = T(0.70710678118654752440);
    constexpr T sg = T(SIGN);
    // o_k *= exp(SIGN 2 pi i k / 8)
    o[1] = Cx<T>{h * (o[1].x - sg * o[1].y), h * (o[1].y + sg * o[1].x)};
    o[2] = c_rot<SIGN>(o[2]);
    o[3] = Cx<T>{h * (-o[3].x - sg * o[3].y), h * (-o[3].y + sg * o[3].x)};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = c_add(e[k], o[k]);
      v[k + 4] = c_sub(e[k], o[k]);
    }
  }
}

// Stockham passes from stride NS on.  On entry to the first pass (NS = 1)
// a[t] holds element q + t P of the lane's transform; every pass leaves its
// result in `buf` (M elements, natural order after the last pass).
template <int M, int SIGN, int NS, class T>
__device__ __forceinline__ void fft_passes(Cx<T>* a, CBuf<T> buf, int q, const Cx<T>* __restrict__ cs) {
  if constexpr (NS < M) {
    constexpr int RL = FdShape<M>::RL, P = FdShape<M>::P;
    constexpr int R = (M / NS) >= 8 ? 8 : (M / NS);
    constexpr int NB = RL / R;  // butterflies per lane
    if constexpr (NS > 1) {
#pragma unroll
      for (int u = 0; u < NB; ++u)
#pragma unroll
        for (int t = 0; t < R; ++t) a[u * R + t] = buf[q + P * u + t * (M / R)];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int j = q + P * u;
      const int k = j & (NS - 1);
      if constexpr (NS > 1) {
#pragma unroll
        for (int t = 1; t < R; ++t) {
          Cx<T> w = cs[2 * t * k * (M / (NS * R))];
          if (SIGN > 0) w.y = -w.y;
          a[u * R + t] = c_mul(a[u * R + t], w);
        }
      }
      dft_reg<R, SIGN>(a + u * R);
    }
    if constexpr (NS > 1) __syncthreads();  // every lane has read this pass's input
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int j = q + P * u;
      const int k = j & (NS - 1);
#pragma unroll
      for (int t = 0; t < R; ++t) buf[(j - k) * R + k + t * NS] = a[u * R + t];
    }
    __syncthreads();
    fft_passes<M, SIGN, NS * R>(a, buf, q, cs);
  }
}

// segmented inclusive prefix sum over the P lanes of a slot
template <int P, class T>
__device__ __forceinline__ T seg_scan(T v, int q) {
#pragma unroll
  for (int d = 1; d < P; d <<= 1) {
    const T o = __shfl_up(v, d, P);
    if (q >= d) v += o;
  }
  return v;
}

template <int P, class T>
__device__ __forceinline__ T seg_sum(T v) {
#pragma unroll
  for (int d = P >> 1; d > 0; d >>= 1) v += __shfl_xor(v, d, P);
  return v;
}

// DST-I pre-processing: a[t] = (y_{2e}, y_{2e+1}) for e = q + t P, x(j) for
// 0 <= j <= N (zero at both ends)
template <int M, class T, class X>
__device__ __forceinline__ void dst1_pre(Cx<T>* a, int q, const T* __restrict__ sn, X x) {
  constexpr int N = 2 * M, RL = FdShape<M>::RL, P = FdShape<M>::P;
#pragma unroll
  for (int t = 0; t < RL; ++t) {
    const int e = q + t * P;
    T y[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = 2 * e + h;
      const T xa = x(j), xb = x(N - j);
      y[h] = sn[j] * (xa + xb) + T(0.5) * (xa - xb);
    }
    a[t] = Cx<T>{y[0], y[1]};
  }
}

// The real DFT bin k (0 <= k <= M) of the packed FFT Z: E + exp(-2 pi i k/N) O.
template <int M, class T>
__device__ __forceinline__ Cx<T> real_bin(CBuf<T> Z, int k, const Cx<T>* __restrict__ cs) {
  const Cx<T> zk = Z[k & (M - 1)], zc = c_conj(Z[(M - k) & (M - 1)]);
  const Cx<T> e{T(0.5) * (zk.x + zc.x), T(0.5) * (zk.y + zc.y)};
  const Cx<T> d = c_sub(zk, zc);
  const Cx<T> o{T(0.5) * d.y, T(-0.5) * d.x};  // -i/2 (zk - zc)
  const Cx<T> w = k < M ? cs[k] : Cx<T>{T(-1), T(0)};
  return c_add(e, c_mul(w, o));
}

// DST-I post-processing: F_f (f = 1..N-1) into cv[f - 1] (cv aliases Z)
template <int M, class T>
__device__ __forceinline__ void dst1_post(CBuf<T> Z, RBuf<T> cv, int q, const Cx<T>* __restrict__ cs) {
  constexpr int RL = FdShape<M>::RL, P = FdShape<M>::P;
  T R[RL], I[RL];
#pragma unroll
  for (int s = 0; s < RL; ++s) {
    const int k = q * RL + s;
    const Cx<T> y = real_bin<M>(Z, k, cs);
    R[s] = (k == 0) ? T(0.5) * y.x : y.x;
    I[s] = -y.y;
  }
#pragma unroll
  for (int s = 1; s < RL; ++s) R[s] += R[s - 1];
  const T tot = seg_scan<P>(R[RL - 1], q);
  const T base = tot - R[RL - 1];
  __syncthreads();  // every lane has read Z
#pragma unroll
  for (int s = 0; s < RL; ++s) {
    const int k = q * RL + s;
    cv[2 * k] = base + R[s];
    if (k > 0) cv[2 * k - 1] = I[s];
  }
  __syncthreads();
}

// DST-II post-processing: S_s (s = 1..N) into cv[s - 1]
template <int M, class T>
__device__ __forceinline__ void dst2_post(CBuf<T> Z, RBuf<T> cv, int q, const Cx<T>* __restrict__ cs,
                                          const Cx<T>* __restrict__ tq) {
  constexpr int N = 2 * M, RL = FdShape<M>::RL;
  T re[RL], im[RL];
  T sm = T(0);
#pragma unroll
  for (int s = 0; s < RL; ++s) {
    const int k = q * RL + s;
    const Cx<T> v = c_mul(tq[k], real_bin<M>(Z, k, cs));
    re[s] = v.x;
    im[s] = -v.y;
  }
  if (q == 0) {
    const Cx<T> z0 = Z[0];
    sm = (tq[M].x * (z0.x - z0.y));  // Re(tq_M (Re Z_0 - Im Z_0))
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < RL; ++s) {
    const int k = q * RL + s;
    cv[N - k - 1] = re[s];
    if (k > 0) cv[k - 1] = im[s];
  }
  if (q == 0) cv[M - 1] = sm;
  __syncthreads();
}

// Z = U~^T S column by column (Algorithm 4, step 5): t = E^T s staged in
// LDS, the sine transform, times g; the V_2 coefficients are plain dot
// products.  S and Z are FP64 in memory; T is the arithmetic type (the
// loads are rounded to it, the results widened back).
template <int M, bool ODD, class T>
__global__ __launch_bounds__(kFdWave) void k_fd_forward(FdDev d, const double* __restrict__ S, int lds_, int r,
                                                        double* __restrict__ Zo) {
  constexpr int N = 2 * M, RL = FdShape<M>::RL, P = FdShape<M>::P, B = FdShape<M>::B;
  constexpr int SL = FdSlot<M>::SIZE;
  __shared__ Cx<T> sm[B * SL];
  const FdTab<T>& tb = fd_tab<T>(d);
  const Cx<T>* cs = reinterpret_cast<const Cx<T>*>(tb.cs);
  const int lane = threadIdx.x, b = lane / P, q = lane % P;
  const int c = blockIdx.x * B + b;
  const bool valid = c < r;
  const double* s = S + (long long)(valid ? c : r - 1) * lds_;
  const CBuf<T> Z{sm + b * SL};
  const RBuf<T> cv{reinterpret_cast<T*>(sm + b * SL)};
  // interior rows of E^T (a shifted copy): at most N = 2 RL P, 2 RL per lane;
  // the loads are clamped into range so that they issue together
  // the B input columns of the workgroup through one resource
  const int c0 = blockIdx.x * B;
  const auto rs = buf_rsrc(S + (long long)c0 * lds_, (long long)(B - 1) * lds_ + d.n);
  const int sb = b * lds_;
  // rows m < N, 2 RL per lane: the interior ones copy s[m + et_sh]
#pragma unroll
  for (int u = 0; u < 2 * RL; ++u) {
    const int m = q + P * u;
    const bool in = valid && m >= d.et_lo && m < d.et_hi;
    cv[m] = T(buf_ld(rs, sb + m + d.et_sh, in));
  }
  // boundary rows [0, et_lo) and [et_hi, n1) through the ELL table, each by
  // the lane that wrote it above
  for (int m = q; m < d.n1; m += P) {
    if (m >= d.et_lo && m < d.et_hi) continue;
    T t = T(0);
    for (int k = 0; k < d.ket; ++k) {
      const int src = d.et_idx[m * d.ket + k];
      if (src >= 0) t += tb.et_val[m * d.ket + k] * T(s[src]);
    }
    cv[m] = t;
  }
  __syncthreads();
  Cx<T> a[RL];
  if constexpr (ODD) {
    dst1_pre<M>(a, q, tb.sn, [&](int j) {
      const T x = cv[min(max(j - 1, 0), N - 2)];
      return (j >= 1 && j < N) ? x : T(0);
    });
  } else {
#pragma unroll
    for (int t = 0; t < RL; ++t) {
      const int e = q + t * P;
      T v[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = 2 * e + h;
        const int m = i < M ? 2 * i : 2 * N - 2 * i - 1;
        v[h] = (m & 1) ? -cv[m] : cv[m];
      }
      a[t] = Cx<T>{v[0], v[1]};
    }
  }
  __syncthreads();  // the staged input is read before the first pass overwrites it
  if constexpr (ODD) {
    fft_passes<M, -1, 1>(a, Z, q, cs);
    dst1_post<M>(Z, cv, q, cs);
  } else {
    fft_passes<M, -1, 1>(a, Z, q, cs);
    dst2_post<M>(Z, cv, q, cs, reinterpret_cast<const Cx<T>*>(tb.tq));
  }
  double* zc = Zo + (long long)c * d.n;
  const auto rz = buf_rsrc(Zo + (long long)c0 * d.n, (long long)B * d.n), rg = buf_rsrc(tb.g, d.n1);
#pragma unroll
  for (int u = 0; u < 2 * RL; ++u) {
    const int mm = q + P * u;
    const bool ok = valid && mm < d.n1;
    buf_st(rz, b * d.n + mm, ok, double(buf_ldt<T>(rg, mm, ok) * cv[mm]));
  }
  for (int a2 = 0; a2 < d.n2; ++a2) {
    const T* v2 = tb.v2u2 + (long long)a2 * d.n;
    const auto rv = buf_rsrc(v2, d.n);
    T part = T(0);
#pragma unroll
    for (int u = 0; u < 2 * RL; ++u) {
      const int i = q + P * u;
      const bool ok = i < d.n;
      part += buf_ldt<T>(rv, i, ok) * T(buf_ld(rs, sb + i, ok && valid));
    }
    for (int i = N + q; i < d.n; i += P) part += v2[i] * T(s[i]);
    part = seg_sum<P>(part);
    if (valid && q == 0) zc[d.n1 + a2] = double(part);
  }
}

// Y[:, j r + c] = U~ D_j Z[:, c] (Algorithm 4, steps 7-8) for j in this
// workgroup's range: the scaled coefficients staged in LDS, the inverse sine
// transform, then E and the V_2 columns.  Z and Y are FP64 in memory; T is
// the arithmetic type.
template <int M, bool ODD, class T>
__global__ __launch_bounds__(kFdWave) void k_fd_backward(FdDev d, const double* __restrict__ Zi, int r,
                                                         double* __restrict__ Y) {
  constexpr int N = 2 * M, RL = FdShape<M>::RL, P = FdShape<M>::P, B = FdShape<M>::B;
  constexpr int SL = FdSlot<M>::SIZE;
  __shared__ Cx<T> sm[B * SL];
  const FdTab<T>& tb = fd_tab<T>(d);
  const Cx<T>* cs = reinterpret_cast<const Cx<T>*>(tb.cs);
  const int lane = threadIdx.x, b = lane / P, q = lane % P;
  // the R_P terms of one column run in consecutive logical workgroups on one
  // XCD (the column is then read from that XCD's L2 after the first)
  const int nj = (d.R + B - 1) / B;
  const int lb = xcd_order(blockIdx.x, gridDim.x);
  const int c = lb / nj, jg = lb - c * nj;
  const int j = jg * B + b;
  const bool valid = j < d.R;
  const double* zc = Zi + (long long)c * d.n;
  const CBuf<T> Z{sm + b * SL};
  const RBuf<T> cv{reinterpret_cast<T*>(sm + b * SL)};
  {
    const auto rg = buf_rsrc(tb.ge, (long long)d.R * d.n), rz = buf_rsrc(zc, d.n);
    const int gb = (valid ? j : 0) * d.n;
    // w_m = ge_m z_m for m < N (for odd p the entry m = n1 = N - 1 is a V_2
    // coefficient the transform never reads)
#pragma unroll
    for (int u = 0; u < 2 * RL; ++u) {
      const int m = q + P * u;
      const bool ok = m < d.n;
      cv[m] = buf_ldt<T>(rg, gb + m, ok) * T(buf_ld(rz, m, ok));
    }
    T w2[kFdMaxV2];
#pragma unroll
    for (int a2 = 0; a2 < kFdMaxV2; ++a2) {
      const bool ok = a2 < d.n2;
      w2[a2] = buf_ldt<T>(rg, gb + d.n1 + a2, ok) * T(buf_ld(rz, d.n1 + a2, ok));
    }
    __syncthreads();
    Cx<T> a[RL];
    if constexpr (ODD) {
      dst1_pre<M>(a, q, tb.sn, [&](int jj) {
        const T x = cv[min(max(jj - 1, 0), N - 2)];
        return (jj >= 1 && jj < N) ? x : T(0);
      });
    } else {
      // inverse of the DST-II steps on S_s = w_{s-1}, the last one doubled
      const Cx<T>* tq = reinterpret_cast<const Cx<T>*>(tb.tq);
#pragma unroll
      for (int t = 0; t < RL; ++t) {
        const int k = q + t * P, km = M - k, k1 = max(k, 1);
        const T sN = cv[N - 1], sa = cv[N - k1 - 1], sb = cv[k1 - 1];
        const Cx<T> qk = k == 0 ? Cx<T>{T(2) * sN, T(0)} : Cx<T>{sa, -sb};
        const Cx<T> qm{cv[N - km - 1], -cv[km - 1]};
        const Cx<T> vk = c_mul(c_conj(tq[k]), qk), vm = c_conj(c_mul(c_conj(tq[km]), qm));
        const Cx<T> e{T(0.5) * (vk.x + vm.x), T(0.5) * (vk.y + vm.y)};
        const Cx<T> o = c_mul(Cx<T>{T(0.5) * (vk.x - vm.x), T(0.5) * (vk.y - vm.y)}, c_conj(cs[k]));
        a[t] = Cx<T>{e.x - o.y, e.y + o.x};  // e + i o
      }
    }
    __syncthreads();  // the staged input is read before the first pass overwrites it
    if constexpr (ODD) {
      fft_passes<M, -1, 1>(a, Z, q, cs);
      dst1_post<M>(Z, cv, q, cs);
    } else {
      fft_passes<M, 1, 1>(a, Z, q, cs);
      // v = the FFT output read as N reals (v_{2i} = Re z_i, v_{2i+1} = Im z_i);
      // T_m = (-1)^m v[m even ? m/2 : N-1-(m-1)/2]
      T tv[2 * RL];
#pragma unroll
      for (int u = 0; u < 2 * RL; ++u) {
        const int m = q + P * u;
        const int i = (m & 1) ? N - 1 - (m >> 1) : (m >> 1);
        const Cx<T> zi = Z[i >> 1];
        const T x = (i & 1) ? zi.y : zi.x;
        tv[u] = (m & 1) ? -x : x;
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 2 * RL; ++u) cv[q + P * u] = tv[u];
      __syncthreads();
    }
    double* yc = Y + ((long long)(valid ? j : 0) * r + c) * d.n;
    auto v2 = [&](int l) {
      T acc = T(0);
#pragma unroll
      for (int a2 = 0; a2 < kFdMaxV2; ++a2)
        if (a2 < d.n2) acc += tb.v2u2[l + (long long)a2 * d.n] * w2[a2];
      return acc;
    };
    // interior rows of E (a shifted copy): at most N = 2 RL P, 2 RL per lane,
    // the loads clamped into range so that they issue together
    if (d.e_hi > d.e_lo) {  // uniform
      // the B output columns of the workgroup (stride r n) through one resource
      const int j0 = jg * B;
      const auto ry = buf_rsrc(Y + ((long long)j0 * r + c) * d.n, ((long long)(B - 1) * r + 1) * d.n);
      const int yb = b * r * d.n;
      T acc[2 * RL];
#pragma unroll
      for (int u = 0; u < 2 * RL; ++u) acc[u] = cv[min(d.e_lo + q + P * u, d.e_hi - 1) + d.e_sh];
#pragma unroll
      for (int a2 = 0; a2 < kFdMaxV2; ++a2) {
        if (a2 < d.n2) {  // uniform
          const auto rv = buf_rsrc(tb.v2u2 + (long long)a2 * d.n, d.n);
#pragma unroll
          for (int u = 0; u < 2 * RL; ++u) acc[u] += buf_ldt<T>(rv, d.e_lo + q + P * u, true) * w2[a2];
        }
      }
#pragma unroll
      for (int u = 0; u < 2 * RL; ++u) {
        const int l = d.e_lo + q + P * u;
        buf_st(ry, yb + l, valid && l < d.e_hi, double(acc[u]));
      }
    }
    // boundary rows [0, e_lo) and [e_hi, n) through the ELL table
    auto ell = [&](int l) {
      T acc = T(0);
      for (int k = 0; k < d.ke; ++k) {
        const int src = d.e_idx[l * d.ke + k];
        if (src >= 0) acc += tb.e_val[l * d.ke + k] * cv[src];
      }
      if (valid) yc[l] = double(acc + v2(l));
    };
    for (int l = q; l < d.e_lo; l += P) ell(l);
    for (int l = d.e_hi + q; l < d.n; l += P) ell(l);
  }
}

// the kernels address a workgroup's columns with 32-bit byte offsets
static void fd_check_span(long long doubles, const char* what) {
  if (doubles * 8 >= (long long)kBufOffHost) throw std::runtime_error(std::string(what) + ": more than 4 GB in one workgroup's reach");
}

template <int M, class T>
static void fd_forward_m(hipStream_t s, const FdDev& d, const double* S, int lds_, int r, double* Z) {
  constexpr int B = FdShape<M>::B;
  fd_check_span((long long)B * lds_ + d.n, "fd_forward");
  const dim3 grid((r + B - 1) / B);
  if (d.odd)
    hipLaunchKernelGGL((k_fd_forward<M, true, T>), grid, dim3(kFdWave), 0, s, d, S, lds_, r, Z);
  else
    hipLaunchKernelGGL((k_fd_forward<M, false, T>), grid, dim3(kFdWave), 0, s, d, S, lds_, r, Z);
}

template <int M, class T>
static void fd_backward_m(hipStream_t s, const FdDev& d, const double* Z, int r, double* Y) {
  constexpr int B = FdShape<M>::B;
  fd_check_span((long long)B * r * d.n + (long long)d.R * d.n, "fd_backward");
  const dim3 grid((unsigned)r * ((d.R + B - 1) / B));
  if (d.odd)
    hipLaunchKernelGGL((k_fd_backward<M, true, T>), grid, dim3(kFdWave), 0, s, d, Z, r, Y);
  else
    hipLaunchKernelGGL((k_fd_backward<M, false, T>), grid, dim3(kFdWave), 0, s, d, Z, r, Y);
}

#define TK_FD_DISPATCH(FN, T, ...)                                         \
  switch (d.N) {                                                           \
    case 4: FN<2, T>(__VA_ARGS__); break;                                  \
    case 8: FN<4, T>(__VA_ARGS__); break;                                  \
    case 16: FN<8, T>(__VA_ARGS__); break;                                 \
    case 32: FN<16, T>(__VA_ARGS__); break;                                \
    case 64: FN<32, T>(__VA_ARGS__); break;                                \
    case 128: FN<64, T>(__VA_ARGS__); break;                               \
    case 256: FN<128, T>(__VA_ARGS__); break;                              \
    case 512: FN<256, T>(__VA_ARGS__); break;                              \
    case 1024: FN<512, T>(__VA_ARGS__); break;                             \
    default: throw std::runtime_error("fd: transform length must be a power of two in [4, 1024]"); \
  }

void fd_forward(hipStream_t s, const FdDev& d, const double* S, int lds_, int r, double* Z, bool f32) {
  if (r <= 0) return;
  if (d.n2 > kFdMaxV2) throw std::runtime_error("fd_forward: more than 4 V_2 columns (degree above 6)");
  if (f32) {
    if (!d.t32.g) throw std::runtime_error("fd_forward: no single-precision tables");
    TK_FD_DISPATCH(fd_forward_m, float, s, d, S, lds_, r, Z);
  } else {
    TK_FD_DISPATCH(fd_forward_m, double, s, d, S, lds_, r, Z);
  }
  check_launch("fd_forward");
}

void fd_backward(hipStream_t s, const FdDev& d, const double* Z, int r, double* Y, bool f32) {
  if (r <= 0 || d.R <= 0) return;
  if (d.n2 > kFdMaxV2) throw std::runtime_error("fd_backward: more than 4 V_2 columns (degree above 6)");
  if (d.R > 65535) throw std::runtime_error("fd_backward: more than 65535 exponential-sum terms");
  if (f32) {
    if (!d.t32.g) throw std::runtime_error("fd_backward: no single-precision tables");
    TK_FD_DISPATCH(fd_backward_m, float, s, d, Z, r, Y);
  } else {
    TK_FD_DISPATCH(fd_backward_m, double, s, d, Z, r, Y);
  }
  check_launch("fd_backward");
}

// ---------------------------------------------------------------------------
// exact-eigenvector FD (Algorithm 4 with the factorizations of Algorithm 3)
// ---------------------------------------------------------------------------

// W[:, j r + c] = E[j, :] .* Z[:, c] for j < R, c < r (n rows); the dense
// products with U before and after are matrix-core GEMMs
__global__ __launch_bounds__(256) void k_fd_exact_scale(int n, int r, int R, const double* __restrict__ E,
                                                        const double* __restrict__ Z, double* __restrict__ W) {
  const long long total = (long long)n * r * R;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < total; e += 256LL * gridDim.x) {
    const int m = (int)(e % n);
    const long long col = e / n;  // j r + c
    const int j = (int)(col / r), c = (int)(col - (long long)j * r);
    W[e] = E[(long long)j * n + m] * Z[(long long)c * n + m];
  }
}

void fd_exact_scale(hipStream_t s, int n, int r, int R, const double* E, const double* Z, double* W) {
  if (n <= 0 || r <= 0 || R <= 0) return;
  const long long total = (long long)n * r * R;
  const int nb = (int)std::min<long long>(4096, (total + 255) / 256);
  hipLaunchKernelGGL(k_fd_exact_scale, dim3(nb), dim3(256), 0, s, n, r, R, E, Z, W);
  check_launch("fd_exact_scale");
}

}  // namespace gpu
}  // namespace tk
