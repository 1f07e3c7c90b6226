// Runtime of the Tucker TPCG library: context, stream-ordered caching
// allocator, lazy Tucker tensors, operator and preconditioner objects,
// relative/dynamic truncation, Tucker scalar products, TPCG, and the C ABI
// declared in include/tk.h.
//
// Paper references: Sec. 2.3 (Tucker format, eq. tt_product, scalar product,
// sums), Sec. 4.1 (Algorithms 1 and 2), Sec. 4.2 (Algorithm 4), Sec. 4.3
// (Algorithm 5, eq. rel_tol_iterates), Sec. 5 (default parameters).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/tk.h"
#include "kernels.h"
#include "tk_internal.h"

namespace tk {

struct Error : std::runtime_error {
  tk_status code;
  Error(tk_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess)                                                              \
      throw ::tk::Error(TK_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_));   \
  } while (0)

// ---------------------------------------------------------------------------
// stream-ordered caching allocator: every kernel of a context runs on one
// stream, so a buffer returned to the cache may be handed out again at once
// (later work on the stream is ordered after earlier uses).
// ---------------------------------------------------------------------------

class Pool {
 public:
  explicit Pool(int dev) : dev_(dev) {}
  ~Pool() { trim(); }
  void* get(size_t bytes) {
    const size_t b = bucket(bytes);
    auto& fl = free_[b];
    if (!fl.empty()) {
      void* p = fl.back();
      fl.pop_back();
      return p;
    }
    void* p = nullptr;
    if (hipMalloc(&p, b) != hipSuccess) {
      (void)hipGetLastError();
      trim();
      if (hipMalloc(&p, b) != hipSuccess) {
        (void)hipGetLastError();
        throw Error(TK_ENOMEM, "device allocation of " + std::to_string(b) + " bytes failed");
      }
    }
    return p;
  }
  void put(void* p, size_t bytes) {
    if (p) free_[bucket(bytes)].push_back(p);
  }
  void trim() {
    for (auto& kv : free_)
      for (void* p : kv.second) (void)hipFree(p);
    free_.clear();
  }

 private:
  static size_t bucket(size_t bytes) {
    size_t b = 256;
    while (b < bytes) b <<= 1;
    return b;
  }
  int dev_;
  std::map<size_t, std::vector<void*>> free_;
};

struct Buf {
  double* p = nullptr;
  size_t bytes = 0;
  Pool* pool = nullptr;
  ~Buf() {
    if (pool) pool->put(p, bytes);
  }
};
using BufP = std::shared_ptr<Buf>;

}  // namespace tk

// ---------------------------------------------------------------------------
// public object types
// ---------------------------------------------------------------------------

namespace tk {
// kernel families timed by the optional HIP-event instrumentation
enum ProfKind { PK_BAND = 0, PK_GEMM, PK_QR, PK_EIG, PK_SELECT, PK_FD_FWD, PK_FD_BWD, PK_MISC, PK_N };
struct ProfRec {
  int kind;
  hipEvent_t a, b;
  double bytes, flops;
};
}  // namespace tk

struct tk_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::unique_ptr<tk::Pool> pool;
  std::string last_error;
  tk::BufP scal;  // device scalars: [0] accumulator + 256 scratch, [300..] misc
  tk::BufP sel;   // rank-selection output (ints)
  double* stage = nullptr;  // pinned host staging for scalar readbacks (kStage doubles)
  // two side streams (default priority) for the speculative ST-HOSVD modes 2
  // and 3, joined to `stream` by events
  hipStream_t side[2] = {nullptr, nullptr};
  hipEvent_t ev_main = nullptr, ev_side[2] = {nullptr, nullptr};
  // instrumentation (off by default)
  bool prof = false;
  std::vector<tk::ProfRec> recs;
  std::vector<hipEvent_t> evpool;
  double p_ms[tk::PK_N] = {}, p_bytes[tk::PK_N] = {}, p_flops[tk::PK_N] = {};
  long long p_n[tk::PK_N] = {};
  long long tail_refinements = 0;  // ST-HOSVD modes whose tail needed a second eigendecomposition
};

namespace tk {

struct Block {
  double c = 1.0;
  BufP core;  // r0 x r1 x r2
  int r[3] = {0, 0, 0};
  int off[3] = {0, 0, 0};
};

}  // namespace tk

struct tk_tucker {
  int n[3] = {0, 0, 0};
  int m[3] = {0, 0, 0};
  tk::BufP U[3];  // n_k x m_k
  std::vector<tk::Block> blocks;
};

struct tk_op {
  int p = 0;
  int n[3] = {0, 0, 0};
  int nmat[3] = {0, 0, 0};
  tk::BufP band[3];
  tk::BufP band_f[3];  // the same bands rounded to FP32 (for FP32 arithmetic)
  std::vector<tk_core_nz> nz;
};

struct tk_prec {
  int R = 0;
  double lam_min = 0, lam_max = 0, err = 0, err_prev = 0;
  std::vector<double> alpha, omega;
  tk::FdDirection dir[3];
  tk::BufP g[3], e_val[3], et_val[3], v2u2[3], ge[3], cs[3], sn[3], tq[3];
  tk::BufP e_idx[3], et_idx[3];  // stored as ints inside double buffers
  tk::BufP f32[3];               // the real tables rounded to FP32, one buffer per direction
  tk::gpu::FdDev dev[3];
  // exact-eigenvector variant (fd_setup_exact): dense M-orthonormal U_k
  // (n_k x n_k) and E_k[j, m] = exp(-alpha_j lam_m / lam_min) (R x n_k)
  bool exact = false;
  int n_exact[3] = {0, 0, 0};
  std::vector<double> lam_exact[3];
  tk::BufP Ud[3], Ed[3];
};

namespace tk {

static BufP alloc(tk_ctx* ctx, size_t count) {
  auto b = std::make_shared<Buf>();
  b->bytes = std::max<size_t>(count, 1) * sizeof(double);
  b->p = static_cast<double*>(ctx->pool->get(b->bytes));
  b->pool = ctx->pool.get();
  return b;
}

static void sync(tk_ctx* ctx) { HIPCHK(hipStreamSynchronize(ctx->stream)); }

static void d2d(tk_ctx* ctx, double* dst, const double* src, size_t count) {
  if (count) HIPCHK(hipMemcpyAsync(dst, src, count * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
}

static void h2d(tk_ctx* ctx, double* dst, const double* src, size_t count) {
  if (count) {
    HIPCHK(hipMemcpyAsync(dst, src, count * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    sync(ctx);  // host memory may be released by the caller after return
  }
}

constexpr size_t kStage = 64;  // doubles of pinned staging per context

// Device -> host copy that synchronises; small reads go through the
// context's pinned staging buffer (one DMA, no pageable-memory staging).
static std::vector<double> d2h(tk_ctx* ctx, const double* src, size_t count) {
  std::vector<double> out(count);
  if (count) {
    double* dst = (count <= kStage && ctx->stage) ? ctx->stage : out.data();
    HIPCHK(hipMemcpyAsync(dst, src, count * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    sync(ctx);
    if (dst != out.data()) std::memcpy(out.data(), dst, count * sizeof(double));
  }
  return out;
}

static long long prod3(const int r[3]) { return (long long)r[0] * r[1] * r[2]; }

// ---------------------------------------------------------------------------
// instrumentation: events around launches of one kernel family
// ---------------------------------------------------------------------------

static hipEvent_t get_event(tk_ctx* ctx) {
  if (!ctx->evpool.empty()) {
    hipEvent_t e = ctx->evpool.back();
    ctx->evpool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIPCHK(hipEventCreate(&e));
  return e;
}

static void prof_flush(tk_ctx* ctx) {
  for (auto& r : ctx->recs) {
    HIPCHK(hipEventSynchronize(r.b));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
    ctx->p_ms[r.kind] += ms;
    ctx->p_bytes[r.kind] += r.bytes;
    ctx->p_flops[r.kind] += r.flops;
    ctx->p_n[r.kind] += 1;
    ctx->evpool.push_back(r.a);
    ctx->evpool.push_back(r.b);
  }
  ctx->recs.clear();
}

struct Prof {
  tk_ctx* ctx;
  ProfRec r{};
  Prof(tk_ctx* c, int kind, double bytes, double flops) : ctx(c) {
    if (!ctx->prof) return;
    r.kind = kind;
    r.bytes = bytes;
    r.flops = flops;
    r.a = get_event(ctx);
    r.b = get_event(ctx);
    HIPCHK(hipEventRecord(r.a, ctx->stream));
  }
  ~Prof() {
    if (!ctx->prof) return;
    if (hipEventRecord(r.b, ctx->stream) != hipSuccess) {
      ctx->evpool.push_back(r.a);
      ctx->evpool.push_back(r.b);
      return;
    }
    ctx->recs.push_back(r);
    if (ctx->recs.size() > 8192) {
      try {
        prof_flush(ctx);
      } catch (...) {
      }
    }
  }
};

// Dense flops of one symmetric eigendecomposition of order a: Householder
// tridiagonalisation (4/3 a^3), two Gram-Schmidt passes (2 a^3 each) and the
// back transformation (2 a^3); bisection and inverse iteration are O(a^2).
static double eig_flops(int a) {
  const double x = a;
  return (4.0 / 3.0 + 4.0 + 2.0) * x * x * x;
}

static void gemm(tk_ctx* ctx, bool ta, bool tb, int M, int N, int K, double alpha, const double* A, int lda,
                 const double* B, int ldb, double beta, double* C, int ldc) {
  Prof pr(ctx, PK_GEMM, 8.0 * ((double)M * K + (double)K * N + (double)M * N * (beta != 0.0 ? 2 : 1)),
          2.0 * M * N * (double)K);
  const int ns = gpu::dgemm_split_count(M, N, K);
  BufP part;
  if (ns > 1) part = alloc(ctx, (size_t)ns * M * N);
  gpu::dgemm(ctx->stream, ta, tb, M, N, K, alpha, A, lda, 0, B, ldb, 0, beta, C, ldc, 0, 1,
             part ? part->p : nullptr, ns);
}

// batched C_i = alpha op(A_i) op(B_i) + beta C_i with element strides
static void gemm_batched(tk_ctx* ctx, bool ta, bool tb, int M, int N, int K, double alpha, const double* A,
                         int lda, long long sA, const double* B, int ldb, long long sB, double beta, double* C,
                         int ldc, long long sC, int batch) {
  Prof pr(ctx, PK_GEMM,
          8.0 * batch * ((double)M * K + (double)K * N + (double)M * N * (beta != 0.0 ? 2 : 1)),
          2.0 * batch * M * N * (double)K);
  gpu::dgemm(ctx->stream, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, nullptr, 1);
}

// ---------------------------------------------------------------------------
// Tucker objects
// ---------------------------------------------------------------------------

static tk_tucker* make_plain(tk_ctx* ctx, const int n[3], const int r[3]) {
  auto* t = new tk_tucker;
  for (int k = 0; k < 3; ++k) {
    t->n[k] = n[k];
    t->m[k] = r[k];
    t->U[k] = alloc(ctx, (size_t)n[k] * r[k]);
  }
  Block b;
  b.core = alloc(ctx, (size_t)prod3(r));
  for (int k = 0; k < 3; ++k) b.r[k] = r[k];
  t->blocks.push_back(b);
  return t;
}

// lazy a*x + b*y: concatenated factors, blocks shifted (Sec. 2.3 sum)
static tk_tucker* lin_comb(tk_ctx* ctx, double a, const tk_tucker* x, double b, const tk_tucker* y) {
  for (int k = 0; k < 3; ++k)
    if (x->n[k] != y->n[k]) throw Error(TK_EINVAL, "sum of Tucker tensors of different sizes");
  auto* t = new tk_tucker;
  gpu::CopySegs cs;  // the six factor copies of the concatenation, one launch
  for (int k = 0; k < 3; ++k) {
    t->n[k] = x->n[k];
    t->m[k] = x->m[k] + y->m[k];
    t->U[k] = alloc(ctx, (size_t)t->n[k] * t->m[k]);
    const long long nx = (long long)x->n[k] * x->m[k], ny = (long long)y->n[k] * y->m[k];
    if (nx) cs.s[cs.n++] = gpu::CopySeg{t->U[k]->p, x->U[k]->p, nx};
    if (ny) cs.s[cs.n++] = gpu::CopySeg{t->U[k]->p + nx, y->U[k]->p, ny};
  }
  gpu::copy_segments(ctx->stream, cs);
  for (const auto& bl : x->blocks) {
    Block c = bl;
    c.c *= a;
    t->blocks.push_back(c);
  }
  for (const auto& bl : y->blocks) {
    Block c = bl;
    c.c *= b;
    for (int k = 0; k < 3; ++k) c.off[k] += x->m[k];
    t->blocks.push_back(c);
  }
  return t;
}

// ---------------------------------------------------------------------------
// scalar products (Sec. 2.3): <X, Y> = vec(Gx)^T vec(Gy x_1 W1 x_2 W2 x_3 W3),
// W_k = X_k^T Y_k; lazy sums are expanded over pairs of blocks.
// ---------------------------------------------------------------------------

// T (r0 x r1 x r2 tensor, ld as matrix r0 x r1r2) x_1 M0 x_2 M1 x_3 M2 by three
// GEMMs that each contract the leading mode and rotate it to the back:
// (a x bc) -> (bc x a') = T^T M^T.  M_k is s_k x r_k with leading dim ldm[k].
static BufP multi_mode_product(tk_ctx* ctx, const double* T, const int r[3], const double* const M[3],
                               const int s[3], const int ldm[3]) {
  int dims[3] = {r[0], r[1], r[2]};
  const double* cur = T;
  BufP hold;
  for (int k = 0; k < 3; ++k) {
    const int a = dims[0], bc = dims[1] * dims[2];
    BufP out = alloc(ctx, (size_t)bc * s[k]);
    gemm(ctx, true, true, bc, s[k], a, 1.0, cur, a, M[k], ldm[k], 0.0, out->p, bc);
    hold = out;
    cur = out->p;
    dims[0] = dims[1];
    dims[1] = dims[2];
    dims[2] = s[k];
  }
  return hold;  // s0 x s1 x s2
}

static double dot(tk_ctx* ctx, const tk_tucker* x, const tk_tucker* y) {
  for (int k = 0; k < 3; ++k)
    if (x->n[k] != y->n[k]) throw Error(TK_EINVAL, "dot of Tucker tensors of different sizes");
  double* acc = ctx->scal->p;
  gpu::fill(ctx->stream, acc, 1, 0.0);
  bool any = false;
  BufP W[3];
  for (int k = 0; k < 3; ++k) {
    if (x->m[k] == 0 || y->m[k] == 0) return 0.0;
    W[k] = alloc(ctx, (size_t)x->m[k] * y->m[k]);  // m_x x m_y
    gemm(ctx, true, false, x->m[k], y->m[k], x->n[k], 1.0, x->U[k]->p, x->n[k], y->U[k]->p, y->n[k], 0.0, W[k]->p, x->m[k]);
  }
  for (const auto& bx : x->blocks)
    for (const auto& by : y->blocks) {
      if (prod3(bx.r) == 0 || prod3(by.r) == 0) continue;
      const double* M[3];
      int ldm[3];
      for (int k = 0; k < 3; ++k) {
        M[k] = W[k]->p + bx.off[k] + (size_t)by.off[k] * x->m[k];
        ldm[k] = x->m[k];
      }
      BufP T = multi_mode_product(ctx, by.core->p, by.r, M, bx.r, ldm);
      gpu::dot_accumulate(ctx->stream, bx.core->p, T->p, prod3(bx.r), bx.c * by.c, acc);
      any = true;
    }
  if (!any) return 0.0;
  auto h = d2h(ctx, acc, 1);
  return h[0];
}

// ---------------------------------------------------------------------------
// Algorithm 1 (relative truncation), steps 1-2 kept for reuse by Algorithm 2
// ---------------------------------------------------------------------------

struct TruncPrep {
  int n[3];
  int q[3];         // rows of R_k = columns of Q_k
  bool ident[3];    // Q_k = I (when m_k >= n_k, R_k = Y_k)
  BufP Q[3];        // n_k x q_k (unless ident)
  BufP Z;           // q0 x q1 x q2
  double norm2 = 0; // ||Z||^2 (set by the first ST-HOSVD mode)
  // the first ST-HOSVD mode depends on Z only: its eigenvectors, projection
  // and energies are kept for the retries of Algorithm 2 on the same tensor
  BufP V0, Pm0, part0;
  // speculative eigenvectors of the Gram matrices of modes 2 and 3 of Z
  // (computed on the side streams; exact for the sequential ST-HOSVD when the
  // earlier modes keep every direction, since an orthogonal rotation in one
  // mode leaves the Gram matrices of the others unchanged, and used as the
  // bases of those modes after a truncation too when the caller asks for it)
  bool spec = false;
  BufP Vs[2];
  std::vector<BufP> spec_keep;
  tk_ctx* spec_ctx = nullptr;  // set once side work is enqueued
  // on every exit (errors included) the main stream waits for the side work
  // before the buffers above go back to the pool
  ~TruncPrep() {
    if (!spec_ctx) return;
    for (int i = 0; i < 2; ++i)
      if (Vs[i]) (void)hipStreamWaitEvent(spec_ctx->stream, spec_ctx->ev_side[i], 0);
  }
};

static TruncPrep truncate_prepare(tk_ctx* ctx, const tk_tucker* y) {
  TruncPrep P;
  BufP R[3];
  gpu::QrJob jobs[3];
  int nj = 0;
  std::vector<BufP> keep;
  for (int k = 0; k < 3; ++k) {
    P.n[k] = y->n[k];
    const int n = y->n[k], m = y->m[k];
    if (m >= n) {
      P.ident[k] = true;
      P.q[k] = n;
      R[k] = y->U[k];  // R_k = Y_k (n x m)
    } else {
      P.ident[k] = false;
      P.q[k] = m;
      BufP A = alloc(ctx, (size_t)n * m);
      d2d(ctx, A->p, y->U[k]->p, (size_t)n * m);
      R[k] = alloc(ctx, (size_t)m * m);
      P.Q[k] = alloc(ctx, (size_t)n * m);
      BufP tau = alloc(ctx, (size_t)m);
      keep.push_back(A);
      keep.push_back(tau);
      if (m > 0) jobs[nj++] = gpu::QrJob{A->p, R[k]->p, P.Q[k]->p, tau->p, n, m};
    }
  }
  {
    double fl = 0.0, by = 0.0;
    for (int i = 0; i < nj; ++i) {
      const double n = jobs[i].n, m = jobs[i].m;
      fl += 2.0 * (2.0 * n * m * m - 2.0 * m * m * m / 3.0);  // factorization + explicit Q
      by += 8.0 * (2.0 * n * m + m * m);
    }
    Prof pr(ctx, PK_QR, by, fl);
    gpu::householder_qr(ctx->stream, jobs, nj);
  }
  // Z = sum_b c_b G_b x_1 R_1[:, b] x_2 R_2[:, b] x_3 R_3[:, b], as one
  // contraction over the stacked mode-1 rank: every block writes
  // W_b = c_b G_b x_2 R_2[:, b] x_3 R_3[:, b] (r1_b x q1 q2, mode-1 unfolding)
  // into rows off1_b.. of W (m1 x q1 q2), then Z_(1) = R_1 W.
  const long long zsz = (long long)P.q[0] * P.q[1] * P.q[2];
  P.Z = alloc(ctx, (size_t)std::max<long long>(zsz, 1));
  const int m1 = y->m[0];
  const long long q12 = (long long)P.q[1] * P.q[2];
  if (zsz == 0) return P;
  if (m1 == 0) {
    gpu::fill(ctx->stream, P.Z->p, zsz, 0.0);
    return P;
  }
  // blocks whose mode-1 column ranges tile [0, m1) exactly can be written
  // with beta = 0; otherwise W starts at zero and blocks accumulate
  std::vector<std::pair<int, int>> ranges;
  for (const auto& b : y->blocks)
    if (prod3(b.r) > 0) ranges.push_back({b.off[0], b.r[0]});
  std::sort(ranges.begin(), ranges.end());
  bool tiles = true;
  int next = 0;
  for (const auto& rg : ranges) {
    if (rg.first != next) tiles = false;
    next = rg.first + rg.second;
  }
  if (next != m1) tiles = false;
  BufP W = alloc(ctx, (size_t)m1 * q12);
  if (!tiles) gpu::fill(ctx->stream, W->p, (long long)m1 * q12, 0.0);
  for (const auto& b : y->blocks) {
    if (prod3(b.r) == 0) continue;
    const int r1 = b.r[0], r2 = b.r[1], r3 = b.r[2];
    const double* R2 = R[1]->p + (size_t)b.off[1] * P.q[1];
    const double* R3 = R[2]->p + (size_t)b.off[2] * P.q[2];
    // T = G_b x_3 R_3[:, b]: (r1 r2 x r3) (q2 x r3)^T
    BufP T = alloc(ctx, (size_t)r1 * r2 * P.q[2]);
    gemm(ctx, false, true, r1 * r2, P.q[2], r3, 1.0, b.core->p, r1 * r2, R3, P.q[2], 0.0, T->p, r1 * r2);
    // W_b[:, :, i2] = c_b T[:, :, i2] R_2[:, b]^T for every i2
    gemm_batched(ctx, false, true, r1, P.q[1], r2, b.c, T->p, r1, (long long)r1 * r2, R2, P.q[1], 0,
                 tiles ? 0.0 : 1.0, W->p + b.off[0], m1, (long long)m1 * P.q[1], P.q[2]);
  }
  gemm(ctx, false, false, P.q[0], (int)q12, m1, 1.0, R[0]->p, P.q[0], W->p, m1, 0.0, P.Z->p, P.q[0]);
  return P;
}

// Steps 3-4: ST-HOSVD of Z with tolerance eps, factors Q_k S_k.
// Modes 2 and 3 of Z on the side streams: G_2 = sum_c Z_c^T Z_c (Z_c the
// q0 x q1 slices), G_3 = Z^T Z with Z viewed as (q0 q1) x q2, and their
// eigenvectors.  The side streams start after everything enqueued on the
// main stream so far (so no pool buffer they receive is still in use there);
// the main stream waits for them before it uses the results and before the
// truncation returns (so their buffers go back to the pool in stream order).
constexpr int kSpecMax = 256;
static void spec_launch(tk_ctx* ctx, TruncPrep& P) {
  if (P.spec) return;
  P.spec = true;
  const int q0 = P.q[0], q1 = P.q[1], q2 = P.q[2];
  if (q0 < 2 || q1 < 2 || q2 < 2 || q1 > kSpecMax || q2 > kSpecMax) return;
  HIPCHK(hipEventRecord(ctx->ev_main, ctx->stream));
  P.spec_ctx = ctx;
  const double* Z = P.Z->p;
  const int a[2] = {q1, q2};
  for (int i = 0; i < 2; ++i) {
    hipStream_t s = ctx->side[i];
    HIPCHK(hipStreamWaitEvent(s, ctx->ev_main, 0));
    const int n = a[i];
    BufP G = alloc(ctx, (size_t)n * n), w = alloc(ctx, (size_t)n), work = alloc(ctx, gpu::sym_eig_work(n));
    P.Vs[i] = alloc(ctx, (size_t)n * n);
    P.spec_keep.insert(P.spec_keep.end(), {G, w, work});
    if (i == 0) {
      BufP part = alloc(ctx, (size_t)q2 * q1 * q1);
      P.spec_keep.push_back(part);
      gpu::dgemm(s, true, false, q1, q1, q0, 1.0, Z, q0, (long long)q0 * q1, Z, q0, (long long)q0 * q1, 0.0,
                 part->p, q1, (long long)q1 * q1, q2);
      gpu::splitk_reduce(s, q1, q1, q2, part->p, 0.0, G->p, q1);
    } else {
      const int K = q0 * q1;
      const int ns = gpu::dgemm_split_count(q2, q2, K);
      BufP part;
      if (ns > 1) {
        part = alloc(ctx, (size_t)ns * q2 * q2);
        P.spec_keep.push_back(part);
      }
      gpu::dgemm(s, true, false, q2, q2, K, 1.0, Z, K, 0, Z, K, 0, 0.0, G->p, q2, 0, 1, part ? part->p : nullptr, ns);
    }
    gpu::sym_eig(s, G->p, n, P.Vs[i]->p, w->p, work->p);
    HIPCHK(hipEventRecord(ctx->ev_side[i], s));
  }
}

static void spec_join(tk_ctx* ctx, const TruncPrep& P, int i) {
  if (P.Vs[i]) HIPCHK(hipStreamWaitEvent(ctx->stream, ctx->ev_side[i], 0));
}

// Second level of one ST-HOSVD mode's eigendecomposition.  The Gram matrix
// G = A A^T of the mode unfolding A (a x bc) carries rounding errors of about
// a eps_mach ||A||^2, so its eigenvectors are reliable only for energies
// well above that (the k1 leading columns of V in the order sel[1..a]); the
// other a - k1 eigenvectors V_r are orthonormal and orthogonal to them but
// mix the small singular directions among themselves.  Their coordinates
// M = V_r^T A are the columns P_r of Pm = A^T V already at hand, whose Gram
// H = P_r^T P_r ((a - k1) x (a - k1)) resolves the tail relative to its own
// norm; with H = Y diag(mu) Y^T the refined basis is [V_k1, V_r Y] and the
// mode coordinates [P_k1, P_r Y].  V (a x a) and Pm (bc x a) are replaced.
// Returns how many leading refined directions are themselves resolved (the
// same test as the rank selection's, on the eigenvalues mu of H).
static int refine_tail(tk_ctx* ctx, int a, int bc, int k1, const int* sel, double budget, BufP& V, BufP& Pm) {
  const int m = a - k1;
  const int* order = sel + 1;  // device: columns in descending energy order
  BufP Vn = alloc(ctx, (size_t)a * a), Pn = alloc(ctx, (size_t)bc * a);
  BufP Vr = alloc(ctx, (size_t)a * m), Pr = alloc(ctx, (size_t)bc * m);
  {
    Prof pr(ctx, PK_SELECT, 16.0 * ((double)a * a + (double)bc * a), 0.0);
    gpu::gather_columns(ctx->stream, V->p, a, order, k1, Vn->p);
    gpu::gather_columns(ctx->stream, Pm->p, bc, order, k1, Pn->p);
    gpu::gather_columns(ctx->stream, V->p, a, order + k1, m, Vr->p);
    gpu::gather_columns(ctx->stream, Pm->p, bc, order + k1, m, Pr->p);
  }
  BufP H = alloc(ctx, (size_t)m * m), Y = alloc(ctx, (size_t)m * m), mu = alloc(ctx, (size_t)m);
  gemm(ctx, true, false, m, m, bc, 1.0, Pr->p, bc, Pr->p, bc, 0.0, H->p, m);
  {
    BufP work = alloc(ctx, gpu::sym_eig_work(m));
    Prof pr(ctx, PK_EIG, 8.0 * 2.0 * m * (double)m, eig_flops(m));
    gpu::sym_eig(ctx->stream, H->p, m, Y->p, mu->p, work->p);
  }
  gemm(ctx, false, false, a, m, m, 1.0, Vr->p, a, Y->p, m, 0.0, Vn->p + (size_t)a * k1, a);
  gemm(ctx, false, false, bc, m, m, 1.0, Pr->p, bc, Y->p, m, 0.0, Pn->p + (size_t)bc * k1, bc);
  V = Vn;
  Pm = Pn;
  const auto hmu = d2h(ctx, mu->p, (size_t)m);  // descending
  double sum = 0.0;
  for (double v : hmu) sum += std::max(v, 0.0);
  const double um = m * 2.220446049250313e-16, top = std::max(hmu[0], 0.0);
  const double thr = budget > 0.0 ? std::max(64.0 * um * sum, 10.0 * (um * top) * (um * top) / budget) : 2.0 * top + 1.0;
  int k_add = 0;
  while (k_add < m && hmu[k_add] >= thr) ++k_add;
  return k_add;
}

// With spec_any, modes 2 and 3 take the eigenvectors of the untruncated
// core's Gram matrices (computed on the side streams while mode 1 runs) even
// after an earlier mode was truncated; the energies are still measured on the
// sequentially truncated core, so ||y - T(y)|| <= eps ||y|| holds exactly,
// and the ranks can only exceed those of the exact ST-HOSVD (Ky Fan) in
// borderline cases.  Without it such modes take a fresh Gram matrix.
static tk_tucker* truncate_finish(tk_ctx* ctx, TruncPrep& P, double eps, double* disc_rel, bool refine = true,
                                  bool spec_any = false) {
  int dims[3] = {P.q[0], P.q[1], P.q[2]};
  BufP cur = P.Z;
  BufP S[3];
  int s_k[3] = {0, 0, 0};
  double disc_total = 0.0;
  double* norm2 = ctx->scal->p + 300;
  double* disc = ctx->scal->p + 301;
  const long long zsz = (long long)dims[0] * dims[1] * dims[2];
  bool zero = (zsz == 0);
  for (int k = 0; k < 3 && !zero; ++k) {
    const int a = dims[0], bc = dims[1] * dims[2];
    const int nseg = gpu::column_energy_parts(bc);
    BufP V, Pm, part;
    if (k == 0) spec_launch(ctx, P);
    // the speculative eigenvectors are the exact ST-HOSVD bases when every earlier
    // mode kept all its directions; with spec_any they serve in any case
    const bool use_spec =
        k > 0 && P.Vs[k - 1] && (spec_any || (s_k[0] == P.q[0] && (k == 1 || s_k[1] == P.q[1])));
    if (k == 0 && P.V0) {
      V = P.V0;
      Pm = P.Pm0;
      part = P.part0;
    } else if (use_spec) {
      spec_join(ctx, P, k - 1);
      V = P.Vs[k - 1];
      Pm = alloc(ctx, (size_t)bc * a);
      gemm(ctx, true, false, bc, a, a, 1.0, cur->p, a, V->p, a, 0.0, Pm->p, bc);
      part = alloc(ctx, (size_t)a * nseg);
      {
        Prof pr(ctx, PK_SELECT, 8.0 * bc * (double)a, 2.0 * bc * (double)a);
        gpu::column_energy(ctx->stream, Pm->p, bc, a, part->p);
      }
    } else {
      // Gram of the mode-k unfolding (the current leading mode)
      BufP G = alloc(ctx, (size_t)a * a);
      gemm(ctx, false, true, a, a, bc, 1.0, cur->p, a, cur->p, a, 0.0, G->p, a);
      V = alloc(ctx, (size_t)a * a);
      BufP w = alloc(ctx, (size_t)a);
      {
        BufP work = alloc(ctx, gpu::sym_eig_work(a));
        Prof pr(ctx, PK_EIG, 8.0 * 2.0 * a * (double)a, eig_flops(a));
        gpu::sym_eig(ctx->stream, G->p, a, V->p, w->p, work->p);
      }
      // P = A^T V (bc x a): columns are the mode-k coordinates in the eigenbasis
      Pm = alloc(ctx, (size_t)bc * a);
      gemm(ctx, true, false, bc, a, a, 1.0, cur->p, a, V->p, a, 0.0, Pm->p, bc);
      part = alloc(ctx, (size_t)a * nseg);
      {
        Prof pr(ctx, PK_SELECT, 8.0 * bc * (double)a, 2.0 * bc * (double)a);
        gpu::column_energy(ctx->stream, Pm->p, bc, a, part->p);
      }
      if (k == 0) {
        P.V0 = V;
        P.Pm0 = Pm;
        P.part0 = part;
      }
    }
    int* sel = reinterpret_cast<int*>(ctx->sel->p);
    {
      Prof pr(ctx, PK_SELECT, 8.0 * a * (double)nseg, 0.0);
      gpu::select_rank(ctx->stream, part->p, nseg, a, eps, norm2, k == 0 ? 1 : 0, sel, disc);
    }
    // one readback of [norm2, tail, s, k1, mode energy] (scal + 300 .. 304)
    auto hv = d2h(ctx, norm2, 5);
    // kept directions that the Gram matrix does not resolve have energies
    // smeared by rounding, which can keep up to all a of them: refine the
    // unresolved tail (up to three levels) while the cut lies inside it
    int k_res = (int)hv[3];
    for (int level = 0; refine && level < 3 && (int)hv[2] > k_res && k_res >= 1 && k_res < a; ++level) {
      const double budget = eps * eps * hv[0] / 3.0;
      const int k_add = refine_tail(ctx, a, bc, k_res, sel, budget, V, Pm);
      part = alloc(ctx, (size_t)a * nseg);
      {
        Prof pr(ctx, PK_SELECT, 8.0 * bc * (double)a + 8.0 * a * (double)nseg, 2.0 * bc * (double)a);
        gpu::column_energy(ctx->stream, Pm->p, bc, a, part->p);
        gpu::select_rank(ctx->stream, part->p, nseg, a, eps, norm2, 0, sel, disc);
      }
      hv = d2h(ctx, norm2, 5);
      k_res += std::max(k_add, 1);
      ++ctx->tail_refinements;
    }
    if (k == 0) P.norm2 = hv[0];
    const double hdisc = hv[1];
    const int hsel = (int)hv[2];
    disc_total += hdisc;
    const int s = hsel;
    s_k[k] = s;
    if (s == 0) {
      zero = true;
      break;
    }
    S[k] = alloc(ctx, (size_t)a * s);
    BufP next = alloc(ctx, (size_t)bc * s);  // rotated core (b, c, s)
    {
      Prof pr(ctx, PK_SELECT, 16.0 * ((double)a * s + (double)bc * s), 0.0);
      gpu::gather_columns(ctx->stream, V->p, a, sel + 1, s, S[k]->p);
      gpu::gather_columns(ctx->stream, Pm->p, bc, sel + 1, s, next->p);
    }
    cur = next;
    dims[0] = dims[1];
    dims[1] = dims[2];
    dims[2] = s;
  }
  // the side streams' buffers may return to the pool only after the main stream has waited for them
  spec_join(ctx, P, 0);
  spec_join(ctx, P, 1);
  if (disc_rel) *disc_rel = (P.norm2 > 0) ? disc_total / P.norm2 : 0.0;
  int n[3] = {P.n[0], P.n[1], P.n[2]};
  if (zero) {
    int r0[3] = {0, 0, 0};
    return make_plain(ctx, n, r0);
  }
  auto* t = new tk_tucker;
  for (int k = 0; k < 3; ++k) {
    t->n[k] = n[k];
    t->m[k] = s_k[k];
    if (P.ident[k]) {
      t->U[k] = S[k];  // Q = I: the factor is S_k (n x s)
    } else {
      t->U[k] = alloc(ctx, (size_t)n[k] * s_k[k]);
      gemm(ctx, false, false, n[k], s_k[k], P.q[k], 1.0, P.Q[k]->p, n[k], S[k]->p, P.q[k], 0.0, t->U[k]->p, n[k]);
    }
  }
  Block b;
  b.core = cur;
  for (int k = 0; k < 3; ++k) b.r[k] = s_k[k];
  t->blocks.push_back(b);
  return t;
}

static tk_tucker* truncate(tk_ctx* ctx, const tk_tucker* y, double eps, double* disc, bool refine = true,
                           bool spec_any = false) {
  TruncPrep P = truncate_prepare(ctx, y);
  return truncate_finish(ctx, P, eps, disc, refine, spec_any);
}

static double core_norm(tk_ctx* ctx, const tk_tucker* t) {
  // plain tensor with orthonormal factors: ||t|| = ||core||_F
  const auto& b = t->blocks[0];
  if (prod3(b.r) == 0) return 0.0;
  double* acc = ctx->scal->p;
  gpu::fill(ctx->stream, acc, 1, 0.0);
  gpu::dot_accumulate(ctx->stream, b.core->p, b.core->p, prod3(b.r), 1.0, acc);
  auto h = d2h(ctx, acc, 1);
  return std::sqrt(std::max(h[0], 0.0)) * std::fabs(b.c);
}

// ---------------------------------------------------------------------------
// operator application (eq. tt_product)
// ---------------------------------------------------------------------------

static tk_tucker* apply_op(tk_ctx* ctx, const tk_op* op, const tk_tucker* x, bool f32 = false) {
  for (int k = 0; k < 3; ++k)
    if (x->n[k] != op->n[k]) throw Error(TK_EINVAL, "operator and tensor sizes differ");
  auto* t = new tk_tucker;
  for (int k = 0; k < 3; ++k) {
    t->n[k] = x->n[k];
    t->m[k] = op->nmat[k] * x->m[k];
    t->U[k] = alloc(ctx, (size_t)t->n[k] * t->m[k]);
    const double nn = x->n[k], mm = x->m[k], R = op->nmat[k], nb = 2 * op->p + 1;
    Prof pr(ctx, PK_BAND, 8.0 * (nn * mm + R * nb * nn + R * nn * mm), 2.0 * R * nb * nn * mm);
    gpu::band_apply(ctx->stream, x->n[k], x->m[k], op->nmat[k], op->p, op->band[k]->p,
                    f32 ? reinterpret_cast<const float*>(op->band_f[k]->p) : nullptr, x->U[k]->p, x->n[k],
                    t->U[k]->p, t->n[k]);
  }
  for (const auto& z : op->nz)
    for (const auto& b : x->blocks) {
      Block c = b;
      c.c = b.c * z.c;
      c.off[0] = z.i1 * x->m[0] + b.off[0];
      c.off[1] = z.i2 * x->m[1] + b.off[1];
      c.off[2] = z.i3 * x->m[2] + b.off[2];
      t->blocks.push_back(c);
    }
  return t;
}

// ---------------------------------------------------------------------------
// low-rank FD application (Algorithm 4, steps 5-9)
// ---------------------------------------------------------------------------

// f32: FP32 arithmetic in the transforms (the exact-eigenvector variant
// always runs in FP64)
static tk_tucker* apply_prec(tk_ctx* ctx, const tk_prec* P, const tk_tucker* s, bool f32 = false) {
  if (s->blocks.size() != 1) throw Error(TK_EINVAL, "fd_precond expects a plain (truncated) Tucker tensor");
  for (int k = 0; k < 3; ++k)
    if (s->n[k] != (P->exact ? P->n_exact[k] : P->dir[k].n))
      throw Error(TK_EINVAL, "preconditioner and tensor sizes differ");
  auto* t = new tk_tucker;
  const Block& sb = s->blocks[0];
  if (P->exact) {
    // Y_(k,j) = U_k D_(k,j) U_k^T S_k: Z = U^T S, W = [D_j Z]_j, Y = U W
    for (int k = 0; k < 3; ++k) {
      const int n = s->n[k], r = s->m[k];
      t->n[k] = n;
      t->m[k] = P->R * r;
      t->U[k] = alloc(ctx, (size_t)n * t->m[k]);
      if (r == 0) continue;
      BufP Z = alloc(ctx, (size_t)n * r), W = alloc(ctx, (size_t)n * t->m[k]);
      gemm(ctx, true, false, n, r, n, 1.0, P->Ud[k]->p, n, s->U[k]->p, n, 0.0, Z->p, n);
      {
        Prof pr(ctx, PK_FD_BWD, 8.0 * ((double)n * r + (double)P->R * n + (double)P->R * n * r),
                (double)P->R * n * r);
        gpu::fd_exact_scale(ctx->stream, n, r, P->R, P->Ed[k]->p, Z->p, W->p);
      }
      gemm(ctx, false, false, n, t->m[k], n, 1.0, P->Ud[k]->p, n, W->p, n, 0.0, t->U[k]->p, n);
    }
    for (int j = 0; j < P->R; ++j) {
      Block c = sb;
      c.c = sb.c * P->omega[j] / P->lam_min;
      for (int k = 0; k < 3; ++k) c.off[k] = j * s->m[k] + sb.off[k];
      t->blocks.push_back(c);
    }
    return t;
  }
  for (int k = 0; k < 3; ++k) {
    const int n = s->n[k], r = s->m[k];
    t->n[k] = n;
    t->m[k] = P->R * r;
    t->U[k] = alloc(ctx, (size_t)n * t->m[k]);
    if (r == 0) continue;
    BufP Z = alloc(ctx, (size_t)n * r);
    const auto& d = P->dev[k];
    // one complex FFT of length N/2 per transform plus O(N) pre- and post-processing
    const double M = 0.5 * d.N, fft = 5.0 * M * std::log2(std::max(M, 2.0)) + 12.0 * d.N;
    {
      // algorithmic bytes: read S, write Z, boundary map and V2U2 columns
      Prof pr(ctx, PK_FD_FWD, 8.0 * (2.0 * n * r + (double)n * d.n2), r * (fft + 2.0 * n * (1 + d.n2)));
      gpu::fd_forward(ctx->stream, d, s->U[k]->p, n, r, Z->p, f32);
    }
    {
      // read Z and the exp table, write R_P r columns
      Prof pr(ctx, PK_FD_BWD, 8.0 * ((double)n * r + (double)P->R * n + (double)P->R * n * r + (double)n * d.n2),
              (double)P->R * r * (fft + n * (1.0 + 2.0 * d.n2)));
      gpu::fd_backward(ctx->stream, d, Z->p, r, t->U[k]->p, f32);
    }
  }
  for (int j = 0; j < P->R; ++j) {
    Block c = sb;
    c.c = sb.c * P->omega[j] / P->lam_min;
    for (int k = 0; k < 3; ++k) c.off[k] = j * s->m[k] + sb.off[k];
    t->blocks.push_back(c);
  }
  return t;
}

// ---------------------------------------------------------------------------
// TPCG (Algorithm 5) with dynamic truncation of the iterate (Algorithm 2)
// ---------------------------------------------------------------------------

struct Owned {
  tk_tucker* t = nullptr;
  Owned() = default;
  explicit Owned(tk_tucker* x) : t(x) {}
  Owned(const Owned&) = delete;
  Owned& operator=(const Owned&) = delete;
  Owned(Owned&& o) noexcept : t(o.t) { o.t = nullptr; }
  Owned& operator=(Owned&& o) noexcept {
    if (this != &o) { delete t; t = o.t; o.t = nullptr; }
    return *this;
  }
  ~Owned() { delete t; }
  tk_tucker* release() { tk_tucker* x = t; t = nullptr; return x; }
};

static tk_tucker* scaled_copy(tk_ctx* ctx, const tk_tucker* x, double a) {
  auto* t = new tk_tucker(*x);  // shares buffers (immutable), scales block coefficients
  for (auto& b : t->blocks) b.c *= a;
  return t;
}

// Precision rule of the mixed mode: the preconditioner application z = P(r)
// and the operator application q = A p (which only steer the search
// direction; the residual is recomputed from x) may run in FP32 arithmetic
// when the relative tolerance eta_k of the truncation that follows is at
// least 10 times the FP32 unit roundoff 2^-24; the update of x, the residual
// f - A x, the scalar products and every truncation stay FP64.
static bool arith_f32(const tk_tpcg_params& prm, double eta) {
  return prm.arith == TK_ARITH_MIXED && eta >= 10.0 * 0x1p-24;
}

static tk_status tpcg(tk_ctx* ctx, const tk_op* op, const tk_prec* P, const tk_tucker* f_in,
                      const tk_tpcg_params& prm, tk_tucker** x_out, tk_tpcg_info* info) {
  tk_tpcg_info inf{};
  const double tol = prm.tol, beta = prm.beta, alpha = prm.alpha, delta = prm.delta;
  const int n[3] = {f_in->n[0], f_in->n[1], f_in->n[2]};
  const double nf = std::sqrt(std::max(dot(ctx, f_in, f_in), 0.0));
  // Sec. 5: eps_min = tol ||f~|| / 10 with the given rhs' norm, at most tol / 10
  const double eps_min = prm.eps_min > 0 ? prm.eps_min : 0.1 * tol * std::min(1.0, nf);
  if (nf == 0.0) {
    int r0[3] = {0, 0, 0};
    *x_out = make_plain(ctx, n, r0);
    inf.converged = 1;
    if (info) *info = inf;
    return TK_OK;
  }
  Owned f(scaled_copy(ctx, f_in, 1.0 / nf));  // ||f|| = 1
  int r0[3] = {0, 0, 0};
  Owned x(make_plain(ctx, n, r0));
  Owned r(scaled_copy(ctx, f.t, 1.0));  // r_0 = f (x_0 = 0)
  double nr = 1.0;
  if (r.t->blocks.size() != 1) {
    r = Owned(truncate(ctx, r.t, 0.0, nullptr, 0.0 < prm.refine_below, prm.reuse_bases != 0));
    nr = core_norm(ctx, r.t);
  }
  double eta = beta * tol / nr;
  auto f32 = [&]() {
    const bool on = arith_f32(prm, eta);
    inf.f32_applications += on ? 1 : 0;
    return on;
  };
  Owned pz(apply_prec(ctx, P, r.t, f32()));
  Owned z(truncate(ctx, pz.t, eta, nullptr, eta < prm.refine_below, prm.reuse_bases != 0));
  pz = Owned();
  Owned p(scaled_copy(ctx, z.t, 1.0));
  Owned ap(apply_op(ctx, op, p.t, f32()));
  Owned q(truncate(ctx, ap.t, eta, nullptr, eta < prm.refine_below, prm.reuse_bases != 0));
  ap = Owned();
  inf.trel_calls = 2;
  double xi = dot(ctx, p.t, q.t);
  double eps = prm.eps0;
  int k = 0;
  tk_status st = TK_OK;
  while (nr > tol && k < prm.maxit) {
    if (!std::isfinite(xi) || xi <= 0.0) { st = TK_EBREAKDOWN; break; }
    const double om = dot(ctx, r.t, p.t) / xi;
    if (!std::isfinite(om)) { st = TK_EBREAKDOWN; break; }
    // Algorithm 2 on y~ = x_k + om p_k with dy~ = om p_k
    Owned yt(lin_comb(ctx, 1.0, x.t, om, p.t));
    TruncPrep prep = truncate_prepare(ctx, yt.t);
    const double den = om * om * dot(ctx, p.t, p.t);
    const double base = om * dot(ctx, p.t, x.t);
    double eps_new = eps;
    Owned x1;
    while (true) {
      x1 = Owned(truncate_finish(ctx, prep, eps_new, nullptr, eps_new < prm.refine_below, prm.reuse_bases != 0));
      ++inf.trel_calls;
      if (den == 0.0) break;
      const double v = (om * dot(ctx, p.t, x1.t) - base) / den;
      if (std::fabs(v - 1.0) < delta) break;
      if (alpha * eps_new > eps_min) eps_new *= alpha;
      else break;
    }
    eps = eps_new;
    x = std::move(x1);
    yt = Owned();
    // r_{k+1} = T^rel(f - A x_{k+1}, eta_k)
    Owned ax(apply_op(ctx, op, x.t));
    Owned res(lin_comb(ctx, 1.0, f.t, -1.0, ax.t));
    ax = Owned();
    r = Owned(truncate(ctx, res.t, eta, nullptr, eta < prm.refine_below, prm.reuse_bases != 0));
    res = Owned();
    ++inf.trel_calls;
    nr = core_norm(ctx, r.t);
    ++k;
    if (prm.verbose)
      std::fprintf(stderr, "tpcg it %d relres %.3e rank (%d,%d,%d) eps %.2e\n", k, nr, x.t->m[0],
                   x.t->m[1], x.t->m[2], eps);
    if (!std::isfinite(nr)) { st = TK_EBREAKDOWN; break; }
    if (nr <= tol) break;
    eta = beta * tol / nr;
    pz = Owned(apply_prec(ctx, P, r.t, f32()));
    z = Owned(truncate(ctx, pz.t, eta, nullptr, eta < prm.refine_below, prm.reuse_bases != 0));
    pz = Owned();
    const double bk = -dot(ctx, z.t, q.t) / xi;
    Owned zp(lin_comb(ctx, 1.0, z.t, bk, p.t));
    p = Owned(truncate(ctx, zp.t, eta, nullptr, eta < prm.refine_below, prm.reuse_bases != 0));
    zp = Owned();
    ap = Owned(apply_op(ctx, op, p.t, f32()));
    q = Owned(truncate(ctx, ap.t, eta, nullptr, eta < prm.refine_below, prm.reuse_bases != 0));
    ap = Owned();
    xi = dot(ctx, p.t, q.t);
    inf.trel_calls += 3;
  }
  inf.iters = k;
  inf.relres = nr;
  inf.converged = nr <= tol;
  inf.eps_final = eps;
  if (st == TK_OK && !inf.converged) st = TK_ENOCONV;
  // scale back: x * ||f||
  tk_tucker* xo = x.release();
  for (auto& b : xo->blocks) b.c *= nf;
  for (int kk = 0; kk < 3; ++kk) inf.rank[kk] = xo->m[kk];
  *x_out = xo;
  if (info) *info = inf;
  return st;
}

// ---------------------------------------------------------------------------
// Block (3-component) systems, Sec. 5.3: products, scalar products, sums and
// truncations act blockwise; the preconditioner is block diagonal.
// ---------------------------------------------------------------------------

// y_a = sum_b A_ab x_b (A row-major 3 x 3, null = zero block)
static void apply_op_block(tk_ctx* ctx, const tk_op* const A[9], tk_tucker* const x[3], Owned y[3],
                           bool f32 = false) {
  for (int a = 0; a < 3; ++a) {
    Owned acc;
    for (int b = 0; b < 3; ++b) {
      if (!A[3 * a + b]) continue;
      Owned t(apply_op(ctx, A[3 * a + b], x[b], f32));
      acc = acc.t ? Owned(lin_comb(ctx, 1.0, acc.t, 1.0, t.t)) : std::move(t);
    }
    if (!acc.t) {
      int r0[3] = {0, 0, 0};
      acc = Owned(make_plain(ctx, x[a]->n, r0));
    }
    y[a] = std::move(acc);
  }
}

static tk_status tpcg_block(tk_ctx* ctx, const tk_op* const A[9], const tk_prec* const P[3],
                            const tk_tucker* const f_in[3], const tk_tpcg_params& prm, tk_tucker* x_out[3],
                            tk_tpcg_info* info) {
  tk_tpcg_info inf{};
  const double tol = prm.tol, beta = prm.beta, alpha = prm.alpha, delta = prm.delta;
  auto bdot = [&](Owned* x, Owned* y) {
    double s = 0.0;
    for (int a = 0; a < 3; ++a) s += dot(ctx, x[a].t, y[a].t);
    return s;
  };
  auto raw = [](Owned* v, tk_tucker* out[3]) {
    for (int a = 0; a < 3; ++a) out[a] = v[a].t;
  };
  auto trunc = [&](Owned* y, double eps, Owned* out) {
    for (int a = 0; a < 3; ++a) out[a] = Owned(truncate(ctx, y[a].t, eps, nullptr, eps < prm.refine_below, prm.reuse_bases != 0));
    inf.trel_calls += 1;
  };
  // ||r|| of a truncated block vector (orthonormal factors per component)
  auto tnorm = [&](Owned* r) {
    double s = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double c = core_norm(ctx, r[a].t);
      s += c * c;
    }
    return std::sqrt(s);
  };
  double nf2 = 0.0;
  for (int a = 0; a < 3; ++a) nf2 += dot(ctx, f_in[a], f_in[a]);
  const double nf = std::sqrt(std::max(nf2, 0.0));
  const double eps_min = prm.eps_min > 0 ? prm.eps_min : 0.1 * tol * std::min(1.0, nf);
  Owned x[3], f[3], r[3], z[3], p[3], q[3], tmp[3];
  int r0[3] = {0, 0, 0};
  for (int a = 0; a < 3; ++a) x[a] = Owned(make_plain(ctx, f_in[a]->n, r0));
  if (nf == 0.0) {
    for (int a = 0; a < 3; ++a) x_out[a] = x[a].release();
    inf.converged = 1;
    if (info) *info = inf;
    return TK_OK;
  }
  for (int a = 0; a < 3; ++a) f[a] = Owned(scaled_copy(ctx, f_in[a], 1.0 / nf));  // ||f|| = 1
  double nr = 1.0;
  bool single = true;
  for (int a = 0; a < 3; ++a) single = single && f[a].t->blocks.size() == 1;
  if (single) {
    for (int a = 0; a < 3; ++a) r[a] = Owned(scaled_copy(ctx, f[a].t, 1.0));  // r_0 = f
  } else {
    trunc(f, 0.0, r);
    nr = tnorm(r);
  }
  double eta = beta * tol / nr;
  // the precision rule of tpcg: P(r) and A p in FP32 arithmetic when allowed
  auto precond = [&](Owned* s, Owned* out) {
    const bool f32 = arith_f32(prm, eta);
    inf.f32_applications += f32 ? 1 : 0;
    for (int a = 0; a < 3; ++a) out[a] = Owned(apply_prec(ctx, P[a], s[a].t, f32));
  };
  auto op_apply = [&](Owned* v, Owned* out, bool direction) {
    const bool f32 = direction && arith_f32(prm, eta);
    inf.f32_applications += f32 ? 1 : 0;
    tk_tucker* vr[3];
    raw(v, vr);
    apply_op_block(ctx, A, vr, out, f32);
  };
  precond(r, tmp);
  trunc(tmp, eta, z);
  for (int a = 0; a < 3; ++a) p[a] = Owned(scaled_copy(ctx, z[a].t, 1.0));
  op_apply(p, tmp, true);
  trunc(tmp, eta, q);
  double xi = bdot(p, q);
  double eps = prm.eps0;
  int k = 0;
  tk_status st = TK_OK;
  while (nr > tol && k < prm.maxit) {
    if (!std::isfinite(xi) || xi <= 0.0) { st = TK_EBREAKDOWN; break; }
    const double om = bdot(r, p) / xi;
    if (!std::isfinite(om)) { st = TK_EBREAKDOWN; break; }
    // Algorithm 2 on the block vector y~ = x_k + om p_k, dy~ = om p_k
    TruncPrep prep[3];
    Owned yt[3];
    for (int a = 0; a < 3; ++a) {
      yt[a] = Owned(lin_comb(ctx, 1.0, x[a].t, om, p[a].t));
      prep[a] = truncate_prepare(ctx, yt[a].t);
    }
    const double den = om * om * bdot(p, p);
    const double base = om * bdot(p, x);
    double eps_new = eps;
    Owned x1[3];
    while (true) {
      for (int a = 0; a < 3; ++a) x1[a] = Owned(truncate_finish(ctx, prep[a], eps_new, nullptr, eps_new < prm.refine_below, prm.reuse_bases != 0));
      ++inf.trel_calls;
      if (den == 0.0) break;
      const double v = (om * bdot(p, x1) - base) / den;
      if (std::fabs(v - 1.0) < delta) break;
      if (alpha * eps_new > eps_min) eps_new *= alpha;
      else break;
    }
    eps = eps_new;
    for (int a = 0; a < 3; ++a) {
      x[a] = std::move(x1[a]);
      yt[a] = Owned();
    }
    // r_{k+1} = T^rel(f - A x_{k+1}, eta_k)
    op_apply(x, tmp, false);
    Owned res[3];
    for (int a = 0; a < 3; ++a) {
      res[a] = Owned(lin_comb(ctx, 1.0, f[a].t, -1.0, tmp[a].t));
      tmp[a] = Owned();
    }
    trunc(res, eta, r);
    nr = tnorm(r);
    ++k;
    if (prm.verbose)
      std::fprintf(stderr, "tpcg-block it %d relres %.3e rank (%d,%d,%d) eps %.2e\n", k, nr, x[0].t->m[0],
                   x[0].t->m[1], x[0].t->m[2], eps);
    if (!std::isfinite(nr)) { st = TK_EBREAKDOWN; break; }
    if (nr <= tol) break;
    eta = beta * tol / nr;
    precond(r, tmp);
    trunc(tmp, eta, z);
    const double bk = -bdot(z, q) / xi;
    for (int a = 0; a < 3; ++a) tmp[a] = Owned(lin_comb(ctx, 1.0, z[a].t, bk, p[a].t));
    trunc(tmp, eta, p);
    op_apply(p, tmp, true);
    trunc(tmp, eta, q);
    xi = bdot(p, q);
  }
  inf.iters = k;
  inf.relres = nr;
  inf.converged = nr <= tol;
  inf.eps_final = eps;
  if (st == TK_OK && !inf.converged) st = TK_ENOCONV;
  for (int a = 0; a < 3; ++a) {
    tk_tucker* xo = x[a].release();
    for (auto& b : xo->blocks) b.c *= nf;
    for (int kk = 0; kk < 3; ++kk) inf.rank[kk] = std::max<int64_t>(inf.rank[kk], xo->m[kk]);
    x_out[a] = xo;
  }
  if (info) *info = inf;
  return st;
}

}  // namespace tk

// ===========================================================================
// C ABI
// ===========================================================================

using namespace tk;

template <class F>
static tk_status guarded(tk_ctx* ctx, F&& f) {
  try {
    if (ctx) HIPCHK(hipSetDevice(ctx->device));
    return f();
  } catch (const Error& e) {
    if (ctx) ctx->last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->last_error = "host allocation failed";
    return TK_ENOMEM;
  } catch (const std::exception& e) {
    if (ctx) ctx->last_error = e.what();
    return TK_EDEVICE;
  }
}

extern "C" {

tk_status tk_ctx_create(int device, void* hip_stream, tk_ctx** out) {
  if (!out) return TK_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return TK_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return TK_EDEVICE;
  auto* c = new tk_ctx;
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->pool = std::make_unique<Pool>(device);
  tk_status st = guarded(c, [&]() {
    c->scal = alloc(c, 512);
    c->sel = alloc(c, 1100);  // 2200 ints
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&c->stage), kStage * sizeof(double), hipHostMallocDefault));
    for (int i = 0; i < 2; ++i) {
      HIPCHK(hipStreamCreateWithFlags(&c->side[i], hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&c->ev_side[i], hipEventDisableTiming));
    }
    HIPCHK(hipEventCreateWithFlags(&c->ev_main, hipEventDisableTiming));
    return TK_OK;
  });
  if (st != TK_OK) {
    delete c;
    return st;
  }
  *out = c;
  return TK_OK;
}

void tk_ctx_destroy(tk_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (int i = 0; i < 2; ++i) {
    if (ctx->side[i]) {
      (void)hipStreamSynchronize(ctx->side[i]);
      (void)hipStreamDestroy(ctx->side[i]);
    }
    if (ctx->ev_side[i]) (void)hipEventDestroy(ctx->ev_side[i]);
  }
  if (ctx->ev_main) (void)hipEventDestroy(ctx->ev_main);
  for (auto& r : ctx->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : ctx->evpool) (void)hipEventDestroy(e);
  ctx->scal.reset();
  ctx->sel.reset();
  if (ctx->stage) (void)hipHostFree(ctx->stage);
  delete ctx;
}

const char* tk_last_error(const tk_ctx* ctx) { return ctx ? ctx->last_error.c_str() : "no context"; }

tk_status tk_ctx_sync(tk_ctx* ctx) {
  if (!ctx) return TK_EINVAL;
  return guarded(ctx, [&]() { sync(ctx); return TK_OK; });
}

tk_status tk_ctx_trim(tk_ctx* ctx) {
  if (!ctx) return TK_EINVAL;
  return guarded(ctx, [&]() { sync(ctx); ctx->pool->trim(); return TK_OK; });
}

tk_status tk_assemble_1d(int32_t n_el, int32_t p, int32_t kind, const double weight[4], double* band) {
  if (n_el < 1 || p < 1 || kind < 0 || kind > 3 || !weight || !band) return TK_EINVAL;
  if (n_el + p - 2 < 1) return TK_EINVAL;
  try {
    assemble_band(n_el, p, kind, weight, band);
  } catch (...) {
    return TK_ENOMEM;
  }
  return TK_OK;
}

tk_status tk_assemble_1d_bc(int32_t n_el, int32_t p, int32_t kind, const double weight[4], int32_t k0, int32_t k1,
                            double* band) {
  if (n_el < 1 || p < 1 || kind < 0 || kind > 3 || !weight || !band) return TK_EINVAL;
  if ((k0 != 0 && k0 != 1) || (k1 != 0 && k1 != 1) || n_el + p - 2 + k0 + k1 < 1) return TK_EINVAL;
  try {
    assemble_band(n_el, p, kind, weight, band, k0, k1);
  } catch (...) {
    return TK_ENOMEM;
  }
  return TK_OK;
}

tk_status tk_assemble_1d_cheb(int32_t n_el, int32_t p, int32_t kind, int32_t nc, const double* c, int32_t k0,
                              int32_t k1, double* band) {
  if (n_el < 1 || p < 1 || kind < 0 || kind > 3 || nc < 1 || nc > 4096 || !c || !band) return TK_EINVAL;
  if ((k0 != 0 && k0 != 1) || (k1 != 0 && k1 != 1) || n_el + p - 2 + k0 + k1 < 1) return TK_EINVAL;
  try {
    assemble_band_cheb(n_el, p, kind, c, nc, band, k0, k1);
  } catch (...) {
    return TK_ENOMEM;
  }
  return TK_OK;
}

tk_status tk_load_vector_1d_cheb(int32_t n_el, int32_t p, int32_t nc, const double* c, int32_t k0, int32_t k1,
                                 double* F) {
  if (n_el < 1 || p < 1 || nc < 1 || nc > 4096 || !c || !F) return TK_EINVAL;
  if ((k0 != 0 && k0 != 1) || (k1 != 0 && k1 != 1) || n_el + p - 2 + k0 + k1 < 1) return TK_EINVAL;
  try {
    load_vector_cheb(n_el, p, c, nc, F, k0, k1);
  } catch (...) {
    return TK_ENOMEM;
  }
  return TK_OK;
}

tk_status tk_basis_values_1d(int32_t n_el, int32_t p, int32_t k0, int32_t k1, int32_t der, int64_t npts,
                             const double* x, double* out) {
  if (n_el < 1 || p < 1 || der < 0 || der > p || npts < 0 || (npts > 0 && (!x || !out))) return TK_EINVAL;
  if ((k0 != 0 && k0 != 1) || (k1 != 0 && k1 != 1) || n_el + p - 2 + k0 + k1 < 1) return TK_EINVAL;
  for (int64_t q = 0; q < npts; ++q)
    if (!(x[q] >= 0.0 && x[q] <= 1.0)) return TK_EINVAL;
  if (npts > INT32_MAX) return TK_EINVAL;
  try {
    basis_values(n_el, p, k0, k1, der, int(npts), x, out);
  } catch (...) {
    return TK_ENOMEM;
  }
  return TK_OK;
}

tk_status tk_load_vector_1d(int32_t n_el, int32_t p, const double weight[4], double* F) {
  if (n_el < 1 || p < 1 || !weight || !F || n_el + p - 2 < 1) return TK_EINVAL;
  try {
    load_vector(n_el, p, weight, F);
  } catch (...) {
    return TK_ENOMEM;
  }
  return TK_OK;
}

tk_status tk_fd_direction_host(int32_t n_el, int32_t p, double coef, int32_t* n, int32_t* n1, int32_t* n2,
                               double* lam, double* g, double* E, double* v2u2) {
  try {
    FdDirection d;
    std::string msg;
    if (!(coef > 0.0) || !fd_direction_setup(n_el, p, coef, d, msg)) return TK_EINVAL;
    if (n) *n = d.n;
    if (n1) *n1 = d.n1;
    if (n2) *n2 = d.n2;
    if (lam) std::copy(d.lam.begin(), d.lam.end(), lam);
    if (g) std::copy(d.g.begin(), d.g.end(), g);
    if (v2u2) std::copy(d.v2u2.begin(), d.v2u2.end(), v2u2);
    if (E) {
      std::fill(E, E + (size_t)d.n * d.n1, 0.0);
      for (int i = 0; i < d.n; ++i)
        for (int c = 0; c < d.ke; ++c) {
          const int j = d.e_idx[(size_t)i * d.ke + c];
          if (j >= 0) E[i + (size_t)j * d.n] = d.e_val[(size_t)i * d.ke + c];
        }
    }
    return TK_OK;
  } catch (...) {
    return TK_ENOMEM;
  }
}

tk_status tk_expsum_host(double M, double eps, int32_t* R, double* alpha, double* omega, double* err,
                         double* err_prev) {
  try {
    ExpSum es;
    std::string msg;
    if (!expsum_for(M, eps, es, msg)) return TK_ENUMERIC;
    if (es.R > 64) return TK_ENUMERIC;
    if (R) *R = es.R;
    for (int j = 0; j < es.R; ++j) {
      if (alpha) alpha[j] = es.alpha[j];
      if (omega) omega[j] = es.omega[j];
    }
    if (err) *err = es.err;
    if (err_prev) *err_prev = es.err_prev;
    return TK_OK;
  } catch (...) {
    return TK_ENOMEM;
  }
}

tk_status tk_tucker_create(tk_ctx* ctx, const int64_t n[3], const int64_t r[3], const double* core,
                           const double* const U[3], int32_t on_device, tk_tucker** out) {
  if (!ctx || !n || !r || !out) return TK_EINVAL;
  *out = nullptr;
  return guarded(ctx, [&]() {
    int nn[3], rr[3];
    for (int k = 0; k < 3; ++k) {
      if (n[k] < 1 || r[k] < 0 || n[k] > (1 << 20) || r[k] > (1 << 16)) throw Error(TK_EINVAL, "bad Tucker shape");
      nn[k] = int(n[k]);
      rr[k] = int(r[k]);
    }
    const bool empty = prod3(rr) == 0;
    if (empty) for (int k = 0; k < 3; ++k) rr[k] = 0;
    if (!empty && (!core || !U || !U[0] || !U[1] || !U[2])) throw Error(TK_EINVAL, "null data pointer");
    Owned t(make_plain(ctx, nn, rr));
    if (!empty) {
      auto cp = [&](double* dst, const double* src, size_t cnt) {
        if (on_device) d2d(ctx, dst, src, cnt);
        else h2d(ctx, dst, src, cnt);
      };
      cp(t.t->blocks[0].core->p, core, (size_t)prod3(rr));
      for (int k = 0; k < 3; ++k) cp(t.t->U[k]->p, U[k], (size_t)nn[k] * rr[k]);
    }
    *out = t.release();
    return TK_OK;
  });
}

void tk_tucker_free(tk_tucker* t) { delete t; }

tk_status tk_tucker_shape(const tk_tucker* t, int64_t n[3], int64_t m[3], int32_t* nblocks) {
  if (!t) return TK_EINVAL;
  for (int k = 0; k < 3; ++k) {
    if (n) n[k] = t->n[k];
    if (m) m[k] = t->m[k];
  }
  if (nblocks) *nblocks = int32_t(t->blocks.size());
  return TK_OK;
}

tk_status tk_tucker_block(const tk_tucker* t, int32_t b, double* coef, int64_t r[3], int64_t off[3]) {
  if (!t || b < 0 || b >= int32_t(t->blocks.size())) return TK_EINVAL;
  const auto& bl = t->blocks[b];
  if (coef) *coef = bl.c;
  for (int k = 0; k < 3; ++k) {
    if (r) r[k] = bl.r[k];
    if (off) off[k] = bl.off[k];
  }
  return TK_OK;
}

tk_status tk_tucker_read(tk_ctx* ctx, const tk_tucker* t, int32_t k, double* U, int32_t b, double* core,
                         int32_t on_device) {
  if (!ctx || !t) return TK_EINVAL;
  return guarded(ctx, [&]() {
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (U) {
      if (k < 0 || k > 2) throw Error(TK_EINVAL, "mode out of range");
      const size_t cnt = (size_t)t->n[k] * t->m[k];
      if (cnt) HIPCHK(hipMemcpyAsync(U, t->U[k]->p, cnt * sizeof(double), kind, ctx->stream));
    }
    if (core) {
      if (b < 0 || b >= int(t->blocks.size())) throw Error(TK_EINVAL, "block out of range");
      const size_t cnt = (size_t)prod3(t->blocks[b].r);
      if (cnt) HIPCHK(hipMemcpyAsync(core, t->blocks[b].core->p, cnt * sizeof(double), kind, ctx->stream));
    }
    sync(ctx);
    return TK_OK;
  });
}

tk_status tk_tucker_dot(tk_ctx* ctx, const tk_tucker* x, const tk_tucker* y, double* out) {
  if (!ctx || !x || !y || !out) return TK_EINVAL;
  return guarded(ctx, [&]() { *out = dot(ctx, x, y); return TK_OK; });
}

tk_status tk_tucker_axpby(tk_ctx* ctx, double a, const tk_tucker* x, double b, const tk_tucker* y,
                          tk_tucker** out) {
  if (!ctx || !x || !y || !out) return TK_EINVAL;
  *out = nullptr;
  return guarded(ctx, [&]() { *out = lin_comb(ctx, a, x, b, y); return TK_OK; });
}

tk_status tk_tucker_rows(tk_ctx* ctx, const tk_tucker* t, const int64_t off[3], const int64_t n[3],
                         tk_tucker** out) {
  if (!ctx || !t || !off || !n || !out) return TK_EINVAL;
  for (int k = 0; k < 3; ++k)
    if (off[k] < 0 || n[k] < 1 || off[k] + n[k] > t->n[k]) return TK_EINVAL;
  *out = nullptr;
  return guarded(ctx, [&]() {
    auto* r = new tk_tucker;
    for (int k = 0; k < 3; ++k) {
      r->n[k] = int(n[k]);
      r->m[k] = t->m[k];
      r->U[k] = alloc(ctx, (size_t)r->n[k] * r->m[k]);
      if (r->m[k] > 0)
        HIPCHK(hipMemcpy2DAsync(r->U[k]->p, sizeof(double) * r->n[k], t->U[k]->p + off[k], sizeof(double) * t->n[k],
                                sizeof(double) * r->n[k], r->m[k], hipMemcpyDeviceToDevice, ctx->stream));
    }
    r->blocks = t->blocks;  // cores are immutable and shared
    *out = r;
    return TK_OK;
  });
}

tk_status tk_op_create(tk_ctx* ctx, int32_t p, const int64_t n[3], const int32_t nmat[3],
                       const double* const bands[3], const tk_core_nz* nz, int64_t nnz, tk_op** out) {
  if (!ctx || !n || !nmat || !bands || !out || (nnz > 0 && !nz) || nnz < 0 || p < 0 || p > 6) return TK_EINVAL;
  *out = nullptr;
  return guarded(ctx, [&]() {
    std::unique_ptr<tk_op> op(new tk_op);
    op->p = p;
    for (int k = 0; k < 3; ++k) {
      if (n[k] < 1 || nmat[k] < 1 || !bands[k]) throw Error(TK_EINVAL, "bad operator mode");
      op->n[k] = int(n[k]);
      op->nmat[k] = nmat[k];
      const size_t cnt = (size_t)nmat[k] * (2 * p + 1) * n[k];
      op->band[k] = alloc(ctx, cnt);
      h2d(ctx, op->band[k]->p, bands[k], cnt);
      std::vector<float> bf(bands[k], bands[k] + cnt);
      op->band_f[k] = alloc(ctx, (cnt + 1) / 2);
      HIPCHK(hipMemcpyAsync(op->band_f[k]->p, bf.data(), cnt * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
      sync(ctx);
    }
    for (int64_t i = 0; i < nnz; ++i) {
      if (nz[i].i1 < 0 || nz[i].i1 >= nmat[0] || nz[i].i2 < 0 || nz[i].i2 >= nmat[1] || nz[i].i3 < 0 ||
          nz[i].i3 >= nmat[2])
        throw Error(TK_EINVAL, "core nonzero index out of range");
      op->nz.push_back(nz[i]);
    }
    *out = op.release();
    return TK_OK;
  });
}

void tk_op_free(tk_op* op) { delete op; }

tk_status tucker_apply_op(tk_ctx* ctx, const tk_op* op, const tk_tucker* x, tk_tucker** y) {
  if (!ctx || !op || !x || !y) return TK_EINVAL;
  *y = nullptr;
  return guarded(ctx, [&]() { *y = apply_op(ctx, op, x); return TK_OK; });
}

tk_status tucker_apply_op_arith(tk_ctx* ctx, const tk_op* op, const tk_tucker* x, int32_t arith, tk_tucker** y) {
  if (!ctx || !op || !x || !y || (arith != TK_ARITH_F64 && arith != TK_ARITH_F32)) return TK_EINVAL;
  *y = nullptr;
  return guarded(ctx, [&]() { *y = apply_op(ctx, op, x, arith == TK_ARITH_F32); return TK_OK; });
}

// The widest range [lo, hi) of rows around the middle of an ELL matrix whose
// rows hold exactly one entry, equal to 1, at column row + sh (sh taken from
// the middle row); lo = hi = 0 when the middle row is not of that kind.
static void interior_rows(const std::vector<int>& idx, const std::vector<double>& val, int k, int rows, int& lo,
                          int& hi, int& sh) {
  auto unit = [&](int i, int s) {
    if (idx[(size_t)i * k] != i + s || val[(size_t)i * k] != 1.0) return false;
    for (int t = 1; t < k; ++t)
      if (idx[(size_t)i * k + t] >= 0) return false;
    return true;
  };
  lo = hi = sh = 0;
  const int mid = rows / 2;
  if (rows == 0 || idx[(size_t)mid * k] < 0) return;
  sh = idx[(size_t)mid * k] - mid;
  if (!unit(mid, sh)) { sh = 0; return; }
  lo = mid;
  hi = mid + 1;
  while (lo > 0 && unit(lo - 1, sh)) --lo;
  while (hi < rows && unit(hi, sh)) ++hi;
}

tk_status fd_setup(tk_ctx* ctx, const int32_t n_el[3], int32_t p, double eps_prec, const double coef[3],
                   tk_prec** out, int32_t* R_P) {
  if (!ctx || !n_el || !out || !(eps_prec > 0.0)) return TK_EINVAL;
  *out = nullptr;
  return guarded(ctx, [&]() {
    std::unique_ptr<tk_prec> P(new tk_prec);
    std::string msg;
    P->lam_min = 0.0;
    P->lam_max = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double c = coef ? coef[k] : 1.0;
      if (!(c > 0.0)) throw Error(TK_EINVAL, "fd_setup: direction coefficients must be positive");
      if (!fd_direction_setup(n_el[k], p, c, P->dir[k], msg)) throw Error(TK_EINVAL, msg);
      const auto& l = P->dir[k].lam;
      P->lam_min += *std::min_element(l.begin(), l.end());
      P->lam_max += *std::max_element(l.begin(), l.end());
    }
    const double MP = P->lam_max / P->lam_min;
    ExpSum es;
    if (!expsum_for(MP, eps_prec, es, msg)) throw Error(TK_ENUMERIC, msg);
    P->R = es.R;
    P->alpha = es.alpha;
    P->omega = es.omega;
    P->err = es.err;
    P->err_prev = es.err_prev;
    const double pi = 3.14159265358979323846;
    for (int k = 0; k < 3; ++k) {
      const auto& d = P->dir[k];
      // exp(-alpha_j lam_m / lam_min), with g_m folded in on the sine part
      std::vector<double> ge((size_t)P->R * d.n);
      for (int j = 0; j < P->R; ++j)
        for (int m = 0; m < d.n; ++m)
          ge[(size_t)j * d.n + m] = std::exp(-P->alpha[j] * d.lam[m] / P->lam_min) * (m < d.n1 ? d.g[m] : 1.0);
      std::vector<double> cs(2 * (size_t)d.N), sn(d.N), tq(2 * (size_t)(d.N / 2 + 1));
      for (int t = 0; t < d.N; ++t) {
        cs[2 * t] = std::cos(2.0 * pi * t / d.N);
        cs[2 * t + 1] = -std::sin(2.0 * pi * t / d.N);
        sn[t] = std::sin(pi * t / d.N);
      }
      for (int t = 0; t <= d.N / 2; ++t) {
        tq[2 * t] = std::cos(pi * t / (2.0 * d.N));
        tq[2 * t + 1] = -std::sin(pi * t / (2.0 * d.N));
      }
      auto up = [&](const std::vector<double>& v) {
        BufP b = alloc(ctx, v.size());
        h2d(ctx, b->p, v.data(), v.size());
        return b;
      };
      auto up_int = [&](const std::vector<int>& v) {
        BufP b = alloc(ctx, (v.size() + 1) / 2);
        if (!v.empty()) {
          HIPCHK(hipMemcpyAsync(b->p, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice, ctx->stream));
          sync(ctx);
        }
        return b;
      };
      P->g[k] = up(d.g);
      P->e_val[k] = up(d.e_val);
      P->et_val[k] = up(d.et_val);
      P->v2u2[k] = up(d.v2u2);
      P->ge[k] = up(ge);
      P->cs[k] = up(cs);
      P->sn[k] = up(sn);
      P->tq[k] = up(tq);
      P->e_idx[k] = up_int(d.e_idx);
      P->et_idx[k] = up_int(d.et_idx);
      gpu::FdDev& dv = P->dev[k];
      dv.n = d.n;
      dv.n1 = d.n1;
      dv.n2 = d.n2;
      dv.N = d.N;
      dv.odd = d.odd ? 1 : 0;
      dv.ke = d.ke;
      dv.ket = d.ket;
      dv.R = P->R;
      dv.e_idx = reinterpret_cast<const int*>(P->e_idx[k]->p);
      dv.et_idx = reinterpret_cast<const int*>(P->et_idx[k]->p);
      dv.t64.g = P->g[k]->p;
      dv.t64.e_val = P->e_val[k]->p;
      dv.t64.et_val = P->et_val[k]->p;
      dv.t64.v2u2 = P->v2u2[k]->p;
      dv.t64.ge = P->ge[k]->p;
      dv.t64.cs = P->cs[k]->p;
      dv.t64.sn = P->sn[k]->p;
      dv.t64.tq = P->tq[k]->p;
      {
        // the same tables rounded to FP32, packed in one buffer (each table
        // starts on a 16-byte boundary)
        const std::vector<double>* tabs[8] = {&d.g, &d.e_val, &d.et_val, &d.v2u2, &ge, &cs, &sn, &tq};
        size_t off[8], tot = 0;
        for (int i = 0; i < 8; ++i) {
          off[i] = tot;
          tot += (tabs[i]->size() + 3) / 4 * 4;
        }
        std::vector<float> hf(std::max<size_t>(tot, 4), 0.0f);
        for (int i = 0; i < 8; ++i)
          for (size_t e = 0; e < tabs[i]->size(); ++e) hf[off[i] + e] = float((*tabs[i])[e]);
        P->f32[k] = alloc(ctx, (hf.size() + 1) / 2);
        HIPCHK(hipMemcpyAsync(P->f32[k]->p, hf.data(), hf.size() * sizeof(float), hipMemcpyHostToDevice,
                              ctx->stream));
        sync(ctx);
        const float* fb = reinterpret_cast<const float*>(P->f32[k]->p);
        dv.t32.g = fb + off[0];
        dv.t32.e_val = fb + off[1];
        dv.t32.et_val = fb + off[2];
        dv.t32.v2u2 = fb + off[3];
        dv.t32.ge = fb + off[4];
        dv.t32.cs = fb + off[5];
        dv.t32.sn = fb + off[6];
        dv.t32.tq = fb + off[7];
      }
      interior_rows(d.e_idx, d.e_val, d.ke, d.n, dv.e_lo, dv.e_hi, dv.e_sh);
      interior_rows(d.et_idx, d.et_val, d.ket, d.n1, dv.et_lo, dv.et_hi, dv.et_sh);
    }
    if (R_P) *R_P = P->R;
    *out = P.release();
    return TK_OK;
  });
}

// fd_setup_exact on the spaces with boundary flags bc[2k], bc[2k+1] (null:
// Dirichlet everywhere)
// approx: the Appendix B eigen-approximations on the same spaces, built
// densely on the host (fd_approx_dense), instead of the exact eigenpairs
static tk_status setup_exact(tk_ctx* ctx, const int32_t n_el[3], int32_t p, double eps_prec, const double coef[3],
                             const int32_t* bc, tk_prec** out, int32_t* R_P, bool approx = false) {
  if (!ctx || !n_el || !out || !(eps_prec > 0.0)) return TK_EINVAL;
  *out = nullptr;
  return guarded(ctx, [&]() {
    std::unique_ptr<tk_prec> P(new tk_prec);
    P->exact = true;
    std::string msg;
    std::vector<double> L[3];
    for (int k = 0; k < 3; ++k) {
      const double c = coef ? coef[k] : 1.0;
      if (!(c > 0.0)) throw Error(TK_EINVAL, "fd_setup_exact: direction coefficients must be positive");
      std::vector<double> C;
      int n = 0;
      const int k0 = bc ? bc[2 * k] : 0, k1 = bc ? bc[2 * k + 1] : 0;
      if (approx) {
        std::vector<double> Ut;
        if (!fd_approx_dense(n_el[k], p, c, k0, k1, Ut, P->lam_exact[k], n, msg)) throw Error(TK_EINVAL, msg);
        P->n_exact[k] = n;
        P->Ud[k] = alloc(ctx, (size_t)n * n);
        h2d(ctx, P->Ud[k]->p, Ut.data(), (size_t)n * n);
        const auto& l = P->lam_exact[k];
        P->lam_min += *std::min_element(l.begin(), l.end());
        P->lam_max += *std::max_element(l.begin(), l.end());
        continue;
      }
      if (!fd_exact_pencil(n_el[k], p, c, C, L[k], n, msg, k0, k1)) throw Error(TK_EINVAL, msg);
      P->n_exact[k] = n;
      // eigenpairs of C with the library's symmetric eigensolver
      BufP Cd = alloc(ctx, (size_t)n * n), V = alloc(ctx, (size_t)n * n), w = alloc(ctx, (size_t)n);
      BufP work = alloc(ctx, gpu::sym_eig_work(n));
      h2d(ctx, Cd->p, C.data(), (size_t)n * n);
      gpu::sym_eig(ctx->stream, Cd->p, n, V->p, w->p, work->p);
      std::vector<double> Q = d2h(ctx, V->p, (size_t)n * n);
      P->lam_exact[k] = d2h(ctx, w->p, (size_t)n);
      // with Neumann at both ends the constants give a zero eigenvalue;
      // computed values below 1e-12 lambda_max are rounding (the smallest
      // nonzero one is about pi^2 coef) and are set to 0
      auto& lk = P->lam_exact[k];
      const double lmax = *std::max_element(lk.begin(), lk.end());
      for (double& v : lk) {
        if (!std::isfinite(v) || v < -1e-8 * std::fabs(lmax)) throw Error(TK_ENUMERIC, "fd_setup_exact: negative eigenvalue");
        if (v < 1e-12 * lmax) v = 0.0;
      }
      fd_exact_vectors(L[k], n, p, Q.data());  // U = L^{-T} Q, M-orthonormal
      P->Ud[k] = alloc(ctx, (size_t)n * n);
      h2d(ctx, P->Ud[k]->p, Q.data(), (size_t)n * n);
      const auto& l = P->lam_exact[k];
      P->lam_min += *std::min_element(l.begin(), l.end());
      P->lam_max += *std::max_element(l.begin(), l.end());
    }
    if (!(P->lam_min > 0.0))
      throw Error(TK_EINVAL, "fd_setup_exact: singular operator (Neumann at both ends of every direction)");
    ExpSum es;
    if (!expsum_for(P->lam_max / P->lam_min, eps_prec, es, msg)) throw Error(TK_ENUMERIC, msg);
    P->R = es.R;
    P->alpha = es.alpha;
    P->omega = es.omega;
    P->err = es.err;
    P->err_prev = es.err_prev;
    for (int k = 0; k < 3; ++k) {
      const int n = P->n_exact[k];
      std::vector<double> E((size_t)P->R * n);
      for (int j = 0; j < P->R; ++j)
        for (int m = 0; m < n; ++m) E[(size_t)j * n + m] = std::exp(-P->alpha[j] * P->lam_exact[k][m] / P->lam_min);
      P->Ed[k] = alloc(ctx, E.size());
      h2d(ctx, P->Ed[k]->p, E.data(), E.size());
    }
    if (R_P) *R_P = P->R;
    *out = P.release();
    return TK_OK;
  });
}

tk_status fd_setup_exact(tk_ctx* ctx, const int32_t n_el[3], int32_t p, double eps_prec, const double coef[3],
                         tk_prec** out, int32_t* R_P) {
  return setup_exact(ctx, n_el, p, eps_prec, coef, nullptr, out, R_P);
}

tk_status fd_setup_exact_bc(tk_ctx* ctx, const int32_t n_el[3], int32_t p, double eps_prec, const double coef[3],
                            const int32_t bc[6], tk_prec** out, int32_t* R_P) {
  if (!bc) return TK_EINVAL;
  for (int i = 0; i < 6; ++i)
    if (bc[i] != 0 && bc[i] != 1) return TK_EINVAL;
  return setup_exact(ctx, n_el, p, eps_prec, coef, bc, out, R_P);
}

tk_status fd_setup_bc(tk_ctx* ctx, const int32_t n_el[3], int32_t p, double eps_prec, const double coef[3],
                      const int32_t bc[6], tk_prec** out, int32_t* R_P) {
  if (!bc) return TK_EINVAL;
  for (int i = 0; i < 6; ++i)
    if (bc[i] != 0 && bc[i] != 1) return TK_EINVAL;
  return setup_exact(ctx, n_el, p, eps_prec, coef, bc, out, R_P, true);
}

tk_status tk_fd_direction_dense_host(int32_t n_el, int32_t p, double coef, int32_t k0, int32_t k1, int32_t* n,
                                     double* lam, double* Ut) {
  try {
    std::vector<double> U, l;
    std::string msg;
    int nn = 0;
    if (!(coef > 0.0) || !fd_approx_dense(n_el, p, coef, k0, k1, U, l, nn, msg)) return TK_EINVAL;
    if (n) *n = nn;
    if (lam) std::copy(l.begin(), l.end(), lam);
    if (Ut) std::copy(U.begin(), U.end(), Ut);
  } catch (...) {
    return TK_ENOMEM;
  }
  return TK_OK;
}

void tk_prec_free(tk_prec* P) { delete P; }

tk_status tk_prec_info(const tk_prec* P, int32_t* R_P, double* lam_min, double* lam_max, double* err,
                       double* alpha, double* omega) {
  if (!P) return TK_EINVAL;
  if (R_P) *R_P = P->R;
  if (lam_min) *lam_min = P->lam_min;
  if (lam_max) *lam_max = P->lam_max;
  if (err) *err = P->err;
  for (int j = 0; j < P->R; ++j) {
    if (alpha) alpha[j] = P->alpha[j];
    if (omega) omega[j] = P->omega[j];
  }
  return TK_OK;
}

tk_status tk_prec_direction(const tk_prec* P, int32_t k, int32_t* n, int32_t* n1, int32_t* n2, double* lam,
                            double* g, double* E, double* v2u2) {
  if (!P || k < 0 || k > 2) return TK_EINVAL;
  if (P->exact) {
    const int ne = P->n_exact[k];
    if (n) *n = ne;
    if (n1) *n1 = ne;
    if (n2) *n2 = 0;
    if (lam) std::copy(P->lam_exact[k].begin(), P->lam_exact[k].end(), lam);
    return TK_OK;
  }
  const auto& d = P->dir[k];
  if (n) *n = d.n;
  if (n1) *n1 = d.n1;
  if (n2) *n2 = d.n2;
  if (lam) std::copy(d.lam.begin(), d.lam.end(), lam);
  if (g) std::copy(d.g.begin(), d.g.end(), g);
  if (v2u2) std::copy(d.v2u2.begin(), d.v2u2.end(), v2u2);
  if (E) {
    std::fill(E, E + (size_t)d.n * d.n1, 0.0);
    for (int i = 0; i < d.n; ++i)
      for (int c = 0; c < d.ke; ++c) {
        const int j = d.e_idx[(size_t)i * d.ke + c];
        if (j >= 0) E[i + (size_t)j * d.n] = d.e_val[(size_t)i * d.ke + c];
      }
  }
  return TK_OK;
}

tk_status fd_precond(tk_ctx* ctx, const tk_prec* P, const tk_tucker* s, tk_tucker** v) {
  if (!ctx || !P || !s || !v) return TK_EINVAL;
  *v = nullptr;
  return guarded(ctx, [&]() { *v = apply_prec(ctx, P, s); return TK_OK; });
}

tk_status fd_precond_arith(tk_ctx* ctx, const tk_prec* P, const tk_tucker* s, int32_t arith, tk_tucker** v) {
  if (!ctx || !P || !s || !v || (arith != TK_ARITH_F64 && arith != TK_ARITH_F32)) return TK_EINVAL;
  *v = nullptr;
  return guarded(ctx, [&]() { *v = apply_prec(ctx, P, s, arith == TK_ARITH_F32); return TK_OK; });
}

tk_status tucker_truncate(tk_ctx* ctx, const tk_tucker* y, double eps, tk_tucker** out, double* discarded) {
  if (!ctx || !y || !out || !(eps >= 0.0)) return TK_EINVAL;
  *out = nullptr;
  return guarded(ctx, [&]() { *out = truncate(ctx, y, eps, discarded); return TK_OK; });
}

tk_status tk_prof_enable(tk_ctx* ctx, int32_t on) {
  if (!ctx) return TK_EINVAL;
  return guarded(ctx, [&]() {
    prof_flush(ctx);
    ctx->prof = on != 0;
    return TK_OK;
  });
}

tk_status tk_truncate_refinements(const tk_ctx* ctx, int64_t* count) {
  if (!ctx || !count) return TK_EINVAL;
  *count = ctx->tail_refinements;
  return TK_OK;
}

tk_status tk_prof_reset(tk_ctx* ctx) {
  if (!ctx) return TK_EINVAL;
  return guarded(ctx, [&]() {
    prof_flush(ctx);
    for (int k = 0; k < PK_N; ++k) ctx->p_ms[k] = ctx->p_bytes[k] = ctx->p_flops[k] = 0.0, ctx->p_n[k] = 0;
    return TK_OK;
  });
}

tk_status tk_prof_read(tk_ctx* ctx, int32_t kind, int64_t* launches, double* ms, double* bytes, double* flops) {
  if (!ctx || kind < 0 || kind >= PK_N) return TK_EINVAL;
  return guarded(ctx, [&]() {
    prof_flush(ctx);
    if (launches) *launches = ctx->p_n[kind];
    if (ms) *ms = ctx->p_ms[kind];
    if (bytes) *bytes = ctx->p_bytes[kind];
    if (flops) *flops = ctx->p_flops[kind];
    return TK_OK;
  });
}

tk_status tk_sym_eig(tk_ctx* ctx, const double* G, int32_t a, double* V, double* w) {
  if (!ctx || !G || !V || !w || a < 1 || a > 2048) return TK_EINVAL;
  return guarded(ctx, [&]() {
    BufP work = alloc(ctx, gpu::sym_eig_work(a));
    Prof pr(ctx, PK_EIG, 8.0 * 2.0 * a * (double)a, eig_flops(a));
    gpu::sym_eig(ctx->stream, G, a, V, w, work->p);
    return TK_OK;
  });
}

// checks of a block system's arguments: three right-hand sides of one shape,
// every nonzero block and every preconditioner of that shape
static bool block_args_ok(const tk_op* const A[9], const tk_prec* const P[3], const tk_tucker* const v[3]) {
  if (!A || !v) return false;
  for (int a = 0; a < 3; ++a) {
    if (!v[a]) return false;
    for (int k = 0; k < 3; ++k)
      if (v[a]->n[k] != v[0]->n[k]) return false;
  }
  bool any = false;
  for (int i = 0; i < 9; ++i) {
    if (!A[i]) continue;
    any = true;
    for (int k = 0; k < 3; ++k)
      if (A[i]->n[k] != v[0]->n[k]) return false;
  }
  if (!any) return false;
  if (P) {
    for (int a = 0; a < 3; ++a) {
      if (!P[a]) return false;
      for (int k = 0; k < 3; ++k)
        if ((P[a]->exact ? P[a]->n_exact[k] : P[a]->dir[k].n) != v[0]->n[k]) return false;
    }
  }
  return true;
}

tk_status tucker_apply_op_block(tk_ctx* ctx, const tk_op* const A[9], tk_tucker* const x[3], tk_tucker* y[3]) {
  if (!ctx || !y || !block_args_ok(A, nullptr, x)) return TK_EINVAL;
  return guarded(ctx, [&]() {
    Owned out[3];
    apply_op_block(ctx, A, x, out);
    for (int a = 0; a < 3; ++a) y[a] = out[a].release();
    return TK_OK;
  });
}

tk_status tpcg_solve_block(tk_ctx* ctx, const tk_op* const A[9], const tk_prec* const P[3],
                           tk_tucker* const f[3], const tk_tpcg_params* params, tk_tucker* x[3],
                           tk_tpcg_info* info) {
  if (!ctx || !x || !P || !block_args_ok(A, P, f)) return TK_EINVAL;
  tk_tpcg_params prm;
  tk_tpcg_defaults(&prm);
  if (params) prm = *params;
  if (!(prm.tol > 0) || !(prm.alpha > 0 && prm.alpha < 1) || !(prm.eps0 > 0) || prm.maxit < 1 ||
      (prm.arith != TK_ARITH_F64 && prm.arith != TK_ARITH_MIXED))
    return TK_EINVAL;
  for (int a = 0; a < 3; ++a) x[a] = nullptr;
  return guarded(ctx, [&]() { return tpcg_block(ctx, A, P, f, prm, x, info); });
}

tk_status tk_dgemm(tk_ctx* ctx, int32_t ta, int32_t tb, int32_t M, int32_t N, int32_t K, double alpha,
                   const double* A, int32_t lda, const double* B, int32_t ldb, double beta, double* C,
                   int32_t ldc) {
  if (!ctx || M < 0 || N < 0 || K < 0) return TK_EINVAL;
  if ((M > 0 && N > 0) && (!C || ldc < M)) return TK_EINVAL;
  if (M > 0 && N > 0 && K > 0) {
    if (!A || !B) return TK_EINVAL;
    if (lda < (ta ? K : M) || ldb < (tb ? N : K)) return TK_EINVAL;
  }
  return guarded(ctx, [&]() {
    gemm(ctx, ta != 0, tb != 0, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    return TK_OK;
  });
}

void tk_tpcg_defaults(tk_tpcg_params* p) {
  if (!p) return;
  p->tol = 1e-6;
  p->beta = 0.1;
  p->eps0 = 0.1;
  p->alpha = 0.5;
  p->eps_min = 0.0;
  p->delta = 1e-3;
  p->maxit = 1000;
  p->verbose = 0;
  p->arith = TK_ARITH_F64;
  p->refine_below = 1e-8;
  p->reuse_bases = 1;
}

tk_status tpcg_solve(tk_ctx* ctx, const tk_op* op, const tk_prec* P, const tk_tucker* f,
                     const tk_tpcg_params* params, tk_tucker** x, tk_tpcg_info* info) {
  if (!ctx || !op || !P || !f || !x) return TK_EINVAL;
  *x = nullptr;
  tk_tpcg_params prm;
  if (params) prm = *params;
  else tk_tpcg_defaults(&prm);
  if (!(prm.tol > 0) || !(prm.beta > 0) || !(prm.eps0 > 0) || !(prm.alpha > 0 && prm.alpha < 1) ||
      !(prm.delta > 0) || prm.maxit < 0 || (prm.arith != TK_ARITH_F64 && prm.arith != TK_ARITH_MIXED)) {
    ctx->last_error = "tpcg_solve: invalid parameters";
    return TK_EINVAL;
  }
  return guarded(ctx, [&]() { return tpcg(ctx, op, P, f, prm, x, info); });
}

}  // extern "C"
