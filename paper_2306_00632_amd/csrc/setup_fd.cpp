// Host setup of the low-rank Fast Diagonalization transform of one direction
// (Sec. 4.2 Algorithm 4, Appendix B, Dirichlet at both ends).
//
// Appendix B approximates the generalized eigenvectors of (K, M) by
//   U~ = [ V1 U1 | V2 U2 ],  Lambda~ = diag((j pi)^2, Lambda2),
// where V1 U1 w is the spline of V_h1 interpolating sum_j w_j sqrt(2) sin(j pi x)
// at the interpolation points (breakpoints for odd p, span midpoints for
// even p), V_h1 = {phi : phi^(2k)(0) = phi^(2k)(1) = 0, 2k <= p-1}, and V_h2 is
// the M-orthogonal complement of V_h1 with its exact small eigenproblem.
//
// This library applies V1 U1 without the collocation solve.  The functions
// of V_h1 are exactly the restrictions to [0,1] of odd, 2-periodic splines on
// the uniform knots (odd reflection keeps C^{p-1} iff the even derivatives
// vanish at the reflection point).  For such splines interpolation at the
// breakpoints/midpoints is diagonal in the sine basis: the interpolant of
// sin(j pi x) is (1/sigma(j pi/N)) sum_k sin(j pi xi_k) B_k(x), with B_k the
// cardinal B-spline translates, xi_k their centres and sigma the symbol
//   sigma(theta) = sum_u N_p(u) cos(theta (u - (p+1)/2))
// over the points u of the interpolation grid inside the support of N_p.  So
//   V1 U1 = E * DST * diag(g),   g_j = sqrt(2) / sigma(j pi / N),
// where DST evaluates the sines at the translate centres (DST-I for odd p,
// DST-III for even p) and the sparse matrix E maps translate coefficients
// (folded by odd symmetry onto the N-1 resp. N basic centres) to the
// Dirichlet B-spline basis: identity in the interior, small dense blocks for
// the translates that cross 0 or 1 (obtained by exact least squares on
// their support).  (V1 U1)^T = diag(g) DST^T E^T.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "tk_internal.h"

namespace tk {
namespace {

constexpr double kPi = 3.14159265358979323846;

// Cardinal B-spline of degree d on [0, d+1] (uniform Cox-de Boor recursion).
double cardinal(int d, double u) {
  if (d == 0) return (u >= 0.0 && u < 1.0) ? 1.0 : 0.0;
  return (u * cardinal(d - 1, u) + (d + 1 - u) * cardinal(d - 1, u - 1.0)) / d;
}

// Dense least squares min ||A x - y|| by Householder QR (A is rows x cols,
// row-major); returns the residual norm.
double lstsq(std::vector<double> A, std::vector<double> y, int rows, int cols,
             std::vector<double>& x) {
  for (int c = 0; c < cols; ++c) {
    double nrm = 0.0;
    for (int i = c; i < rows; ++i) nrm += A[i * cols + c] * A[i * cols + c];
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) continue;
    const double alpha = (A[c * cols + c] > 0) ? -nrm : nrm;
    std::vector<double> v(rows - c);
    for (int i = c; i < rows; ++i) v[i - c] = A[i * cols + c];
    v[0] -= alpha;
    double vv = 0.0;
    for (double t : v) vv += t * t;
    if (vv == 0.0) continue;
    for (int k = c; k < cols; ++k) {
      double s = 0.0;
      for (int i = c; i < rows; ++i) s += v[i - c] * A[i * cols + k];
      s = 2.0 * s / vv;
      for (int i = c; i < rows; ++i) A[i * cols + k] -= s * v[i - c];
    }
    double s = 0.0;
    for (int i = c; i < rows; ++i) s += v[i - c] * y[i];
    s = 2.0 * s / vv;
    for (int i = c; i < rows; ++i) y[i] -= s * v[i - c];
  }
  x.assign(cols, 0.0);
  for (int c = cols - 1; c >= 0; --c) {
    double s = y[c];
    for (int k = c + 1; k < cols; ++k) s -= A[c * cols + k] * x[k];
    x[c] = (A[c * cols + c] != 0.0) ? s / A[c * cols + c] : 0.0;
  }
  double r = 0.0;
  for (int i = cols; i < rows; ++i) r += y[i] * y[i];
  return std::sqrt(r);
}

// Banded SPD Cholesky: A given in DIA form (2p+1) x n; returns lower factor
// L[(i)*(p+1) + (i-j)] for j in [i-p, i].
bool band_cholesky(const std::vector<double>& band, int n, int p, std::vector<double>& L) {
  L.assign(size_t(n) * (p + 1), 0.0);
  auto Aij = [&](int i, int j) { return band[size_t(j - i + p) * n + i]; };
  for (int i = 0; i < n; ++i) {
    for (int j = std::max(0, i - p); j <= i; ++j) {
      double s = Aij(i, j);
      for (int k = std::max(0, i - p); k < j; ++k)
        s -= L[size_t(i) * (p + 1) + (i - k)] * L[size_t(j) * (p + 1) + (j - k)];
      if (i == j) {
        if (s <= 0.0) return false;
        L[size_t(i) * (p + 1)] = std::sqrt(s);
      } else {
        L[size_t(i) * (p + 1) + (i - j)] = s / L[size_t(j) * (p + 1)];
      }
    }
  }
  return true;
}

void band_cholesky_solve(const std::vector<double>& L, int n, int p, std::vector<double>& x) {
  for (int i = 0; i < n; ++i) {
    double s = x[i];
    for (int k = std::max(0, i - p); k < i; ++k) s -= L[size_t(i) * (p + 1) + (i - k)] * x[k];
    x[i] = s / L[size_t(i) * (p + 1)];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = x[i];
    for (int k = i + 1; k <= std::min(n - 1, i + p); ++k) s -= L[size_t(k) * (p + 1) + (k - i)] * x[k];
    x[i] = s / L[size_t(i) * (p + 1)];
  }
}

void band_matvec(const std::vector<double>& band, int n, int p, const double* x, double* y) {
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int o = -p; o <= p; ++o) {
      const int j = i + o;
      if (j >= 0 && j < n) s += band[size_t(o + p) * n + i] * x[j];
    }
    y[i] = s;
  }
}

// Cyclic Jacobi for a small symmetric matrix (row-major, in place); V gets
// the eigenvectors as columns.
void small_jacobi(std::vector<double>& A, int n, std::vector<double>& V) {
  V.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += A[i * n + j] * A[i * n + j];
        if (i != j) off += A[i * n + j] * A[i * n + j];
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (apq == 0.0) continue;
        const double tau = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
}

}  // namespace

bool fd_direction_setup(int n_el, int p, double coef, FdDirection& d, std::string& msg) {
  if (p < 1 || n_el <= p) {
    msg = "fd_setup: need p >= 1 and n_el > p";
    return false;
  }
  if ((n_el & (n_el - 1)) != 0 || n_el < 4 || n_el > 1024) {
    msg = "fd_setup: n_el must be a power of two in [4, 1024] (radix-2 FFT length 2*n_el)";
    return false;
  }
  const int N = n_el;
  d.n_el = n_el;
  d.p = p;
  d.N = N;
  d.n = n_el + p - 2;
  d.odd = (p % 2) == 1;
  d.n1 = d.odd ? N - 1 : N;
  d.n2 = d.odd ? p - 1 : p - 2;
  const int n = d.n, n1 = d.n1, n2 = d.n2;
  const auto knots = open_knots(n_el, p);
  const int nfull = n_el + p;

  // symbol sigma(theta) on the interpolation grid and g_j = sqrt(2)/sigma_j
  std::vector<double> uu, nu;
  for (int i = 0; i <= 2 * (p + 1); ++i) {
    const double u = d.odd ? double(i) : i + 0.5;
    if (u > 0.0 && u < p + 1.0) {
      uu.push_back(u);
      nu.push_back(cardinal(p, u));
    }
  }
  d.g.resize(n1);
  for (int j = 1; j <= n1; ++j) {
    const double th = kPi * j / N;
    double s = 0.0;
    for (size_t k = 0; k < uu.size(); ++k) s += nu[k] * std::cos(th * (uu[k] - 0.5 * (p + 1)));
    if (!(std::fabs(s) > 1e-12)) {
      msg = "fd_setup: vanishing interpolation symbol";
      return false;
    }
    d.g[j - 1] = std::sqrt(2.0) / s;
  }

  // E: translates k = -p .. N-1 (B_k supported on [k/N, (k+p+1)/N])
  std::vector<double> E(size_t(n) * n1, 0.0), dropped(2 * size_t(n1), 0.0);
  std::vector<double> vals(p + 1);
  const int q = d.odd ? (p - 1) / 2 : p / 2;
  for (int k = -p; k <= N - 1; ++k) {
    // fold the translate's centre index onto a basic centre, with sign
    const int m = d.odd ? k + q + 1 : k + q;
    int base = -1;
    double sgn = 1.0;
    if (d.odd) {
      int mm = m;
      if (mm < 0) { mm = -mm; sgn = -1.0; }
      if (mm > N) { mm = 2 * N - mm; sgn = -sgn; }
      if (mm == 0 || mm == N) continue;  // the sine vanishes there
      base = mm - 1;
    } else {
      int mm = m;
      if (mm < 0) { mm = -mm - 1; sgn = -1.0; }
      if (mm >= N) { mm = 2 * N - 1 - mm; sgn = -sgn; }
      base = mm;
    }
    // open-basis coefficients of B_k restricted to [0, 1]
    std::vector<std::pair<int, double>> coeffs;
    if (k >= 0 && k <= N - p - 1) {
      coeffs.push_back({k + p, 1.0});
    } else {
      const double a = std::max(0.0, double(k) / N), b = std::min(1.0, double(k + p + 1) / N);
      std::vector<int> cand;
      for (int l = 0; l < nfull; ++l)
        if (knots[l] < b && knots[l + p + 1] > a) cand.push_back(l);
      const int S = 8 * (p + 1);
      std::vector<double> A(size_t(S) * cand.size(), 0.0), y(S);
      for (int s = 0; s < S; ++s) {
        const double x = a + (b - a) * (s + 0.5) / S;
        const int span = find_span(knots, p, x);
        span_basis(knots, p, span, x, 0, vals.data());
        for (size_t c = 0; c < cand.size(); ++c) {
          const int loc = cand[c] - (span - p);
          A[s * cand.size() + c] = (loc >= 0 && loc <= p) ? vals[loc] : 0.0;
        }
        y[s] = cardinal(p, x * N - k);
      }
      std::vector<double> xs;
      const double res = lstsq(A, y, S, int(cand.size()), xs);
      if (res > 1e-10) {
        msg = "fd_setup: boundary translate not representable";
        return false;
      }
      for (size_t c = 0; c < cand.size(); ++c)
        if (std::fabs(xs[c]) > 1e-10) coeffs.push_back({cand[c], xs[c]});  // exact coefficients are O(1e-3) or more; drop least-squares noise
    }
    for (auto& lc : coeffs) {
      const int l = lc.first;
      if (l == 0) dropped[base] += sgn * lc.second;
      else if (l == nfull - 1) dropped[n1 + base] += sgn * lc.second;
      else E[size_t(l - 1) * n1 + base] += sgn * lc.second;
    }
  }
  for (double v : dropped)
    if (std::fabs(v) > 1e-9) {
      msg = "fd_setup: odd extension does not vanish at the boundary";
      return false;
    }
  // ELL forms of E and E^T
  int ke = 1, ket = 1;
  for (int i = 0; i < n; ++i) {
    int c = 0;
    for (int j = 0; j < n1; ++j) c += (E[size_t(i) * n1 + j] != 0.0);
    ke = std::max(ke, c);
  }
  for (int j = 0; j < n1; ++j) {
    int c = 0;
    for (int i = 0; i < n; ++i) c += (E[size_t(i) * n1 + j] != 0.0);
    ket = std::max(ket, c);
  }
  d.ke = ke;
  d.ket = ket;
  d.e_idx.assign(size_t(n) * ke, -1);
  d.e_val.assign(size_t(n) * ke, 0.0);
  d.et_idx.assign(size_t(n1) * ket, -1);
  d.et_val.assign(size_t(n1) * ket, 0.0);
  for (int i = 0; i < n; ++i) {
    int c = 0;
    for (int j = 0; j < n1; ++j)
      if (E[size_t(i) * n1 + j] != 0.0) {
        d.e_idx[size_t(i) * ke + c] = j;
        d.e_val[size_t(i) * ke + c] = E[size_t(i) * n1 + j];
        ++c;
      }
  }
  for (int j = 0; j < n1; ++j) {
    int c = 0;
    for (int i = 0; i < n; ++i)
      if (E[size_t(i) * n1 + j] != 0.0) {
        d.et_idx[size_t(j) * ket + c] = i;
        d.et_val[size_t(j) * ket + c] = E[size_t(i) * n1 + j];
        ++c;
      }
  }

  // unit L^2 norm (M-norm) of every approximate eigenvector function: column
  // k of V1 U1 is g_k E s_k with s_k the sine vector of the transform (DST-I
  // samples sin(pi j k / N) for odd p, DST-II samples sin(pi (2m+1) k / 2N)
  // for even p), so g_k becomes sign(g_k) / ||E s_k||_M
  {
    const double unit[4] = {1.0, 0.0, 0.0, 0.0};
    std::vector<double> Mb(size_t(2 * p + 1) * n), sk(n1), v(n), Mv(n);
    assemble_band(n_el, p, 0, unit, Mb.data());
    for (int k = 1; k <= n1; ++k) {
      for (int m = 0; m < n1; ++m)
        sk[m] = d.odd ? std::sin(kPi * double(m + 1) * k / N) : std::sin(kPi * double(2 * m + 1) * k / (2.0 * N));
      for (int i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int c = 0; c < ke; ++c) {
          const int j = d.e_idx[size_t(i) * ke + c];
          if (j >= 0) acc += d.e_val[size_t(i) * ke + c] * sk[j];
        }
        v[i] = acc;
      }
      band_matvec(Mb, n, p, v.data(), Mv.data());
      double nrm2 = 0.0;
      for (int i = 0; i < n; ++i) nrm2 += v[i] * Mv[i];
      if (!(nrm2 > 0.0)) {
        msg = "fd_setup: interpolated sine with zero norm";
        return false;
      }
      d.g[k - 1] = (d.g[k - 1] >= 0.0 ? 1.0 : -1.0) / std::sqrt(nrm2);
    }
  }

  // eigenvalue approximations on V_h1
  d.lam.assign(n, 0.0);
  for (int j = 1; j <= n1; ++j) d.lam[j - 1] = coef * (kPi * j) * (kPi * j);

  // V_h2 = M^{-1} D^T with the even-derivative constraints D, and its pencil
  d.v2u2.assign(size_t(n) * n2, 0.0);
  if (n2 > 0) {
    const double unit[4] = {1.0, 0.0, 0.0, 0.0};
    std::vector<double> Mb(size_t(2 * p + 1) * n), Kb(size_t(2 * p + 1) * n), L;
    assemble_band(n_el, p, 0, unit, Mb.data());
    assemble_band(n_el, p, 1, unit, Kb.data());
    if (!band_cholesky(Mb, n, p, L)) {
      msg = "fd_setup: mass matrix not positive definite";
      return false;
    }
    std::vector<double> V2(size_t(n) * n2);  // column-major n x n2
    int row = 0;
    for (int end = 0; end < 2; ++end)
      for (int k = 1; 2 * k <= p - 1; ++k) {
        std::vector<double> col(n);
        dirichlet_basis_at(n_el, p, end ? 1.0 : 0.0, 2 * k, col.data());
        band_cholesky_solve(L, n, p, col);
        std::copy(col.begin(), col.end(), V2.begin() + size_t(row) * n);
        ++row;
      }
    // small pencil (V2^T K V2, V2^T M V2)
    std::vector<double> K2(n2 * n2), M2(n2 * n2), tmp(n);
    for (int b = 0; b < n2; ++b) {
      band_matvec(Kb, n, p, &V2[size_t(b) * n], tmp.data());
      for (int a = 0; a < n2; ++a) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += V2[size_t(a) * n + i] * tmp[i];
        K2[a * n2 + b] = s;
      }
      band_matvec(Mb, n, p, &V2[size_t(b) * n], tmp.data());
      for (int a = 0; a < n2; ++a) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += V2[size_t(a) * n + i] * tmp[i];
        M2[a * n2 + b] = s;
      }
    }
    // M2 = C C^T (dense Cholesky), then eig of C^{-1} K2 C^{-T}
    std::vector<double> C(n2 * n2, 0.0);
    for (int i = 0; i < n2; ++i)
      for (int j = 0; j <= i; ++j) {
        double s = M2[i * n2 + j];
        for (int k = 0; k < j; ++k) s -= C[i * n2 + k] * C[j * n2 + k];
        if (i == j) {
          if (s <= 0) { msg = "fd_setup: V_h2 mass not SPD"; return false; }
          C[i * n2 + i] = std::sqrt(s);
        } else {
          C[i * n2 + j] = s / C[j * n2 + j];
        }
      }
    auto lower_solve = [&](std::vector<double>& X) {  // X <- C^{-1} X (n2 x n2 row-major)
      for (int c = 0; c < n2; ++c)
        for (int i = 0; i < n2; ++i) {
          double s = X[i * n2 + c];
          for (int k = 0; k < i; ++k) s -= C[i * n2 + k] * X[k * n2 + c];
          X[i * n2 + c] = s / C[i * n2 + i];
        }
    };
    std::vector<double> T = K2;
    lower_solve(T);  // C^{-1} K2
    std::vector<double> Tt(n2 * n2);
    for (int i = 0; i < n2; ++i)
      for (int j = 0; j < n2; ++j) Tt[i * n2 + j] = T[j * n2 + i];
    lower_solve(Tt);  // C^{-1} (C^{-1} K2)^T = C^{-1} K2 C^{-T}
    std::vector<double> Q;
    small_jacobi(Tt, n2, Q);
    std::vector<int> ord(n2);
    for (int i = 0; i < n2; ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return Tt[a * n2 + a] < Tt[b * n2 + b]; });
    // U2 = C^{-T} Q  (upper solve with C^T)
    std::vector<double> U2(n2 * n2);
    for (int c = 0; c < n2; ++c)
      for (int i = n2 - 1; i >= 0; --i) {
        double s = Q[i * n2 + ord[c]];
        for (int k = i + 1; k < n2; ++k) s -= C[k * n2 + i] * U2[k * n2 + c];
        U2[i * n2 + c] = s / C[i * n2 + i];
      }
    for (int c = 0; c < n2; ++c) {
      d.lam[n1 + c] = coef * Tt[ord[c] * n2 + ord[c]];
      for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int a = 0; a < n2; ++a) s += V2[size_t(a) * n + i] * U2[a * n2 + c];
        d.v2u2[size_t(c) * n + i] = s;
      }
    }
  }
  return true;
}

// ---------------------------------------------------------------------------
// exact eigenpairs (Algorithm 3's factorizations) for the exact-FD variant
// ---------------------------------------------------------------------------

bool fd_exact_pencil(int n_el, int p, double coef, std::vector<double>& C, std::vector<double>& L, int& n,
                     std::string& msg, int k0, int k1) {
  if (p < 1 || n_el <= p || n_el > 4096) {
    msg = "fd_setup_exact: need p >= 1 and p < n_el <= 4096";
    return false;
  }
  if ((k0 != 0 && k0 != 1) || (k1 != 0 && k1 != 1)) {
    msg = "fd_setup_exact: boundary flags must be 0 (Dirichlet) or 1 (Neumann)";
    return false;
  }
  n = n_el + p - 2 + k0 + k1;
  const double unit[4] = {1.0, 0.0, 0.0, 0.0};
  std::vector<double> Mb(size_t(2 * p + 1) * n), Kb(size_t(2 * p + 1) * n);
  assemble_band(n_el, p, 0, unit, Mb.data(), k0, k1);
  assemble_band(n_el, p, 1, unit, Kb.data(), k0, k1);
  if (!band_cholesky(Mb, n, p, L)) {
    msg = "fd_setup_exact: mass matrix not positive definite";
    return false;
  }
  auto lower_solve = [&](double* x) {  // x <- L^{-1} x
    for (int i = 0; i < n; ++i) {
      double s = x[i];
      for (int k = std::max(0, i - p); k < i; ++k) s -= L[size_t(i) * (p + 1) + (i - k)] * x[k];
      x[i] = s / L[size_t(i) * (p + 1)];
    }
  };
  // X = L^{-1} (coef K), column by column (K symmetric, banded)
  std::vector<double> X(size_t(n) * n, 0.0);
  for (int c = 0; c < n; ++c) {
    double* col = X.data() + size_t(c) * n;
    for (int o = -p; o <= p; ++o) {
      const int r = c - o;  // K[r, c] = band[(c - r + p) n + r]
      if (r >= 0 && r < n) col[r] = coef * Kb[size_t(o + p) * n + r];
    }
    lower_solve(col);
  }
  // C = L^{-1} X^T (= L^{-1} K L^{-T}), then symmetrized
  C.assign(size_t(n) * n, 0.0);
  std::vector<double> tmp(n);
  for (int c = 0; c < n; ++c) {
    for (int r = 0; r < n; ++r) tmp[r] = X[size_t(r) * n + c];
    lower_solve(tmp.data());
    for (int r = 0; r < n; ++r) C[size_t(c) * n + r] = tmp[r];
  }
  for (int c = 0; c < n; ++c)
    for (int r = c + 1; r < n; ++r) {
      const double v = 0.5 * (C[size_t(c) * n + r] + C[size_t(r) * n + c]);
      C[size_t(c) * n + r] = v;
      C[size_t(r) * n + c] = v;
    }
  return true;
}

// Appendix B on the space with boundary flags (k0, k1), built densely:
// V_h1 = {phi : phi^(d)(e) = 0 for the constrained orders d at each end e}
// (even orders >= 2 at a Dirichlet end, odd orders at a Neumann end, all
// d <= p - 1), spanned by Phi0 (combinations of the first e0 functions in
// the kernel of the constraints at 0), single functions in the middle and
// Phi1 (the last e1 functions, constraints at 1); the sines
// sqrt(2) sin((j - (k0+k1)/2) pi x + k0 pi/2) interpolated in V_h1 at the
// breakpoints (odd p; an end only where it is Neumann) or span midpoints
// (even p), each scaled to unit M-norm, with Lambda1 = ((j - (k0+k1)/2) pi)^2;
// V2 = M^{-1} D^T spans the M-orthogonal complement and carries the exact
// eigenpairs of its projected pencil.  Ut (n x n, column-major) =
// [V1 U1 | V2 U2] and lam (n) are for (coef K, M).
bool fd_approx_dense(int n_el, int p, double coef, int k0, int k1, std::vector<double>& Ut,
                     std::vector<double>& lam, int& n, std::string& msg) {
  if (p < 2 || n_el <= p || n_el > 4096) {
    msg = "fd_setup_bc: need p >= 2 and p < n_el <= 4096";
    return false;
  }
  if ((k0 != 0 && k0 != 1) || (k1 != 0 && k1 != 1)) {
    msg = "fd_setup_bc: boundary flags must be 0 (Dirichlet) or 1 (Neumann)";
    return false;
  }
  n = n_el + p - 2 + k0 + k1;
  const int n1 = (p % 2 == 1) ? n_el - 1 + k0 + k1 : n_el;
  const int n2 = n - n1;
  const int sh = 1 - k0;  // full-basis index of space index 0
  const double unit[4] = {1.0, 0.0, 0.0, 0.0};
  std::vector<double> Mb(size_t(2 * p + 1) * n), Kb(size_t(2 * p + 1) * n);
  assemble_band(n_el, p, 0, unit, Mb.data(), k0, k1);
  assemble_band(n_el, p, 1, unit, Kb.data(), k0, k1);
  std::vector<double> LM;
  if (!band_cholesky(Mb, n, p, LM)) {
    msg = "fd_setup_bc: mass matrix not positive definite";
    return false;
  }
  const auto kn = open_knots(n_el, p);
  // constraint rows (over the space's n functions) at an end
  auto orders = [&](int neumann) {
    std::vector<int> o;
    for (int d = neumann ? 1 : 2; d < p; d += 2) o.push_back(d);
    return o;
  };
  auto rows_at = [&](double x, int neumann) {
    const auto od = orders(neumann);
    const int span = find_span(kn, p, x);
    std::vector<double> vals(size_t(p + 1) * (p + 1));
    span_basis(kn, p, span, x, p, vals.data());
    std::vector<std::vector<double>> R;
    for (int d : od) {
      std::vector<double> r(n, 0.0);
      for (int a = 0; a <= p; ++a) {
        const int i = span - p + a - sh;
        if (i >= 0 && i < n) r[i] = vals[size_t(d) * (p + 1) + a];
      }
      R.push_back(r);
    }
    return R;
  };
  const auto D0 = rows_at(0.0, k0), D1 = rows_at(1.0, k1);
  if (int(D0.size() + D1.size()) != n2) {
    msg = "fd_setup_bc: constraint count does not match the interpolation points";
    return false;
  }
  const auto o0 = orders(k0), o1 = orders(k1);
  const int e0 = o0.empty() ? 0 : o0.back() + k0, e1 = o1.empty() ? 0 : o1.back() + k1;
  // kernel of a c x e block (rows of D restricted to columns [c0, c0 + e)):
  // the last e - c columns of the full Q of a Householder QR of its transpose
  auto kernel = [&](const std::vector<std::vector<double>>& D, int col0, int e) {
    const int c = int(D.size());
    std::vector<double> A(size_t(e) * c);  // e x c, column-major
    for (int r = 0; r < c; ++r)
      for (int i = 0; i < e; ++i) A[size_t(r) * e + i] = D[r][col0 + i];
    std::vector<double> Q(size_t(e) * e, 0.0);
    for (int i = 0; i < e; ++i) Q[size_t(i) * e + i] = 1.0;
    for (int k = 0; k < c; ++k) {
      std::vector<double> v(e, 0.0);
      double nrm = 0.0;
      for (int i = k; i < e; ++i) nrm += A[size_t(k) * e + i] * A[size_t(k) * e + i];
      nrm = std::sqrt(nrm);
      if (nrm == 0.0) continue;
      const double alpha = A[size_t(k) * e + k] > 0 ? -nrm : nrm;
      for (int i = k; i < e; ++i) v[i] = A[size_t(k) * e + i];
      v[k] -= alpha;
      double vv = 0.0;
      for (double t : v) vv += t * t;
      if (vv == 0.0) continue;
      for (int j = k; j < c; ++j) {  // A <- H A
        double sdot = 0.0;
        for (int i = k; i < e; ++i) sdot += v[i] * A[size_t(j) * e + i];
        sdot = 2.0 * sdot / vv;
        for (int i = k; i < e; ++i) A[size_t(j) * e + i] -= sdot * v[i];
      }
      for (int j = 0; j < e; ++j) {  // G <- H G: G = H_{c-1} ... H_0 = Q^T
        double sdot = 0.0;
        for (int i = k; i < e; ++i) sdot += Q[size_t(i) * e + j] * v[i];
        sdot = 2.0 * sdot / vv;
        for (int i = k; i < e; ++i) Q[size_t(i) * e + j] -= sdot * v[i];
      }
    }
    return Q;  // Q^T, row-major e x e: kernel vector j (j >= c) is its row j
  };
  // V1 as (row, column, value) triplets
  struct Ent { int r, c; double v; };
  std::vector<Ent> V1;
  int col = 0;
  if (e0 > 0) {
    const auto Q = kernel(D0, 0, e0);
    for (int j = int(D0.size()); j < e0; ++j, ++col)
      for (int i = 0; i < e0; ++i) V1.push_back({i, col, Q[size_t(j) * e0 + i]});
  }
  for (int r = e0; r < n - e1; ++r, ++col) V1.push_back({r, col, 1.0});
  if (e1 > 0) {
    const auto Q = kernel(D1, n - e1, e1);
    for (int j = int(D1.size()); j < e1; ++j, ++col)
      for (int i = 0; i < e1; ++i) V1.push_back({n - e1 + i, col, Q[size_t(j) * e1 + i]});
  }
  if (col != n1) {
    msg = "fd_setup_bc: V_h1 basis has the wrong dimension";
    return false;
  }
  // A = Bx V1 (n1 x n1, row-major): the V_h1 basis at the interpolation points
  std::vector<double> xs(n1);
  for (int i = 0; i < n1; ++i) xs[i] = (p % 2 == 1) ? double(i + 1 - k0) / n_el : (i + 0.5) / n_el;
  std::vector<std::vector<Ent>> byrow(n);
  for (const auto& t : V1) byrow[t.r].push_back(t);
  std::vector<double> A(size_t(n1) * n1, 0.0), vals(p + 1);
  for (int i = 0; i < n1; ++i) {
    const int span = find_span(kn, p, xs[i]);
    span_basis(kn, p, span, xs[i], 0, vals.data());
    for (int a = 0; a <= p; ++a) {
      const int r = span - p + a - sh;
      if (r < 0 || r >= n) continue;
      for (const auto& t : byrow[r]) A[size_t(i) * n1 + t.c] += vals[a] * t.v;
    }
  }
  // U1 = A^{-1} Udft (LU with partial pivoting), row-major n1 x n1
  const double kPi = 3.14159265358979323846, kap = 0.5 * (k0 + k1);
  std::vector<double> U1(size_t(n1) * n1);
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n1; ++j)
      U1[size_t(i) * n1 + j] = std::sqrt(2.0) * std::sin(kPi * (j + 1 - kap) * xs[i] + 0.5 * kPi * k0);
  std::vector<int> piv(n1);
  for (int k = 0; k < n1; ++k) {
    int pr = k;
    for (int i = k + 1; i < n1; ++i)
      if (std::fabs(A[size_t(i) * n1 + k]) > std::fabs(A[size_t(pr) * n1 + k])) pr = i;
    if (A[size_t(pr) * n1 + k] == 0.0) {
      msg = "fd_setup_bc: singular collocation matrix";
      return false;
    }
    if (pr != k) {
      for (int j = 0; j < n1; ++j) std::swap(A[size_t(k) * n1 + j], A[size_t(pr) * n1 + j]);
      for (int j = 0; j < n1; ++j) std::swap(U1[size_t(k) * n1 + j], U1[size_t(pr) * n1 + j]);
    }
    const double d = A[size_t(k) * n1 + k];
    for (int i = k + 1; i < n1; ++i) {
      const double f = A[size_t(i) * n1 + k] / d;
      if (f == 0.0) continue;
      for (int j = k + 1; j < n1; ++j) A[size_t(i) * n1 + j] -= f * A[size_t(k) * n1 + j];
      for (int j = 0; j < n1; ++j) U1[size_t(i) * n1 + j] -= f * U1[size_t(k) * n1 + j];
    }
  }
  for (int k = n1 - 1; k >= 0; --k) {
    for (int j = 0; j < n1; ++j) {
      double sacc = U1[size_t(k) * n1 + j];
      for (int i = k + 1; i < n1; ++i) sacc -= A[size_t(k) * n1 + i] * U1[size_t(i) * n1 + j];
      U1[size_t(k) * n1 + j] = sacc / A[size_t(k) * n1 + k];
    }
  }
  // W1 = V1 U1, columns scaled to unit M-norm
  Ut.assign(size_t(n) * n, 0.0);
  lam.assign(n, 0.0);
  for (const auto& t : V1)
    for (int j = 0; j < n1; ++j) Ut[size_t(j) * n + t.r] += t.v * U1[size_t(t.c) * n1 + j];
  std::vector<double> mw(n);
  for (int j = 0; j < n1; ++j) {
    double* w = Ut.data() + size_t(j) * n;
    band_matvec(Mb, n, p, w, mw.data());
    double nm = 0.0;
    for (int i = 0; i < n; ++i) nm += w[i] * mw[i];
    if (!(nm > 0.0)) {
      msg = "fd_setup_bc: an interpolated sine has zero norm";
      return false;
    }
    const double sc = 1.0 / std::sqrt(nm);
    for (int i = 0; i < n; ++i) w[i] *= sc;
    const double f = kPi * (j + 1 - kap);
    lam[j] = coef * f * f;
  }
  if (n2 > 0) {
    // V2 = M^{-1} D^T, then the pencil (V2^T K V2, V2^T M V2) by Cholesky and Jacobi
    std::vector<std::vector<double>> D(D0);
    D.insert(D.end(), D1.begin(), D1.end());
    std::vector<std::vector<double>> V2(n2);
    for (int c = 0; c < n2; ++c) {
      V2[c] = D[c];
      band_cholesky_solve(LM, n, p, V2[c]);
    }
    std::vector<double> K2(size_t(n2) * n2), M2(size_t(n2) * n2), kv(n), mv(n);
    for (int b = 0; b < n2; ++b) {
      band_matvec(Kb, n, p, V2[b].data(), kv.data());
      band_matvec(Mb, n, p, V2[b].data(), mv.data());
      for (int a = 0; a < n2; ++a) {
        double sk = 0.0, sm = 0.0;
        for (int i = 0; i < n; ++i) {
          sk += V2[a][i] * kv[i];
          sm += V2[a][i] * mv[i];
        }
        K2[size_t(a) * n2 + b] = sk;
        M2[size_t(a) * n2 + b] = sm;
      }
    }
    std::vector<double> L2(size_t(n2) * n2, 0.0);  // M2 = L2 L2^T, row-major lower
    for (int i = 0; i < n2; ++i)
      for (int j = 0; j <= i; ++j) {
        double sacc = M2[size_t(i) * n2 + j];
        for (int k = 0; k < j; ++k) sacc -= L2[size_t(i) * n2 + k] * L2[size_t(j) * n2 + k];
        if (i == j) {
          if (!(sacc > 0.0)) {
            msg = "fd_setup_bc: V2 Gram matrix not positive definite";
            return false;
          }
          L2[size_t(i) * n2 + i] = std::sqrt(sacc);
        } else {
          L2[size_t(i) * n2 + j] = sacc / L2[size_t(j) * n2 + j];
        }
      }
    // C2 = L2^{-1} K2 L2^{-T}
    std::vector<double> X(K2);
    for (int c = 0; c < n2; ++c)  // X <- L2^{-1} X (column c)
      for (int i = 0; i < n2; ++i) {
        double sacc = X[size_t(i) * n2 + c];
        for (int k = 0; k < i; ++k) sacc -= L2[size_t(i) * n2 + k] * X[size_t(k) * n2 + c];
        X[size_t(i) * n2 + c] = sacc / L2[size_t(i) * n2 + i];
      }
    std::vector<double> C2(size_t(n2) * n2);
    for (int r = 0; r < n2; ++r)  // C2 <- X L2^{-T} (row r: solve L2 y = X[r, :]^T)
      for (int i = 0; i < n2; ++i) {
        double sacc = X[size_t(r) * n2 + i];
        for (int k = 0; k < i; ++k) sacc -= L2[size_t(i) * n2 + k] * C2[size_t(r) * n2 + k];
        C2[size_t(r) * n2 + i] = sacc / L2[size_t(i) * n2 + i];
      }
    for (int a = 0; a < n2; ++a)
      for (int b = a + 1; b < n2; ++b) {
        const double v = 0.5 * (C2[size_t(a) * n2 + b] + C2[size_t(b) * n2 + a]);
        C2[size_t(a) * n2 + b] = C2[size_t(b) * n2 + a] = v;
      }
    std::vector<double> Qs;
    small_jacobi(C2, n2, Qs);
    for (int c = 0; c < n2; ++c) {
      // U2 column c = L2^{-T} Qs[:, c]
      std::vector<double> u(n2);
      for (int i = n2 - 1; i >= 0; --i) {
        double sacc = Qs[size_t(i) * n2 + c];
        for (int k = i + 1; k < n2; ++k) sacc -= L2[size_t(k) * n2 + i] * u[k];
        u[i] = sacc / L2[size_t(i) * n2 + i];
      }
      double* out = Ut.data() + size_t(n1 + c) * n;
      for (int b = 0; b < n2; ++b)
        for (int i = 0; i < n; ++i) out[i] += V2[b][i] * u[b];
      lam[n1 + c] = coef * C2[size_t(c) * n2 + c];
    }
  }
  return true;
}

void fd_exact_vectors(const std::vector<double>& L, int n, int p, double* Q) {
  for (int c = 0; c < n; ++c) {
    double* x = Q + size_t(c) * n;
    for (int i = n - 1; i >= 0; --i) {
      double s = x[i];
      for (int k = i + 1; k <= std::min(n - 1, i + p); ++k) s -= L[size_t(k) * (p + 1) + (k - i)] * x[k];
      x[i] = s / L[size_t(i) * (p + 1)];
    }
  }
}

}  // namespace tk
