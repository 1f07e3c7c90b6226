// Host setup: univariate B-splines on open uniform knot vectors and the 1D
// Galerkin integrals of the weighted matrices and load vectors.
//
// Sec. 2.1 of the paper defines the knot vectors and the B-splines; the
// weighted univariate integrals int delta(b_i) delta(b_j) w dx are those of
// Appendix A.  Values and derivatives on a knot span are computed with the
// triangular scheme of de Boor (all p+1 nonzero functions at once) and the
// integrals with Gauss-Legendre quadrature, p + 5 points per span.
#include <cmath>
#include <cstring>
#include <vector>

#include "tk_internal.h"

namespace tk {

std::vector<double> open_knots(int n_el, int p) {
  std::vector<double> k;
  k.reserve(n_el + 2 * p + 1);
  for (int i = 0; i <= p; ++i) k.push_back(0.0);
  for (int i = 1; i < n_el; ++i) k.push_back(double(i) / n_el);
  for (int i = 0; i <= p; ++i) k.push_back(1.0);
  return k;
}

int find_span(const std::vector<double>& knots, int p, double x) {
  const int m = int(knots.size()) - p - 1;  // number of basis functions
  if (x >= knots[m]) return m - 1;         // right end: last non-empty span
  if (x <= knots[p]) return p;
  int lo = p, hi = m;                      // knots[lo] <= x < knots[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (x < knots[mid]) hi = mid; else lo = mid;
  }
  return lo;
}

void span_basis(const std::vector<double>& knots, int p, int span, double x,
                int nder, double* out) {
  // ndu: upper triangle holds basis values of increasing degree, lower
  // triangle the knot differences used as denominators.
  std::vector<double> ndu((p + 1) * (p + 1)), left(p + 1), right(p + 1);
  auto NDU = [&](int i, int j) -> double& { return ndu[i * (p + 1) + j]; };
  NDU(0, 0) = 1.0;
  for (int j = 1; j <= p; ++j) {
    left[j] = x - knots[span + 1 - j];
    right[j] = knots[span + j] - x;
    double saved = 0.0;
    for (int r = 0; r < j; ++r) {
      NDU(j, r) = right[r + 1] + left[j - r];
      const double t = NDU(r, j - 1) / NDU(j, r);
      NDU(r, j) = saved + right[r + 1] * t;
      saved = left[j - r] * t;
    }
    NDU(j, j) = saved;
  }
  for (int r = 0; r <= p; ++r) out[r] = NDU(r, p);
  if (nder == 0) return;
  std::vector<double> a(2 * (p + 1));
  auto A = [&](int s, int j) -> double& { return a[s * (p + 1) + j]; };
  for (int r = 0; r <= p; ++r) {
    int s1 = 0, s2 = 1;
    A(0, 0) = 1.0;
    for (int k = 1; k <= nder; ++k) {
      double d = 0.0;
      const int rk = r - k, pk = p - k;
      if (k > p) { out[k * (p + 1) + r] = 0.0; continue; }
      if (r >= k) {
        A(s2, 0) = A(s1, 0) / NDU(pk + 1, rk);
        d = A(s2, 0) * NDU(rk, pk);
      }
      const int j1 = (rk >= -1) ? 1 : -rk;
      const int j2 = (r - 1 <= pk) ? k - 1 : p - r;
      for (int j = j1; j <= j2; ++j) {
        A(s2, j) = (A(s1, j) - A(s1, j - 1)) / NDU(pk + 1, rk + j);
        d += A(s2, j) * NDU(rk + j, pk);
      }
      if (r <= pk) {
        A(s2, k) = -A(s1, k - 1) / NDU(pk + 1, r);
        d += A(s2, k) * NDU(r, pk);
      }
      out[k * (p + 1) + r] = d;
      std::swap(s1, s2);
    }
  }
  double fac = p;
  for (int k = 1; k <= nder; ++k) {
    for (int r = 0; r <= p; ++r) out[k * (p + 1) + r] *= (k <= p ? fac : 0.0);
    fac *= (p - k);
  }
}

void gauss_legendre(int nq, std::vector<double>& x, std::vector<double>& w) {
  x.assign(nq, 0.0);
  w.assign(nq, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < nq; ++i) {
    double z = std::cos(pi * (i + 0.75) / (nq + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;  // Legendre recurrence
      for (int k = 2; k <= nq; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (nq == 1) { p1 = z; p0 = 1.0; }
      dp = nq * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= nq; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    if (nq == 1) { p1 = z; p0 = 1.0; }
    dp = nq * (z * p1 - p0) / (z * z - 1.0);
    x[nq - 1 - i] = z;
    w[nq - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

static inline double weight_at(const double w[4], double x) {
  return w[0] + w[1] * std::cos(w[2] * x + w[3]);
}

// w(x) = sum_m c[m] T_m(2x - 1) (three-term recurrence)
static double cheb_weight(const double* c, int nc, double x) {
  const double t = 2.0 * x - 1.0;
  double t0 = 1.0, t1 = t, s = nc > 0 ? c[0] : 0.0;
  if (nc > 1) s += c[1] * t1;
  for (int m = 2; m < nc; ++m) {
    const double t2 = 2.0 * t * t1 - t0;
    s += c[m] * t2;
    t0 = t1;
    t1 = t2;
  }
  return s;
}

void assemble_band_cheb(int n_el, int p, int kind, const double* c, int nc, double* band, int k0, int k1) {
  const int n = n_el + p - 2 + k0 + k1;
  const int sh = 1 - k0;
  const int nb = 2 * p + 1;
  std::memset(band, 0, sizeof(double) * nb * n);
  const auto kn = open_knots(n_el, p);
  std::vector<double> gx, gw;
  // exact for the polynomial weight of degree nc - 1 times the basis products
  gauss_legendre(p + 1 + (nc + 1) / 2 + 2, gx, gw);
  const int da = (kind == 1 || kind == 2) ? 1 : 0;
  const int db = (kind == 1 || kind == 3) ? 1 : 0;
  std::vector<double> vals(2 * (p + 1));
  const double h = 1.0 / n_el;
  for (int e = 0; e < n_el; ++e) {
    const int span = e + p;
    for (size_t q = 0; q < gx.size(); ++q) {
      const double x = e * h + 0.5 * h * (gx[q] + 1.0);
      const double wq = 0.5 * h * gw[q] * cheb_weight(c, nc, x);
      span_basis(kn, p, span, x, 1, vals.data());
      for (int a = 0; a <= p; ++a) {
        const int i = span - p + a - sh;
        if (i < 0 || i >= n) continue;
        const double va = vals[da * (p + 1) + a];
        for (int b = 0; b <= p; ++b) {
          const int j = span - p + b - sh;
          if (j < 0 || j >= n) continue;
          band[(j - i + p) * n + i] += wq * va * vals[db * (p + 1) + b];
        }
      }
    }
  }
}

void load_vector_cheb(int n_el, int p, const double* c, int nc, double* F, int k0, int k1) {
  const int n = n_el + p - 2 + k0 + k1;
  const int sh = 1 - k0;
  std::memset(F, 0, sizeof(double) * n);
  const auto kn = open_knots(n_el, p);
  std::vector<double> gx, gw;
  gauss_legendre(p + 1 + (nc + 1) / 2 + 2, gx, gw);
  std::vector<double> vals(p + 1);
  const double h = 1.0 / n_el;
  for (int e = 0; e < n_el; ++e) {
    const int span = e + p;
    for (size_t q = 0; q < gx.size(); ++q) {
      const double x = e * h + 0.5 * h * (gx[q] + 1.0);
      const double wq = 0.5 * h * gw[q] * cheb_weight(c, nc, x);
      span_basis(kn, p, span, x, 0, vals.data());
      for (int a = 0; a <= p; ++a) {
        const int i = span - p + a - sh;
        if (i >= 0 && i < n) F[i] += wq * vals[a];
      }
    }
  }
}

void assemble_band(int n_el, int p, int kind, const double weight[4], double* band, int k0, int k1) {
  const int n = n_el + p - 2 + k0 + k1;
  const int sh = 1 - k0;  // full-basis index of space index 0
  const int nb = 2 * p + 1;
  std::memset(band, 0, sizeof(double) * nb * n);
  const auto kn = open_knots(n_el, p);
  std::vector<double> gx, gw;
  gauss_legendre(p + 5, gx, gw);
  const int da = (kind == 1 || kind == 2) ? 1 : 0;  // derivative on test function i
  const int db = (kind == 1 || kind == 3) ? 1 : 0;  // derivative on trial function j
  std::vector<double> vals(2 * (p + 1));
  const double h = 1.0 / n_el;
  for (int e = 0; e < n_el; ++e) {
    const int span = e + p;
    const double x0 = e * h;
    for (size_t q = 0; q < gx.size(); ++q) {
      const double x = x0 + 0.5 * h * (gx[q] + 1.0);
      const double wq = 0.5 * h * gw[q] * weight_at(weight, x);
      span_basis(kn, p, span, x, 1, vals.data());
      for (int a = 0; a <= p; ++a) {
        const int i = span - p + a - sh;  // space index (full index - sh)
        if (i < 0 || i >= n) continue;
        const double va = vals[da * (p + 1) + a];
        for (int b = 0; b <= p; ++b) {
          const int j = span - p + b - sh;
          if (j < 0 || j >= n) continue;
          const int o = j - i;
          band[(o + p) * n + i] += wq * va * vals[db * (p + 1) + b];
        }
      }
    }
  }
}

void load_vector(int n_el, int p, const double weight[4], double* F) {
  const int n = n_el + p - 2;
  std::memset(F, 0, sizeof(double) * n);
  const auto kn = open_knots(n_el, p);
  std::vector<double> gx, gw;
  gauss_legendre(p + 5, gx, gw);
  std::vector<double> vals(p + 1);
  const double h = 1.0 / n_el;
  for (int e = 0; e < n_el; ++e) {
    const int span = e + p;
    for (size_t q = 0; q < gx.size(); ++q) {
      const double x = e * h + 0.5 * h * (gx[q] + 1.0);
      const double wq = 0.5 * h * gw[q] * weight_at(weight, x);
      span_basis(kn, p, span, x, 0, vals.data());
      for (int a = 0; a <= p; ++a) {
        const int i = span - p + a - 1;
        if (i >= 0 && i < n) F[i] += wq * vals[a];
      }
    }
  }
}

void basis_values(int n_el, int p, int k0, int k1, int der, int npts, const double* x, double* out) {
  const int n = n_el + p - 2 + k0 + k1;
  const int sh = 1 - k0;
  std::memset(out, 0, sizeof(double) * size_t(npts) * n);
  const auto kn = open_knots(n_el, p);
  std::vector<double> tmp((der + 1) * (p + 1));
  for (int q = 0; q < npts; ++q) {
    const int span = find_span(kn, p, x[q]);
    span_basis(kn, p, span, x[q], der, tmp.data());
    for (int a = 0; a <= p; ++a) {
      const int i = span - p + a - sh;
      if (i >= 0 && i < n) out[q + size_t(npts) * i] = tmp[der * (p + 1) + a];
    }
  }
}

void dirichlet_basis_at(int n_el, int p, double x, int der, double* vals) {
  const int n = n_el + p - 2;
  for (int i = 0; i < n; ++i) vals[i] = 0.0;
  const auto kn = open_knots(n_el, p);
  const int span = find_span(kn, p, x);
  std::vector<double> tmp((der + 1) * (p + 1));
  span_basis(kn, p, span, x, der, tmp.data());
  for (int a = 0; a <= p; ++a) {
    const int i = span - p + a - 1;
    if (i >= 0 && i < n) vals[i] = tmp[der * (p + 1) + a];
  }
}

}  // namespace tk
