// Host setup: best uniform exponential sums s_R(x) = sum_j omega_j exp(-alpha_j x)
// for 1/x on [1, M] (Sec. 4.2, Proposition 1), and R_P = min{R : E_R(M) <= eps/M}
// (eq. estimate_prec_rel).
//
// The minimax parameters are characterised by equioscillation of the error
// e(x) = 1/x - s_R(x) at 2R+1 points of [1, M]; they are computed by the
// Remez exchange: Newton's method on e(x_i) = (-1)^i E for the current
// reference x_0 < ... < x_2R, followed by moving the reference to the
// alternating extrema of the new error.  Parameters are kept as
// a_j = log alpha_j and b_j = log omega_j (positivity by construction).
// Starting values: R = 1 from the trapezoidal (sinc) rule for
// 1/x = int exp(t - x e^t) dt; R -> R+1 by extending the R-term optimum
// (its node spacings are kept from the slow end and one node is added at the
// fast end), with simpler extensions as alternatives.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "tk_internal.h"

namespace tk {
namespace {

using Vec = std::vector<double>;
constexpr int kGrid = 6000;

double err_at(const Vec& a, const Vec& b, double x) {
  double s = 0.0;
  for (size_t j = 0; j < a.size(); ++j) s += std::exp(b[j] - std::exp(a[j]) * x);
  return 1.0 / x - s;
}

// first and second derivative of e with respect to t = log x
void err_dt(const Vec& a, const Vec& b, double x, double& d1, double& d2) {
  double s1 = 0.0, s2 = 0.0;
  for (size_t j = 0; j < a.size(); ++j) {
    const double al = std::exp(a[j]);
    const double t = std::exp(b[j] - al * x) * al;
    s1 += t;
    s2 += t * al;
  }
  d1 = -1.0 / x + x * s1;
  d2 = 1.0 / x + x * s1 - x * x * s2;
}

Vec extrema(const Vec& a, const Vec& b, double M) {
  const double L = std::log(M);
  Vec t(kGrid), e(kGrid);
  for (int i = 0; i < kGrid; ++i) {
    t[i] = L * i / (kGrid - 1);
    e[i] = err_at(a, b, std::exp(t[i]));
  }
  Vec pts;
  int start = 0;
  for (int i = 1; i <= kGrid; ++i) {
    const bool cut = (i == kGrid) || ((e[i] >= 0) != (e[i - 1] >= 0));
    if (!cut) continue;
    int j = start;
    for (int k = start; k < i; ++k)
      if (std::fabs(e[k]) > std::fabs(e[j])) j = k;
    double tt = t[j];
    if (j > 0 && j < kGrid - 1) {
      const double lo = t[j - 1], hi = t[j + 1];
      for (int it = 0; it < 30; ++it) {
        double d1, d2;
        err_dt(a, b, std::exp(tt), d1, d2);
        if (d2 == 0.0) break;
        double tn = std::min(std::max(tt - d1 / d2, lo), hi);
        const bool done = std::fabs(tn - tt) < 1e-14;
        tt = tn;
        if (done) break;
      }
    }
    pts.push_back(std::exp(tt));
    start = i;
  }
  return pts;
}

// Solve A x = r in place (partial pivoting); false if singular.
bool lu_solve(std::vector<double>& A, Vec& r, int n) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int i = c + 1; i < n; ++i)
      if (std::fabs(A[i * n + c]) > std::fabs(A[piv * n + c])) piv = i;
    if (A[piv * n + c] == 0.0) return false;
    if (piv != c) {
      for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[piv * n + k]);
      std::swap(r[c], r[piv]);
    }
    for (int i = c + 1; i < n; ++i) {
      const double f = A[i * n + c] / A[c * n + c];
      if (f == 0.0) continue;
      for (int k = c; k < n; ++k) A[i * n + k] -= f * A[c * n + k];
      r[i] -= f * r[c];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = r[i];
    for (int k = i + 1; k < n; ++k) s -= A[i * n + k] * r[k];
    r[i] = s / A[i * n + i];
  }
  return true;
}

double residual(const Vec& z, int R, const Vec& xr, Vec& f) {
  const int n = 2 * R + 1;
  f.assign(n, 0.0);
  double nrm = 0.0;
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 0; j < R; ++j) s += std::exp(z[R + j] - std::exp(z[j]) * xr[i]);
    const double sg = (i % 2 == 0) ? 1.0 : -1.0;
    f[i] = (1.0 / xr[i] - s - sg * z[2 * R]) * xr[i];
    if (!std::isfinite(f[i])) return INFINITY;
    nrm += f[i] * f[i];
  }
  return std::sqrt(nrm);
}

// Newton on the reference equations; z = (a, b, E).
bool solve_reference(Vec& z, int R, const Vec& xr) {
  const int n = 2 * R + 1;
  Vec f, fn, dz(n), zn(n);
  double f0 = residual(z, R, xr, f);
  if (!std::isfinite(f0)) return false;
  std::vector<double> J(n * n);
  for (int it = 0; it < 60; ++it) {
    for (int i = 0; i < n; ++i) {
      const double x = xr[i];
      for (int j = 0; j < R; ++j) {
        const double al = std::exp(z[j]);
        const double tj = std::exp(z[R + j] - al * x);
        J[i * n + j] = tj * al * x * x;      // d/da_j (row scaled by x)
        J[i * n + R + j] = -tj * x;          // d/db_j
      }
      J[i * n + 2 * R] = -((i % 2 == 0) ? 1.0 : -1.0) * x;
    }
    for (int i = 0; i < n; ++i) dz[i] = -f[i];
    if (!lu_solve(J, dz, n)) return false;
    double mx = 0.0;
    for (int j = 0; j < 2 * R; ++j) mx = std::max(mx, std::fabs(dz[j]));
    double lam = std::min(1.0, 2.0 / std::max(mx, 1e-300));
    double fnew;
    while (true) {
      for (int i = 0; i < n; ++i) zn[i] = z[i] + lam * dz[i];
      fnew = residual(zn, R, xr, fn);
      if (std::isfinite(fnew) && fnew < f0 * (1.0 - 1e-4 * lam)) break;
      lam *= 0.5;
      if (lam < 1e-6) return f0 < 1e-10;
    }
    double step = 0.0, zn2 = 0.0;
    for (int i = 0; i < n; ++i) {
      step += (lam * dz[i]) * (lam * dz[i]);
      zn2 += zn[i] * zn[i];
    }
    z = zn;
    f = fn;
    f0 = fnew;
    if (std::sqrt(step) < 1e-14 * (1.0 + std::sqrt(zn2))) break;
  }
  return f0 < 1e-10;
}

struct Sol {
  Vec a, b;
  double E = 0.0;
  Vec xr;
};

bool remez(const Vec& a0, const Vec& b0, double M, const Vec* xr0, Sol& out) {
  const int R = int(a0.size());
  Vec xr = xr0 ? *xr0 : extrema(a0, b0, M);
  if (int(xr.size()) != 2 * R + 1) return false;
  Vec z(2 * R + 1);
  for (int j = 0; j < R; ++j) { z[j] = a0[j]; z[R + j] = b0[j]; }
  z[2 * R] = 0.0;
  const double L = std::log(M);
  for (int it = 0; it < 80; ++it) {
    if (!solve_reference(z, R, xr)) return false;
    Vec a(z.begin(), z.begin() + R), b(z.begin() + R, z.begin() + 2 * R);
    Vec xn = extrema(a, b, M);
    if (int(xn.size()) != 2 * R + 1) return false;
    double emax = 0.0;
    for (double x : xn) emax = std::max(emax, std::fabs(err_at(a, b, x)));
    for (int i = 0; i < 4 * kGrid; ++i)
      emax = std::max(emax, std::fabs(err_at(a, b, std::exp(L * i / (4 * kGrid - 1)))));
    const double E = std::fabs(z[2 * R]);
    if (emax - E <= 1e-7 * E) {
      out.a = a;
      out.b = b;
      out.E = E;
      out.xr = xn;
      return true;
    }
    xr = xn;
  }
  return false;
}

bool fresh(int R, double M, Sol& out) {
  const double L = std::log(M);
  double best = INFINITY;
  Vec ba, bb;
  Vec a(R), b(R);
  for (int i0 = 0; i0 < 60; ++i0) {
    const double t0 = (-L - 3.0) + (L + 5.0) * i0 / 59.0;
    for (int ih = 0; ih < 28; ++ih) {
      const double h = 0.3 + 2.7 * ih / 27.0;
      for (int j = 0; j < R; ++j) { a[j] = t0 + h * j; b[j] = std::log(h) + a[j]; }
      double v = 0.0;
      for (int i = 0; i < 2000; ++i)
        v = std::max(v, std::fabs(err_at(a, b, std::exp(L * i / 1999.0))));
      if (v < best) { best = v; ba = a; bb = b; }
    }
  }
  return remez(ba, bb, M, nullptr, out);
}

std::vector<std::pair<Vec, Vec>> grow_candidates(Vec a, Vec b) {
  const int R = int(a.size());
  std::vector<int> ord(R);
  for (int i = 0; i < R; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int i, int j) { return a[i] < a[j]; });
  Vec as(R), bs(R);
  for (int i = 0; i < R; ++i) { as[i] = a[ord[i]]; bs[i] = b[ord[i]]; }
  std::vector<std::pair<Vec, Vec>> out;
  if (R >= 3) {  // keep spacings from the slow end, add a node at the fast end
    Vec d(R - 1), c(R);
    for (int i = 0; i + 1 < R; ++i) d[i] = as[i + 1] - as[i];
    for (int i = 0; i < R; ++i) c[i] = bs[i] - as[i];
    Vec dn(d.begin(), d.end() - 1);
    dn.push_back(d[R - 3]);
    dn.push_back(d[R - 2]);
    Vec an(R + 1), cn(c.begin(), c.end() - 1);
    an[R] = as[R - 1] + 0.04;
    for (int i = R - 1; i >= 0; --i) an[i] = an[i + 1] - dn[i];
    cn.push_back(2.0 * c[R - 2] - c[R - 3]);
    cn.push_back(c[R - 1]);
    Vec bn(R + 1);
    for (int i = 0; i <= R; ++i) bn[i] = an[i] + cn[i];
    out.push_back({an, bn});
  }
  if (R >= 2) {
    Vec an(R + 1), bn(R + 1);
    for (int i = 0; i <= R; ++i) {  // interpolate over a normalised index
      const double s = double(i) * (R - 1) / R;
      const int k = std::min(int(s), R - 2);
      const double f = s - k;
      an[i] = (1 - f) * as[k] + f * as[k + 1];
      bn[i] = (1 - f) * bs[k] + f * bs[k + 1] + std::log(double(R) / (R + 1));
    }
    out.push_back({an, bn});
    Vec al = as, bl = bs;
    al.insert(al.begin(), as[0] - (as[1] - as[0]));
    bl.insert(bl.begin(), bs[0] - (bs[1] - bs[0]));
    out.push_back({al, bl});
    Vec ar = as, br = bs;
    ar.push_back(as[R - 1] + (as[R - 1] - as[R - 2]));
    br.push_back(bs[R - 1] + (bs[R - 1] - bs[R - 2]));
    out.push_back({ar, br});
  }
  for (double dd : {0.5, 1.0, 2.0}) {  // split the slowest term
    Vec an = as, bn = bs;
    an[0] = as[0] - dd;
    bn[0] = bs[0] - dd - std::log(2.0);
    an.insert(an.begin() + 1, as[0] + dd);
    bn.insert(bn.begin() + 1, bs[0] + dd - std::log(2.0));
    out.push_back({an, bn});
  }
  return out;
}

}  // namespace

bool expsum_for(double M, double eps, ExpSum& out, std::string& msg) {
  if (!(M >= 1.0) || !(eps > 0.0)) {
    msg = "exponential sum: need M >= 1 and eps > 0";
    return false;
  }
  if (M < 1.0 + 1e-12) M = 1.0 + 1e-12;
  Sol cur;
  if (!fresh(1, M, cur)) {
    msg = "exponential sum: Remez failed for R = 1";
    return false;
  }
  double prev = INFINITY;
  for (int R = 1; R <= 60; ++R) {
    if (cur.E <= eps / M) {
      std::vector<int> ord(R);
      for (int i = 0; i < R; ++i) ord[i] = i;
      std::sort(ord.begin(), ord.end(), [&](int i, int j) { return cur.a[i] < cur.a[j]; });
      out.R = R;
      out.alpha.resize(R);
      out.omega.resize(R);
      for (int i = 0; i < R; ++i) {
        out.alpha[i] = std::exp(cur.a[ord[i]]);
        out.omega[i] = std::exp(cur.b[ord[i]]);
      }
      out.err = cur.E;
      out.err_prev = prev;
      return true;
    }
    prev = cur.E;
    // reference for R+1: stretch the current one over 2R+3 points (log scale)
    Vec tref(2 * R + 3);
    for (int i = 0; i < 2 * R + 3; ++i) {
      const double s = double(i) * (2 * R) / (2 * R + 2);
      const int k = std::min(int(s), 2 * R - 1);
      const double f = s - k;
      tref[i] = std::exp((1 - f) * std::log(cur.xr[k]) + f * std::log(cur.xr[k + 1]));
    }
    Sol next;
    bool ok = false;
    const auto cands = grow_candidates(cur.a, cur.b);
    for (const auto& c : cands)
      if ((ok = remez(c.first, c.second, M, &tref, next))) break;
    if (!ok)
      for (const auto& c : cands)
        if ((ok = remez(c.first, c.second, M, nullptr, next))) break;
    if (!ok) ok = fresh(R + 1, M, next);
    if (!ok) {
      msg = "exponential sum: Remez failed for R = " + std::to_string(R + 1);
      return false;
    }
    cur = next;
  }
  msg = "exponential sum: tolerance not reached with R <= 60";
  return false;
}

}  // namespace tk
