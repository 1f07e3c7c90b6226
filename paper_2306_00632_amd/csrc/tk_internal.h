// Internal declarations shared by the host setup, the runtime and the HIP
// kernels of the Tucker TPCG library.  Not part of the public C ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

namespace tk {

// ---------------------------------------------------------------------------
// host setup (setup_bspline.cpp): univariate B-splines on open uniform knots
// ---------------------------------------------------------------------------

// Knot vector of the open uniform spline space on [0,1] with n_el spans.
std::vector<double> open_knots(int n_el, int p);

// Values and derivatives up to order `nder` of the p+1 B-splines that are
// nonzero on the knot span `span` (knots[span] <= x < knots[span+1]) at x.
// out[d*(p+1) + i] = d-th derivative of B_{span-p+i}.
void span_basis(const std::vector<double>& knots, int p, int span, double x,
                int nder, double* out);

// Index of the span containing x (last non-empty span for x == 1).
int find_span(const std::vector<double>& knots, int p, double x);

// Gauss-Legendre nodes/weights on [-1, 1].
void gauss_legendre(int nq, std::vector<double>& x, std::vector<double>& w);

// Banded matrix int delta_a(b_i) delta_b(b_j) w dx with w(x) = c0 + c1 cos(a x + b)
// on the space with boundary flags (k0, k1) (1 = Neumann: the end basis
// function is kept; 0 = Dirichlet: it is dropped), n = n_el + p - 2 + k0 + k1;
// the default is the Dirichlet space.  DIA layout band[(o+p)*n + i] = A[i, i+o].
// kind: 0 mass, 1 stiffness, 2 mixed (d/dx on test function i), 3 mixed (trial j).
void assemble_band(int n_el, int p, int kind, const double weight[4], double* band, int k0 = 0, int k1 = 0);

// The same integrals with the weight w(x) = sum_{m < nc} c[m] T_m(2x - 1) (a
// Chebyshev series on [0, 1], Appendix A), Gauss-Legendre exact for it.
void assemble_band_cheb(int n_el, int p, int kind, const double* c, int nc, double* band, int k0, int k1);
void load_vector_cheb(int n_el, int p, const double* c, int nc, double* F, int k0, int k1);

// Dirichlet-space load vector F_i = int b_i g dx, g from the weight family.
void load_vector(int n_el, int p, const double weight[4], double* F);

// Derivative `der` of the n = n_el + p - 2 + k0 + k1 basis functions of the
// space with flags (k0, k1) at npts points x in [0, 1]: out (npts x n,
// column-major).
void basis_values(int n_el, int p, int k0, int k1, int der, int npts, const double* x, double* out);

// Dirichlet basis (n = n_el + p - 2 functions) derivative `der` at x.
void dirichlet_basis_at(int n_el, int p, double x, int der, double* vals);

// ---------------------------------------------------------------------------
// host setup (setup_expsum.cpp): best exponential sums for 1/x on [1, M]
// ---------------------------------------------------------------------------

struct ExpSum {
  int R = 0;
  std::vector<double> alpha, omega;  // alpha ascending
  double err = 0.0;                  // E_R(M)
  double err_prev = 0.0;             // E_{R-1}(M)
};

// R_P = min{R : E_R(M) <= eps / M} with the minimax parameters (Remez).
// Returns false (and a message) if the exchange iteration fails.
bool expsum_for(double M, double eps, ExpSum& out, std::string& msg);

// ---------------------------------------------------------------------------
// host setup (setup_fd.cpp): data of the low-rank FD transform of one direction
// ---------------------------------------------------------------------------

struct FdDirection {
  int n_el = 0, p = 0, n = 0, n1 = 0, n2 = 0;
  int N = 0;        // n_el; the FFT length is 2N
  bool odd = true;  // odd p: DST-I of length N-1; even p: DST-II / DST-III of length N
  std::vector<double> lam;          // approximate eigenvalues, length n (Lambda1, Lambda2)
  std::vector<double> g;            // sqrt(2)/sigma(j pi/N), length n1
  // sparse E (n x n1): coefficient map from periodic-spline coefficients to
  // the Dirichlet basis, as ELL with `ke` entries per row, and its transpose
  int ke = 0, ket = 0;
  std::vector<int> e_idx, et_idx;   // n*ke, n1*ket (column index, -1 = empty)
  std::vector<double> e_val, et_val;
  std::vector<double> v2u2;         // n x n2, column-major
};

bool fd_direction_setup(int n_el, int p, double coef, FdDirection& d, std::string& msg);

// Exact generalized eigenpairs of (coef K, M) on the space with boundary
// flags (k0, k1) (default: the Dirichlet space), eq.
// (factorizations): with the banded Cholesky factor M = L L^T (L in the band
// layout of band_cholesky), C = L^{-1} (coef K) L^{-T} (n x n, column-major,
// symmetrized) has the same eigenvalues, and U = L^{-T} Q for its orthonormal
// eigenvectors Q is M-orthonormal.
bool fd_exact_pencil(int n_el, int p, double coef, std::vector<double>& C, std::vector<double>& L, int& n,
                     std::string& msg, int k0 = 0, int k1 = 0);
// Appendix B eigen-approximations (U~, Lambda~) of (coef K, M) on the space
// with boundary flags (k0, k1), built densely on the host: Ut n x n
// column-major (M-orthonormal interpolated sines, then V2 U2), lam n.
bool fd_approx_dense(int n_el, int p, double coef, int k0, int k1, std::vector<double>& Ut,
                     std::vector<double>& lam, int& n, std::string& msg);
// Q (n x n, column-major) <- L^{-T} Q
void fd_exact_vectors(const std::vector<double>& L, int n, int p, double* Q);

}  // namespace tk
