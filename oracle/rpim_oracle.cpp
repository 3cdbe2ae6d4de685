// RPIM stiffness-assembly ORACLE -- test infrastructure only.
//
// A plain, serial, obviously-correct CPU implementation of what the GPU
// library computes.  Only the tests, the smoke check and the benchmark's
// CPU-baseline leg may load it; the product path never does.  It shares no
// code, header, table or constant with the GPU library.
//
// What it computes (GeoMFree3D Sec. 2: stage 1 assembly, stage 2 penalty
// boundary conditions; the method is the RPIM of Liu cited in Sec. 1, and the
// paper prints no equations, so it is the standard polynomial-augmented radial
// point interpolation in its Galerkin form for 3D linear elasticity):
//
//   K = sum_g  w_g |J_g| E_c(g)  B_g^T  D(E=1, nu)  B_g            (stage 1)
//
// where B_g holds the gradients of the RPIM shape functions of the nodes in
// the support of Gauss point g.  Each shape-function gradient comes from one
// moment-matrix solve per Gauss point:
//
//   G = [[R, P], [P^T, 0]],  R_ab = (|x_a - x_b|^2 + (alpha_c d_c)^2)^q,
//   P_a = [1, x_a - x_g],   G gamma_k = r_k,  r_k = d/dx_k [R(x); p(x)] at x_g,
//   dphi_a/dx_k = gamma_k[a].
//
// Stage 2 (penalty boundary conditions) adds alpha = factor * max_i K_ii to
// each fixed diagonal and alpha * u_bar to the right-hand side.
//
// Arithmetic sequence (shared *contract*, not shared code): both this file
// and the GPU kernels follow the same floating-point operation order so that
// the FP64 results are bitwise equal despite cond(G) ~ 1e10:
//   C2  d = x_i - x_j per component; s = fma(dz,dz, fma(dy,dy, dx*dx));
//       support membership s <= fl(d_s*d_s).
//   C3  supports sorted by ascending node id.
//   C4  R = correctly rounded (fl(s + C^2))^q, C^2 = fl(fl(alpha_c*d_c)^2).
//   C5  RHS: t = fl(s + C^2); coef = fl(fl(2q)*CR(t^q)) / t;
//       r_k[a] = coef * fl(x_g - x_a)_k.
//   C6  LU with partial pivoting: pivot = first max |a_rk| (r >= k) in current
//       row order; swap whole rows; l = a_rk / a_kk (IEEE division);
//       a_rj = fma(-l, a_kj, a_rj).  Singular if |u_kk| <= N*eps*max|G|.
//   C7  Forward substitution rides along as extra columns; back substitution
//       for k descending: b_k /= u_kk, then b_r = fma(-u_rk, b_k, b_r), r < k.
//   C8  block entry e = fma(lc, m1, mc*m2) with m1 = pa_al*pb_be,
//       m2 = pa_be*pb_al (+ dot if al == be), dot = fma(pa2,pb2, fma(pa1,pb1, pa0*pb0)),
//       lc = fl(c*lam), mc = fl(c*mu), c = fl(w*E), lam = nu/((1+nu)(1-2nu)),
//       mu = 1/(2(1+nu)).
//   C9  every K entry is +0 + e_g1 + e_g2 + ... in ascending Gauss-point id.
//   C10 no other contraction (built with -ffp-contract=off).
//   C11 mixed precision: FP64 up to dphi (moment matrix and LU stay FP64);
//       dphi, lc, mc rounded to float; C8 evaluated in float (fmaf); each
//       entry is a compensated (Kahan) float sum of its terms in ascending g:
//       s = c = +0; per term e: y = e - c, t = s + y, c = (t - s) - y, s = t;
//       the entry is s.
//
// An extended-precision (__float128) evaluation of the same formulas, with the
// supports frozen, backs the finite-difference gradient checks.
//
// Moving-least-squares and Shepard shape functions (Sec. 4) can replace the
// RPIM ones for assembly, body force and stresses; their operation order
// (M1-M6) is written out above gp_mls.

#include <quadmath.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

namespace {

enum {
  OK = 0,
  E_ARG = -1,
  E_SUPPORT = -4,
  E_SINGULAR = -5,
  E_RANGE = -6,
  E_POW = -7,
  E_STATE = -8,
};

// ---------------------------------------------------------------------------
// Correctly rounded x^q (C4).  An 80-bit powl value is accepted when it lies
// farther than 16 of its own ulps from the nearest midpoint between doubles;
// otherwise the value is recomputed with quad-precision powq and the same
// test is applied with a 2^-100 relative margin.  A value that is still
// ambiguous is reported (never seen in practice).
// ---------------------------------------------------------------------------
long g_pow_fallbacks = 0;
long g_pow_hard = 0;

double round_checked_ld(long double y, long double margin, bool* ok) {
  double d = (double)y;  // round to nearest even
  long double dl = d;
  double nb = (y > dl) ? std::nextafter(d, INFINITY) : std::nextafter(d, -INFINITY);
  long double mid = (dl + (long double)nb) * 0.5L;  // exact in 64-bit mantissa
  *ok = fabsl(y - mid) > margin;
  return d;
}

double pow_cr(double x, double q) {
  long double y = powl((long double)x, (long double)q);
  bool ok = false;
  long double ulp = fabsl(y) * LDBL_EPSILON;  // 2^-63 relative
  double d = round_checked_ld(y, 16.0L * ulp, &ok);
  if (ok) return d;
  g_pow_fallbacks++;
  __float128 yq = powq((__float128)x, (__float128)q);
  double dq = (double)yq;
  __float128 dql = dq;
  double nb = (yq > dql) ? std::nextafter(dq, INFINITY) : std::nextafter(dq, -INFINITY);
  __float128 mid = (dql + (__float128)nb) * (__float128)0.5;
  __float128 gap = fabsq(yq - mid);
  if (!(gap > fabsq(yq) * (__float128)ldexp(1.0, -100))) g_pow_hard++;  // 2^-100
  return dq;
}

// ---------------------------------------------------------------------------
// Scalar helpers: T = double follows the contract; T = __float128 is the
// extended-precision evaluation (rounding order immaterial there).
// ---------------------------------------------------------------------------
inline double fmaT(double a, double b, double c) { return std::fma(a, b, c); }
inline __float128 fmaT(__float128 a, __float128 b, __float128 c) { return a * b + c; }
inline double absT(double a) { return std::fabs(a); }
inline __float128 absT(__float128 a) { return fabsq(a); }
inline double powT(double t, double q) { return pow_cr(t, q); }
inline __float128 powT(__float128 t, __float128 q) { return powq(t, q); }

struct Model {
  int64_t N = 0, G = 0, C = 0;
  std::vector<double> node, gp, wdet;
  std::vector<int32_t> cell;
  double ds = 0, alpha_c = 0, dc = 0, q = 0;
  int shape_kind = 0;  // 0 RPIM, 1 moving least squares (linear basis), 2 Shepard
  bool built = false;
  // supports (C3): gp_ptr[G+1], gp_nbr[sum n]
  std::vector<int64_t> gp_ptr;
  std::vector<int32_t> gp_nbr;
  // node-block pattern: blk_ptr[N+1], blk_col[]
  std::vector<int64_t> blk_ptr;
  std::vector<int32_t> blk_col;
};

inline double sqdist(const double* a, const double* b) {
  double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
  return std::fma(dz, dz, std::fma(dy, dy, dx * dx));  // C2
}

// Position of scalar column `col` in the sorted CSR row `row`.
int64_t find_col(const int64_t* row_ptr, const int32_t* col_idx, int64_t row, int32_t col) {
  const int32_t* b = col_idx + row_ptr[row];
  const int32_t* e = col_idx + row_ptr[row + 1];
  const int32_t* p = std::lower_bound(b, e, col);
  if (p == e || *p != col) return -1;
  return p - col_idx;
}

// ---------------------------------------------------------------------------
// Per-Gauss-point RPIM solve.  Builds the moment matrix G (N x N, N = n + 4)
// augmented with the three derivative right-hand sides (and optionally the
// value right-hand side), runs LU with partial pivoting (C6) with forward
// elimination of the extra columns, then back substitution (C7).
// On return sol[k*Nn + i] holds the full solution gamma_k (i < N).
// ---------------------------------------------------------------------------
template <class T>
int gp_solve(const Model& m, const double* X, int64_t g, int nrhs, std::vector<T>& sol,
             std::vector<T>* lu_out = nullptr, std::vector<int>* piv_out = nullptr) {
  const int64_t b0 = m.gp_ptr[g];
  const int n = (int)(m.gp_ptr[g + 1] - b0);
  const int32_t* S = &m.gp_nbr[b0];
  const int Nn = n + 4;
  const int W = Nn + nrhs;  // augmented row width
  std::vector<T> A((size_t)Nn * W, T(0));
  const T C2 = (T)(m.alpha_c * m.dc) * (T)(m.alpha_c * m.dc);
  const double C2d = (m.alpha_c * m.dc) * (m.alpha_c * m.dc);
  const T q = (T)m.q;
  const double* xg = &m.gp[3 * g];

  // R block (C2, C4): G[a][b] = CR(fl(s_ab + C^2)^q)
  for (int a = 0; a < n; ++a) {
    const double* xa = &X[3 * (int64_t)S[a]];
    for (int b = 0; b < n; ++b) {
      const double* xb = &X[3 * (int64_t)S[b]];
      T t;
      if constexpr (sizeof(T) == sizeof(double)) {
        t = (T)(sqdist(xa, xb) + C2d);
      } else {
        T dx = (T)xa[0] - (T)xb[0], dy = (T)xa[1] - (T)xb[1], dz = (T)xa[2] - (T)xb[2];
        t = dx * dx + dy * dy + dz * dz + C2;
      }
      A[(size_t)a * W + b] = powT(t, q);
    }
    // P block: [1, x_a - x_g]
    A[(size_t)a * W + n] = T(1);
    A[(size_t)n * W + a] = T(1);
    for (int k = 0; k < 3; ++k) {
      T d = (T)xa[k] - (T)xg[k];
      A[(size_t)a * W + n + 1 + k] = d;
      A[(size_t)(n + 1 + k) * W + a] = d;
    }
  }
  // right-hand sides (C5): derivative of [R(x); p(x)] at x_g, and optionally the value
  for (int a = 0; a < n; ++a) {
    const double* xa = &X[3 * (int64_t)S[a]];
    T t;
    if constexpr (sizeof(T) == sizeof(double)) {
      t = (T)(sqdist(xa, xg) + C2d);
    } else {
      T dx = (T)xa[0] - (T)xg[0], dy = (T)xa[1] - (T)xg[1], dz = (T)xa[2] - (T)xg[2];
      t = dx * dx + dy * dy + dz * dz + C2;
    }
    T R = powT(t, q);
    T coef = ((T)2 * q * R) / t;  // fl(fl(2q) * R) / t
    for (int k = 0; k < 3; ++k) A[(size_t)a * W + Nn + k] = coef * ((T)xg[k] - (T)xa[k]);
    if (nrhs > 3) A[(size_t)a * W + Nn + 3] = R;
  }
  for (int k = 0; k < 3; ++k) A[(size_t)(n + 1 + k) * W + Nn + k] = T(1);
  if (nrhs > 3) A[(size_t)n * W + Nn + 3] = T(1);

  // C6: LU with partial pivoting, extra columns eliminated alongside.
  T maxabs = T(0);
  for (int r = 0; r < Nn; ++r)
    for (int c = 0; c < Nn; ++c) maxabs = std::max(maxabs, absT(A[(size_t)r * W + c]));
  const double tiny = ((double)Nn * DBL_EPSILON) * (double)maxabs;
  std::vector<int> piv(Nn);
  for (int k = 0; k < Nn; ++k) {
    int p = k;
    T best = absT(A[(size_t)k * W + k]);
    for (int r = k + 1; r < Nn; ++r) {
      T v = absT(A[(size_t)r * W + k]);
      if (v > best) { best = v; p = r; }
    }
    piv[k] = p;
    if constexpr (sizeof(T) == sizeof(double)) {
      if (!(best > tiny)) return E_SINGULAR;
    }
    if (p != k)
      for (int c = 0; c < W; ++c) std::swap(A[(size_t)k * W + c], A[(size_t)p * W + c]);
    const T piv_v = A[(size_t)k * W + k];
    for (int r = k + 1; r < Nn; ++r) {
      T l = A[(size_t)r * W + k] / piv_v;
      A[(size_t)r * W + k] = l;
      for (int c = k + 1; c < W; ++c)
        A[(size_t)r * W + c] = fmaT(-l, A[(size_t)k * W + c], A[(size_t)r * W + c]);
    }
  }
  // C7: back substitution, column oriented, k descending.
  sol.assign((size_t)nrhs * Nn, T(0));
  for (int j = 0; j < nrhs; ++j) {
    std::vector<T> b(Nn);
    for (int r = 0; r < Nn; ++r) b[r] = A[(size_t)r * W + Nn + j];
    for (int k = Nn - 1; k >= 0; --k) {
      b[k] = b[k] / A[(size_t)k * W + k];
      for (int r = 0; r < k; ++r) b[r] = fmaT(-A[(size_t)r * W + k], b[k], b[r]);
    }
    for (int r = 0; r < Nn; ++r) sol[(size_t)j * Nn + r] = b[r];
  }
  if (lu_out) {
    lu_out->assign((size_t)Nn * Nn, T(0));
    for (int r = 0; r < Nn; ++r)
      for (int c = 0; c < Nn; ++c) (*lu_out)[(size_t)r * Nn + c] = A[(size_t)r * W + c];
  }
  if (piv_out) *piv_out = piv;
  return OK;
}

// Solve G y = rhs with the stored factors (L rows carry every later swap) and
// pivots: all row swaps in factorisation order, then forward and back
// substitution (C7 order).
void lu_solve(int Nn, const std::vector<double>& lu, const std::vector<int>& piv, std::vector<double>& b) {
  for (int k = 0; k < Nn; ++k)
    if (piv[k] != k) std::swap(b[k], b[piv[k]]);
  for (int k = 0; k < Nn; ++k)
    for (int r = k + 1; r < Nn; ++r) b[r] = std::fma(-lu[(size_t)r * Nn + k], b[k], b[r]);
  for (int k = Nn - 1; k >= 0; --k) {
    b[k] = b[k] / lu[(size_t)k * Nn + k];
    for (int r = 0; r < k; ++r) b[r] = std::fma(-lu[(size_t)r * Nn + k], b[k], b[r]);
  }
}

// ---------------------------------------------------------------------------
// Moving-least-squares shape functions (named in Sec. 4 as the package's next
// shape functions): linear basis (M = 4) or constant basis (M = 1, Shepard's
// functions), with the cubic-spline weight over the support radius d_s.
//   M1  d = x_g - x_i per component; s = fma(dz,dz, fma(dy,dy, dx*dx));
//       r = sqrt(s) / d_s; basis p = [1, x_i - x_g] (M = 4) or [1] (M = 1).
//   M2  r2 = r*r; r <= 1/2: W = (fl(2/3) - 4*r2) + (4*r2)*r, Wr = fma(12, r, -8);
//       1/2 < r <= 1: W = ((fl(4/3) - 4*r) + 4*r2) - fl(4/3)*(r2*r),
//       Wr = (8 - 4/r) - 4*r; otherwise W = Wr = 0.  Wr = W'(r)/r, and the
//       weight's gradient at x_g is w_k = (Wr*d_k) / fl(d_s*d_s).
//   M3  A_jl (j <= l) = +0 + t_1 + t_2 + ... in ascending support order,
//       t = (W*p_j)*p_l; the derivative matrices A^k likewise with
//       t = (w_k*p_j)*p_l; A_lj = A_jl.
//   M4  A = LU by C6 (singular if |u_kk| <= M*eps*max|A|); gamma = A^-1 e_0:
//       interchanges applied to the right-hand side in step order, forward
//       b_r = fma(-l_rk, b_k, b_r), back substitution by C7.
//   M5  gamma_k = A^-1 rhs with the same factors, rhs_j = [j == k+1] - s_j,
//       s_j the fma chain over l ascending of A^k_jl gamma_l from +0 (the
//       term [j == k+1] only exists for M = 4).
//   M6  c = gamma^T p = fma(g3,p3, fma(g2,p2, fma(g1,p1, g0))) (g0 for M = 1),
//       c_k likewise from gamma_k; phi = W*c, dphi_k = fma(W, c_k, w_k*c).
// ---------------------------------------------------------------------------
int gp_mls(const Model& m, const double* X, int64_t g, int M, std::vector<double>& phi, std::vector<double>& dphi) {
  const int64_t b0 = m.gp_ptr[g];
  const int n = (int)(m.gp_ptr[g + 1] - b0);
  const int32_t* S = &m.gp_nbr[b0];
  const double* xg = &m.gp[3 * g];
  const double C23 = 2.0 / 3.0, C43 = 4.0 / 3.0;
  const double dw2 = m.ds * m.ds;
  std::vector<double> W(n), wk(3 * (size_t)n), P(4 * (size_t)n);
  for (int a = 0; a < n; ++a) {  // M1, M2
    const double* xi = &X[3 * (int64_t)S[a]];
    double d[3];
    for (int k = 0; k < 3; ++k) d[k] = xg[k] - xi[k];
    const double s = std::fma(d[2], d[2], std::fma(d[1], d[1], d[0] * d[0]));
    const double r = std::sqrt(s) / m.ds;
    const double r2 = r * r;
    double Wa = 0.0, Wr = 0.0;
    if (r <= 0.5) {
      Wa = (C23 - 4.0 * r2) + (4.0 * r2) * r;
      Wr = std::fma(12.0, r, -8.0);
    } else if (r <= 1.0) {
      Wa = ((C43 - 4.0 * r) + 4.0 * r2) - C43 * (r2 * r);
      Wr = (8.0 - 4.0 / r) - 4.0 * r;
    }
    W[a] = Wa;
    for (int k = 0; k < 3; ++k) wk[3 * a + k] = (Wr * d[k]) / dw2;
    P[4 * a] = 1.0;
    for (int k = 0; k < 3; ++k) P[4 * a + 1 + k] = xi[k] - xg[k];
  }
  double A[4][4] = {}, Ak[3][4][4] = {};
  for (int j = 0; j < M; ++j)  // M3
    for (int l = j; l < M; ++l) {
      double s0 = 0.0, s1[3] = {0.0, 0.0, 0.0};
      for (int a = 0; a < n; ++a) {
        s0 = s0 + (W[a] * P[4 * a + j]) * P[4 * a + l];
        for (int k = 0; k < 3; ++k) s1[k] = s1[k] + (wk[3 * a + k] * P[4 * a + j]) * P[4 * a + l];
      }
      A[j][l] = A[l][j] = s0;
      for (int k = 0; k < 3; ++k) Ak[k][j][l] = Ak[k][l][j] = s1[k];
    }
  double LU[4][4];  // M4
  double mx = 0.0;
  for (int j = 0; j < M; ++j)
    for (int l = 0; l < M; ++l) {
      LU[j][l] = A[j][l];
      mx = std::max(mx, std::fabs(A[j][l]));
    }
  const double tiny = ((double)M * DBL_EPSILON) * mx;
  int piv[4];
  for (int k = 0; k < M; ++k) {
    int p = k;
    double best = std::fabs(LU[k][k]);
    for (int r = k + 1; r < M; ++r) {
      const double v = std::fabs(LU[r][k]);
      if (v > best) { best = v; p = r; }
    }
    piv[k] = p;
    if (!(best > tiny)) return E_SINGULAR;
    if (p != k)
      for (int c = 0; c < M; ++c) std::swap(LU[k][c], LU[p][c]);
    for (int r = k + 1; r < M; ++r) {
      const double l = LU[r][k] / LU[k][k];
      LU[r][k] = l;
      for (int c = k + 1; c < M; ++c) LU[r][c] = std::fma(-l, LU[k][c], LU[r][c]);
    }
  }
  const auto solve = [&](double* b) {
    for (int k = 0; k < M; ++k)
      if (piv[k] != k) std::swap(b[k], b[piv[k]]);
    for (int k = 0; k < M; ++k)
      for (int r = k + 1; r < M; ++r) b[r] = std::fma(-LU[r][k], b[k], b[r]);
    for (int k = M - 1; k >= 0; --k) {
      b[k] = b[k] / LU[k][k];
      for (int r = 0; r < k; ++r) b[r] = std::fma(-LU[r][k], b[k], b[r]);
    }
  };
  double gam[4] = {1.0, 0.0, 0.0, 0.0};
  solve(gam);
  double gk[3][4];
  for (int k = 0; k < 3; ++k) {  // M5
    for (int j = 0; j < M; ++j) {
      double s = 0.0;
      for (int l = 0; l < M; ++l) s = std::fma(Ak[k][j][l], gam[l], s);
      gk[k][j] = (j == k + 1 ? 1.0 : 0.0) - s;
    }
    solve(gk[k]);
  }
  phi.assign(n, 0.0);
  dphi.assign(3 * (size_t)n, 0.0);
  for (int a = 0; a < n; ++a) {  // M6
    const double* pa = &P[4 * a];
    double c = gam[0];
    if (M == 4) c = std::fma(gam[3], pa[3], std::fma(gam[2], pa[2], std::fma(gam[1], pa[1], c)));
    phi[a] = W[a] * c;
    for (int k = 0; k < 3; ++k) {
      double ck = gk[k][0];
      if (M == 4) ck = std::fma(gk[k][3], pa[3], std::fma(gk[k][2], pa[2], std::fma(gk[k][1], pa[1], ck)));
      dphi[3 * a + k] = std::fma(W[a], ck, wk[3 * a + k] * c);
    }
  }
  return OK;
}

// Shape functions of point g under the model's kind: phi[a] (RPIM: only when
// want_phi, from the value right-hand side) and dphi[3a+k].
int point_shapes(const Model& m, const double* X, int64_t g, bool want_phi, std::vector<double>& phi,
                 std::vector<double>& dphi) {
  if (m.shape_kind != 0) return gp_mls(m, X, g, m.shape_kind == 1 ? 4 : 1, phi, dphi);
  std::vector<double> sol;
  const int st = gp_solve<double>(m, X, g, want_phi ? 4 : 3, sol);
  if (st != OK) return st;
  const int n = (int)(m.gp_ptr[g + 1] - m.gp_ptr[g]), Nn = n + 4;
  phi.assign(n, 0.0);
  dphi.assign(3 * (size_t)n, 0.0);
  for (int a = 0; a < n; ++a) {
    if (want_phi) phi[a] = sol[(size_t)3 * Nn + a];
    for (int k = 0; k < 3; ++k) dphi[3 * a + k] = sol[(size_t)k * Nn + a];
  }
  return OK;
}

// Isotropic elasticity constants for E = 1 (C8), evaluated left to right.
void lame_hat(double nu, double* lam, double* mu) {
  double onep = 1.0 + nu;
  double onem = 1.0 - 2.0 * nu;
  *lam = nu / (onep * onem);
  *mu = 1.0 / (2.0 * onep);
}

}  // namespace

extern "C" {

void* orcl_model_create(int64_t N, const double* node_xyz, int64_t G, const double* gp_xyz,
                        const double* gp_wdet, const int32_t* gp_cell, int64_t C, double ds,
                        double alpha_c, double dc, double q) {
  if (N <= 0 || G < 0 || C <= 0 || !(ds > 0) || !(alpha_c > 0) || !(dc > 0) || !(q > 0)) return nullptr;
  Model* m = new Model;
  m->N = N; m->G = G; m->C = C;
  m->node.assign(node_xyz, node_xyz + 3 * N);
  m->gp.assign(gp_xyz, gp_xyz + 3 * G);
  m->wdet.assign(gp_wdet, gp_wdet + G);
  m->cell.assign(gp_cell, gp_cell + G);
  m->ds = ds; m->alpha_c = alpha_c; m->dc = dc; m->q = q;
  return m;
}

void orcl_model_destroy(void* h) { delete (Model*)h; }

// Shape functions of the model: 0 RPIM (default), 1 moving least squares with a
// linear basis, 2 Shepard's functions (constant basis); both MLS kinds use the
// cubic-spline weight over the support radius.  The adjoint is RPIM only.
int orcl_set_shape(void* h, int kind) {
  if (!h || kind < 0 || kind > 2) return E_ARG;
  ((Model*)h)->shape_kind = kind;
  return OK;
}

// Support search (brute force over all nodes, ascending id: C2, C3) and the
// node-block pattern: cols(I) = union of S_g over Gauss points g with I in S_g.
int orcl_build_pattern(void* h, int64_t* nnz, int64_t* sum_n, int64_t* first_bad_gp) {
  Model& m = *(Model*)h;
  const double r2 = m.ds * m.ds;
  m.gp_ptr.assign(m.G + 1, 0);
  m.gp_nbr.clear();
  int64_t bad = -1;
  for (int64_t g = 0; g < m.G; ++g) {
    for (int64_t i = 0; i < m.N; ++i)
      if (sqdist(&m.node[3 * i], &m.gp[3 * g]) <= r2) m.gp_nbr.push_back((int32_t)i);
    m.gp_ptr[g + 1] = (int64_t)m.gp_nbr.size();
    if (bad < 0 && m.gp_ptr[g + 1] - m.gp_ptr[g] < 5) bad = g;  // needs n >= m + 1 = 5
  }
  if (first_bad_gp) *first_bad_gp = bad;
  if (bad >= 0) return E_SUPPORT;
  // inverse lists node -> Gauss points (ascending g)
  std::vector<std::vector<int64_t>> inv(m.N);
  for (int64_t g = 0; g < m.G; ++g)
    for (int64_t e = m.gp_ptr[g]; e < m.gp_ptr[g + 1]; ++e) inv[m.gp_nbr[e]].push_back(g);
  m.blk_ptr.assign(m.N + 1, 0);
  m.blk_col.clear();
  std::vector<int64_t> mark(m.N, -1);
  std::vector<int32_t> row;
  for (int64_t I = 0; I < m.N; ++I) {
    row.clear();
    for (int64_t g : inv[I])
      for (int64_t e = m.gp_ptr[g]; e < m.gp_ptr[g + 1]; ++e) {
        int32_t J = m.gp_nbr[e];
        if (mark[J] != I) { mark[J] = I; row.push_back(J); }
      }
    std::sort(row.begin(), row.end());
    m.blk_col.insert(m.blk_col.end(), row.begin(), row.end());
    m.blk_ptr[I + 1] = (int64_t)m.blk_col.size();
  }
  m.built = true;
  if (nnz) *nnz = 9 * (int64_t)m.blk_col.size();
  if (sum_n) *sum_n = (int64_t)m.gp_nbr.size();
  return OK;
}

int orcl_get_support(void* h, int64_t* gp_ptr, int32_t* gp_nbr) {
  Model& m = *(Model*)h;
  if (!m.built) return E_STATE;
  std::memcpy(gp_ptr, m.gp_ptr.data(), sizeof(int64_t) * (m.G + 1));
  std::memcpy(gp_nbr, m.gp_nbr.data(), sizeof(int32_t) * m.gp_nbr.size());
  return OK;
}

// Scalar CSR with dof = 3*node + component; row 3I+al lists 3J+be for J in
// cols(I) (ascending) and be = 0, 1, 2.
int orcl_get_pattern(void* h, int64_t* row_ptr, int32_t* col_idx) {
  Model& m = *(Model*)h;
  if (!m.built) return E_STATE;
  int64_t pos = 0;
  row_ptr[0] = 0;
  for (int64_t I = 0; I < m.N; ++I) {
    for (int al = 0; al < 3; ++al) {
      for (int64_t e = m.blk_ptr[I]; e < m.blk_ptr[I + 1]; ++e)
        for (int be = 0; be < 3; ++be) col_idx[pos++] = 3 * m.blk_col[e] + be;
      row_ptr[3 * I + al + 1] = pos;
    }
  }
  return OK;
}

// Shape functions at Gauss point g: phi[a] (values, test use) and dphi[a*3+k].
int orcl_shape(void* h, int64_t g, const double* node_xyz, double* phi, double* dphi) {
  Model& m = *(Model*)h;
  if (!m.built || g < 0 || g >= m.G) return E_ARG;
  const double* X = node_xyz ? node_xyz : m.node.data();
  std::vector<double> ph, dph;
  int st = point_shapes(m, X, g, true, ph, dph);
  if (st != OK) return st;
  const int n = (int)(m.gp_ptr[g + 1] - m.gp_ptr[g]);
  for (int a = 0; a < n; ++a) {
    if (phi) phi[a] = ph[a];
    for (int k = 0; k < 3; ++k) dphi[3 * a + k] = dph[3 * a + k];
  }
  return OK;
}

// Stage 1: K over the listed Gauss points (all when gps == NULL), ascending g.
// precision 0: K is double[nnz] (C8, C9).  precision 1: K is float[nnz], the
// compensated float sums of C11.
int orcl_assemble(void* h, const double* node_xyz, const double* cell_E, double nu, int precision,
                  void* K_vals, const int64_t* gps, int64_t n_gps, int64_t* first_bad_gp) {
  Model& m = *(Model*)h;
  if (!m.built) return E_STATE;
  if (precision != 0 && precision != 1) return E_ARG;
  if (!(nu > -1.0 && nu < 0.5)) return E_ARG;
  const double* X = node_xyz ? node_xyz : m.node.data();
  const int64_t ndof = 3 * m.N;
  std::vector<int64_t> row_ptr(ndof + 1);
  std::vector<int32_t> col_idx(9 * m.blk_col.size());
  orcl_get_pattern(h, row_ptr.data(), col_idx.data());
  const int64_t nnz = (int64_t)col_idx.size();
  double* K64 = (double*)K_vals;
  float* K32 = (float*)K_vals;
  std::vector<float> kc;  // C11: Kahan compensation per entry (the running sum is K32 itself)
  if (precision == 0) std::fill(K64, K64 + nnz, 0.0);
  else {
    std::fill(K32, K32 + nnz, 0.0f);
    kc.assign(nnz, 0.0f);
  }
  double lam, mu;
  lame_hat(nu, &lam, &mu);
  const int64_t count = gps ? n_gps : m.G;
  if (first_bad_gp) *first_bad_gp = -1;
  std::vector<double> phi, dphi;
  for (int64_t it = 0; it < count; ++it) {
    const int64_t g = gps ? gps[it] : it;
    int st = point_shapes(m, X, g, false, phi, dphi);
    if (st != OK) { if (first_bad_gp) *first_bad_gp = g; return st; }
    const int64_t b0 = m.gp_ptr[g];
    const int n = (int)(m.gp_ptr[g + 1] - b0);
    const int32_t* S = &m.gp_nbr[b0];
    const double c = m.wdet[g] * cell_E[m.cell[g]];
    const double lc = c * lam, mc = c * mu;
    for (int a = 0; a < n; ++a) {
      const double pa[3] = {dphi[3 * a], dphi[3 * a + 1], dphi[3 * a + 2]};
      for (int b = 0; b < n; ++b) {
        const double pb[3] = {dphi[3 * b], dphi[3 * b + 1], dphi[3 * b + 2]};
        for (int al = 0; al < 3; ++al)
          for (int be = 0; be < 3; ++be) {
            int64_t pos = find_col(row_ptr.data(), col_idx.data(), 3 * (int64_t)S[a] + al, 3 * S[b] + be);
            if (pos < 0) return E_STATE;
            if (precision == 0) {
              double dot = std::fma(pa[2], pb[2], std::fma(pa[1], pb[1], pa[0] * pb[0]));
              double m1 = pa[al] * pb[be];
              double m2 = pa[be] * pb[al];
              if (al == be) m2 = m2 + dot;
              K64[pos] = K64[pos] + std::fma(lc, m1, mc * m2);
            } else {
              const float fa[3] = {(float)pa[0], (float)pa[1], (float)pa[2]};
              const float fb[3] = {(float)pb[0], (float)pb[1], (float)pb[2]};
              const float flc = (float)lc, fmc = (float)mc;
              float dot = std::fmaf(fa[2], fb[2], std::fmaf(fa[1], fb[1], fa[0] * fb[0]));
              float m1 = fa[al] * fb[be];
              float m2 = fa[be] * fb[al];
              if (al == be) m2 = m2 + dot;
              float e = std::fmaf(flc, m1, fmc * m2);
              // compensated float sum (Kahan): the compensation carries the
              // low-order part lost when e joins the running sum
              float y = e - kc[pos];
              float t = K32[pos] + y;
              kc[pos] = (t - K32[pos]) - y;
              K32[pos] = t;
            }
          }
      }
    }
  }
  return OK;
}

// After the solve (GeoMFree3D Sec. 2: the displacements are found first, the
// stresses from them).  Body force: f_I = sum_g w_g phi_I(x_g) b_g, b_g the
// force per unit volume at Gauss point g, summed per node in ascending g:
// e = fl(w_g * phi_a) * b_k, f = f + e.  phi comes from the value right-hand
// side [R(x_g); 1, 0, 0, 0] of the same solve (gp_solve with four columns).
int orcl_body_force(void* h, const double* node_xyz, const double* gp_force, double* f) {
  Model& m = *(Model*)h;
  if (!m.built) return E_STATE;
  const double* X = node_xyz ? node_xyz : m.node.data();
  std::fill(f, f + 3 * m.N, 0.0);
  std::vector<double> phi, dphi;
  for (int64_t g = 0; g < m.G; ++g) {
    int st = point_shapes(m, X, g, true, phi, dphi);
    if (st != OK) return st;
    const int64_t b0 = m.gp_ptr[g];
    const int n = (int)(m.gp_ptr[g + 1] - b0);
    for (int a = 0; a < n; ++a) {
      const double c = m.wdet[g] * phi[a];
      for (int k = 0; k < 3; ++k) {
        const int64_t d = 3 * (int64_t)m.gp_nbr[b0 + a] + k;
        f[d] = f[d] + c * gp_force[3 * g + k];
      }
    }
  }
  return OK;
}

// Stress at every Gauss point from nodal displacements u (dof 3*node + comp):
// H_ij = sum_a u_{S[a], i} dphi_a/dx_j as fma(u, dphi, H) in ascending a from
// +0; eps_ij = 0.5 * (H_ij + H_ji); tr = (eps_00 + eps_11) + eps_22;
// with lc = fl(E_c * lam_hat), mc = fl(E_c * mu_hat):
// sigma_ii = fma(lc, tr, fl(2 mc) * eps_ii), sigma_ij = fl(2 mc) * eps_ij;
// stored as [xx, yy, zz, yz, xz, xy] per point.
int orcl_gauss_stress(void* h, const double* node_xyz, const double* cell_E, double nu, const double* u,
                      double* sigma) {
  Model& m = *(Model*)h;
  if (!m.built) return E_STATE;
  if (!(nu > -1.0 && nu < 0.5)) return E_ARG;
  const double* X = node_xyz ? node_xyz : m.node.data();
  double lam, mu;
  lame_hat(nu, &lam, &mu);
  std::vector<double> phi, dphi;
  for (int64_t g = 0; g < m.G; ++g) {
    int st = point_shapes(m, X, g, false, phi, dphi);
    if (st != OK) return st;
    const int64_t b0 = m.gp_ptr[g];
    const int n = (int)(m.gp_ptr[g + 1] - b0);
    double H[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    for (int a = 0; a < n; ++a) {
      const int64_t I = m.gp_nbr[b0 + a];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) H[i][j] = std::fma(u[3 * I + i], dphi[3 * a + j], H[i][j]);
    }
    double e[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) e[i][j] = 0.5 * (H[i][j] + H[j][i]);
    const double tr = (e[0][0] + e[1][1]) + e[2][2];
    const double c = cell_E[m.cell[g]];
    const double lc = c * lam, mc2 = 2.0 * (c * mu);
    double* s = sigma + 6 * g;
    for (int i = 0; i < 3; ++i) s[i] = std::fma(lc, tr, mc2 * e[i][i]);
    s[3] = mc2 * e[1][2];
    s[4] = mc2 * e[0][2];
    s[5] = mc2 * e[0][1];
  }
  return OK;
}

// Stage 2: penalty BCs.  alpha = factor * max_i K_ii over all dofs (before the
// update); K_dd += alpha and rhs_d += alpha * u_bar_d for each fixed dof d.
int orcl_penalty(const int64_t* row_ptr, const int32_t* col_idx, void* K_vals, int precision,
                 int64_t n_dof, const int32_t* fixed, const double* ubar, int64_t n_fixed,
                 double factor, double* rhs, double* alpha_out) {
  if (n_dof <= 0 || n_fixed < 0 || !(factor > 0)) return E_ARG;
  std::vector<char> seen(n_dof, 0);
  for (int64_t i = 0; i < n_fixed; ++i) {
    if (fixed[i] < 0 || fixed[i] >= n_dof || seen[fixed[i]]) return E_ARG;
    seen[fixed[i]] = 1;
  }
  double mx = -INFINITY;
  for (int64_t d = 0; d < n_dof; ++d) {
    int64_t p = find_col(row_ptr, col_idx, d, (int32_t)d);
    if (p < 0) return E_ARG;
    double v = precision == 0 ? ((double*)K_vals)[p] : (double)((float*)K_vals)[p];
    mx = std::max(mx, v);
  }
  const double alpha = factor * mx;
  for (int64_t i = 0; i < n_fixed; ++i) {
    int64_t d = fixed[i];
    int64_t p = find_col(row_ptr, col_idx, d, (int32_t)d);
    if (precision == 0) ((double*)K_vals)[p] = ((double*)K_vals)[p] + alpha;
    else ((float*)K_vals)[p] = ((float*)K_vals)[p] + (float)alpha;
    if (rhs) rhs[d] = rhs[d] + alpha * (ubar ? ubar[i] : 0.0);
  }
  if (alpha_out) *alpha_out = alpha;
  return OK;
}

// Adjoint of stage 1: given Kbar = dL/dK on the pattern, dE[c] = dL/dE_c and
// dX[i][k] = dL/dx_{i,k} with Gauss points, weights and supports held fixed.
// Per Gauss point: Phibar = dL_g/dphi; lambda_k = G^{-T} [Phibar_k; 0]
// (G is symmetric, so its own LU serves); Gbar = -sum_k lambda_k gamma_k^T;
// then the chain rule through R(s_ab), the polynomial block and the
// derivative right-hand sides.  Accumulated in ascending g over the listed
// Gauss points (all when gps == NULL): a node's or a cell's value is complete
// when every Gauss point whose support holds the node, or that lies in the
// cell, is listed.
int orcl_assemble_backward(void* h, const double* node_xyz, const double* cell_E, double nu,
                           const double* Kbar, const int64_t* gps, int64_t n_gps, double* dE, double* dX) {
  Model& m = *(Model*)h;
  if (!m.built || m.shape_kind != 0) return E_STATE;
  const double* X = node_xyz ? node_xyz : m.node.data();
  const int64_t ndof = 3 * m.N;
  std::vector<int64_t> row_ptr(ndof + 1);
  std::vector<int32_t> col_idx(9 * m.blk_col.size());
  orcl_get_pattern(h, row_ptr.data(), col_idx.data());
  double lam, mu;
  lame_hat(nu, &lam, &mu);
  std::fill(dE, dE + m.C, 0.0);
  std::fill(dX, dX + 3 * m.N, 0.0);
  const double C2 = (m.alpha_c * m.dc) * (m.alpha_c * m.dc);
  const double q = m.q;
  std::vector<double> sol, lu;
  std::vector<int> piv;
  const int64_t count = gps ? n_gps : m.G;
  for (int64_t it = 0; it < count; ++it) {
    const int64_t g = gps ? gps[it] : it;
    if (g < 0 || g >= m.G) return E_ARG;
    int st = gp_solve<double>(m, X, g, 3, sol, &lu, &piv);
    if (st != OK) return st;
    const int64_t b0 = m.gp_ptr[g];
    const int n = (int)(m.gp_ptr[g + 1] - b0), Nn = n + 4;
    const int32_t* S = &m.gp_nbr[b0];
    const double w = m.wdet[g];
    const double E = cell_E[m.cell[g]];
    const double c = w * E;
    auto phi = [&](int a, int k) { return sol[(size_t)k * Nn + a]; };
    // Mb = Kbar_ab + Kbar_ba^T per block; Phibar[c][ga] = sum_b lc (Mb pb)_ga + mc (Mb^T pb)_ga + mc tr(Mb) pb_ga
    std::vector<double> pbar((size_t)n * 3, 0.0);
    double Lw = 0.0;  // sum <Kbar, k^g> / E
    for (int a = 0; a < n; ++a) {
      for (int b = 0; b < n; ++b) {
        double M[3][3], Kab[3][3];
        for (int al = 0; al < 3; ++al)
          for (int be = 0; be < 3; ++be) {
            int64_t p1 = find_col(row_ptr.data(), col_idx.data(), 3 * (int64_t)S[a] + al, 3 * S[b] + be);
            int64_t p2 = find_col(row_ptr.data(), col_idx.data(), 3 * (int64_t)S[b] + be, 3 * S[a] + al);
            Kab[al][be] = Kbar[p1];
            M[al][be] = Kbar[p1] + Kbar[p2];
          }
        const double pb[3] = {phi(b, 0), phi(b, 1), phi(b, 2)};
        const double pa[3] = {phi(a, 0), phi(a, 1), phi(a, 2)};
        double tr = M[0][0] + M[1][1] + M[2][2];
        for (int ga = 0; ga < 3; ++ga) {
          double s1 = 0, s2 = 0;
          for (int be = 0; be < 3; ++be) { s1 += M[ga][be] * pb[be]; s2 += M[be][ga] * pb[be]; }
          pbar[3 * a + ga] += c * lam * s1 + c * mu * s2 + c * mu * tr * pb[ga];
        }
        double dot = pa[0] * pb[0] + pa[1] * pb[1] + pa[2] * pb[2];
        for (int al = 0; al < 3; ++al)
          for (int be = 0; be < 3; ++be) {
            double kk = w * (lam * pa[al] * pb[be] + mu * pa[be] * pb[al] + (al == be ? mu * dot : 0.0));
            Lw += Kab[al][be] * kk;
          }
      }
    }
    (void)E;
    dE[m.cell[g]] += Lw;
    // adjoint solves lambda_k = G^{-1} [Phibar_k; 0]
    std::vector<double> lamv((size_t)3 * Nn);
    for (int k = 0; k < 3; ++k) {
      std::vector<double> b(Nn, 0.0);
      for (int a = 0; a < n; ++a) b[a] = pbar[3 * a + k];
      lu_solve(Nn, lu, piv, b);
      for (int i = 0; i < Nn; ++i) lamv[(size_t)k * Nn + i] = b[i];
    }
    auto Gbar = [&](int i, int j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s -= lamv[(size_t)k * Nn + i] * sol[(size_t)k * Nn + j];
      return s;
    };
    const double* xg = &m.gp[3 * g];
    for (int a = 0; a < n; ++a) {
      const double* xa = &X[3 * (int64_t)S[a]];
      double acc[3] = {0, 0, 0};
      // (i) R block: both G[a][b] and G[b][a] depend on x_a
      for (int b = 0; b < n; ++b) {
        if (b == a) continue;
        const double* xb = &X[3 * (int64_t)S[b]];
        double t = sqdist(xa, xb) + C2;
        double R = pow_cr(t, q);
        double dR = q * R / t;  // d rho / d s
        double gsum = Gbar(a, b) + Gbar(b, a);
        for (int k = 0; k < 3; ++k) acc[k] += gsum * dR * 2.0 * (xa[k] - xb[k]);
      }
      // (ii) polynomial block: d(x_a - x_g)_k / dx_{a,k} = 1 in both G[a][n+1+k] and its mirror
      for (int k = 0; k < 3; ++k) acc[k] += Gbar(a, n + 1 + k) + Gbar(n + 1 + k, a);
      // (iii) derivative right-hand sides r_k[a] = 2q t^(q-1) (x_g - x_a)_k
      double t = sqdist(xa, xg) + C2;
      double R = pow_cr(t, q);
      double tq1 = R / t, tq2 = R / (t * t);
      for (int cc = 0; cc < 3; ++cc) {
        double s = 0;
        for (int k = 0; k < 3; ++k) {
          double dgc = xg[cc] - xa[cc], dgk = xg[k] - xa[k];
          double dr = -(4.0 * q * (q - 1.0) * tq2 * dgc * dgk + (k == cc ? 2.0 * q * tq1 : 0.0));
          s += lamv[(size_t)k * Nn + a] * dr;
        }
        acc[cc] += s;
      }
      for (int k = 0; k < 3; ++k) dX[3 * (int64_t)S[a] + k] += acc[k];
    }
  }
  return OK;
}

// Extended precision: sum over the listed Gauss points of <Kbar, k^g> in
// __float128, with the build-time supports frozen and node coordinates taken
// from node_xyz.  Result returned as hi + lo doubles.  Backs the central
// finite-difference checks of the coordinate gradient.
int orcl_dot_q(void* h, const double* node_xyz, const double* cell_E, double nu, const double* Kbar,
               const int64_t* gps, int64_t n_gps, double* out_hi_lo) {
  Model& m = *(Model*)h;
  if (!m.built || m.shape_kind != 0) return E_STATE;
  const int64_t ndof = 3 * m.N;
  std::vector<int64_t> row_ptr(ndof + 1);
  std::vector<int32_t> col_idx(9 * m.blk_col.size());
  orcl_get_pattern(h, row_ptr.data(), col_idx.data());
  const __float128 nuq = nu;
  const __float128 lam = nuq / ((1 + nuq) * (1 - 2 * nuq));
  const __float128 mu = 1 / (2 * (1 + nuq));
  __float128 total = 0;
  std::vector<__float128> sol;
  for (int64_t it = 0; it < n_gps; ++it) {
    const int64_t g = gps[it];
    int st = gp_solve<__float128>(m, node_xyz, g, 3, sol);
    if (st != OK) return st;
    const int64_t b0 = m.gp_ptr[g];
    const int n = (int)(m.gp_ptr[g + 1] - b0), Nn = n + 4;
    const int32_t* S = &m.gp_nbr[b0];
    const __float128 c = (__float128)m.wdet[g] * (__float128)cell_E[m.cell[g]];
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        __float128 pa[3], pb[3];
        for (int k = 0; k < 3; ++k) { pa[k] = sol[(size_t)k * Nn + a]; pb[k] = sol[(size_t)k * Nn + b]; }
        __float128 dot = pa[0] * pb[0] + pa[1] * pb[1] + pa[2] * pb[2];
        for (int al = 0; al < 3; ++al)
          for (int be = 0; be < 3; ++be) {
            int64_t p = find_col(row_ptr.data(), col_idx.data(), 3 * (int64_t)S[a] + al, 3 * S[b] + be);
            __float128 e = c * (lam * pa[al] * pb[be] + mu * pa[be] * pb[al] + (al == be ? mu * dot : 0));
            total += (__float128)Kbar[p] * e;
          }
      }
  }
  double hi = (double)total;
  double lo = (double)(total - (__float128)hi);
  out_hi_lo[0] = hi;
  out_hi_lo[1] = lo;
  return OK;
}

// Exposed for the pow pins.
double orcl_pow_cr(double x, double q) { return pow_cr(x, q); }
long orcl_pow_fallbacks(void) { return g_pow_fallbacks; }
long orcl_pow_hard_cases(void) { return g_pow_hard; }

// Quad-precision reference value of x^q split as hi + lo (pins the CR rounding).
void orcl_pow_q(double x, double q, double* hi_lo) {
  __float128 y = powq((__float128)x, (__float128)q);
  hi_lo[0] = (double)y;
  hi_lo[1] = (double)(y - (__float128)hi_lo[0]);
}

}  // extern "C"
