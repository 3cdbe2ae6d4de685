// Moving-least-squares shape functions (GeoMFree3D Sec. 4 names moving least
// squares as the package's next shape functions): linear basis (M = 4) or
// constant basis (M = 1, Shepard's functions), with the cubic-spline weight
// over the support radius.  They replace the RPIM moment-matrix solve for a
// plan that selects them; the row gather then assembles K from the same
// gradient array.
//
// Operation order (the written contract the CPU checker follows as well):
//   M1  d = x_g - x_i; s = fma(dz,dz, fma(dy,dy, dx*dx)); r = sqrt(s) / d_s;
//       basis p = [1, x_i - x_g] (M = 4) or [1] (M = 1).
//   M2  r2 = r*r; r <= 1/2: W = (fl(2/3) - 4*r2) + (4*r2)*r, Wr = fma(12, r, -8);
//       1/2 < r <= 1: W = ((fl(4/3) - 4*r) + 4*r2) - fl(4/3)*(r2*r),
//       Wr = (8 - 4/r) - 4*r; else W = Wr = 0; w_k = (Wr*d_k) / fl(d_s*d_s).
//   M3  A_jl (j <= l) = +0 + t_1 + t_2 + ... in ascending support order,
//       t = (W*p_j)*p_l; A^k with t = (w_k*p_j)*p_l; A_lj = A_jl.
//   M4  A = LU with partial pivoting (first largest |a_rk|, whole-row swaps,
//       l = a_rk/a_kk, a_rj = fma(-l, a_kj, a_rj); singular if
//       |u_kk| <= M*eps*max|A|); gamma = A^-1 e_0: interchanges applied to
//       the right-hand side in step order, forward b_r = fma(-l_rk, b_k, b_r),
//       back b_k = b_k / u_kk then b_r = fma(-u_rk, b_k, b_r), k descending.
//   M5  gamma_k = A^-1 rhs, rhs_j = [j == k+1] - s_j, s_j = fma chain over l
//       ascending of A^k_jl gamma_l from +0 ([j == k+1] only for M = 4).
//   M6  c = fma(g3,p3, fma(g2,p2, fma(g1,p1, g0))) (g0 for M = 1), c_k from
//       gamma_k likewise; phi = W*c, dphi_k = fma(W, c_k, w_k*c).
//
// One wave per Gauss point: lanes take support entries for M1/M2 and M6; the
// 4 M (M + 1) / 2 ascending sums of M3 run one per lane; every lane then
// forms the same 4 x 4 factorisation from those sums (a few hundred flops).
// The kernel reads the support's coordinates and writes the gradients: its
// bound is memory latency and traffic, not arithmetic.
#include <cfloat>

#include "rpim_internal.h"

namespace rpim {
namespace {

constexpr int kMlsMaxN = kMaxSupport;

__device__ __forceinline__ void flag_error(DevStatus* st, unsigned flag, int64_t g) {
  atomicOr(&st->flags, flag);
  if (g >= 0) atomicMin(&st->first_bad, (unsigned long long)g);
}

template <int M>
__global__ void __launch_bounds__(64) k_mls(int64_t G, const int64_t* gp_ptr, const int32_t* gp_nbr, const double* X,
                                            const double* gp_xyz, double ds, double* dphi, float* dphi32,
                                            double* phi, DevStatus* st) {
  constexpr int NU = M * (M + 1) / 2;  // upper entries of one symmetric M x M matrix
  __shared__ double Wv[kMlsMaxN], wk[3][kMlsMaxN], qv[3][kMlsMaxN];
  __shared__ double sums[4 * NU];      // A, then A^0, A^1, A^2 (upper entries)
  const int lane = threadIdx.x;
  const int64_t g = blockIdx.x;
  if (g >= G) return;
  const int64_t b0 = gp_ptr[g];
  const int n = (int)(gp_ptr[g + 1] - b0);
  const double xg[3] = {gp_xyz[3 * g], gp_xyz[3 * g + 1], gp_xyz[3 * g + 2]};
  const double C23 = 2.0 / 3.0, C43 = 4.0 / 3.0;
  const double dw2 = ds * ds;
  // M1, M2
  for (int a = lane; a < n; a += 64) {
    const double* xi = X + 3 * (int64_t)gp_nbr[b0 + a];
    double d[3];
    for (int k = 0; k < 3; ++k) d[k] = xg[k] - xi[k];
    const double s = __builtin_fma(d[2], d[2], __builtin_fma(d[1], d[1], d[0] * d[0]));
    const double r = __builtin_sqrt(s) / ds;
    const double r2 = r * r;
    double W = 0.0, Wr = 0.0;
    if (r <= 0.5) {
      W = (C23 - 4.0 * r2) + (4.0 * r2) * r;
      Wr = __builtin_fma(12.0, r, -8.0);
    } else if (r <= 1.0) {
      W = ((C43 - 4.0 * r) + 4.0 * r2) - C43 * (r2 * r);
      Wr = (8.0 - 4.0 / r) - 4.0 * r;
    }
    Wv[a] = W;
    for (int k = 0; k < 3; ++k) {
      wk[k][a] = (Wr * d[k]) / dw2;
      qv[k][a] = xi[k] - xg[k];
    }
  }
  __syncthreads();
  // M3: sum e = c * NU + u, c = 0 for A and 1 + k for A^k, u the upper entry (j, l) in row order
  if (lane < 4 * NU) {
    const int c = lane / NU, u = lane - c * NU;
    int j = 0, l = 0;
    for (int e = 0, jj = 0; jj < M; ++jj)
      for (int ll = jj; ll < M; ++ll, ++e)
        if (e == u) {
          j = jj;
          l = ll;
        }
    double s = 0.0;
#pragma unroll 8
    for (int a = 0; a < n; ++a) {  // the loads run ahead, the sum stays in order
      const double wa = c == 0 ? Wv[a] : wk[c - 1][a];
      const double pj = j == 0 ? 1.0 : qv[j - 1][a];
      const double pl = l == 0 ? 1.0 : qv[l - 1][a];
      s = s + (wa * pj) * pl;
    }
    sums[lane] = s;
  }
  __syncthreads();
  const auto entry = [&](int c, int j, int l) {  // symmetric access to the upper entries
    if (j > l) {
      const int t = j;
      j = l;
      l = t;
    }
    const int u = j * M - j * (j - 1) / 2 + (l - j);
    return sums[c * NU + u];
  };
  // M4: every lane factors the same matrix
  double LU[M][M];
  double mx = 0.0;
  for (int j = 0; j < M; ++j)
    for (int l = 0; l < M; ++l) {
      LU[j][l] = entry(0, j, l);
      mx = fmax(mx, fabs(LU[j][l]));
    }
  const double tiny = ((double)M * DBL_EPSILON) * mx;
  int piv[M];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    int p = k;
    double best = fabs(LU[k][k]);
#pragma unroll
    for (int r = k + 1; r < M; ++r) {
      const double v = fabs(LU[r][k]);
      if (v > best) {
        best = v;
        p = r;
      }
    }
    piv[k] = p;
    if (!(best > tiny)) {  // uniform
      if (lane == 0) flag_error(st, kFlagSingular, g);
      return;
    }
#pragma unroll
    for (int r = 0; r < M; ++r)
      if (r == p && p != k)
#pragma unroll
        for (int c = 0; c < M; ++c) {
          const double t = LU[k][c];
          LU[k][c] = LU[r][c];
          LU[r][c] = t;
        }
#pragma unroll
    for (int r = k + 1; r < M; ++r) {
      const double l = LU[r][k] / LU[k][k];
      LU[r][k] = l;
#pragma unroll
      for (int c = k + 1; c < M; ++c) LU[r][c] = __builtin_fma(-l, LU[k][c], LU[r][c]);
    }
  }
  const auto solve = [&](double(&b)[M]) {
#pragma unroll
    for (int k = 0; k < M; ++k) {
#pragma unroll
      for (int r = k + 1; r < M; ++r)
        if (piv[k] == r) {
          const double t = b[k];
          b[k] = b[r];
          b[r] = t;
        }
    }
#pragma unroll
    for (int k = 0; k < M; ++k)
#pragma unroll
      for (int r = k + 1; r < M; ++r) b[r] = __builtin_fma(-LU[r][k], b[k], b[r]);
#pragma unroll
    for (int k = M - 1; k >= 0; --k) {
      b[k] = b[k] / LU[k][k];
#pragma unroll
      for (int r = 0; r < k; ++r) b[r] = __builtin_fma(-LU[r][k], b[k], b[r]);
    }
  };
  double gam[M];
#pragma unroll
  for (int j = 0; j < M; ++j) gam[j] = j == 0 ? 1.0 : 0.0;
  solve(gam);
  // M5
  double gk[3][M];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
#pragma unroll
    for (int j = 0; j < M; ++j) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < M; ++l) s = __builtin_fma(entry(1 + k, j, l), gam[l], s);
      gk[k][j] = (j == k + 1 ? 1.0 : 0.0) - s;
    }
    solve(gk[k]);
  }
  // M6
  for (int a = lane; a < n; a += 64) {
    const double q[3] = {qv[0][a], qv[1][a], qv[2][a]};
    double c = gam[0];
    if constexpr (M == 4) c = __builtin_fma(gam[3], q[2], __builtin_fma(gam[2], q[1], __builtin_fma(gam[1], q[0], c)));
    const double W = Wv[a];
    if (phi) phi[b0 + a] = W * c;
    if (dphi) {
      for (int k = 0; k < 3; ++k) {
        double ck = gk[k][0];
        if constexpr (M == 4)
          ck = __builtin_fma(gk[k][3], q[2], __builtin_fma(gk[k][2], q[1], __builtin_fma(gk[k][1], q[0], ck)));
        const double v = __builtin_fma(W, ck, wk[k][a] * c);
        dphi[3 * (b0 + a) + k] = v;
        if (dphi32) dphi32[3 * (b0 + a) + k] = (float)v;
      }
    }
  }
}

}  // namespace

rpim_status launch_mls(rpim_plan* p, const double* X, double* dphi, float* dphi32, double* phi, hipStream_t s) {
  if (p->G == 0) return RPIM_OK;
  if (p->max_n > kMlsMaxN) return RPIM_E_RANGE;
  const double ds = p->radius.empty() ? 0.0 : p->radius[0];
  for (double r : p->radius)
    if (r != ds) return RPIM_E_ARG;  // one weight radius for the whole plan
  if (p->shape_kind == RPIM_SHAPE_MLS)
    hipLaunchKernelGGL(k_mls<4>, dim3((unsigned)p->G), dim3(64), 0, s, p->G, (const int64_t*)p->gp_ptr,
                       (const int32_t*)p->gp_nbr, X, (const double*)p->gp_xyz, ds, dphi, dphi32, phi, p->status);
  else
    hipLaunchKernelGGL(k_mls<1>, dim3((unsigned)p->G), dim3(64), 0, s, p->G, (const int64_t*)p->gp_ptr,
                       (const int32_t*)p->gp_nbr, X, (const double*)p->gp_xyz, ds, dphi, dphi32, phi, p->status);
  RPIM_HIP(hipGetLastError());
  return RPIM_OK;
}

}  // namespace rpim
