// After the solve (GeoMFree3D Sec. 2: the displacements are found first, the
// stresses from them; Sec. 3, Example 1, loads a cube by its own weight):
//   shape-function values  phi_g = G_g^-1 [R(x_g); 1, 0, 0, 0] (first n
//                          entries), from the kept LU factors of the assembly;
//   body force             f_I = sum_g w_g phi_I(x_g) b_g, per node in
//                          ascending g: e = fl(w_g phi) * b_k, f = f + e;
//   Gauss-point stress     H_ij = sum_a u_{S[a],i} dphi_a/dx_j (fma chain in
//                          ascending a from +0), eps = (H + H^T) / 2,
//                          tr = (eps_00 + eps_11) + eps_22, lc = E lam,
//                          mc2 = 2 (E mu): sigma_ii = fma(lc, tr, mc2 eps_ii),
//                          sigma_ij = mc2 eps_ij; [xx, yy, zz, yz, xz, xy].
// The operation orders are the written contract the CPU checker follows too,
// so results are bitwise equal to a serial evaluation.
#include "dd_pow.h"
#include "kept_solve.h"
#include "rpim_internal.h"

namespace rpim {
namespace {

constexpr int kT = 256;

__device__ __forceinline__ void flag_error(DevStatus* st, unsigned flag, int64_t g) {
  atomicOr(&st->flags, flag);
  if (g >= 0) atomicMin(&st->first_bad, (unsigned long long)g);
}

// One workgroup per Gauss point (whole waves, one thread per unknown).
__global__ void __launch_bounds__(kT) k_shape_values(const int32_t* gp_order, int64_t order_begin,
                                                     const int64_t* gp_ptr, const int32_t* gp_nbr, const double* X,
                                                     const double* gp_xyz, double C2, double q,
                                                     const int64_t* lu_off, const double* lu, const int32_t* piv,
                                                     double* phi, DevStatus* st) {
  extern __shared__ double smem[];
  const int tid = threadIdx.x;
  const int nT = blockDim.x;
  const int64_t g = gp_order[order_begin + blockIdx.x];
  const int64_t b0 = gp_ptr[g];
  const int n = (int)(gp_ptr[g + 1] - b0);
  const int N = n + 4;
  double* y = smem;             // [N] forward values by position
  double* x = y + N;            // [N] solution by unknown
  int* ppos = (int*)(x + N);    // [N] pivot positions
  const int64_t o = b0 + 4 * g;
  for (int i = tid; i < N; i += nT) ppos[i] = piv[o + i];
  // value right-hand side of my original row: R(x_g) for support rows, then [1, 0, 0, 0]
  double b[1] = {0.0};
  bool hard = false;
  if (tid < n) {
    const double* xa = X + 3 * (int64_t)gp_nbr[b0 + tid];
    const double* xq = gp_xyz + 3 * g;
    const double dx = xa[0] - xq[0], dy = xa[1] - xq[1], dz = xa[2] - xq[2];
    const double t = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx)) + C2;
    b[0] = pow_cr(t, q, &hard);
  } else if (tid == n) {
    b[0] = 1.0;
  }
  if (hard) flag_error(st, kFlagPow, g);
  __syncthreads();
  kept_solve<1>(lu + lu_off[g], ppos, N, tid, b, y, x);
  for (int a = tid; a < n; a += nT) phi[b0 + a] = x[a];
}

// One thread per node: its three components summed over the points whose
// support holds it, in ascending g (the inverse list order).
__global__ void k_body_force(int64_t N, const int64_t* inv_ptr, const uint64_t* inv_key, const int64_t* gp_ptr,
                             const double* wdet, const double* phi, const double* gp_force, double* f) {
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= N) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int64_t e = inv_ptr[I]; e < inv_ptr[I + 1]; ++e) {
    const uint64_t key = inv_key[e];
    const int64_t g = (int64_t)(key >> 8);
    const double c = wdet[g] * phi[gp_ptr[g] + (int64_t)(key & 255)];
    s0 = s0 + c * gp_force[3 * g];
    s1 = s1 + c * gp_force[3 * g + 1];
    s2 = s2 + c * gp_force[3 * g + 2];
  }
  f[3 * I] = s0;
  f[3 * I + 1] = s1;
  f[3 * I + 2] = s2;
}

// One thread per Gauss point.
__global__ void k_gauss_stress(int64_t G, const int64_t* gp_ptr, const int32_t* gp_nbr, const double* dphi,
                               const int32_t* gp_cell, const double* E, double lam, double mu, const double* u,
                               double* sigma) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  double H[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
  for (int64_t e = gp_ptr[g]; e < gp_ptr[g + 1]; ++e) {
    const int64_t I = gp_nbr[e];
    const double ui[3] = {u[3 * I], u[3 * I + 1], u[3 * I + 2]};
    const double dj[3] = {dphi[3 * e], dphi[3 * e + 1], dphi[3 * e + 2]};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) H[i][j] = __builtin_fma(ui[i], dj[j], H[i][j]);
  }
  double ep[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) ep[i][j] = 0.5 * (H[i][j] + H[j][i]);
  const double tr = (ep[0][0] + ep[1][1]) + ep[2][2];
  const double c = E[gp_cell[g]];
  const double lc = c * lam, mc2 = 2.0 * (c * mu);
  double* s = sigma + 6 * g;
#pragma unroll
  for (int i = 0; i < 3; ++i) s[i] = __builtin_fma(lc, tr, mc2 * ep[i][i]);
  s[3] = mc2 * ep[1][2];
  s[4] = mc2 * ep[0][2];
  s[5] = mc2 * ep[0][1];
}

inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

rpim_status launch_shape_values(rpim_plan* p, const double* X, double* phi, hipStream_t s) {
  const double ac = p->alpha_c * p->d_c;
  const double C2 = ac * ac;
  for (const Bucket& b : p->buckets) {
    const int N = b.nmax;
    const int threads = 64 * ((N + 63) / 64);
    if (threads > kT) return RPIM_E_RANGE;
    const size_t lds = sizeof(double) * 2 * (size_t)N + sizeof(int) * (size_t)N;
    hipLaunchKernelGGL(k_shape_values, dim3((unsigned)b.count), dim3(threads), lds, s, (const int32_t*)p->gp_order,
                       b.begin, (const int64_t*)p->gp_ptr, (const int32_t*)p->gp_nbr, X,
                       (const double*)p->gp_xyz, C2, p->q, (const int64_t*)p->lu_off, (const double*)p->lu,
                       (const int32_t*)p->piv, phi, p->status);
    RPIM_HIP(hipGetLastError());
  }
  return RPIM_OK;
}

rpim_status launch_body_force(rpim_plan* p, const double* phi, const double* gp_force, double* f, hipStream_t s) {
  hipLaunchKernelGGL(k_body_force, dim3(nblocks(p->N, 64)), dim3(64), 0, s, p->N, (const int64_t*)p->inv_ptr,
                     (const uint64_t*)p->inv_key, (const int64_t*)p->gp_ptr, (const double*)p->gp_wdet, phi,
                     gp_force, f);
  RPIM_HIP(hipGetLastError());
  return RPIM_OK;
}

rpim_status launch_gauss_stress(rpim_plan* p, const double* E, double nu, const double* u, double* sigma,
                                hipStream_t s) {
  const double onep = 1.0 + nu;
  const double onem = 1.0 - 2.0 * nu;
  const double lam = nu / (onep * onem);
  const double mu = 1.0 / (2.0 * onep);
  if (p->G == 0) return RPIM_OK;
  hipLaunchKernelGGL(k_gauss_stress, dim3(nblocks(p->G, kT)), dim3(kT), 0, s, p->G, (const int64_t*)p->gp_ptr,
                     (const int32_t*)p->gp_nbr, (const double*)p->dphi, (const int32_t*)p->gp_cell, E, lam, mu, u,
                     sigma);
  RPIM_HIP(hipGetLastError());
  return RPIM_OK;
}

}  // namespace rpim
