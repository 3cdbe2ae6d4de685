// Stage 1 adjoint: dL/dK on the pattern -> dL/dE per cell and dL/dx per node.
//
// With Gauss points, weights and supports fixed, K depends on the node
// coordinates only through each point's shape-function gradients
// phi = G^{-1} r, where G (moment matrix) and r (derivative right-hand sides)
// depend on the coordinates.  For one Gauss point, with M = Kbar + Kbar^T:
//   Phibar[a] = sum_b lc (M_ab phi_b) + mc (M_ab^T phi_b) + mc tr(M_ab) phi_b
//   dL/dE_c  += (1/2) sum_ab <M_ab, k_ab> / E_c
//   lambda_k  = G^{-1} [Phibar_k; 0]          (G is symmetric: reuse its LU)
//   Gbar      = -sum_k lambda_k gamma_k^T,   rbar_k = lambda_k
//   dL/dx_a  += sum_b (Gbar_ab + Gbar_ba) R'(s_ab) 2 (x_a - x_b)
//             + sum_k (Gbar[a][n+1+k] + Gbar[n+1+k][a]) e_k
//             + sum_k lambda_k[a] dr_k[a]/dx_a
// Kernels: (1) symmetrise Kbar on the pattern; (2) row gather per node I
// (M's row held in LDS) producing Phibar and the dE share for every slot
// (g, local index of I); (3) one workgroup per Gauss point for the adjoint
// solves and the chain rule, writing per-slot coordinate gradients;
// (4) deterministic reductions of the slots to nodes (ascending g) and to
// cells (ascending g).  No atomics.
#include <cfloat>

#include "dd_pow.h"
#include "rpim_internal.h"

namespace rpim {
namespace {

constexpr int kT = 256;

__device__ __forceinline__ int64_t find_sorted(const int32_t* v, int64_t b, int64_t e, int32_t key) {
  while (b < e) {
    const int64_t m = (b + e) >> 1;
    if (v[m] < key) b = m + 1; else e = m;
  }
  return b;
}

// M = Kbar + Kbar^T, stored on the scalar CSR layout of K.
__global__ void k_symmetrize(int64_t nblk, const int64_t* blk_ptr, const int32_t* blk_row, const int32_t* blk_col,
                             const int32_t* row_lo, const int64_t* rbm_off, const uint2* rbm, const double* dK,
                             double* M) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nblk) return;
  const int32_t I = blk_row[e], J = blk_col[e];
  const int64_t bI = blk_ptr[I], LI = blk_ptr[I + 1] - bI, pI = e - bI;
  const int64_t bJ = blk_ptr[J], LJ = blk_ptr[J + 1] - bJ;
  const int64_t pJ = block_pos(blk_ptr, row_lo, rbm_off, rbm, J, I) - bJ;
  for (int al = 0; al < 3; ++al)
    for (int be = 0; be < 3; ++be) {
      const int64_t o = 9 * bI + 3 * al * LI + 3 * pI + be;
      const int64_t t = 9 * bJ + 3 * be * LJ + 3 * pJ + al;
      M[o] = dK[o] + dK[t];
    }
}

// Sum of 4 values over the block; result valid in every thread.
__device__ __forceinline__ void block_sum4(double v[4], double (*sh)[kT / 64]) {
  for (int o = 32; o > 0; o >>= 1)
    for (int i = 0; i < 4; ++i) v[i] += __shfl_xor(v[i], o, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int i = 0; i < 4; ++i) sh[i][w] = v[i];
  __syncthreads();
  for (int i = 0; i < 4; ++i) {
    double s = 0.0;
    for (int k = 0; k < kT / 64; ++k) s += sh[i][k];
    v[i] = s;
  }
  __syncthreads();
}

// Row gather: Phibar and dE share for each slot (g, a_I), I = blockIdx.x.
__global__ void __launch_bounds__(kT) k_bwd_rows(const int64_t* blk_ptr, const int32_t* row_lo,
                                                 const int64_t* rbm_off, const uint2* rbm,
                                                 const int64_t* inv_ptr, const uint64_t* inv_key,
                                                 const int64_t* gp_ptr, const int32_t* gp_nbr, const double* dphi,
                                                 const double* wdet, const int32_t* gp_cell, const double* E,
                                                 double lam, double mu, const double* M, double* pbar, double* dEs) {
  extern __shared__ double smem[];
  __shared__ double red[4][kT / 64];
  const int64_t I = blockIdx.x;
  const int64_t rb = blk_ptr[I];
  const int L = (int)(blk_ptr[I + 1] - rb);
  double* Mrow = smem;                  // [L][9]  M_IJ blocks of row I
  uint2* bm = (uint2*)(Mrow + 9 * L);   // row I's rank bitmap
  const int tid = threadIdx.x;
  const int lo_I = row_lo[I];
  const int64_t wb = rbm_off[I];
  const int nw = (int)(rbm_off[I + 1] - wb);
  for (int i = tid; i < nw; i += kT) bm[i] = rbm[wb + i];
  for (int idx = tid; idx < 9 * L; idx += kT) {
    const int pos = idx / 9, r = idx - 9 * pos, al = r / 3, be = r - 3 * al;
    Mrow[idx] = M[9 * rb + 3 * (int64_t)al * L + 3 * pos + be];
  }
  __syncthreads();
  for (int64_t e = inv_ptr[I]; e < inv_ptr[I + 1]; ++e) {
    const uint64_t key = inv_key[e];
    const int64_t g = (int64_t)(key >> 8);
    const int aI = (int)(key & 255);
    const int64_t b0 = gp_ptr[g];
    const int n = (int)(gp_ptr[g + 1] - b0);
    const double w = wdet[g];
    const double c = w * E[gp_cell[g]];
    const double lc = c * lam, mc = c * mu;
    const double pI[3] = {dphi[3 * (b0 + aI)], dphi[3 * (b0 + aI) + 1], dphi[3 * (b0 + aI) + 2]};
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = tid; b < n; b += kT) {
      const int32_t J = gp_nbr[b0 + b];
      const int r = J - lo_I;
      const uint2 wv = bm[r >> 5];
      const int lo = (int)wv.y + __popc(wv.x & ((1u << (r & 31)) - 1u));
      const double* Mb = Mrow + 9 * lo;
      const double pb[3] = {dphi[3 * (b0 + b)], dphi[3 * (b0 + b) + 1], dphi[3 * (b0 + b) + 2]};
      const double tr = Mb[0] + Mb[4] + Mb[8];
      for (int ga = 0; ga < 3; ++ga) {
        const double s1 = Mb[3 * ga] * pb[0] + Mb[3 * ga + 1] * pb[1] + Mb[3 * ga + 2] * pb[2];
        const double s2 = Mb[ga] * pb[0] + Mb[3 + ga] * pb[1] + Mb[6 + ga] * pb[2];
        v[ga] += lc * s1 + mc * s2 + mc * tr * pb[ga];
      }
      const double dot = pI[0] * pb[0] + pI[1] * pb[1] + pI[2] * pb[2];
      double kk = 0.0;
      for (int al = 0; al < 3; ++al)
        for (int be = 0; be < 3; ++be) {
          const double kv = lam * pI[al] * pb[be] + mu * pI[be] * pb[al] + (al == be ? mu * dot : 0.0);
          kk += Mb[3 * al + be] * kv;
        }
      v[3] += 0.5 * w * kk;
    }
    block_sum4(v, red);
    if (tid == 0) {
      const int64_t slot = b0 + aI;
      pbar[3 * slot] = v[0];
      pbar[3 * slot + 1] = v[1];
      pbar[3 * slot + 2] = v[2];
      dEs[slot] = v[3];
    }
  }
}

// Per Gauss point: adjoint solves with the kept LU, then the chain rule.
// LDS: lambda[3][N], gamma[3][N], S[n].
__global__ void __launch_bounds__(kT) k_bwd_gp(const int32_t* gp_order, int64_t order_begin, const int64_t* gp_ptr,
                                               const int32_t* gp_nbr, const int64_t* blk_ptr,
                                               const int32_t* row_lo, const int64_t* rbm_off, const uint2* rbm,
                                               const double* R, const double* X,
                                               const double* gp_xyz, double C2, double q, const int64_t* lu_off,
                                               const double* lu, const int32_t* piv, const double* gam,
                                               const double* pbar, double* dXs) {
  extern __shared__ double smem[];
  __shared__ double xg[3];
  const int tid = threadIdx.x;
  const int64_t g = gp_order[order_begin + blockIdx.x];
  const int64_t b0 = gp_ptr[g];
  const int n = (int)(gp_ptr[g + 1] - b0);
  const int N = n + 4;
  double* lamv = smem;          // [3][N]
  double* gm = lamv + 3 * N;    // [3][N]
  int* S = (int*)(gm + 3 * N);  // [n]
  const int64_t o = b0 + 4 * g;
  const double* LU = lu + lu_off[g];  // column-major
  for (int idx = tid; idx < 3 * N; idx += kT) {
    const int k = idx / N, i = idx - k * N;
    lamv[idx] = i < n ? pbar[3 * (b0 + i) + k] : 0.0;
    gm[idx] = gam[3 * o + idx];
  }
  for (int i = tid; i < n; i += kT) S[i] = gp_nbr[b0 + i];
  if (tid < 3) xg[tid] = gp_xyz[3 * g + tid];
  __syncthreads();
  // row swaps in factorisation order
  if (tid < 3) {
    double* b = lamv + tid * N;
    for (int k = 0; k < N; ++k) {
      const int p = piv[o + k];
      if (p != k) { const double t = b[k]; b[k] = b[p]; b[p] = t; }
    }
  }
  __syncthreads();
  // forward substitution with unit lower L
  for (int k = 0; k < N - 1; ++k) {
    for (int idx = tid; idx < 3 * (N - k - 1); idx += kT) {
      const int j = idx / (N - k - 1), r = k + 1 + idx % (N - k - 1);
      lamv[j * N + r] = __builtin_fma(-LU[(int64_t)k * N + r], lamv[j * N + k], lamv[j * N + r]);
    }
    __syncthreads();
  }
  // back substitution with U
  for (int k = N - 1; k >= 0; --k) {
    if (tid < 3) lamv[tid * N + k] = lamv[tid * N + k] / LU[(int64_t)k * N + k];
    __syncthreads();
    for (int idx = tid; idx < 3 * k; idx += kT) {
      const int j = idx / k, r = idx - j * k;
      lamv[j * N + r] = __builtin_fma(-LU[(int64_t)k * N + r], lamv[j * N + k], lamv[j * N + r]);
    }
    __syncthreads();
  }
  // chain rule per support node a
  for (int a = tid; a < n; a += kT) {
    const double* xa = X + 3 * (int64_t)S[a];
    double acc[3] = {0.0, 0.0, 0.0};
    const double la[3] = {lamv[a], lamv[N + a], lamv[2 * N + a]};
    const double ga[3] = {gm[a], gm[N + a], gm[2 * N + a]};
    for (int b = 0; b < n; ++b) {
      if (b == a) continue;
      const double* xb = X + 3 * (int64_t)S[b];
      const double gsum = -(la[0] * gm[b] + la[1] * gm[N + b] + la[2] * gm[2 * N + b] + lamv[b] * ga[0] +
                            lamv[N + b] * ga[1] + lamv[2 * N + b] * ga[2]);
      const double dx = xa[0] - xb[0], dy = xa[1] - xb[1], dz = xa[2] - xb[2];
      const double t = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx)) + C2;
      const double Rab = R[block_pos(blk_ptr, row_lo, rbm_off, rbm, S[a], S[b])];
      const double f = gsum * (q * Rab / t) * 2.0;
      acc[0] += f * dx;
      acc[1] += f * dy;
      acc[2] += f * dz;
    }
    for (int k = 0; k < 3; ++k) {
      const int i = n + 1 + k;
      acc[k] -= la[0] * gm[i] + la[1] * gm[N + i] + la[2] * gm[2 * N + i] + lamv[i] * ga[0] + lamv[N + i] * ga[1] +
                lamv[2 * N + i] * ga[2];
    }
    const double dgx[3] = {xg[0] - xa[0], xg[1] - xa[1], xg[2] - xa[2]};
    const double t = __builtin_fma(-dgx[2], -dgx[2], __builtin_fma(-dgx[1], -dgx[1], dgx[0] * dgx[0])) + C2;
    bool hard = false;
    const double Rg = pow_cr(t, q, &hard);
    const double tq1 = Rg / t, tq2 = Rg / (t * t);
    for (int cc = 0; cc < 3; ++cc) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) {
        const double dr = -(4.0 * q * (q - 1.0) * tq2 * dgx[cc] * dgx[k] + (k == cc ? 2.0 * q * tq1 : 0.0));
        s += la[k] * dr;
      }
      acc[cc] += s;
    }
    for (int k = 0; k < 3; ++k) dXs[3 * (b0 + a) + k] = acc[k];
  }
}

__global__ void k_reduce_nodes(int64_t N, const int64_t* inv_ptr, const uint64_t* inv_key, const int64_t* gp_ptr,
                               const double* dXs, double* dX) {
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= N) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int64_t e = inv_ptr[I]; e < inv_ptr[I + 1]; ++e) {
    const uint64_t key = inv_key[e];
    const int64_t slot = gp_ptr[(int64_t)(key >> 8)] + (int64_t)(key & 255);
    s0 += dXs[3 * slot];
    s1 += dXs[3 * slot + 1];
    s2 += dXs[3 * slot + 2];
  }
  dX[3 * I] = s0;
  dX[3 * I + 1] = s1;
  dX[3 * I + 2] = s2;
}

__global__ void k_reduce_gp(int64_t G, const int64_t* gp_ptr, const double* dEs, double* dEg) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  double s = 0.0;
  for (int64_t e = gp_ptr[g]; e < gp_ptr[g + 1]; ++e) s += dEs[e];
  dEg[g] = s;
}

__global__ void k_reduce_cells(int64_t C, const int64_t* cell_ptr, const int32_t* cell_gp, const double* dEg,
                               double* dE) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  double s = 0.0;
  for (int64_t e = cell_ptr[c]; e < cell_ptr[c + 1]; ++e) s += dEg[cell_gp[e]];
  dE[c] = s;
}

inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

rpim_status launch_backward(rpim_plan* p, const double* X, const double* E, double nu, const double* dK, double* dE,
                            double* dX, hipStream_t s) {
  rpim_status st;
  if ((st = ensure(&p->msym, &p->cap_msym, p->nnz)) || (st = ensure(&p->pbar, &p->cap_pbar, 3 * p->sum_n)) ||
      (st = ensure(&p->dEs, &p->cap_dEs, p->sum_n)) || (st = ensure(&p->dEg, &p->cap_dEg, p->G)) ||
      (st = ensure(&p->dXs, &p->cap_dXs, 3 * p->sum_n)))
    return st;
  const double onep = 1.0 + nu;
  const double onem = 1.0 - 2.0 * nu;
  const double lam = nu / (onep * onem);
  const double mu = 1.0 / (2.0 * onep);
  const double ac = p->alpha_c * p->d_c;
  const double C2 = ac * ac;
  phase_begin(p, RPIM_PHASE_BWD_ROWS, s);
  if (p->nblk > 0)
    hipLaunchKernelGGL(k_symmetrize, dim3(nblocks(p->nblk, 256)), dim3(256), 0, s, p->nblk,
                       (const int64_t*)p->blk_ptr, (const int32_t*)p->blk_row, (const int32_t*)p->blk_col,
                       (const int32_t*)p->row_lo, (const int64_t*)p->rbm_off, (const uint2*)p->rbm, dK, p->msym);
  const int L = (int)p->max_row_blocks;
  const size_t lds_rows = sizeof(double) * 9 * (size_t)L + sizeof(uint2) * (size_t)p->max_row_words;
  if (lds_rows > 160 * 1024) return RPIM_E_RANGE;
  RPIM_HIP(hipFuncSetAttribute((const void*)k_bwd_rows, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_rows));
  hipLaunchKernelGGL(k_bwd_rows, dim3((unsigned)p->N), dim3(kT), lds_rows, s, (const int64_t*)p->blk_ptr,
                     (const int32_t*)p->row_lo, (const int64_t*)p->rbm_off, (const uint2*)p->rbm,
                     (const int64_t*)p->inv_ptr, (const uint64_t*)p->inv_key,
                     (const int64_t*)p->gp_ptr, (const int32_t*)p->gp_nbr, (const double*)p->dphi,
                     (const double*)p->gp_wdet, (const int32_t*)p->gp_cell, E, lam, mu, (const double*)p->msym,
                     p->pbar, p->dEs);
  RPIM_HIP(hipGetLastError());
  phase_end(p, RPIM_PHASE_BWD_ROWS, s);
  phase_begin(p, RPIM_PHASE_BWD_GP, s);
  for (const Bucket& b : p->buckets) {
    const int N = b.nmax;
    const size_t lds = sizeof(double) * 6 * (size_t)N + sizeof(int) * (size_t)N;
    hipLaunchKernelGGL(k_bwd_gp, dim3((unsigned)b.count), dim3(kT), lds, s, (const int32_t*)p->gp_order, b.begin,
                       (const int64_t*)p->gp_ptr, (const int32_t*)p->gp_nbr, (const int64_t*)p->blk_ptr,
                       (const int32_t*)p->row_lo, (const int64_t*)p->rbm_off, (const uint2*)p->rbm,
                       (const double*)p->R, X, (const double*)p->gp_xyz, C2, p->q,
                       (const int64_t*)p->lu_off, (const double*)p->lu, (const int32_t*)p->piv,
                       (const double*)p->gam, (const double*)p->pbar, p->dXs);
    RPIM_HIP(hipGetLastError());
  }
  phase_end(p, RPIM_PHASE_BWD_GP, s);
  phase_begin(p, RPIM_PHASE_BWD_REDUCE, s);
  hipLaunchKernelGGL(k_reduce_nodes, dim3(nblocks(p->N, 256)), dim3(256), 0, s, p->N, (const int64_t*)p->inv_ptr,
                     (const uint64_t*)p->inv_key, (const int64_t*)p->gp_ptr, (const double*)p->dXs, dX);
  hipLaunchKernelGGL(k_reduce_gp, dim3(nblocks(p->G, 256)), dim3(256), 0, s, p->G, (const int64_t*)p->gp_ptr,
                     (const double*)p->dEs, p->dEg);
  hipLaunchKernelGGL(k_reduce_cells, dim3(nblocks(p->C, 256)), dim3(256), 0, s, p->C, (const int64_t*)p->cell_ptr,
                     (const int32_t*)p->cell_gp, (const double*)p->dEg, dE);
  RPIM_HIP(hipGetLastError());
  phase_end(p, RPIM_PHASE_BWD_REDUCE, s);
  return RPIM_OK;
}

}  // namespace rpim
