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
// (4) deterministic reductions of the slots to nodes (fixed-order per-lane
// sums and butterfly) and to cells (ascending g).  No atomics.
#include <cfloat>

#include "dd_pow.h"
#include "kept_solve.h"
#include "rpim_internal.h"

namespace rpim {
namespace {

constexpr int kT = 256;

// Sum over each row of sixteen lanes, delivered to the row's lane 15: an
// inclusive scan with DPP row shifts (lanes shifted in from outside the row
// read zero).  Fixed order, so deterministic; every lane must be active.
__device__ __forceinline__ double row16_sum(double v) {
  long long x;
  x = __builtin_amdgcn_update_dpp(0ll, __double_as_longlong(v), 0x111, 0xF, 0xF, true);
  v += __longlong_as_double(x);
  x = __builtin_amdgcn_update_dpp(0ll, __double_as_longlong(v), 0x112, 0xF, 0xF, true);
  v += __longlong_as_double(x);
  x = __builtin_amdgcn_update_dpp(0ll, __double_as_longlong(v), 0x114, 0xF, 0xF, true);
  v += __longlong_as_double(x);
  x = __builtin_amdgcn_update_dpp(0ll, __double_as_longlong(v), 0x118, 0xF, 0xF, true);
  v += __longlong_as_double(x);
  return v;
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

// Row gather: Phibar and dE share for each slot (g, a_I), I = blockIdx.x.
// Slots are independent, so each wave takes its own Gauss points and reduces
// within the wave: no barriers after the row load.
__global__ void __launch_bounds__(kT) k_bwd_rows(const int64_t* blk_ptr, const int32_t* row_lo,
                                                 const int64_t* rbm_off, const uint2* rbm,
                                                 const int64_t* inv_ptr, const uint64_t* inv_key,
                                                 const int64_t* gp_ptr, const int32_t* gp_nbr, const double* dphi,
                                                 const double* wdet, const int32_t* gp_cell, const double* E,
                                                 double lam, double mu, const double* M, double* pbar, double* dEs) {
  extern __shared__ double smem[];
  const int64_t I = blockIdx.x;
  const int64_t rb = blk_ptr[I];
  const int L = (int)(blk_ptr[I + 1] - rb);
  double* Mrow = smem;                  // [L][9]  M_IJ blocks of row I
  uint2* bm = (uint2*)(Mrow + 9 * L);   // row I's rank bitmap
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int lo_I = row_lo[I];
  const int64_t wb = rbm_off[I];
  const int nw = (int)(rbm_off[I + 1] - wb);
  for (int i = tid; i < nw; i += kT) bm[i] = rbm[wb + i];
  for (int idx = tid; idx < 9 * L; idx += kT) {
    const int pos = idx / 9, r = idx - 9 * pos, al = r / 3, be = r - 3 * al;
    Mrow[idx] = M[9 * rb + 3 * (int64_t)al * L + 3 * pos + be];
  }
  __syncthreads();
  // Each wave takes four slots at a time, sixteen lanes per slot (lanes over
  // the support of the slot's point), so four independent chains of dependent
  // loads are in flight per wave.  Wave wv's groups start at slots
  // s_beg + 4 wv + 16 t; the metadata of sixteen groups (64 slots, one per
  // lane) is loaded at once and handed to each group's lanes by shuffle.
  const int q = lane >> 4, ql = lane & 15;
  const int64_t s_beg = inv_ptr[I], e_end = inv_ptr[I + 1];
  for (int64_t gbase = s_beg + 4 * wv; gbase < e_end; gbase += 16 * (kT / 16)) {
    // lane l: slot gbase + 16 (l / 4) + l % 4 (past the end: the last slot)
    const int64_t sl = gbase + 16 * (lane >> 2) + (lane & 3);
    const uint64_t keyl = inv_key[sl < e_end ? sl : e_end - 1];
    const int64_t gl = (int64_t)(keyl >> 8);
    const int64_t b0l = gp_ptr[gl];
    const int nl = (int)(gp_ptr[gl + 1] - b0l);
    const double wl = wdet[gl];
    const double cl = wl * E[gp_cell[gl]];
    for (int t = 0; t < 16 && gbase + 16 * t < e_end; ++t) {  // uniform
      const int64_t e = gbase + 16 * t + q;
      const bool live = e < e_end;
      const int src = 4 * t + q;
      double v[4] = {0.0, 0.0, 0.0, 0.0};
      const int64_t b0 = __shfl(b0l, src, 64);
      const int aI = (int)(__shfl((long long)keyl, src, 64) & 255);
      const int n = __shfl(nl, src, 64);
      const double w = __shfl(wl, src, 64);
      const double c = __shfl(cl, src, 64);
      if (live) {
        const double lc = c * lam, mc = c * mu, hw = 0.5 * w;
        const double pI[3] = {dphi[3 * (b0 + aI)], dphi[3 * (b0 + aI) + 1], dphi[3 * (b0 + aI) + 2]};
#pragma unroll 2
        for (int b = ql; b < n; b += 16) {
          const int32_t J = gp_nbr[b0 + b];
          const int r = J - lo_I;
          const uint2 bw = bm[r >> 5];
          const int pos = (int)bw.y + __popc(bw.x & ((1u << (r & 31)) - 1u));
          const double* Mb = Mrow + 9 * pos;
          const double pb[3] = {dphi[3 * (b0 + b)], dphi[3 * (b0 + b) + 1], dphi[3 * (b0 + b) + 2]};
          const double tr = Mb[0] + Mb[4] + Mb[8];
          // <M_IJ, k_IJ> with k_IJ = lam pI pb^T + mu pb pI^T + mu (pI . pb) 1 is
          // lam pI.(M pb) + mu pI.(M^T pb) + mu tr(M) (pI . pb): the products s1 = M pb
          // and s2 = M^T pb serve both sums
          // (fused multiply-adds throughout: these sums carry no rounding contract)
          const double mtr = mc * tr;
          double d1 = 0.0, d2 = 0.0;
          for (int ga = 0; ga < 3; ++ga) {
            const double s1 = __builtin_fma(Mb[3 * ga + 2], pb[2], __builtin_fma(Mb[3 * ga + 1], pb[1], Mb[3 * ga] * pb[0]));
            const double s2 = __builtin_fma(Mb[6 + ga], pb[2], __builtin_fma(Mb[3 + ga], pb[1], Mb[ga] * pb[0]));
            v[ga] = __builtin_fma(lc, s1, __builtin_fma(mc, s2, __builtin_fma(mtr, pb[ga], v[ga])));
            d1 = __builtin_fma(pI[ga], s1, d1);
            d2 = __builtin_fma(pI[ga], s2, d2);
          }
          const double dot = __builtin_fma(pI[2], pb[2], __builtin_fma(pI[1], pb[1], pI[0] * pb[0]));
          v[3] = __builtin_fma(hw, __builtin_fma(lam, d1, __builtin_fma(mu, d2, (mu * tr) * dot)), v[3]);
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = row16_sum(v[i]);
      if (live && ql == 15) {
        const int64_t slot = b0 + aI;
        pbar[3 * slot] = v[0];
        pbar[3 * slot + 1] = v[1];
        pbar[3 * slot + 2] = v[2];
        dEs[slot] = v[3];
      }
    }
  }
}

// Per Gauss point: adjoint solves with the kept LU, then the chain rule.
// Thread r owns original row r for the forward substitution and position r
// for the back substitution (right-hand sides in registers); each step's
// factor entry is loaded before the step's barrier.  The chain rule runs over
// (a, b) pairs with four threads per support node a and a fixed-order
// shuffle reduction of their partial sums.  The kernel is bound by the
// latency of its dependent chains (substitution steps, the pair-table
// gathers), so it is held to five waves per SIMD: faster, measured, than four
// waves without the few registers' worth of spills that five cost.
__global__ void __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(5))) k_bwd_gp(const int32_t* gp_order, int64_t order_begin, const int64_t* gp_ptr,
                                               const int32_t* gp_nbr, const int64_t* blk_ptr,
                                               const int32_t* row_lo, const int64_t* rbm_off, const uint2* rbm,
                                               const double* R, const double* X,
                                               const double* gp_xyz, double C2, double q, const int64_t* lu_off,
                                               const double* lu, const int32_t* piv, const double* gam,
                                               const double* pbar, double* dXs) {
  extern __shared__ double smem[];
  __shared__ double xg[3];
  const int tid = threadIdx.x;
  const int nT = blockDim.x;  // 64 * ceil(N / 64): one thread per unknown, whole waves
  const int64_t g = gp_order[order_begin + blockIdx.x];
  const int64_t b0 = gp_ptr[g];
  const int n = (int)(gp_ptr[g + 1] - b0);
  const int N = n + 4;
  double* lamv = smem;            // [3][N] solution lambda_k (by unknown)
  double* gm = lamv + 3 * N;      // [3][N] gamma_k
  double* y = gm + 3 * N;         // [3][N] forward values by position
  double* xs = y + 3 * N;         // [n][3] support coordinates
  double* tq = xs + 3 * n;        // [2][n] R/t and R/t^2 of the RPIM basis at the point, per support node
  int64_t* rwbS = (int64_t*)(tq + 2 * n);  // [n] rank-word offset of each support node's row
  int64_t* rbpS = rwbS + n;                // [n] pattern start of each support node's row
  int* S = (int*)(rbpS + n);      // [n]
  int* ppos = S + n;              // [N] position of each step's pivot before its interchange
  int* rloS = ppos + N;           // [n] window start of each support node's row
  const int64_t o = b0 + 4 * g;
  // packed factors, column-major F[c*N + p]: u_pc for p <= c; for p > c the
  // multiplier of step c for the row at position p after that step's interchange
  const double* Fm = lu + lu_off[g];
  for (int idx = tid; idx < 3 * N; idx += nT) gm[idx] = gam[3 * o + idx];
  for (int i = tid; i < n; i += nT) {
    const int32_t sidx = gp_nbr[b0 + i];
    S[i] = sidx;
    rloS[i] = row_lo[sidx];
    rwbS[i] = rbm_off[sidx];
    rbpS[i] = blk_ptr[sidx];
    for (int k = 0; k < 3; ++k) xs[3 * i + k] = X[3 * (int64_t)sidx + k];
  }
  for (int i = tid; i < N; i += nT) ppos[i] = piv[o + i];
  if (tid < 3) xg[tid] = gp_xyz[3 * g + tid];
  // right-hand side [Phibar_k; 0] of my original row
  const bool own = tid < N;
  double b[3] = {0.0, 0.0, 0.0};
  if (own && tid < n)
    for (int k = 0; k < 3; ++k) b[k] = pbar[3 * (b0 + tid) + k];
  __syncthreads();
  // the basis R(x_g, x_a) = t^q and its two quotients, one lane per support
  // node (kept apart from the chain rule's live values); the solve's barriers
  // order these LDS writes before their use
  for (int a = tid; a < n; a += nT) {
    const double dgx[3] = {xg[0] - xs[3 * a], xg[1] - xs[3 * a + 1], xg[2] - xs[3 * a + 2]};
    const double t = __builtin_fma(-dgx[2], -dgx[2], __builtin_fma(-dgx[1], -dgx[1], dgx[0] * dgx[0])) + C2;
    bool hard = false;
    const double Rg = pow_cr(t, q, &hard);
    tq[a] = Rg / t;
    tq[n + a] = Rg / (t * t);
  }
  // lambda_k = G^-1 [Phibar_k; 0] with the kept factors (G symmetric)
  kept_solve<3>(Fm, ppos, N, tid, b, y, lamv);
  // chain rule: four threads per support node a, partial sums over b = sub mod 4
  // in ascending b.  R_ab is read as entry (S[b], S[a]) of row S[b] of the pair
  // table (symmetric bit for bit), four b at a time with the loads first: one
  // load instruction touches four rows (one per sub) at the columns of sixteen
  // consecutive support nodes.
  for (int a0 = 0; a0 < n; a0 += nT / 4) {
    const int a = a0 + tid / 4, sub = tid & 3;
    double acc[3] = {0.0, 0.0, 0.0};
    if (a < n) {
      const double xa[3] = {xs[3 * a], xs[3 * a + 1], xs[3 * a + 2]};
      const double la[3] = {lamv[a], lamv[N + a], lamv[2 * N + a]};
      const double ga[3] = {gm[a], gm[N + a], gm[2 * N + a]};
      const int32_t Ia = S[a];
      for (int bb0 = sub; bb0 < n; bb0 += 16) {
        uint2 wv[4];
        int rr[4];
        double Rv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int bb = bb0 + 4 * j, bs = bb < n ? bb : sub;
          rr[j] = Ia - rloS[bs];
          wv[j] = rbm[rwbS[bs] + (rr[j] >> 5)];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int bb = bb0 + 4 * j, bs = bb < n ? bb : sub;
          Rv[j] = R[rbpS[bs] + (int64_t)wv[j].y + __popc(wv[j].x & ((1u << (rr[j] & 31)) - 1u))];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int bb = bb0 + 4 * j;
          if (bb < n && bb != a) {  // (fused multiply-adds: no rounding contract here)
            const double gsum = -__builtin_fma(
                lamv[2 * N + bb], ga[2],
                __builtin_fma(lamv[N + bb], ga[1],
                              __builtin_fma(lamv[bb], ga[0],
                                            __builtin_fma(la[2], gm[2 * N + bb],
                                                          __builtin_fma(la[1], gm[N + bb], la[0] * gm[bb])))));
            const double dx = xa[0] - xs[3 * bb], dy = xa[1] - xs[3 * bb + 1], dz = xa[2] - xs[3 * bb + 2];
            const double t = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx)) + C2;
            const double f = gsum * (q * Rv[j] / t) * 2.0;
            acc[0] = __builtin_fma(f, dx, acc[0]);
            acc[1] = __builtin_fma(f, dy, acc[1]);
            acc[2] = __builtin_fma(f, dz, acc[2]);
          }
        }
      }
    }
    // fixed-order reduction over the four threads of each node
    for (int k = 0; k < 3; ++k) {
      acc[k] += __shfl_xor(acc[k], 1, 64);
      acc[k] += __shfl_xor(acc[k], 2, 64);
    }
    if (a < n && sub == 0) {
      const double xa[3] = {xs[3 * a], xs[3 * a + 1], xs[3 * a + 2]};
      const double la[3] = {lamv[a], lamv[N + a], lamv[2 * N + a]};
      const double ga[3] = {gm[a], gm[N + a], gm[2 * N + a]};
      for (int k = 0; k < 3; ++k) {
        const int i = n + 1 + k;
        acc[k] -= la[0] * gm[i] + la[1] * gm[N + i] + la[2] * gm[2 * N + i] + lamv[i] * ga[0] +
                  lamv[N + i] * ga[1] + lamv[2 * N + i] * ga[2];
      }
      const double dgx[3] = {xg[0] - xa[0], xg[1] - xa[1], xg[2] - xa[2]};
      const double tq1 = tq[a], tq2 = tq[n + a];
      for (int cc = 0; cc < 3; ++cc) {
        double s2 = 0.0;
        for (int k = 0; k < 3; ++k) {
          const double dr = -(4.0 * q * (q - 1.0) * tq2 * dgx[cc] * dgx[k] + (k == cc ? 2.0 * q * tq1 : 0.0));
          s2 += la[k] * dr;
        }
        acc[cc] += s2;
      }
      for (int k = 0; k < 3; ++k) dXs[3 * (b0 + a) + k] = acc[k];
    }
  }
}

// dL/dx of node I: sum of its slots' contributions.  One wave per node: lane l
// sums entries l, l + 64, ... in ascending order, then a fixed butterfly adds
// the lanes (deterministic, no atomics).
__global__ void __launch_bounds__(256) k_reduce_nodes(int64_t N, const int64_t* inv_ptr, const uint64_t* inv_key,
                                                      const int64_t* gp_ptr, const double* dXs, double* dX) {
  const int64_t I = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (I >= N) return;  // uniform per wave
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int64_t e = inv_ptr[I] + lane; e < inv_ptr[I + 1]; e += 64) {
    const uint64_t key = inv_key[e];
    const int64_t slot = gp_ptr[(int64_t)(key >> 8)] + (int64_t)(key & 255);
    s0 += dXs[3 * slot];
    s1 += dXs[3 * slot + 1];
    s2 += dXs[3 * slot + 2];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    s0 += __shfl_xor(s0, o, 64);
    s1 += __shfl_xor(s1, o, 64);
    s2 += __shfl_xor(s2, o, 64);
  }
  if (lane == 0) {
    dX[3 * I] = s0;
    dX[3 * I + 1] = s1;
    dX[3 * I + 2] = s2;
  }
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
  if ((st = raise_lds_limit((const void*)k_bwd_rows, lds_rows, p->device)) != RPIM_OK) return st;
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
    const size_t lds = sizeof(double) * 14 * (size_t)N + sizeof(int64_t) * 2 * (size_t)N + sizeof(int) * (size_t)(3 * N);
    const int threads = 64 * ((N + 63) / 64);  // whole waves, at least one thread per unknown
    if (threads > kT) return RPIM_E_RANGE;
    hipLaunchKernelGGL(k_bwd_gp, dim3((unsigned)b.count), dim3(threads), lds, s, (const int32_t*)p->gp_order, b.begin,
                       (const int64_t*)p->gp_ptr, (const int32_t*)p->gp_nbr, (const int64_t*)p->blk_ptr,
                       (const int32_t*)p->row_lo, (const int64_t*)p->rbm_off, (const uint2*)p->rbm,
                       (const double*)p->R, X, (const double*)p->gp_xyz, C2, p->q,
                       (const int64_t*)p->lu_off, (const double*)p->lu, (const int32_t*)p->piv,
                       (const double*)p->gam, (const double*)p->pbar, p->dXs);
    RPIM_HIP(hipGetLastError());
  }
  phase_end(p, RPIM_PHASE_BWD_GP, s);
  phase_begin(p, RPIM_PHASE_BWD_REDUCE, s);
  hipLaunchKernelGGL(k_reduce_nodes, dim3(nblocks(p->N, 4)), dim3(256), 0, s, p->N, (const int64_t*)p->inv_ptr,
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
