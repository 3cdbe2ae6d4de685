// Device pieces shared by the register-resident moment-matrix solvers
// (shape_reg.hip, shape_panel.hip): wave reductions and broadcasts, and the
// build of one row of the augmented moment matrix [G | r_0 r_1 r_2] per
// thread.  Included by those two sources only.
#pragma once

#include <cfloat>
#include <climits>

#include "dd_pow.h"
#include "rpim_internal.h"

namespace rpim {
namespace solver {

__device__ __forceinline__ void flag_error(DevStatus* st, unsigned flag, int64_t g) {
  atomicOr(&st->flags, flag);
  if (g >= 0) atomicMin(&st->first_bad, (unsigned long long)g);
}

// Wave reductions on 32-bit values with DPP: inclusive row scans (row_shr 1, 2,
// 4, 8), then row_bcast 15 / 31 carry the row results up to lane 63.
template <bool kMax>
__device__ __forceinline__ unsigned dpp_step(unsigned v, unsigned id, int ctrl_sel) {
  unsigned o;
  switch (ctrl_sel) {
    case 0: o = __builtin_amdgcn_update_dpp(id, v, 0x111, 0xF, 0xF, false); break;
    case 1: o = __builtin_amdgcn_update_dpp(id, v, 0x112, 0xF, 0xF, false); break;
    case 2: o = __builtin_amdgcn_update_dpp(id, v, 0x114, 0xF, 0xF, false); break;
    case 3: o = __builtin_amdgcn_update_dpp(id, v, 0x118, 0xF, 0xF, false); break;
    case 4: o = __builtin_amdgcn_update_dpp(id, v, 0x142, 0xA, 0xF, false); break;
    default: o = __builtin_amdgcn_update_dpp(id, v, 0x143, 0xC, 0xF, false); break;
  }
  return kMax ? (o > v ? o : v) : (o < v ? o : v);
}

template <bool kMax>
__device__ __forceinline__ unsigned wave_reduce_u32(unsigned v) {
  const unsigned id = kMax ? 0u : 0xFFFFFFFFu;
#pragma unroll
  for (int i = 0; i < 6; ++i) v = dpp_step<kMax>(v, id, i);
  return __builtin_amdgcn_readlane(v, 63);
}

// Wave argmax of |x| over active lanes (value desc, key asc), exact on the
// bit pattern of the non-negative double; returns the value (-1 if none) and
// the winning key.
__device__ __forceinline__ void wave_argmax(double ax, bool active, unsigned key, double* best, unsigned* bkey) {
  const unsigned long long bits = __double_as_longlong(ax);
  const unsigned hi = active ? (unsigned)(bits >> 32) : 0u;
  const unsigned lo = (unsigned)bits;
  const unsigned mhi = wave_reduce_u32<true>(hi);
  // usually a single lane holds the largest high word: it is the winner, and
  // the low-word and key passes (which only break ties) are skipped
  const unsigned long long c1 = __ballot(active && hi == mhi);
  unsigned mlo, mkey;
  if (__popcll(c1) == 1) {
    const int L = __ffsll((long long)c1) - 1;
    mlo = (unsigned)__builtin_amdgcn_readlane((int)lo, L);
    mkey = (unsigned)__builtin_amdgcn_readlane((int)key, L);
  } else {
    mlo = wave_reduce_u32<true>((active && hi == mhi) ? lo : 0u);
    const bool cand = active && hi == mhi && lo == mlo;
    mkey = wave_reduce_u32<false>(cand ? key : 0xFFFFFFFFu);
  }
  *bkey = mkey;
  *best = (mkey == 0xFFFFFFFFu) ? -1.0 : __longlong_as_double(((unsigned long long)mhi << 32) | mlo);
}

__device__ __forceinline__ double wave_max_nonneg(double x) {
  double b;
  unsigned k;
  wave_argmax(x, true, 0u, &b, &k);
  return b;
}

// The winner's window as U row k: dst[j] = a[j] for the 16-column blocks in
// use (dst 16-byte aligned; the U storage is padded past its last row).
template <int NB, int WC>
__device__ __forceinline__ void write_row(const double (&a)[WC], double* dst, int len) {
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (16 * c < len) {
#pragma unroll
      for (int e = 0; e < 16; e += 2) {
        const int j = 16 * c + e;
        if (j + 1 < WC) *reinterpret_cast<double2*>(dst + j) = make_double2(a[j], a[j + 1]);
        else if (j < WC) dst[j] = a[j];
      }
    }
  }
}

// Lane e of each row of sixteen lanes broadcast to the whole row (64-bit DPP
// row_newbcast).  e must fold to a constant; every lane of the row must be
// active, since a disabled source lane reads as zero.
__device__ __forceinline__ double row_bcast(double v, int e) {
  const long long x = __double_as_longlong(v);
  long long r;
  switch (e) {
    case 0: r = __builtin_amdgcn_update_dpp(x, x, 0x150, 0xF, 0xF, true); break;
    case 1: r = __builtin_amdgcn_update_dpp(x, x, 0x151, 0xF, 0xF, true); break;
    case 2: r = __builtin_amdgcn_update_dpp(x, x, 0x152, 0xF, 0xF, true); break;
    case 3: r = __builtin_amdgcn_update_dpp(x, x, 0x153, 0xF, 0xF, true); break;
    case 4: r = __builtin_amdgcn_update_dpp(x, x, 0x154, 0xF, 0xF, true); break;
    case 5: r = __builtin_amdgcn_update_dpp(x, x, 0x155, 0xF, 0xF, true); break;
    case 6: r = __builtin_amdgcn_update_dpp(x, x, 0x156, 0xF, 0xF, true); break;
    case 7: r = __builtin_amdgcn_update_dpp(x, x, 0x157, 0xF, 0xF, true); break;
    case 8: r = __builtin_amdgcn_update_dpp(x, x, 0x158, 0xF, 0xF, true); break;
    case 9: r = __builtin_amdgcn_update_dpp(x, x, 0x159, 0xF, 0xF, true); break;
    case 10: r = __builtin_amdgcn_update_dpp(x, x, 0x15A, 0xF, 0xF, true); break;
    case 11: r = __builtin_amdgcn_update_dpp(x, x, 0x15B, 0xF, 0xF, true); break;
    case 12: r = __builtin_amdgcn_update_dpp(x, x, 0x15C, 0xF, 0xF, true); break;
    case 13: r = __builtin_amdgcn_update_dpp(x, x, 0x15D, 0xF, 0xF, true); break;
    case 14: r = __builtin_amdgcn_update_dpp(x, x, 0x15E, 0xF, 0xF, true); break;
    default: r = __builtin_amdgcn_update_dpp(x, x, 0x15F, 0xF, 0xF, true); break;
  }
  return __longlong_as_double(r);
}

// Update-and-shift, a[j] <- fma(-l, u[j], a[j + 1]) for the 16-column blocks
// in use; the window's last element becomes zero.  The pivot row comes from
// LDS one element per lane: lane c of every row of sixteen lanes reads
// element c of a block, and the fma takes element e from lane e of its row
// by DPP, so a block costs one 8-byte LDS read per lane instead of sixteen.
// The next block is requested before the current block's fmas (the buffer is
// padded to whole blocks).  Runs with every lane active (see row_bcast).
template <int NB, int WC>
__device__ __forceinline__ void shift_update(double (&a)[WC], double nl, const double* u, int len, int c16) {
  double ub[2];
  ub[0] = u[c16];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (16 * b < len) {
      if (b + 1 < NB) ub[(b + 1) & 1] = u[16 * (b + 1) + c16];
      // broadcasts four elements ahead of their multiply-adds, so a wave
      // running alone does not wait on each DPP result in turn
#pragma unroll
      for (int e0 = 0; e0 < 16; e0 += 4) {
        double u4[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) u4[e] = row_bcast(ub[b & 1], e0 + e);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int j = 16 * b + e0 + e;
          if (j + 1 < WC) a[j] = __builtin_fma(nl, u4[e], a[j + 1]);
          else if (j < WC) a[j] = 0.0;
        }
      }
    }
  }
}


// Per-support-node data of the build phase, kept in LDS (the solvers place
// them inside their U storage, which is written only after the build).
struct BuildLds {
  double* xs;     // [3 NMAX] support node coordinates
  double* coefs;  // [NMAX] right-hand-side coefficients
  int64_t* rwb;   // [NMAX] rank-bitmap word offset of each support node's pattern row
  int64_t* rbp;   // [NMAX] start of that row in the pair table
  int* S;         // [NMAX] support node ids
  int* rlo;       // [NMAX] first node id of that row's window
};

template <int NMAX>
__device__ __forceinline__ BuildLds build_lds(double* lds) {
  BuildLds b;
  b.xs = lds;
  b.coefs = lds + 3 * NMAX;
  b.rwb = reinterpret_cast<int64_t*>(lds + 4 * NMAX);
  b.rbp = reinterpret_cast<int64_t*>(lds + 5 * NMAX);
  b.S = reinterpret_cast<int*>(lds + 6 * NMAX);
  b.rlo = b.S + NMAX;
  return b;
}

// Stage the support of point g into LDS and compute the derivative
// right-hand-side coefficients fl(fl(2q) * R) / t (one power per support
// node).  Ends with a barrier.  Sets *hard when a power was not roundable.
template <int T>
__device__ __forceinline__ void stage_support(const BuildLds& bl, double* xg, int t, int64_t g, int64_t b0, int n,
                                              const int32_t* gp_nbr, const int32_t* row_lo, const int64_t* rbm_off,
                                              const int64_t* blk_ptr, const double* X, const double* gp_xyz,
                                              double C2, double q, bool* hard) {
  for (int i = t; i < n; i += T) {
    const int32_t I = gp_nbr[b0 + i];
    bl.S[i] = I;
    bl.rlo[i] = row_lo[I];
    bl.rwb[i] = rbm_off[I];
    bl.rbp[i] = blk_ptr[I];
    for (int k = 0; k < 3; ++k) bl.xs[3 * i + k] = X[3 * (int64_t)I + k];
  }
  if (t < 3) xg[t] = gp_xyz[3 * g + t];
  __syncthreads();
  for (int r = t; r < n; r += T) {
    const double* xa = bl.xs + 3 * r;
    const double dx = xa[0] - xg[0], dy = xa[1] - xg[1], dz = xa[2] - xg[2];
    const double tt = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx)) + C2;
    const double Rv = pow_cr(tt, q, hard);
    bl.coefs[r] = ((2.0 * q) * Rv) / tt;
  }
  __syncthreads();
}

// Thread t fills row t of [G | rhs] in registers: columns 0..N-1 of G (zero
// padding up to NMAX), then the three right-hand sides at NMAX..NMAX+2, then
// zeros up to WC.  The radial-basis block is symmetric bit for bit (the pair
// table evaluates each ordered pair from x_I - x_J, and squares do not see the
// sign), so lane t reads entry (S[c], S[t]) from row S[c] of the pair table:
// the row's window, rank words and start are uniform over the workgroup, and
// the lanes' loads fall into a few adjacent words and values of that one row.
// The loads run branch-free in batches of CB columns (past-the-end columns
// look up column 0 and are overwritten), so each batch's rank words are all in
// flight before its values are needed.  Rows t >= N are zero.
template <int NMAX, int WAVES, int WC>
__device__ __forceinline__ void build_row(double (&a)[WC], const BuildLds& bl, const double* xg, int t, int n,
                                          int N, const uint2* rbm, const double* R) {
  if (t < n) {
    // two dependent global loads per batch: bigger batches where registers
    // allow it without lowering occupancy (the two-wave kernels)
    constexpr int CB = WAVES > 1 ? 16 : 8;
    const int my_id = bl.S[t];
#pragma unroll
    for (int c0 = 0; c0 < NMAX; c0 += CB) {
      uint2 wd[CB];
      int rl[CB];
#pragma unroll
      for (int e = 0; e < CB; ++e) {
        if (c0 + e < NMAX) {
          const int cs = c0 + e < n ? c0 + e : 0;
          rl[e] = my_id - bl.rlo[cs];
          wd[e] = rbm[bl.rwb[cs] + (rl[e] >> 5)];
        }
      }
#pragma unroll
      for (int e = 0; e < CB; ++e) {
        if (c0 + e < NMAX) {
          const int cs = c0 + e < n ? c0 + e : 0;
          a[c0 + e] = R[bl.rbp[cs] + (int64_t)wd[e].y + __popc(wd[e].x & ((1u << (rl[e] & 31)) - 1u))];
        }
      }
      __builtin_amdgcn_sched_barrier(0);  // keep batches apart: bounded registers in flight
    }
    // columns n..N-1: [1, x_t - x_g]; zero padding after them
    const double xr0 = bl.xs[3 * t], xr1 = bl.xs[3 * t + 1], xr2 = bl.xs[3 * t + 2];
    const double d0 = xr0 - xg[0], d1 = xr1 - xg[1], d2 = xr2 - xg[2];
#pragma unroll
    for (int c = 0; c < NMAX; ++c) {
      if (c >= n) {  // uniform
        const int kk = c - n;
        a[c] = kk == 0 ? 1.0 : (kk == 1 ? d0 : (kk == 2 ? d1 : (kk == 3 ? d2 : 0.0)));
      }
    }
    const double cf = bl.coefs[t];
    a[NMAX] = cf * (xg[0] - xr0);
    a[NMAX + 1] = cf * (xg[1] - xr1);
    a[NMAX + 2] = cf * (xg[2] - xr2);
  } else if (t < N) {
    const int k = t - n - 1;  // -1 for the row of ones
#pragma unroll
    for (int c = 0; c < NMAX; ++c) a[c] = c < n ? (k < 0 ? 1.0 : bl.xs[3 * c + k] - xg[k]) : 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) a[NMAX + j] = (k == j) ? 1.0 : 0.0;
  } else {
#pragma unroll
    for (int c = 0; c < NMAX + 3; ++c) a[c] = 0.0;
  }
#pragma unroll
  for (int c = NMAX + 3; c < WC; ++c) a[c] = 0.0;
}

// Singularity threshold N * eps * max|G| over the workgroup (right-hand sides
// excluded); rmax holds WAVES doubles of LDS.  Contains a barrier.
template <int NMAX, int WAVES, int WC>
__device__ __forceinline__ double singular_threshold(const double (&a)[WC], int N, int lane, int w, double* rmax) {
  double mx = 0.0;
#pragma unroll
  for (int j = 0; j < NMAX; ++j)
    if (j < N) mx = fmax(mx, fabs(a[j]));
  mx = wave_max_nonneg(mx);
  if (lane == 0) rmax[w] = mx;
  __syncthreads();
  mx = rmax[0];
#pragma unroll
  for (int i = 1; i < WAVES; ++i) mx = fmax(mx, rmax[i]);
  return ((double)N * DBL_EPSILON) * mx;
}

// Back substitution by position from the U rows in LDS, k descending, then
// the outputs (gradients, and with keep the U entries of the packed factor
// matrix F, the pivot positions and the full solutions).  U row t starts at lds[my_off] (thread t's own row, t < N):
// its element j is column t + j and its right-hand sides sit at
// NMAX - t + (0, 1, 2).  At step k the thread at position k forms x_k = b_k / u_kk; the other threads
// of its wave take x_k by readlane (no barrier), and threads t < k update
// b_t <- fma(-u_tk, x_k, b_t).  With two waves, positions 64 and up belong
// to wave 1, which runs them first on its own; after one barrier wave 0
// applies those x_k in the same descending order and finishes.
template <int NMAX, int WAVES>
__device__ __forceinline__ void back_substitute_and_store(const double* lds, int my_off, double (*xsol)[NMAX],
                                                          const int* pivpos, int t, int N, int n, int64_t g,
                                                          int64_t b0, double* dphi, float* dphi32, int keep,
                                                          double* F, int32_t* piv_out, double* gam) {
  constexpr int T = 64 * WAVES;
  const int w = t >> 6;
  double bb[3] = {0.0, 0.0, 0.0};
  double ud = 1.0;
  if (t < N) {
    ud = lds[my_off];
#pragma unroll
    for (int j = 0; j < 3; ++j) bb[j] = lds[my_off + (NMAX - t) + j];
  }
  double myx[3] = {0.0, 0.0, 0.0};  // thread t: x at position t
  const auto bsub_step = [&](int k) {
    const int src = k & 63;
    const double urk = t < k ? lds[my_off + (k - t)] : 0.0;
    const double ukk = readlane_f64(ud, src);
    double x[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) x[j] = readlane_f64(bb[j], src) / ukk;
    if (t == k) {
#pragma unroll
      for (int j = 0; j < 3; ++j) myx[j] = x[j];
    }
    if (t < k) {
#pragma unroll
      for (int j = 0; j < 3; ++j) bb[j] = __builtin_fma(-urk, x[j], bb[j]);
    }
  };
  if constexpr (WAVES == 1) {
#pragma unroll 1
    for (int k = N - 1; k >= 0; --k) bsub_step(k);
  } else {
    static_assert(WAVES == 2, "waves");
    if (w == 1) {
#pragma unroll 1
      for (int k = N - 1; k >= 64; --k) bsub_step(k);
      if (t < N) {
#pragma unroll
        for (int j = 0; j < 3; ++j) xsol[j][t] = myx[j];
      }
    }
    __syncthreads();
    if (w == 0) {
#pragma unroll 1
      for (int k = N - 1; k >= 64; --k) {
        const double urk = lds[my_off + (k - t)];
#pragma unroll
        for (int j = 0; j < 3; ++j) bb[j] = __builtin_fma(-urk, xsol[j][k], bb[j]);
      }
#pragma unroll 1
      for (int k = (N < 64 ? N : 64) - 1; k >= 0; --k) bsub_step(k);
    }
  }
  if (t < N && (WAVES == 1 || w == 0)) {
#pragma unroll
    for (int j = 0; j < 3; ++j) xsol[j][t] = myx[j];
  }
  __syncthreads();

  // ---- outputs ---------------------------------------------------------------
  for (int idx = t; idx < 3 * n; idx += T) {
    const int aa = idx / 3, j = idx - 3 * aa;
    dphi[3 * (b0 + aa) + j] = xsol[j][aa];
    if (dphi32) dphi32[3 * (b0 + aa) + j] = (float)xsol[j][aa];
  }
  if (keep) {
    // U by position into the packed factor matrix: F[c*N + p] = u_pc, c >= p;
    // row c of F in one store per wave (lane p writes column p)
    if (t < N) {
#pragma unroll 4
      for (int c = t & ~63; c < N; ++c)
        if (t <= c) F[(int64_t)c * N + t] = lds[my_off + (c - t)];
    }
    const int64_t o = b0 + 4 * g;
    for (int i = t; i < N; i += T) piv_out[o + i] = pivpos[i];
    for (int idx = t; idx < 3 * N; idx += T) {
      const int j = idx / N, i = idx - j * N;
      gam[3 * o + idx] = xsol[j][i];
    }
  }
}

}  // namespace solver
}  // namespace rpim
