// Moment-matrix solve with rows held in registers (gfx950).
//
// One workgroup of 64*WAVES threads per Gauss point; thread t owns row t of
// the augmented moment matrix [G | r_0 r_1 r_2] as a register *window*: at
// step k the window holds the row's columns k, k+1, ..., N-1 followed by its
// three right-hand sides (then zeros).  Rows never move; partial pivoting is
// done on row *positions* (the row order the textbook algorithm has after
// its swaps), which yields the same pivot choices, multipliers and fma
// sequence as whole-row swapping:
//   step k: the pivot is the active row with the largest |a_k| (window
//           element 0), ties to the smaller position; it takes position k,
//           the row that held position k takes the pivot's old position.
//           The pivot publishes its window through LDS; every other active
//           row computes l = a_k / u_kk and updates-and-shifts its window in
//           one pass: w_j <- fma(-l, u_{j+1}, w_{j+1}), so column k+1 becomes
//           element 0.  The pivot row's window (its U row) is kept in LDS.
// Back substitution then runs by position from the U rows in LDS, k
// descending: x_k = b_k / u_kk, b_r = fma(-u_rk, x_k, b_r) for r < k.
//
// Every register index is static: element 0 is always the pivot column.  The
// publish and the shifted update walk the window in blocks of BLK columns and
// skip blocks past the row's end under uniform branches; the update requests
// block c+1 of the pivot row from LDS before it issues the fmas of block c.
// Code size is O(NMAX).
#include <cfloat>
#include <climits>

#include "dd_pow.h"
#include "rpim_internal.h"

namespace rpim {
namespace {

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
  const unsigned mlo = wave_reduce_u32<true>((active && hi == mhi) ? lo : 0u);
  const bool cand = active && hi == mhi && lo == mlo;
  const unsigned mkey = wave_reduce_u32<false>(cand ? key : 0xFFFFFFFFu);
  *bkey = mkey;
  *best = (mkey == 0xFFFFFFFFu) ? -1.0 : __longlong_as_double(((unsigned long long)mhi << 32) | mlo);
}

__device__ __forceinline__ double wave_max_nonneg(double x) {
  double b;
  unsigned k;
  wave_argmax(x, true, 0u, &b, &k);
  return b;
}

// Candidate publish: dst[j] = a[j + 1] for the blocks in use.
template <int NBLK, int BLK, int WC>
__device__ __forceinline__ void publish_window(const double (&a)[WC], double* dst, int len) {
#pragma unroll
  for (int c = 0; c < NBLK; ++c) {
    if (BLK * c < len) {
#pragma unroll
      for (int e = 0; e < BLK; e += 2) {
        const int j = BLK * c + e;
        if (j + 2 < WC) *reinterpret_cast<double2*>(dst + j) = make_double2(a[j + 1], a[j + 2]);
        else if (j + 1 < WC) dst[j] = a[j + 1];
      }
    }
  }
}

// Update-and-shift, a[j] <- fma(-l, u[j], a[j + 1]) for the blocks in use; the
// window's last element becomes zero.  Each block requests the next block of
// the pivot row from LDS before it issues its own fmas (the pivot-row buffer
// is padded to whole blocks, so the request past the row's end stays inside
// it).
template <int NBLK, int BLK, int WC>
__device__ __forceinline__ void shift_update(double (&a)[WC], double nl, const double* u, int len) {
  double ub[2][BLK];
#pragma unroll
  for (int e = 0; e < BLK; e += 2) {
    const double2 v = *reinterpret_cast<const double2*>(u + e);
    ub[0][e] = v.x;
    ub[0][e + 1] = v.y;
  }
#pragma unroll
  for (int c = 0; c < NBLK; ++c) {
    if (BLK * c < len) {
      if (c + 1 < NBLK) {
#pragma unroll
        for (int e = 0; e < BLK; e += 2) {
          const double2 v = *reinterpret_cast<const double2*>(u + BLK * (c + 1) + e);
          ub[(c + 1) & 1][e] = v.x;
          ub[(c + 1) & 1][e + 1] = v.y;
        }
      }
#pragma unroll
      for (int e = 0; e < BLK; ++e) {
        const int j = BLK * c + e;
        if (j + 1 < WC) a[j] = __builtin_fma(nl, ub[c & 1][e], a[j + 1]);
        else if (j < WC) a[j] = 0.0;
      }
    }
  }
}

template <int NMAX>
constexpr int u_size() {
  return NMAX * (NMAX + 7) / 2 + 8;  // sum over positions k < N <= NMAX of (NMAX + 3 - k)
}

template <int NMAX, int WAVES, int BLK>
__global__ void __launch_bounds__(64 * WAVES) k_shape_win(
    const int32_t* gp_order, int64_t order_begin, const int64_t* gp_ptr, const int32_t* gp_nbr,
    const int64_t* blk_ptr, const int32_t* row_lo, const int64_t* rbm_off, const uint2* rbm, const double* R,
    const double* X, const double* gp_xyz, double C2, double q, double* dphi, int keep, const int64_t* lu_off,
    double* lu, int32_t* piv_out, double* gam, DevStatus* st) {
  constexpr int T = 64 * WAVES;
  constexpr int WC = NMAX + 4;   // window: matrix columns + 3 right-hand sides + 1 zero
  constexpr int NBLK = (WC + BLK - 1) / BLK;
  constexpr int US = u_size<NMAX>();
  constexpr int LDSD = US;
  static_assert(T >= NMAX && NMAX % 8 == 0 && BLK % 2 == 0, "shape");
  __shared__ __align__(16) double lds[LDSD];            // the U rows
  __shared__ __align__(16) double prow[2][WAVES][NBLK * BLK];  // candidate windows shifted by one: prow[j] = w[j+1]
  __shared__ double cval[2][WAVES];
  __shared__ double cpiv[2][WAVES];                     // candidate's w[0]
  __shared__ unsigned ckey[2][WAVES];
  __shared__ double xsol[3][NMAX];
  __shared__ int S[NMAX];
  __shared__ int rlo[NMAX];          // per support node: first id of its row window,
  __shared__ int64_t rwb[NMAX];      // its rank-bitmap word offset,
  __shared__ int64_t rbp[NMAX];      // and its pattern row start
  __shared__ double xs[3 * NMAX];    // support node coordinates
  __shared__ int rowat[NMAX];
  __shared__ double xg[3];
  __shared__ double rmax[WAVES];
  __shared__ double coefs[NMAX];

  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t g = gp_order[order_begin + blockIdx.x];
  const int64_t b0 = gp_ptr[g];
  const int n = (int)(gp_ptr[g + 1] - b0);
  const int N = n + 4;
  for (int i = t; i < n; i += T) {
    const int32_t I = gp_nbr[b0 + i];
    S[i] = I;
    rlo[i] = row_lo[I];
    rwb[i] = rbm_off[I];
    rbp[i] = blk_ptr[I];
    for (int k = 0; k < 3; ++k) xs[3 * i + k] = X[3 * (int64_t)I + k];
  }
  if (t < 3) xg[t] = gp_xyz[3 * g + t];
  __syncthreads();
  // derivative right-hand-side coefficients fl(fl(2q) * R) / t, one power per support node
  bool hard = false;
  for (int r = t; r < n; r += T) {
    const double* xa = xs + 3 * r;
    const double dx = xa[0] - xg[0], dy = xa[1] - xg[1], dz = xa[2] - xg[2];
    const double tt = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx)) + C2;
    const double Rv = pow_cr(tt, q, &hard);
    coefs[r] = ((2.0 * q) * Rv) / tt;
  }
  __syncthreads();

  // ---- build: thread t fills row t of [G | rhs] in registers ---------------------
  // Columns 0..N-1 of G (zero padding up to NMAX), then the three right-hand
  // sides at NMAX..NMAX+2.  The radial-basis block is symmetric bit for bit
  // (the pair table evaluates each ordered pair from x_I - x_J, and squares
  // do not see the sign), so lane t reads entry (S[c], S[t]) from row S[c] of
  // the pair table: the row's window, rank words and start are uniform over
  // the workgroup, and the lanes' loads fall into a few adjacent words and
  // values of that one row.  The loads run branch-free in batches of CB
  // columns (past-the-end columns look up column 0 and are overwritten), so
  // each batch's rank words are all in flight before its values are needed.
  double a[WC];
  if (t < n) {
    constexpr int CB = 8;
    static_assert(NMAX % CB == 0, "batch");
    const int my_id = S[t];
#pragma unroll
    for (int c0 = 0; c0 < NMAX; c0 += CB) {
      uint2 wd[CB];
      int rl[CB];
#pragma unroll
      for (int e = 0; e < CB; ++e) {
        const int cs = c0 + e < n ? c0 + e : 0;
        rl[e] = my_id - rlo[cs];
        wd[e] = rbm[rwb[cs] + (rl[e] >> 5)];
      }
#pragma unroll
      for (int e = 0; e < CB; ++e) {
        const int cs = c0 + e < n ? c0 + e : 0;
        a[c0 + e] = R[rbp[cs] + (int64_t)wd[e].y + __popc(wd[e].x & ((1u << (rl[e] & 31)) - 1u))];
      }
      __builtin_amdgcn_sched_barrier(0);  // keep batches apart: bounded registers in flight
    }
    // columns n..N-1: [1, x_t - x_g]; zero padding after them
    const double xr0 = xs[3 * t], xr1 = xs[3 * t + 1], xr2 = xs[3 * t + 2];
    const double d0 = xr0 - xg[0], d1 = xr1 - xg[1], d2 = xr2 - xg[2];
#pragma unroll
    for (int c = 0; c < NMAX; ++c) {
      if (c >= n) {  // uniform
        const int kk = c - n;
        a[c] = kk == 0 ? 1.0 : (kk == 1 ? d0 : (kk == 2 ? d1 : (kk == 3 ? d2 : 0.0)));
      }
    }
    const double cf = coefs[t];
    a[NMAX] = cf * (xg[0] - xr0);
    a[NMAX + 1] = cf * (xg[1] - xr1);
    a[NMAX + 2] = cf * (xg[2] - xr2);
  } else if (t < N) {
    const int k = t - n - 1;  // -1 for the row of ones
#pragma unroll
    for (int c = 0; c < NMAX; ++c) a[c] = c < n ? (k < 0 ? 1.0 : xs[3 * c + k] - xg[k]) : 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) a[NMAX + j] = (k == j) ? 1.0 : 0.0;
  } else {
#pragma unroll
    for (int c = 0; c < NMAX + 3; ++c) a[c] = 0.0;
  }
#pragma unroll
  for (int c = NMAX + 3; c < WC; ++c) a[c] = 0.0;
  if (hard) flag_error(st, kFlagPow, g);

  // singularity threshold N * eps * max|G| (the right-hand sides excluded)
  double mx = 0.0;
#pragma unroll
  for (int j = 0; j < NMAX; ++j)
    if (j < N) mx = fmax(mx, fabs(a[j]));
  {
    mx = wave_max_nonneg(mx);
    if (lane == 0) rmax[w] = mx;
    __syncthreads();
    mx = rmax[0];
#pragma unroll
    for (int i = 1; i < WAVES; ++i) mx = fmax(mx, rmax[i]);
  }
  const double tiny = ((double)N * DBL_EPSILON) * mx;

  // ---- LU with partial pivoting on positions; windows shift each step ----------
  int pos = t;              // current position of my row
  const bool real = t < N;  // padding rows never take part
  double* Lkeep = keep ? lu + lu_off[g] : nullptr;      // multipliers, column-major by original row
  int uoff = 0;                                           // offset of U row k in lds
#pragma unroll 1
  for (int k = 0; k < N; ++k) {
    const int buf = k & 1;
    const int len = NMAX + 3 - k;  // window elements in use (columns k..NMAX-1 and 3 rhs)
    const bool active = real && pos >= k;
    double v;
    unsigned key;
    wave_argmax(fabs(a[0]), active, ((unsigned)pos << 8) | (unsigned)t, &v, &key);
    if ((key & 255u) == (unsigned)t) {  // this wave's candidate publishes its window
      publish_window<NBLK, BLK, WC>(a, prow[buf][w], len);
      cpiv[buf][w] = a[0];
    }
    if (lane == 0) {
      cval[buf][w] = v;
      ckey[buf][w] = key;
    }
    __syncthreads();
    double best = cval[buf][0];
    unsigned bkey = ckey[buf][0];
    int bw = 0;
#pragma unroll
    for (int i = 1; i < WAVES; ++i) {
      const double v2 = cval[buf][i];
      const unsigned k2 = ckey[buf][i];
      const bool take = v2 > best || (v2 == best && k2 < bkey);
      best = take ? v2 : best;
      bkey = take ? k2 : bkey;
      bw = take ? i : bw;
    }
    if (!(best > tiny)) {
      if (t == 0) flag_error(st, kFlagSingular, g);
      return;  // uniform: every thread saw the same best
    }
    const int prow_id = (int)(bkey & 255u), ppos = (int)(bkey >> 8);
    if (t == 0) rowat[k] = prow_id;
    if (t == prow_id) pos = k;
    else if (pos == k) pos = ppos;
    if (real && pos > k) {
      const double l = a[0] / cpiv[buf][bw];
      if (keep) Lkeep[(int64_t)k * N + t] = l;
      shift_update<NBLK, BLK, WC>(a, -l, prow[buf][bw], len);  // prow[j] = pivot column k+1+j
    }
    // keep the pivot's window as U row k, one element per thread; the buffer is
    // not written again before the next step's barrier
    if (t == 0) lds[uoff] = cpiv[buf][bw];
    for (int i = t; i < len - 1; i += T) lds[uoff + 1 + i] = prow[buf][bw][i];
    uoff += len;
  }
  __syncthreads();

  // ---- back substitution by position from the U rows, k descending ------------
  // U row k starts at k (NMAX + 3) - k (k - 1) / 2; its element j is column k + j
  // and its right-hand sides sit at NMAX - k + (0, 1, 2).
  int my_off = 0;
  double bb[3] = {0.0, 0.0, 0.0};
  if (t < N) {
    my_off = t * (NMAX + 3) - (t * (t - 1)) / 2;
#pragma unroll
    for (int j = 0; j < 3; ++j) bb[j] = lds[my_off + (NMAX - t) + j];
  }
  int koff = (N - 1) * (NMAX + 3) - ((N - 1) * (N - 2)) / 2;
#pragma unroll 1
  for (int k = N - 1; k >= 0; --k) {
    if (t == k) {
      const double ukk = lds[koff];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        bb[j] = bb[j] / ukk;
        xsol[j][k] = bb[j];
      }
    }
    __syncthreads();
    if (t < k) {
      const double urk = lds[my_off + (k - t)];
#pragma unroll
      for (int j = 0; j < 3; ++j) bb[j] = __builtin_fma(-urk, xsol[j][k], bb[j]);
    }
    koff -= (NMAX + 3 - (k - 1));
  }
  __syncthreads();

  // ---- outputs ---------------------------------------------------------------
  for (int idx = t; idx < 3 * n; idx += T) {
    const int aa = idx / 3, j = idx - 3 * aa;
    dphi[3 * (b0 + aa) + j] = xsol[j][aa];
  }
  if (keep) {
    // U by position, column-major (U[c*N + p] = u_pc), after the multipliers
    double* U = Lkeep + (int64_t)N * N;
    if (t < N) {
      const int off = t * (NMAX + 3) - (t * (t - 1)) / 2;
      for (int c = 0; c < N; ++c)
        if (t <= c) U[(int64_t)c * N + t] = lds[off + (c - t)];
    }
    const int64_t o = b0 + 4 * g;
    for (int i = t; i < N; i += T) piv_out[o + i] = rowat[i];
    for (int idx = t; idx < 3 * N; idx += T) {
      const int j = idx / N, i = idx - j * N;
      gam[3 * o + idx] = xsol[j][i];
    }
  }
}

template <int NMAX, int WAVES, int BLK>
rpim_status launch_one(rpim_plan* p, const Bucket& bk, const double* X, double C2, int keep, hipStream_t s) {
  hipLaunchKernelGGL((k_shape_win<NMAX, WAVES, BLK>), dim3((unsigned)bk.count), dim3(64 * WAVES), 0, s,
                     (const int32_t*)p->gp_order, bk.begin, (const int64_t*)p->gp_ptr, (const int32_t*)p->gp_nbr,
                     (const int64_t*)p->blk_ptr, (const int32_t*)p->row_lo, (const int64_t*)p->rbm_off,
                     (const uint2*)p->rbm, (const double*)p->R, X, (const double*)p->gp_xyz, C2, p->q, p->dphi,
                     keep, (const int64_t*)p->lu_off, p->lu, p->piv, p->gam, p->status);
  RPIM_HIP(hipGetLastError());
  return RPIM_OK;
}

}  // namespace

// Largest padded size handled in registers; bigger buckets use the LDS kernel.
int shape_reg_max() { return 104; }

rpim_status launch_shape_reg(rpim_plan* p, const Bucket& b, const double* X, double C2, int keep, hipStream_t s) {
  switch (b.nmax) {
    case 8: case 16: return launch_one<16, 1, 16>(p, b, X, C2, keep, s);
    case 24: return launch_one<24, 1, 16>(p, b, X, C2, keep, s);
    case 32: return launch_one<32, 1, 16>(p, b, X, C2, keep, s);
    case 40: return launch_one<40, 1, 16>(p, b, X, C2, keep, s);
    case 48: return launch_one<48, 1, 16>(p, b, X, C2, keep, s);
    case 56: return launch_one<56, 1, 16>(p, b, X, C2, keep, s);
    case 64: return launch_one<64, 1, 16>(p, b, X, C2, keep, s);
    case 72: return launch_one<72, 2, 8>(p, b, X, C2, keep, s);
    case 80: return launch_one<80, 2, 8>(p, b, X, C2, keep, s);
    case 88: return launch_one<88, 2, 8>(p, b, X, C2, keep, s);
    case 96: return launch_one<96, 2, 8>(p, b, X, C2, keep, s);
    case 104: return launch_one<104, 2, 8>(p, b, X, C2, keep, s);
    default: return RPIM_E_RANGE;
  }
}

}  // namespace rpim
