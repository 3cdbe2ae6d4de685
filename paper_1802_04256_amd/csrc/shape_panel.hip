// Moment-matrix solve by blocked (panel) elimination, rows held in registers
// (gfx950).
//
// The elimination order is the one of the row-by-row kernel (shape_reg.hip)
// and of the arithmetic contract: pivot = first largest |a_rk| in current
// row order, l = a_rk / u_kk (IEEE division), every element updated by
// a_rj <- fma(-l, u_kj, a_rj) in ascending k, the three right-hand sides
// carried as extra columns.  What changes is when each update is applied.
//
// One workgroup of 64*WAVES threads per Gauss point; thread t owns row t of
// [G | r_0 r_1 r_2] as a register window whose element 0 is column k0, the
// first column of the current panel of kPanel = 16 columns.  Per panel:
//   1. Sixteen pivot steps that touch only the panel's columns: the pivot
//      search (wave reductions; with two waves each wave's candidate also posts
//      the sixteen panel elements of its row, so one barrier per step serves
//      both the choice and the broadcast), then every eliminated row forms its
//      multiplier, keeps it in place of the panel column, and updates the rest
//      of its panel columns.  Nothing outside the panel is touched, so a step
//      costs a handful of instructions besides the exchange.
//   2. The panel's pivot rows publish their windows: the panel part (their
//      multipliers and their U entries) to a 16 x 16 buffer, the trailing part
//      (columns right of the panel, not yet updated by this panel) straight
//      into their U rows.
//   3. The trailing parts of the sixteen U rows are completed column by column,
//      one thread per column: u_ij <- fma(-l_ii', u_i'j, u_ij) for i' < i in
//      ascending i', which is exactly the sequence of updates those elements
//      receive in the row-by-row order.
//   4. Every row still active applies the panel's sixteen updates to its
//      trailing columns, again in ascending step order, reading the new U rows
//      from LDS (all lanes read the same address: a broadcast), and shifts its
//      window by sixteen columns.
// The result, multipliers and U rows are bitwise those of the row-by-row
// kernel; the per-step chain that bounds that kernel (a full row written and
// read through LDS at every step) is replaced by two barriers per panel and a
// trailing update with sixteen independent multiply-add chains per block.
// U rows are stored compactly (row k from its diagonal: NMAX + 3 - k doubles
// rounded up to even), and back substitution is shared with the row-by-row
// kernel.
#include "shape_common.h"

namespace rpim {
namespace {

using namespace solver;

constexpr int kPanel = 16;

// Start of compact U row k (rows of (NMAX + 3 - k) doubles rounded up to even;
// NMAX is a multiple of 8): sum_{i<k} ((NMAX + 4 - i) & ~1).
template <int NMAX>
__host__ __device__ constexpr int uoff(int k) {
  return k * (NMAX + 4) - k * (k - 1) / 2 - k / 2;
}

template <int NMAX, int WAVES>
__global__ void __launch_bounds__(64 * WAVES, NMAX <= 88 ? 2 : 1) k_shape_panel(
    const int32_t* gp_order, int64_t order_begin, const int64_t* gp_ptr, const int32_t* gp_nbr,
    const int64_t* blk_ptr, const int32_t* row_lo, const int64_t* rbm_off, const uint2* rbm, const double* R,
    const double* X, const double* gp_xyz, double C2, double q, double* dphi, float* dphi32, int keep,
    const int64_t* lu_off, double* lu, int32_t* piv_out, double* gam, DevStatus* st) {
  constexpr int T = 64 * WAVES;
  constexpr int NB = kPanel;
  constexpr int WC = NMAX + 4;             // window: columns + 3 right-hand sides + 1 zero
  constexpr int NBLK = (WC + 15) / 16;     // blocks of sixteen window elements
  constexpr int US = uoff<NMAX>(NMAX) + 16;  // compact U rows (+ slack for a block's tail reads)
  static_assert(T >= NMAX && NMAX % 8 == 0 && NB == 16, "shape");
  static_assert(7 * NMAX <= US, "build data fit in the U storage");
  struct __align__(16) Cand {
    double v;      // |a_k| of the wave's candidate (-1: no active row)
    unsigned key;  // (position << 8) | row
    unsigned pad;
  };
  __shared__ __align__(16) double lds[US];             // U rows (build data before them)
  __shared__ __align__(16) double p11[NB][NB];         // panel part of the panel's pivot rows
  __shared__ __align__(16) double prow[2][WAVES][NB];  // each wave's candidate panel part (two steps in flight)
  __shared__ Cand cand[2][WAVES];
  __shared__ double xsol[3][NMAX];
  __shared__ int pivpos[NMAX];  // position the pivot of each step held before it
  __shared__ double xg[3];
  __shared__ double rmax[WAVES];
  __shared__ int mpos[64];  // hand-over: positions of the rows that move
  __shared__ int mcount, hstate;
  const BuildLds bl = build_lds<NMAX>(lds);

  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t g = gp_order[order_begin + blockIdx.x];
  const int64_t b0 = gp_ptr[g];
  const int n = (int)(gp_ptr[g + 1] - b0);
  const int N = n + 4;
  bool hard = false;
  stage_support<T>(bl, xg, t, g, b0, n, gp_nbr, row_lo, rbm_off, blk_ptr, X, gp_xyz, C2, q, &hard);
  double a[WC];
  build_row<NMAX, WAVES, WC>(a, bl, xg, t, n, N, rbm, R);
  if (hard) flag_error(st, kFlagPow, g);
  const double tiny = singular_threshold<NMAX, WAVES, WC>(a, N, lane, w, rmax);

  int pos = t;        // current position of my row
  bool real = t < N;  // padding rows never take part (a row handed over is real in its new lane)
  double* F = keep ? lu + lu_off[g] : nullptr;  // packed factors (multipliers by position)
  // One panel from column k0 on, by every wave of the workgroup or (ONE) by
  // wave 0 alone once it holds every row still active.  Returns 1 when every
  // row is pivoted, 2 on a singular pivot (flagged), 0 otherwise.
  auto panel = [&](auto one_tag, const int k0) -> int {
    constexpr bool ONE = decltype(one_tag)::value || WAVES == 1;
    constexpr int TT = ONE ? 64 : T;  // threads at work
    const auto sync = [&] {
      if constexpr (ONE && WAVES > 1) {  // wave 0 alone: its LDS accesses complete in program order
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      } else {
        __syncthreads();
      }
    };
      const int len = NMAX + 3 - k0;            // window elements in use (columns k0..NMAX-1, 3 rhs)
      const int nbe = N - k0 < NB ? N - k0 : NB;  // pivot steps in this panel
      // ---- 1. pivot steps inside the panel ---------------------------------------------
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        if (i < nbe) {  // uniform
          const int k = k0 + i;
          const bool active = real && pos >= k;
          double v;
          unsigned key;
          wave_argmax(fabs(a[i]), active, ((unsigned)pos << 8) | (unsigned)t, &v, &key);
          double best = v;
          unsigned bkey = key;
          double u[NB];  // pivot row, window elements i..NB-1 (panel columns k..k0+NB-1)
          if constexpr (WAVES > 1 && !ONE) {  // candidates and the pivot row through LDS
            const int buf = i & 1;
            if (lane == 0) {
              Cand c;
              c.v = key == 0xFFFFFFFFu ? -1.0 : v;
              c.key = key;
              c.pad = 0;
              cand[buf][w] = c;
            }
            if (key != 0xFFFFFFFFu && t == (int)(key & 255u)) {
#pragma unroll
              for (int j = 0; j < NB - i; ++j) prow[buf][w][j] = a[i + j];
            }
            sync();
            int wb = 0;
            best = cand[buf][0].v;
            bkey = cand[buf][0].key;
#pragma unroll
            for (int x = 1; x < (ONE ? 1 : WAVES); ++x) {
              const Cand c = cand[buf][x];
              const bool take = c.v > best || (c.v == best && c.key < bkey);
              best = take ? c.v : best;
              bkey = take ? c.key : bkey;
              wb = take ? x : wb;
            }
#pragma unroll
            for (int j = 0; j < NB - i; ++j) u[j] = prow[buf][wb][j];
          } else {
            if (key == 0xFFFFFFFFu) best = -1.0;
            const int L = (int)(key & 63u);
#pragma unroll
            for (int j = 0; j < NB - i; ++j) u[j] = readlane_f64(a[i + j], L);
          }
          if (!(best > tiny)) {
            if (t == 0) flag_error(st, kFlagSingular, g);
            return 2;  // uniform: every working thread saw the same best
          }
          const int prow_id = (int)(bkey & 255u), ppos = (int)(bkey >> 8);
          if (t == 0) pivpos[k] = ppos;
          if (t == prow_id) pos = k;
          else if (pos == k) pos = ppos;
          if (real && pos > k) {  // eliminated at this step
            const double l = a[i] / u[0];
            a[i] = l;  // kept in place of the panel column for steps 3 and 4
#pragma unroll
            for (int j = 1; j < NB - i; ++j) a[i + j] = __builtin_fma(-l, u[j], a[i + j]);
            if (keep) F[(int64_t)k * N + pos] = l;
          }
        }
      }
      // ---- 2. the panel's pivot rows publish their windows ------------------------------
      {
        const int pp = pos - k0;  // position inside the panel
        if (real && pp >= 0 && pp < nbe) {
#pragma unroll
          for (int j = 0; j < NB; j += 2)
            *reinterpret_cast<double2*>(&p11[pp][j]) = make_double2(a[j], a[j + 1]);
          double* dst = lds + uoff<NMAX>(k0 + pp) - pp;  // element j of the window -> dst[j]
#pragma unroll
          for (int j = NB; j < WC; ++j)
            if (j < len) dst[j] = a[j];
        }
      }
      sync();
      // ---- 3. trailing parts of the panel's U rows, one thread per column ---------------
      // The earlier rows' finished elements are read back from LDS rather than
      // kept in registers (the window stays live here), one row at a time.
      for (int j = NB + t; j < len; j += TT) {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          if (i < nbe) {  // uniform
            double* e = lds + uoff<NMAX>(k0 + i) + (j - i);
            double v = *e;
#pragma unroll
            for (int i2 = 0; i2 < i; ++i2) {
              v = __builtin_fma(-p11[i][i2], lds[uoff<NMAX>(k0 + i2) + (j - i2)], v);
              if ((i2 & 3) == 3) __builtin_amdgcn_sched_barrier(0);  // four terms' loads in flight at most
            }
            *e = v;
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
      // U rows' panel part: row k0+i from its diagonal (in the last panel the
      // right-hand sides may sit inside the panel's sixteen window elements)
      for (int idx = t; idx < NB * NB; idx += TT) {
        const int i = idx / NB, e = idx - i * NB;
        if (i < nbe && e >= i && e < len) lds[uoff<NMAX>(k0 + i) + (e - i)] = p11[i][e];
      }
      sync();
      if (k0 + NB >= N) return 1;  // uniform: every row is pivoted
      // ---- 4. trailing update and shift for the rows still active -----------------------
      // Each half block of the window (eight elements from 8 h) takes the
      // sixteen updates in ascending step order; the U values of step i + 1 are
      // loaded while step i's multiply-adds run (two sets of eight in flight).
      if (real && pos >= k0 + NB) {
#pragma unroll
        for (int h = 2; h < 2 * NBLK; ++h) {
          if (8 * h < len) {  // uniform
            double ub[2][8];
            auto load = [&](int i, double(&dst)[8]) {
              const double* urow = lds + uoff<NMAX>(k0 + i) + (8 * h - i);  // U_{k0+i} at window column 8 h
#pragma unroll
              for (int e = 0; e < 8; ++e)
                if (8 * h + e < WC) dst[e] = urow[e];
            };
            load(0, ub[0]);
#pragma unroll
            for (int i = 0; i < NB; ++i) {
              if (i + 1 < NB) load(i + 1, ub[(i + 1) & 1]);
              const double nl = -a[i];
#pragma unroll
              for (int e = 0; e < 8; ++e)
                if (8 * h + e < WC) a[8 * h + e] = __builtin_fma(nl, ub[i & 1][e], a[8 * h + e]);
              __builtin_amdgcn_sched_barrier(0);
            }
          }
        }
#pragma unroll
        for (int j = 0; j + NB < WC; ++j) a[j] = a[j + NB];
      }
      return 0;
  };

  int state = 0;
  int k0 = 0;
  // the hand-over's extra registers would cost the largest window its spill-free fit
  constexpr bool kHandOver = WAVES > 1 && NMAX <= 88;
  if constexpr (!kHandOver) {
#pragma unroll 1
    for (;; k0 += NB)
      if ((state = panel(std::false_type{}, k0)) != 0) break;
  } else {
#pragma unroll 1
    for (;; k0 += NB) {
      state = panel(std::false_type{}, k0);
      if (state != 0 || N - (k0 + NB) <= 64) break;  // uniform
    }
    if (state == 0) {
      // ---- hand-over: the rows still active fit in one wave -------------------------
      // Wave 1's active rows move, sixteen window elements at a time through
      // the U storage of rows not yet reached, to lanes of wave 0 whose rows
      // are pivoted; wave 0 then runs the remaining panels alone (no barrier
      // per pivot step) and wave 1 waits for the back substitution.  A row's
      // lane carries no meaning past the build: factors are stored by position.
      k0 += NB;
      constexpr int KH = 16 * ((NMAX - 64 + 15) / 16);  // latest hand-over column
      static_assert(uoff<NMAX>(NMAX) + 16 - uoff<NMAX>(KH) >= 64 * 16, "hand-over buffer fits");
      double* hb = lds + uoff<NMAX>(k0);
      const int lenn = NMAX + 3 - k0;  // window elements in use from column k0 on
      const bool act = real && pos >= k0;
      const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
      const unsigned long long mask = __ballot(w == 1 ? act : !act);  // wave 1: movers; wave 0: free lanes
      const int r = __popcll(mask & below);
      if (w == 1) {
        if (act) mpos[r] = pos;
        if (lane == 0) mcount = __popcll(mask);
      }
      __syncthreads();
      const bool take = w == 0 && !act && r < mcount;
#pragma unroll
      for (int c = 0; c < NBLK; ++c) {
        if (16 * c < lenn) {  // uniform
          if (w == 1 && act) {
#pragma unroll
            for (int e = 0; e < 16; ++e)
              if (16 * c + e < WC) hb[16 * r + e] = a[16 * c + e];
          }
          __syncthreads();
          if (take) {
#pragma unroll
            for (int e = 0; e < 16; ++e)
              if (16 * c + e < WC) a[16 * c + e] = hb[16 * r + e];
          }
          __syncthreads();
        }
      }
      if (take) {
        pos = mpos[r];
        real = true;
      }
      if (w == 0) {
#pragma unroll 1
        for (;; k0 += NB)
          if ((state = panel(std::true_type{}, k0)) != 0) break;
        if (t == 0) hstate = state;
      }
      __syncthreads();  // wave 1 waits here for wave 0's factorization
      state = hstate;
    }
  }
  if (state == 2) return;  // singular (uniform)

  // ---- back substitution by position from the U rows, then the outputs ----------
  back_substitute_and_store<NMAX, WAVES>(lds, t < N ? uoff<NMAX>(t) : 0, xsol, pivpos, t, N, n, g, b0, dphi, dphi32,
                                         keep, F, piv_out, gam);
}

template <int NMAX, int WAVES>
rpim_status launch_one(rpim_plan* p, const Bucket& bk, const double* X, double C2, int keep, float* dphi32,
                       hipStream_t s) {
  hipLaunchKernelGGL((k_shape_panel<NMAX, WAVES>), dim3((unsigned)bk.count), dim3(64 * WAVES), 0, s,
                     (const int32_t*)p->gp_order, bk.begin, (const int64_t*)p->gp_ptr, (const int32_t*)p->gp_nbr,
                     (const int64_t*)p->blk_ptr, (const int32_t*)p->row_lo, (const int64_t*)p->rbm_off,
                     (const uint2*)p->rbm, (const double*)p->R, X, (const double*)p->gp_xyz, C2, p->q, p->dphi,
                     dphi32, keep, (const int64_t*)p->lu_off, p->lu, p->piv, p->gam, p->status);
  RPIM_HIP(hipGetLastError());
  return RPIM_OK;
}

}  // namespace

int shape_panel_max() { return 96; }

rpim_status launch_shape_panel(rpim_plan* p, const Bucket& b, const double* X, double C2, int keep, float* dphi32,
                               hipStream_t s) {
  switch (b.nmax) {
    case 8: case 16: return launch_one<16, 1>(p, b, X, C2, keep, dphi32, s);
    case 24: return launch_one<24, 1>(p, b, X, C2, keep, dphi32, s);
    case 32: return launch_one<32, 1>(p, b, X, C2, keep, dphi32, s);
    case 40: return launch_one<40, 1>(p, b, X, C2, keep, dphi32, s);
    case 48: return launch_one<48, 1>(p, b, X, C2, keep, dphi32, s);
    case 56: return launch_one<56, 1>(p, b, X, C2, keep, dphi32, s);
    case 64: return launch_one<64, 1>(p, b, X, C2, keep, dphi32, s);
    case 72: return launch_one<72, 2>(p, b, X, C2, keep, dphi32, s);
    case 80: return launch_one<80, 2>(p, b, X, C2, keep, dphi32, s);
    case 88: return launch_one<88, 2>(p, b, X, C2, keep, dphi32, s);
    case 96: return launch_one<96, 2>(p, b, X, C2, keep, dphi32, s);
    default: return RPIM_E_RANGE;
  }
}

}  // namespace rpim
