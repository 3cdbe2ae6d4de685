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
//           Each wave's candidate posts (|a_k|, key) in one 16-byte LDS
//           write; after a barrier every wave picks the winner, and the
//           winner writes its window once, as U row k, into LDS.  After a
//           second barrier every other active row computes l = a_k / u_kk and
//           updates-and-shifts its window in one pass:
//           w_j <- fma(-l, u_{j+1}, w_{j+1}), so column k+1 becomes element 0.
//           (With one wave per point both barriers are unnecessary: a wave's
//           LDS accesses complete in program order.)
// Back substitution then runs by position from the U rows in LDS, k
// descending: x_k = b_k / u_kk, b_r = fma(-u_rk, x_k, b_r) for r < k; x_k
// reaches the other threads of its wave by readlane.
//
// Every register index is static: element 0 is always the pivot column.  The
// winner's write and the update walk the window in blocks of sixteen columns,
// skipping blocks past the row's end under uniform branches.  The pivot row
// reaches the other rows one element per lane from LDS and is spread across
// each row of sixteen lanes by DPP broadcasts.  A workgroup's time is the
// latency of its chain of N steps (pivot search, exchange, row write,
// division, update): a workgroup alone on a CU takes as long per step as one
// among a full load, so the step is kept short rather than lean, and
// throughput comes from the points resident per CU.  Code size is O(NMAX).
#include "shape_common.h"

namespace rpim {
namespace {

using namespace solver;

// U storage: row k (k < N <= NMAX) holds NMAX + 3 - k doubles rounded up to
// even (16-byte aligned rows), followed by padding for the update's read-ahead.
template <int NMAX>
constexpr int u_size() {
  int s = 0;
  for (int k = 0; k < NMAX; ++k) s += (NMAX + 3 - k + 1) & ~1;
  return s + 16 * ((NMAX + 4 + 15) / 16) + 32;
}

template <int NMAX, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) k_shape_win(
    const int32_t* gp_order, int64_t order_begin, const int64_t* gp_ptr, const int32_t* gp_nbr,
    const int64_t* blk_ptr, const int32_t* row_lo, const int64_t* rbm_off, const uint2* rbm, const double* R,
    const double* X, const double* gp_xyz, double C2, double q, double* dphi, float* dphi32, int keep,
    const int64_t* lu_off,
    double* lu, int32_t* piv_out, double* gam, DevStatus* st) {
  constexpr int T = 64 * WAVES;
  constexpr int WC = NMAX + 4;   // window: matrix columns + 3 right-hand sides + 1 zero
  constexpr int NB = (WC + 15) / 16;  // blocks of sixteen columns
  constexpr int US = u_size<NMAX>();
  constexpr int LDSD = US;
  static_assert(T >= NMAX && NMAX % 8 == 0, "shape");
  struct __align__(16) Cand {
    double v;      // |a_k| of the wave's candidate (-1: no active row)
    unsigned key;  // (position << 8) | row
    unsigned pad;
  };
  __shared__ __align__(16) double lds[LDSD];  // the U rows
  __shared__ Cand cand[2][WAVES];
  __shared__ int uoffs[NMAX];                 // start of U row k in lds
  __shared__ double xsol[3][NMAX];
  __shared__ int pivpos[NMAX];                // position the pivot of each step held before it
  __shared__ double xg[3];
  __shared__ double rmax[WAVES];
  // Per-support-node data of the build phase share the U storage: every read
  // of them comes before the barrier that ends the build, and U is written
  // only after it.  The smaller footprint lets more points reside per CU,
  // which is what the latency-bound elimination needs.
  static_assert(7 * NMAX <= US, "build data fit in the U storage");
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

  // ---- LU with partial pivoting on positions; windows shift each step ----------
  int pos = t;              // current position of my row
  const bool real = t < N;  // padding rows never take part
  double* F = keep ? lu + lu_off[g] : nullptr;          // packed factors (multipliers by position)
  int uoff = 0;                                           // start of U row k in lds
#pragma unroll 1
  for (int k = 0; k < N; ++k) {
    const int len = NMAX + 3 - k;  // window elements in use (columns k..NMAX-1 and 3 rhs)
    const bool active = real && pos >= k;
    double v;
    unsigned key;
    wave_argmax(fabs(a[0]), active, ((unsigned)pos << 8) | (unsigned)t, &v, &key);
    double best = v;
    unsigned bkey = key;
    if constexpr (WAVES > 1) {
      const int buf = k & 1;
      if (lane == 0) {
        Cand c;
        c.v = key == 0xFFFFFFFFu ? -1.0 : v;
        c.key = key;
        c.pad = 0;
        cand[buf][w] = c;
      }
      __syncthreads();
      best = cand[buf][0].v;
      bkey = cand[buf][0].key;
#pragma unroll
      for (int i = 1; i < WAVES; ++i) {
        const Cand c = cand[buf][i];
        const bool take = c.v > best || (c.v == best && c.key < bkey);
        best = take ? c.v : best;
        bkey = take ? c.key : bkey;
      }
    } else {
      if (key == 0xFFFFFFFFu) best = -1.0;
    }
    if (!(best > tiny)) {
      if (t == 0) flag_error(st, kFlagSingular, g);
      return;  // uniform: every thread saw the same best
    }
    const int prow_id = (int)(bkey & 255u), ppos = (int)(bkey >> 8);
    double* urow = lds + uoff;  // urow[0] = u_kk, urow[1 + j] = pivot column k+1+j
    if (t == prow_id) write_row<NB, WC>(a, urow, len);
    if (t == 0) {
      pivpos[k] = ppos;
      uoffs[k] = uoff;
    }
    if (t == prow_id) pos = k;
    else if (pos == k) pos = ppos;
    if constexpr (WAVES > 1) __syncthreads();
    {
      // every lane runs the update (the DPP broadcast reads all lanes); rows that
      // are not eliminated this step take l = 0, which only shifts their windows
      // (the pivot's window is already stored as its U row)
      const bool upd = real && pos > k;
      const double l = upd ? a[0] / urow[0] : 0.0;
      shift_update<NB, WC>(a, -l, urow + 1, len, lane & 15);
      if (keep && upd) F[(int64_t)k * N + pos] = l;  // after the update: no branch between the two
    }
    uoff += (len + 1) & ~1;
  }
  __syncthreads();

  // ---- back substitution by position from the U rows, then the outputs ----------
  back_substitute_and_store<NMAX, WAVES>(lds, t < N ? uoffs[t] : 0, xsol, pivpos, t, N, n, g, b0, dphi, dphi32, keep,
                                         F, piv_out, gam);
}

template <int NMAX, int WAVES>
rpim_status launch_one(rpim_plan* p, const Bucket& bk, const double* X, double C2, int keep, float* dphi32,
                       hipStream_t s) {
  hipLaunchKernelGGL((k_shape_win<NMAX, WAVES>), dim3((unsigned)bk.count), dim3(64 * WAVES), 0, s,
                     (const int32_t*)p->gp_order, bk.begin, (const int64_t*)p->gp_ptr, (const int32_t*)p->gp_nbr,
                     (const int64_t*)p->blk_ptr, (const int32_t*)p->row_lo, (const int64_t*)p->rbm_off,
                     (const uint2*)p->rbm, (const double*)p->R, X, (const double*)p->gp_xyz, C2, p->q, p->dphi,
                     dphi32, keep, (const int64_t*)p->lu_off, p->lu, p->piv, p->gam, p->status);
  RPIM_HIP(hipGetLastError());
  return RPIM_OK;
}

}  // namespace

// Largest padded size handled in registers; bigger buckets use the LDS kernel.
int shape_reg_max() { return 104; }

rpim_status launch_shape_reg(rpim_plan* p, const Bucket& b, const double* X, double C2, int keep, float* dphi32,
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
    case 104: return launch_one<104, 2>(p, b, X, C2, keep, dphi32, s);
    default: return RPIM_E_RANGE;
  }
}

}  // namespace rpim
