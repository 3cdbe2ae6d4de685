// Stage 1 forward: radial-basis pair table, per-point moment-matrix solve,
// and the deterministic row-gather reduction of B^T D B into K.
//
// Arithmetic follows one fixed operation order (shared with the CPU checker
// as a written contract, not as code):
//   s   = fma(dz,dz, fma(dy,dy, dx*dx)),  d = x_a - x_b
//   R   = correctly rounded (fl(s + C^2))^q                   (dd_pow.h)
//   rhs = fl(fl(2q) * R) / t * fl(x_g - x_a)_k,  t = fl(s_ag + C^2)
//   LU  : pivot = first largest |a_rk| in current row order, whole-row swap,
//         l = a_rk / a_kk (IEEE), a_rj = fma(-l, a_kj, a_rj); right-hand
//         sides eliminated as extra columns; back substitution k descending.
//   k_IJ: e = fma(lc, m1, mc*m2), m1 = pI_al pJ_be, m2 = pI_be pJ_al (+ dot),
//         dot = fma(pI2,pJ2, fma(pI1,pJ1, pI0 pJ0)).
//   K   : +0 + e_g1 + e_g2 + ... over contributing points in ascending g;
//         mixed: float terms, one compensated (Kahan) float sum per entry,
//         also in ascending g.
#include <cfloat>
#include <climits>
#include <type_traits>

#include "dd_pow.h"
#include "rpim_internal.h"

namespace rpim {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ void flag_error(DevStatus* st, unsigned flag, int64_t g) {
  atomicOr(&st->flags, flag);
  if (g >= 0) atomicMin(&st->first_bad, (unsigned long long)g);
}

__device__ __forceinline__ double sqdist(const double* a, const double* b) {
  const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
  return __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
}

// ---- radial basis on every node pair of the pattern -------------------------
__global__ void k_pair_table(int64_t nblk, const int32_t* blk_row, const int32_t* blk_col, const double* X,
                             double C2, double q, double* R, DevStatus* st) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nblk) return;
  const int64_t I = blk_row[e], J = blk_col[e];
  const double t = sqdist(X + 3 * I, X + 3 * J) + C2;
  bool hard = false;
  R[e] = pow_cr(t, q, &hard);
  if (hard) flag_error(st, kFlagPow, -1);
}

__global__ void k_pow_test(const double* x, double q, double* y, int64_t n, DevStatus* st) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bool hard = false;
  y[i] = pow_cr(x[i], q, &hard);
  if (hard && st) flag_error(st, kFlagPow, -1);
}

// Block-wide argmax of (value, row) with ties to the smaller row.
__device__ __forceinline__ void argmax_pair(double v, int r, double* sv, int* sr, double* out_v, int* out_r) {
  for (int o = 32; o > 0; o >>= 1) {
    const double v2 = __shfl_xor(v, o, 64);
    const int r2 = __shfl_xor(r, o, 64);
    if (v2 > v || (v2 == v && r2 < r)) { v = v2; r = r2; }
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { sv[w] = v; sr[w] = r; }
  __syncthreads();
  double bv = sv[0];
  int br = sr[0];
  for (int i = 1; i < kThreads / 64; ++i)
    if (sv[i] > bv || (sv[i] == bv && sr[i] < br)) { bv = sv[i]; br = sr[i]; }
  *out_v = bv;
  *out_r = br;
  __syncthreads();
}

// ---- one workgroup per Gauss point: moment matrix, LU, three solves --------
// LDS: A[N][ld] (augmented with 3 right-hand sides), S[n], pivots[N].
__global__ void __launch_bounds__(kThreads) k_shape(const int32_t* gp_order, int64_t order_begin,
                                                    const int64_t* gp_ptr, const int32_t* gp_nbr,
                                                    const int64_t* blk_ptr, const int32_t* row_lo,
                                                    const int64_t* rbm_off, const uint2* rbm, const double* R,
                                                    const double* X, const double* gp_xyz, double C2, double q,
                                                    int ld, double* dphi, float* dphi32, int keep,
                                                    const int64_t* lu_off,
                                                    double* lu, int32_t* piv_out, double* gam, DevStatus* st) {
  extern __shared__ double smem[];
  __shared__ double red_v[kThreads / 64];
  __shared__ int red_r[kThreads / 64];
  __shared__ double xg[3];
  const int tid = threadIdx.x;
  const int64_t g = gp_order[order_begin + blockIdx.x];
  const int64_t b0 = gp_ptr[g];
  const int n = (int)(gp_ptr[g + 1] - b0);
  const int N = n + 4, W = N + 3;
  double* A = smem;
  int* S = (int*)(A + (size_t)N * ld);
  int* pv = S + n;  // pivot position of each step, before its interchange
  double* F = keep ? lu + lu_off[g] : nullptr;  // packed factors: multipliers by position, then U
  for (int i = tid; i < n; i += kThreads) S[i] = gp_nbr[b0 + i];
  for (int i = tid; i < N * ld; i += kThreads) A[i] = 0.0;
  if (tid < 3) xg[tid] = gp_xyz[3 * g + tid];
  __syncthreads();

  // R block from the pair table: G[a][b] = G[b][a] = R(S[a], S[b]), a <= b
  for (int idx = tid; idx < n * n; idx += kThreads) {
    const int a = idx / n, b = idx - a * n;
    if (b < a) continue;
    const double v = R[block_pos(blk_ptr, row_lo, rbm_off, rbm, S[a], S[b])];
    A[a * ld + b] = v;
    A[b * ld + a] = v;
  }
  // polynomial block and right-hand sides
  const double two_q = 2.0 * q;
  for (int a = tid; a < n; a += kThreads) {
    const double* xa = X + 3 * (int64_t)S[a];
    A[a * ld + n] = 1.0;
    A[n * ld + a] = 1.0;
    for (int k = 0; k < 3; ++k) {
      const double d = xa[k] - xg[k];
      A[a * ld + n + 1 + k] = d;
      A[(n + 1 + k) * ld + a] = d;
    }
    const double t = sqdist(xa, xg) + C2;
    bool hard = false;
    const double Rv = pow_cr(t, q, &hard);
    if (hard) flag_error(st, kFlagPow, g);
    const double coef = (two_q * Rv) / t;
    for (int k = 0; k < 3; ++k) A[a * ld + N + k] = coef * (xg[k] - xa[k]);
  }
  if (tid < 3) A[(n + 1 + tid) * ld + N + tid] = 1.0;
  __syncthreads();

  // singularity threshold N * eps * max|G|
  double mx = 0.0;
  for (int idx = tid; idx < N * N; idx += kThreads) {
    const int r = idx / N, c = idx - r * N;
    mx = fmax(mx, fabs(A[r * ld + c]));
  }
  double maxabs;
  int dummy;
  argmax_pair(mx, 0, red_v, red_r, &maxabs, &dummy);
  const double tiny = ((double)N * DBL_EPSILON) * maxabs;

  bool singular = false;
  for (int k = 0; k < N; ++k) {
    double v = -1.0;
    int r = N;
    for (int i = k + tid; i < N; i += kThreads) {
      const double a = fabs(A[i * ld + k]);
      if (a > v) { v = a; r = i; }
    }
    double best;
    int p;
    argmax_pair(v, r, red_v, red_r, &best, &p);
    if (!(best > tiny)) { singular = true; break; }
    if (tid == 0) pv[k] = p;  // the pivot's position before the interchange
    if (p != k)
      for (int c = tid; c < W; c += kThreads) {
        const double t = A[k * ld + c];
        A[k * ld + c] = A[p * ld + c];
        A[p * ld + c] = t;
      }
    __syncthreads();
    const double piv = A[k * ld + k];
    for (int i = k + 1 + tid; i < N; i += kThreads) {
      const double l = A[i * ld + k] / piv;
      A[i * ld + k] = l;
      if (F) F[(int64_t)k * N + i] = l;  // multiplier of the row now at position i
    }
    __syncthreads();
    const int m = N - k - 1, wc = W - k - 1;
    for (int idx = tid; idx < m * wc; idx += kThreads) {
      const int i = k + 1 + idx / wc, c = k + 1 + idx % wc;
      A[i * ld + c] = __builtin_fma(-A[i * ld + k], A[k * ld + c], A[i * ld + c]);
    }
    __syncthreads();
  }
  if (singular) {
    if (tid == 0) flag_error(st, kFlagSingular, g);
    return;
  }
  // back substitution on the three right-hand sides
  for (int k = N - 1; k >= 0; --k) {
    if (tid < 3) A[k * ld + N + tid] = A[k * ld + N + tid] / A[k * ld + k];
    __syncthreads();
    for (int idx = tid; idx < 3 * k; idx += kThreads) {
      const int i = idx / 3, j = idx - 3 * i;
      A[i * ld + N + j] = __builtin_fma(-A[i * ld + k], A[k * ld + N + j], A[i * ld + N + j]);
    }
    __syncthreads();
  }
  for (int idx = tid; idx < 3 * n; idx += kThreads) {
    const int a = idx / 3, k = idx - 3 * a;
    dphi[3 * (b0 + a) + k] = A[a * ld + N + k];
    if (dphi32) dphi32[3 * (b0 + a) + k] = (float)A[a * ld + N + k];
  }
  if (keep) {
    for (int idx = tid; idx < N * N; idx += kThreads) {
      const int r = idx / N, c = idx - r * N;  // position r, column c
      if (c >= r) F[(int64_t)c * N + r] = A[r * ld + c];
    }
    const int64_t o = b0 + 4 * g;
    for (int i = tid; i < N; i += kThreads) piv_out[o + i] = pv[i];
    for (int idx = tid; idx < 3 * N; idx += kThreads) {
      const int k = idx / N, i = idx - k * N;
      gam[3 * o + idx] = A[i * ld + N + k];
    }
  }
}

// ---- row gather: one workgroup per node row I --------------------------------
// K is symmetric bit for bit: each point's block (J, I) is the transpose of its
// block (I, J) with every entry rounded identically (the contract's products
// commute), and both entries sum the same points in the same order.  So row I
// assembles only its blocks J >= I and also writes each one, transposed, into
// row J: half the work and half the LDS of a full row.
// acc[s][9] over the row's upper blocks (s = rank of J in row I minus the rank
// of I).  Those columns are cut into GW ranges of node ids and wave w owns the
// slots of its range, so no slot is touched by two waves.  Each wave walks the
// row's Gauss points in ascending g; since supports are sorted, the part of a
// point's support inside the wave's range is a contiguous run, found with two
// ballots (with GW = 1 it is the support from I's own entry on), and its
// entries go one per lane, each lane adding all nine entries of its 3x3 block.
// A wave's LDS accesses execute in program order, so every slot receives its
// contributions in ascending g without barriers.  GW = 1 reads each point's
// metadata once per row instead of once per wave; more waves per row shorten
// the row's serial walk when rows are few.
template <bool kMixed, int GW>
__global__ void __launch_bounds__(64 * GW) k_rowgather(const int64_t* blk_ptr, const int32_t* blk_col,
                                                              const int32_t* row_lo,
                                                              const int64_t* rbm_off, const uint2* rbm,
                                                              const int64_t* inv_ptr, const uint64_t* inv_key,
                                                              const int64_t* gp_ptr, const int32_t* gp_nbr,
                                                              const void* dphi_any, const double* wdet,
                                                              const int32_t* gp_cell, const double* E, double lam,
                                                              double mu, void* Kout) {
  extern __shared__ double smem[];
  // gradients: FP64, or rounded to float by the solver for the mixed path
  using T = typename std::conditional<kMixed, float, double>::type;
  const T* dphi = static_cast<const T*>(dphi_any);
  const int64_t I = blockIdx.x;
  const int64_t rb = blk_ptr[I];
  const int L = (int)(blk_ptr[I + 1] - rb);
  if (L == 0) return;  // a node in no support has an empty row (uniform)
  const int tid = threadIdx.x;
  const int w = tid >> 6, lane = tid & 63;
  const int lo_I = row_lo[I];
  const int64_t wb = rbm_off[I];
  const int nw = (int)(rbm_off[I + 1] - wb);
  // rank of the diagonal block in row I; the upper blocks follow it
  const int rI = (int)I - lo_I;
  const uint2 wI = rbm[wb + (rI >> 5)];
  const int pd = (int)wI.y + __popc(wI.x & ((1u << (rI & 31)) - 1u));
  const int Lu = L - pd;
  double* acc = smem;                  // [Lu][9] double sums, or (sum, compensation) float pairs (mixed)
  uint2* bm = (uint2*)(acc + 9 * Lu);  // row I's rank bitmap
  constexpr int kThreadsG = 64 * GW;
  for (int i = tid; i < nw; i += kThreadsG) bm[i] = rbm[wb + i];
  for (int i = tid; i < 9 * Lu; i += kThreadsG) acc[i] = 0.0;  // +0 sums and compensations
  // this wave's columns: node ids in [thr_lo, thr_hi), from I upwards
  const int32_t thr_lo = w == 0 ? (int32_t)I : blk_col[rb + pd + (int64_t)w * Lu / GW];
  const int32_t thr_hi = w + 1 == GW ? INT_MAX : blk_col[rb + pd + (int64_t)(w + 1) * Lu / GW];
  __syncthreads();

  // Several waves per row (GW > 1): a software pipeline over the row's Gauss
  // points, point metadata (scalar) three points ahead, the support ids that locate the wave's run two points
  // ahead, the run's entries one point ahead.  Loads past the row's last point
  // re-read the last point, loads past a support's end re-read its last entry
  // (no branch around a load).
  struct Meta {
    int64_t b0;
    int n, aI;
    double lc, mc;
  };
  struct Split {
    int32_t J0, J1;  // support ids at b = lane and b = lane + 64
  };
  struct Run {
    int lo, hi;      // the wave's part of the support: b in [lo, hi)
    int32_t J;       // entry b = lo + lane
    T p[3];
    T pI[3];
  };
  const int64_t e_beg = inv_ptr[I], e_end = inv_ptr[I + 1];
  auto meta = [&](int64_t e) {
    Meta m;
    const uint64_t key = inv_key[e];
    const int64_t g = (int64_t)(key >> 8);
    m.aI = (int)(key & 255);
    m.b0 = gp_ptr[g];
    m.n = (int)(gp_ptr[g + 1] - m.b0);
    const double c = wdet[g] * E[gp_cell[g]];
    m.lc = c * lam;
    m.mc = c * mu;
    return m;
  };
  auto split = [&](const Meta& m) {
    Split sp;
    if constexpr (GW == 1) {  // one wave owns every upper column: no run to locate
      sp.J0 = sp.J1 = 0;
      return sp;
    }
    const int b1 = lane + 64 < m.n ? lane + 64 : m.n - 1;
    sp.J0 = gp_nbr[m.b0 + (lane < m.n ? lane : m.n - 1)];
    sp.J1 = gp_nbr[m.b0 + b1];
    return sp;
  };
  auto run = [&](const Meta& m, const Split& sp) {
    Run r;
    // supports are sorted: the count of ids below a threshold is a position
    if constexpr (GW == 1) {  // the upper part starts at I's own entry
      r.lo = m.aI;
      r.hi = m.n;
    } else {
      const bool v0 = lane < m.n, v1 = lane + 64 < m.n;
      r.lo = __popcll(__ballot(v0 && sp.J0 < thr_lo)) + __popcll(__ballot(v1 && sp.J1 < thr_lo));
      r.hi = __popcll(__ballot(v0 && sp.J0 < thr_hi)) + __popcll(__ballot(v1 && sp.J1 < thr_hi));
    }
    const int b = r.lo + lane;
    const int bc = b < m.n ? b : m.n - 1;
    r.J = gp_nbr[m.b0 + bc];
    for (int k = 0; k < 3; ++k) r.p[k] = dphi[3 * (m.b0 + bc) + k];
    for (int k = 0; k < 3; ++k) r.pI[k] = dphi[3 * (m.b0 + m.aI) + k];
    return r;
  };
  // all nine entries of block (I, J) of one point, added to its slot
  auto accum = [&](int32_t J, const T (&pJ)[3], const T (&pI)[3], double lc, double mc) {
    const int r = J - lo_I;
    const uint2 wv = bm[r >> 5];
    const int pos = (int)wv.y + __popc(wv.x & ((1u << (r & 31)) - 1u)) - pd;  // upper slot
    if constexpr (!kMixed) {
      const double dot = __builtin_fma(pI[2], pJ[2], __builtin_fma(pI[1], pJ[1], pI[0] * pJ[0]));
      double m[3][3];
#pragma unroll
      for (int al = 0; al < 3; ++al)
#pragma unroll
        for (int be = 0; be < 3; ++be) m[al][be] = pI[al] * pJ[be];
      double* a = acc + 9 * pos;
#pragma unroll
      for (int al = 0; al < 3; ++al)
#pragma unroll
        for (int be = 0; be < 3; ++be) {
          double m2 = m[be][al];  // phi_I,beta * phi_J,alpha
          if (al == be) m2 = m2 + dot;
          // LDS FP64 add (ds_add_f64): no read round trip; a wave's LDS
          // operations execute in program order and no two lanes or waves
          // share a slot, so each slot still sums in ascending g
          __hip_atomic_fetch_add(a + 3 * al + be, __builtin_fma(lc, m[al][be], mc * m2), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    } else {
      const float flc = (float)lc, fmc = (float)mc;
      const float dot = __builtin_fmaf(pI[2], pJ[2], __builtin_fmaf(pI[1], pJ[1], pI[0] * pJ[0]));
      float m[3][3];
#pragma unroll
      for (int al = 0; al < 3; ++al)
#pragma unroll
        for (int be = 0; be < 3; ++be) m[al][be] = pI[al] * pJ[be];
      float2* a = reinterpret_cast<float2*>(acc) + 9 * pos;
#pragma unroll
      for (int al = 0; al < 3; ++al)
#pragma unroll
        for (int be = 0; be < 3; ++be) {
          float m2 = m[be][al];
          if (al == be) m2 = m2 + dot;
          const float ev = __builtin_fmaf(flc, m[al][be], fmc * m2);
          // compensated float sum (Kahan): the slot holds (sum, compensation);
          // the compensation keeps the low-order part that the rounded sum
          // dropped and feeds it back with the next term.  The lane owns the
          // slot for this point and the wave's LDS operations run in program
          // order, so the next point's read sees this write (ascending g).
          float2 sc = a[3 * al + be];
          const float y = ev - sc.y;
          const float t = sc.x + y;
          sc.y = (t - sc.x) - y;
          sc.x = t;
          a[3 * al + be] = sc;
        }
    }
  };
  if constexpr (GW == 1) {
    // One wave owns the whole upper row.  Point metadata comes 64 points at
    // a time, one point per lane (the key -> point -> cell -> modulus loads
    // run once per 64 points), the next 64 loaded while these are used; each
    // point's fields are then taken by readlane.  The support entries of a
    // point are loaded kAhead points before its turn (a ring of kAhead runs).
    constexpr int kAhead = 8;  // divides 64
    struct LaneMeta {          // lane l: point e0 + l of the batch starting at e0
      int64_t b0;
      int n, aI;
      double lc, mc;
    };
    const int64_t cnt = e_end - e_beg;
    auto load_batch = [&](int64_t i0) {  // points i0 .. i0 + 63 of the row (past the end: the last)
      LaneMeta v;
      const int64_t i = i0 + lane < cnt ? i0 + lane : cnt - 1;
      const uint64_t key = inv_key[e_beg + i];
      const int64_t g = (int64_t)(key >> 8);
      v.aI = (int)(key & 255);
      v.b0 = gp_ptr[g];
      v.n = (int)(gp_ptr[g + 1] - v.b0);
      const double c = wdet[g] * E[gp_cell[g]];
      v.lc = c * lam;
      v.mc = c * mu;
      return v;
    };
    auto pick = [&](const LaneMeta& v, int j) {  // the batch's point j (j uniform)
      Meta m;
      m.b0 = readlane_i64(v.b0, j);
      m.n = __builtin_amdgcn_readlane(v.n, j);
      m.aI = __builtin_amdgcn_readlane(v.aI, j);
      m.lc = readlane_f64(v.lc, j);
      m.mc = readlane_f64(v.mc, j);
      return m;
    };
    auto run1 = [&](const Meta& m) {  // the upper part of the support: from I's own entry on
      Run r;
      r.lo = m.aI;
      r.hi = m.n;
      const int b = r.lo + lane;
      const int bc = b < m.n ? b : m.n - 1;
      r.J = gp_nbr[m.b0 + bc];
      for (int k = 0; k < 3; ++k) r.p[k] = dphi[3 * (m.b0 + bc) + k];
      for (int k = 0; k < 3; ++k) r.pI[k] = dphi[3 * (m.b0 + m.aI) + k];
      return r;
    };
    if (cnt > 0) {
      LaneMeta cur = load_batch(0), nxt = cur;
      if (cnt > 64) nxt = load_batch(64);
      Run ring[kAhead];
#pragma unroll
      for (int u = 0; u < kAhead; ++u) ring[u] = run1(pick(cur, u < cnt ? u : (int)cnt - 1));
      for (int64_t i0 = 0; i0 < cnt; i0 += kAhead) {
        if (i0 > 0 && (i0 & 63) == 0) {  // next batch (uniform)
          cur = nxt;
          if (i0 + 64 < cnt) nxt = load_batch(i0 + 64);
        }
#pragma unroll
        for (int u = 0; u < kAhead; ++u) {
          const int64_t i = i0 + u;
          if (i < cnt) {  // uniform
            const Meta m = pick(cur, (int)(i & 63));
            const Run& r = ring[u];
            if (r.lo + lane < r.hi) accum(r.J, r.p, r.pI, m.lc, m.mc);
            // upper parts longer than one wave (over 64 entries) continue in a plain loop
            for (int b = r.lo + 64 + lane; b < r.hi; b += 64) {
              const int64_t eb = m.b0 + b;
              const T pJ[3] = {dphi[3 * eb], dphi[3 * eb + 1], dphi[3 * eb + 2]};
              accum(gp_nbr[eb], pJ, r.pI, m.lc, m.mc);
            }
            // refill with point i + kAhead (past the end: the last point again)
            const int64_t ip = i + kAhead < cnt ? i + kAhead : cnt - 1;
            const Meta mp = (ip >> 6) == (i0 >> 6) ? pick(cur, (int)(ip & 63)) : pick(nxt, (int)(ip & 63));
            ring[u] = run1(mp);
          }
        }
      }
    }
  } else {
    const int64_t e_last = e_end - 1;
    auto clampe = [&](int64_t e) { return e < e_last ? e : e_last; };
    Meta m_cur = {}, m_nxt = {}, m_n2 = {};
    Split s_nxt = {}, s_n2 = {};
    Run r_cur = {};
    if (e_beg < e_end) {
      m_cur = meta(e_beg);
      m_nxt = meta(clampe(e_beg + 1));
      const Split s_cur = split(m_cur);
      m_n2 = meta(clampe(e_beg + 2));
      s_nxt = split(m_nxt);
      r_cur = run(m_cur, s_cur);
    }
    for (int64_t e = e_beg; e < e_end; ++e) {
      const Meta m_n3 = meta(clampe(e + 3));
      s_n2 = split(m_n2);
      const Run r_nxt = run(m_nxt, s_nxt);
      if (r_cur.lo + lane < r_cur.hi) accum(r_cur.J, r_cur.p, r_cur.pI, m_cur.lc, m_cur.mc);
      // runs longer than one wave (supports beyond ~128 nodes) continue in a plain loop
      for (int b = r_cur.lo + 64 + lane; b < r_cur.hi; b += 64) {
        const int64_t eb = m_cur.b0 + b;
        const T pJ[3] = {dphi[3 * eb], dphi[3 * eb + 1], dphi[3 * eb + 2]};
        accum(gp_nbr[eb], pJ, r_cur.pI, m_cur.lc, m_cur.mc);
      }
      m_cur = m_nxt;
      m_nxt = m_n2;
      m_n2 = m_n3;
      s_nxt = s_n2;
      r_cur = r_nxt;
    }
  }
  __syncthreads();
  // row I: its upper blocks, three contiguous runs of 3 Lu entries (one per row alpha)
  auto slot = [&](int i) -> T {
    if constexpr (!kMixed) return acc[i];
    else return reinterpret_cast<const float2*>(acc)[i].x;  // the compensated sum
  };
  T* K = static_cast<T*>(Kout);
  const int64_t base = 9 * rb + 3 * (int64_t)pd;
  for (int idx = tid; idx < 9 * Lu; idx += kThreadsG) {
    const int a = idx / (3 * Lu), rem = idx - 3 * Lu * a, sl = rem / 3, be = rem - 3 * sl;
    K[base + 3 * (int64_t)a * L + rem] = slot(9 * sl + 3 * a + be);
  }
  // row J > I: block (J, I) is block (I, J) transposed, at I's rank in row J
  for (int sl = 1 + tid; sl < Lu; sl += kThreadsG) {
    const int32_t J = blk_col[rb + pd + sl];
    const int64_t bJ = blk_ptr[J];
    const int64_t LJ = blk_ptr[J + 1] - bJ;
    const int rJ = (int)I - row_lo[J];
    const uint2 wJ = rbm[rbm_off[J] + (rJ >> 5)];
    const int64_t pJ = (int64_t)wJ.y + __popc(wJ.x & ((1u << (rJ & 31)) - 1u));
    const int64_t oJ = 9 * bJ + 3 * pJ;
#pragma unroll
    for (int be = 0; be < 3; ++be)
#pragma unroll
      for (int a = 0; a < 3; ++a) K[oJ + 3 * be * LJ + a] = slot(9 * sl + 3 * a + be);
  }
}

inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }


}  // namespace

rpim_status launch_pair_table(rpim_plan* p, const double* X, hipStream_t s) {
  const double ac = p->alpha_c * p->d_c;
  const double C2 = ac * ac;
  if (p->nblk == 0) return RPIM_OK;
  hipLaunchKernelGGL(k_pair_table, dim3(nblocks(p->nblk, 256)), dim3(256), 0, s, p->nblk,
                     (const int32_t*)p->blk_row, (const int32_t*)p->blk_col, X, C2, p->q, p->R, p->status);
  RPIM_HIP(hipGetLastError());
  return RPIM_OK;
}

rpim_status launch_shape_bucket(rpim_plan* p, const Bucket& b, const double* X, int keep, float* dphi32,
                                hipStream_t s) {
  const double ac = p->alpha_c * p->d_c;
  const double C2 = ac * ac;
  const int kind = p->solver_kind[b.nmax / kBucketStep];
  if (kind == RPIM_SOLVER_PANEL && b.nmax <= shape_panel_max())
    return launch_shape_panel(p, b, X, C2, keep, dphi32, s);
  if (kind != RPIM_SOLVER_LDS && b.nmax <= shape_reg_max()) return launch_shape_reg(p, b, X, C2, keep, dphi32, s);
  const int N = b.nmax;
  const int ld = ((N + 3) | 1);  // odd row stride in doubles
  const size_t lds = sizeof(double) * (size_t)N * ld + sizeof(int) * (size_t)(2 * N);
  if (lds > 160 * 1024) return RPIM_E_RANGE;
  if (rpim_status st = raise_lds_limit((const void*)k_shape, lds, p->device)) return st;
  hipLaunchKernelGGL(k_shape, dim3((unsigned)b.count), dim3(kThreads), lds, s, (const int32_t*)p->gp_order,
                     b.begin, (const int64_t*)p->gp_ptr, (const int32_t*)p->gp_nbr, (const int64_t*)p->blk_ptr,
                     (const int32_t*)p->row_lo, (const int64_t*)p->rbm_off, (const uint2*)p->rbm,
                     (const double*)p->R, X, (const double*)p->gp_xyz, C2, p->q, ld,
                     p->dphi, dphi32, keep, (const int64_t*)p->lu_off, p->lu, p->piv, p->gam, p->status);
  RPIM_HIP(hipGetLastError());
  return RPIM_OK;
}

rpim_status launch_shape(rpim_plan* p, const double* X, int keep, float* dphi32, hipStream_t s) {
  for (const Bucket& b : p->buckets)
    if (rpim_status st = launch_shape_bucket(p, b, X, keep, dphi32, s)) return st;
  return RPIM_OK;
}

template <bool kMixed, int GW>
rpim_status launch_gather_t(rpim_plan* p, const double* E, double lam, double mu, void* K, size_t lds, hipStream_t s) {
  if (rpim_status st = raise_lds_limit((const void*)k_rowgather<kMixed, GW>, lds, p->device)) return st;
  hipLaunchKernelGGL((k_rowgather<kMixed, GW>), dim3((unsigned)p->N), dim3(64 * GW), lds, s,
                     (const int64_t*)p->blk_ptr, (const int32_t*)p->blk_col, (const int32_t*)p->row_lo,
                     (const int64_t*)p->rbm_off, (const uint2*)p->rbm, (const int64_t*)p->inv_ptr,
                     (const uint64_t*)p->inv_key, (const int64_t*)p->gp_ptr, (const int32_t*)p->gp_nbr,
                     kMixed ? (const void*)p->dphi32 : (const void*)p->dphi, (const double*)p->gp_wdet,
                     (const int32_t*)p->gp_cell, E, lam, mu, K);
  RPIM_HIP(hipGetLastError());
  return RPIM_OK;
}

int gather_waves_valid(int gw) { return gw >= 1 && gw <= 4; }

rpim_status launch_rowgather(rpim_plan* p, const double* E, double nu, int precision, void* K, hipStream_t s,
                             int gather_waves) {
  const double onep = 1.0 + nu;
  const double onem = 1.0 - 2.0 * nu;
  const double lam = nu / (onep * onem);
  const double mu = 1.0 / (2.0 * onep);
  const int Lu = (int)p->max_row_upper;
  const size_t lds = sizeof(double) * 9 * (size_t)Lu + sizeof(uint2) * (size_t)p->max_row_words;
  if (lds > 160 * 1024) return RPIM_E_RANGE;
  const int gw = gather_waves > 0 ? gather_waves : p->gather_waves[precision == RPIM_MIXED ? 1 : 0];
  if (precision == RPIM_FP64) {
    switch (gw) {
      case 2: return launch_gather_t<false, 2>(p, E, lam, mu, K, lds, s);
      case 3: return launch_gather_t<false, 3>(p, E, lam, mu, K, lds, s);
      case 4: return launch_gather_t<false, 4>(p, E, lam, mu, K, lds, s);
      default: return launch_gather_t<false, 1>(p, E, lam, mu, K, lds, s);
    }
  }
  switch (gw) {
    case 2: return launch_gather_t<true, 2>(p, E, lam, mu, K, lds, s);
    case 3: return launch_gather_t<true, 3>(p, E, lam, mu, K, lds, s);
    case 4: return launch_gather_t<true, 4>(p, E, lam, mu, K, lds, s);
    default: return launch_gather_t<true, 1>(p, E, lam, mu, K, lds, s);
  }
}

rpim_status launch_pow_test(const double* x, double q, double* y, int64_t n, hipStream_t s) {
  if (n <= 0) return RPIM_OK;
  hipLaunchKernelGGL(k_pow_test, dim3(nblocks(n, 256)), dim3(256), 0, s, x, q, y, n, (DevStatus*)nullptr);
  RPIM_HIP(hipGetLastError());
  return RPIM_OK;
}

}  // namespace rpim
