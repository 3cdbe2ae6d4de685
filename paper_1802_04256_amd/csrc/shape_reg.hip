// Moment-matrix solve with rows held in registers (gfx950).
//
// One workgroup of 64*WAVES threads per Gauss point; thread t owns row t of
// the augmented moment matrix [G | r_0 r_1 r_2] in VGPRs: NMAX doubles of
// matrix columns (columns n+4..NMAX-1 are zero padding) plus 3 right-hand
// sides.  Rows never move: partial pivoting is done on row *positions* (the
// row order the textbook algorithm has after its swaps), which yields the
// same pivot choices, multipliers and fma sequence as whole-row swapping:
//   step k: pivot = active row with the largest |a_k|, ties to the smaller
//           position; it takes position k and the row that held position k
//           takes the pivot's old position; the pivot row is broadcast through
//           LDS; every other active row does l = a_k / u_kk and
//           a_j = fma(-l, u_j, a_j) for j > k.
// Back substitution runs by position, k descending: x_k = b_k / u_kk is
// broadcast and every row at a smaller position does b = fma(-u_rk, x_k, b).
//
// Code size stays O(NMAX): the step loop is a runtime loop; row columns are
// updated in blocks of 8 under uniform branches, and the element of column k
// is read or written through a switch on the (uniform) step index, so no
// register is ever indexed dynamically.  In the block that contains column
// k, columns < k are updated with a pivot-row value of +0, which leaves them
// unchanged (x + (+-0) = x up to the sign of an exact-zero multiplier, which
// nothing downstream reads).  The matrix is built through a small LDS staging
// buffer a few rows at a time; a 76 x 79 system costs ~6 KB of LDS.
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

// Wave argmax of (value desc, key asc).
__device__ __forceinline__ void wave_argmax(double& v, int& key) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double v2 = __shfl_xor(v, o, 64);
    const int k2 = __shfl_xor(key, o, 64);
    const bool take = (v2 > v) || (v2 == v && k2 < key);
    v = take ? v2 : v;
    key = take ? k2 : key;
  }
}

#define RPIM_C8(b, X) X(b + 0) X(b + 1) X(b + 2) X(b + 3) X(b + 4) X(b + 5) X(b + 6) X(b + 7)
#define RPIM_C128(X)                                                                                      \
  RPIM_C8(0, X) RPIM_C8(8, X) RPIM_C8(16, X) RPIM_C8(24, X) RPIM_C8(32, X) RPIM_C8(40, X) RPIM_C8(48, X) \
  RPIM_C8(56, X) RPIM_C8(64, X) RPIM_C8(72, X) RPIM_C8(80, X) RPIM_C8(88, X) RPIM_C8(96, X) RPIM_C8(104, X) \
  RPIM_C8(112, X) RPIM_C8(120, X)

// a[k] for a uniform k (jump on k; each case reads one fixed register).
template <int NMAX>
__device__ __forceinline__ double get_col(const double (&a)[NMAX], int k) {
  double v = 0.0;
  switch (k) {
#define RPIM_GET(c)                         \
  case (c):                                 \
    if constexpr ((c) < NMAX) v = a[(c)];   \
    break;
    RPIM_C128(RPIM_GET)
#undef RPIM_GET
    default:
      break;
  }
  return v;
}

template <int NMAX>
__device__ __forceinline__ void set_col(double (&a)[NMAX], int k, double v) {
  switch (k) {
#define RPIM_SET(c)                         \
  case (c):                                 \
    if constexpr ((c) < NMAX) a[(c)] = v;   \
    break;
    RPIM_C128(RPIM_SET)
#undef RPIM_SET
    default:
      break;
  }
}

template <int NMAX, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) k_shape_reg(
    const int32_t* gp_order, int64_t order_begin, const int64_t* gp_ptr, const int32_t* gp_nbr,
    const int64_t* blk_ptr, const int32_t* row_lo, const int64_t* rbm_off, const uint2* rbm, const double* R,
    const double* X, const double* gp_xyz, double C2, double q, double* dphi, int keep, const int64_t* lu_off,
    double* lu, int32_t* piv_out, double* gam, DevStatus* st) {
  constexpr int T = 64 * WAVES;
  constexpr int NB = NMAX / 8;
  constexpr int WC = NMAX + 3;  // staging row width: matrix + 3 right-hand sides
  constexpr int CH = 16;        // staging rows per chunk
  static_assert(T >= NMAX && NMAX % 8 == 0 && NMAX <= 128, "shape");
  __shared__ double stage[CH][WC];
  __shared__ __align__(16) double prow[2][WAVES][NMAX];  // candidate pivot rows (zeros at columns < k)
  __shared__ double prhs[2][WAVES][3];
  __shared__ double cval[2][WAVES];
  __shared__ double cpiv[2][WAVES];
  __shared__ int ckey[2][WAVES];
  __shared__ double xsol[3][NMAX];
  __shared__ int S[NMAX];
  __shared__ int ipiv[NMAX];
  __shared__ int rowat[NMAX];
  __shared__ double xg[3];
  __shared__ double rmax[WAVES];
  __shared__ double coefs[NMAX];

  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t g = gp_order[order_begin + blockIdx.x];
  const int64_t b0 = gp_ptr[g];
  const int n = (int)(gp_ptr[g + 1] - b0);
  const int N = n + 4;
  for (int i = t; i < n; i += T) S[i] = gp_nbr[b0 + i];
  if (t < 3) xg[t] = gp_xyz[3 * g + t];
  __syncthreads();
  // derivative right-hand-side coefficients fl(fl(2q) * R) / t, one power per support node
  bool hard = false;
  for (int r = t; r < n; r += T) {
    const double* xa = X + 3 * (int64_t)S[r];
    const double dx = xa[0] - xg[0], dy = xa[1] - xg[1], dz = xa[2] - xg[2];
    const double tt = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx)) + C2;
    const double Rv = pow_cr(tt, q, &hard);
    coefs[r] = ((2.0 * q) * Rv) / tt;
  }
  __syncthreads();

  // ---- build rows through the staging buffer --------------------------------
  double a[NMAX];
  double b[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < NMAX; ++j) a[j] = 0.0;
  for (int r0 = 0; r0 < N; r0 += CH) {
    for (int idx = t; idx < CH * WC; idx += T) {
      const int rr = idx / WC, c = idx - rr * WC;
      const int r = r0 + rr;
      double v = 0.0;
      if (r < n) {
        if (c < n) {
          v = R[block_pos(blk_ptr, row_lo, rbm_off, rbm, S[r], S[c])];
        } else if (c == n) {
          v = 1.0;
        } else if (c < N) {
          v = X[3 * (int64_t)S[r] + (c - n - 1)] - xg[c - n - 1];
        } else if (c >= NMAX) {
          v = coefs[r] * (xg[c - NMAX] - X[3 * (int64_t)S[r] + (c - NMAX)]);
        }
      } else if (r == n) {
        v = c < n ? 1.0 : 0.0;
      } else if (r < N) {
        const int k = r - n - 1;
        if (c < n) v = X[3 * (int64_t)S[c] + k] - xg[k];
        else if (c == NMAX + k) v = 1.0;
      }
      stage[rr][c] = v;
    }
    __syncthreads();
    if (t >= r0 && t < r0 + CH && t < N) {
#pragma unroll
      for (int j = 0; j < NMAX; ++j) a[j] = stage[t - r0][j];
#pragma unroll
      for (int j = 0; j < 3; ++j) b[j] = stage[t - r0][NMAX + j];
    }
    __syncthreads();
  }
  if (hard) flag_error(st, kFlagPow, g);

  // singularity threshold N * eps * max|G|
  double mx = 0.0;
#pragma unroll
  for (int j = 0; j < NMAX; ++j) mx = fmax(mx, fabs(a[j]));
  {
    int dummy = 0;
    wave_argmax(mx, dummy);
    if (lane == 0) rmax[w] = mx;
    __syncthreads();
    mx = rmax[0];
#pragma unroll
    for (int i = 1; i < WAVES; ++i) mx = fmax(mx, rmax[i]);
  }
  const double tiny = ((double)N * DBL_EPSILON) * mx;

  // ---- LU with partial pivoting on positions ----------------------------------
  int pos = t;              // current position of my row
  const bool real = t < N;  // padding rows never take part
#pragma unroll 1
  for (int k = 0; k < N; ++k) {
    const int buf = k & 1;
    const int kb = k >> 3;  // block holding column k
    const bool active = real && pos >= k;
    const double ak = get_col<NMAX>(a, k);
    double v = active ? fabs(ak) : -1.0;
    int key = active ? (pos << 8) | t : INT_MAX;
    wave_argmax(v, key);
    // the wave's candidate publishes its row (zeros at columns < k)
    if ((key & 255) == t) {
#pragma unroll
      for (int bb = 0; bb < NB; ++bb) {
        if (bb == kb) {
#pragma unroll
          for (int e = 0; e < 8; ++e) prow[buf][w][8 * bb + e] = (8 * bb + e > k) ? a[8 * bb + e] : 0.0;
        } else if (bb > kb && 8 * bb < N) {
#pragma unroll
          for (int e = 0; e < 8; ++e) prow[buf][w][8 * bb + e] = a[8 * bb + e];
        }
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int j = 0; j < 3; ++j) prhs[buf][w][j] = b[j];
      cpiv[buf][w] = ak;
    }
    if (lane == 0) {
      cval[buf][w] = v;
      ckey[buf][w] = key;
    }
    __syncthreads();
    double best = cval[buf][0];
    int bkey = ckey[buf][0];
    int bw = 0;
#pragma unroll
    for (int i = 1; i < WAVES; ++i) {
      const double v2 = cval[buf][i];
      const int k2 = ckey[buf][i];
      if (v2 > best || (v2 == best && k2 < bkey)) { best = v2; bkey = k2; bw = i; }
    }
    if (!(best > tiny)) {
      if (t == 0) flag_error(st, kFlagSingular, g);
      return;  // uniform: every thread saw the same best
    }
    const int prow_id = bkey & 255, ppos = bkey >> 8;
    if (t == 0) {
      ipiv[k] = ppos;
      rowat[k] = prow_id;
    }
    if (t == prow_id) pos = k;
    else if (pos == k) pos = ppos;
    if (real && pos > k) {
      const double l = ak / cpiv[buf][bw];
      const double* u = prow[buf][bw];
#pragma unroll
      for (int bb = 0; bb < NB; ++bb) {
        if (bb >= kb && 8 * bb < N) {
#pragma unroll
          for (int e = 0; e < 8; ++e) a[8 * bb + e] = __builtin_fma(-l, u[8 * bb + e], a[8 * bb + e]);
        }
        __builtin_amdgcn_sched_barrier(0);  // keep each block's loads next to its fmas
      }
      set_col<NMAX>(a, k, l);  // column k holds the multiplier (u_k was 0 above)
#pragma unroll
      for (int j = 0; j < 3; ++j) b[j] = __builtin_fma(-l, prhs[buf][bw][j], b[j]);
    }
  }
  __syncthreads();

  // ---- back substitution by position, k descending ----------------------------
#pragma unroll 1
  for (int k = N - 1; k >= 0; --k) {
    const double ak = get_col<NMAX>(a, k);
    if (t == rowat[k]) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        b[j] = b[j] / ak;
        xsol[j][k] = b[j];
      }
    }
    __syncthreads();
    if (real && pos < k) {
#pragma unroll
      for (int j = 0; j < 3; ++j) b[j] = __builtin_fma(-ak, xsol[j][k], b[j]);
    }
  }
  __syncthreads();

  // ---- outputs ---------------------------------------------------------------
  for (int idx = t; idx < 3 * n; idx += T) {
    const int aa = idx / 3, j = idx - 3 * aa;
    dphi[3 * (b0 + aa) + j] = xsol[j][aa];
  }
  if (keep) {
    double* L = lu + lu_off[g];  // column-major by position
    if (real) {
#pragma unroll
      for (int c = 0; c < NMAX; ++c)
        if (c < N) L[(int64_t)c * N + pos] = a[c];
    }
    const int64_t o = b0 + 4 * g;
    for (int i = t; i < N; i += T) piv_out[o + i] = ipiv[i];
    for (int idx = t; idx < 3 * N; idx += T) {
      const int j = idx / N, i = idx - j * N;
      gam[3 * o + idx] = xsol[j][i];
    }
  }
}

template <int NMAX, int WAVES>
rpim_status launch_one(rpim_plan* p, const Bucket& bk, const double* X, double C2, int keep, hipStream_t s) {
  hipLaunchKernelGGL((k_shape_reg<NMAX, WAVES>), dim3((unsigned)bk.count), dim3(64 * WAVES), 0, s,
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
    case 8: case 16: return launch_one<16, 1>(p, b, X, C2, keep, s);
    case 24: return launch_one<24, 1>(p, b, X, C2, keep, s);
    case 32: return launch_one<32, 1>(p, b, X, C2, keep, s);
    case 40: return launch_one<40, 1>(p, b, X, C2, keep, s);
    case 48: return launch_one<48, 1>(p, b, X, C2, keep, s);
    case 56: return launch_one<56, 1>(p, b, X, C2, keep, s);
    case 64: return launch_one<64, 1>(p, b, X, C2, keep, s);
    case 72: return launch_one<72, 2>(p, b, X, C2, keep, s);
    case 80: return launch_one<80, 2>(p, b, X, C2, keep, s);
    case 88: return launch_one<88, 2>(p, b, X, C2, keep, s);
    case 96: return launch_one<96, 2>(p, b, X, C2, keep, s);
    case 104: return launch_one<104, 2>(p, b, X, C2, keep, s);
    default: return RPIM_E_RANGE;
  }
}

}  // namespace rpim
