// Solves with the kept factors of one point's moment matrix (shared by the
// adjoint and by the shape-function values; included by backward.hip and
// post.hip only).
//
// F is the packed factor matrix, column-major F[c*N + p]: for p <= c the U
// entry u_pc (rows by position), for p > c the multiplier applied at step c
// to the row that held position p after that step's interchange; ppos[k] is
// the position the pivot of step k held before its interchange.  The
// arithmetic is the elimination order of the arithmetic contract applied to
// extra right-hand-side columns: forward, for k ascending, b_r = fma(-l_rk,
// b_k, b_r) for the rows below the pivot; back, for k descending,
// x_k = b_k / u_kk, then b_r = fma(-u_rk, x_k, b_r) for r < k.
#pragma once

#include "rpim_internal.h"

namespace rpim {

// One workgroup of whole waves, thread t < N owning original row t.  b holds
// thread t's NR right-hand-side entries (rows t >= N: ignored).  y and x are
// LDS arrays of NR * N doubles; on return x[c*N + k] is unknown k of
// solution c.  ppos is LDS.  Contains barriers: every thread calls it.
template <int NR>
__device__ __forceinline__ void kept_solve(const double* F, const int* ppos, int N, int tid, double (&b)[NR],
                                           double* y, double* x) {
  const bool own = tid < N;
  // Forward substitution on original rows, replaying the interchanges: thread r
  // tracks the position of its row (the pivot of step k takes position k, the
  // row that held k takes the pivot's old position).  Factor entries are read
  // PF steps ahead; a second tracker replays the interchanges PF steps ahead of
  // the first, so each entry is read at the position the row will hold then.
  constexpr int PF = 8;
  const auto interchange = [&](int k, int q) {  // position after step k of a row at q before it
    const int pk = ppos[k];
    return q == pk ? k : (q == k ? pk : q);
  };
  int pos = own ? tid : N;   // position before the current step
  int posa = pos;            // position after the steps already prefetched
  double fcur[PF], fnxt[PF];
  const auto fetch = [&](int k, int q) { return F[(int64_t)k * N + (q < N ? q : N - 1)]; };
#pragma unroll
  for (int j = 0; j < PF; ++j) {
    if (j < N) {
      posa = interchange(j, posa);
      fcur[j] = fetch(j, posa);
    }
  }
  for (int k0 = 0; k0 < N; k0 += PF) {
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      const int kk = k0 + PF + j;
      if (kk < N) {  // uniform
        posa = interchange(kk, posa);
        fnxt[j] = fetch(kk, posa);
      }
    }
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      const int k = k0 + j;
      if (k < N) {  // uniform
        const int after = interchange(k, pos);
        if (own && after == k) {  // my row is the pivot of step k
          for (int c = 0; c < NR; ++c) y[c * N + k] = b[c];
        }
        pos = after;
        __syncthreads();
        if (own && pos > k)
          for (int c = 0; c < NR; ++c) b[c] = __builtin_fma(-fcur[j], y[c * N + k], b[c]);
      }
    }
#pragma unroll
    for (int j = 0; j < PF; ++j) fcur[j] = fnxt[j];
  }
  __syncthreads();
  // back substitution by position: thread p holds y_p; u_{p,k} read PF steps ahead
  const int trow = own ? tid : 0;
  double yp[NR];
  for (int c = 0; c < NR; ++c) yp[c] = 0.0;
  if (own)
    for (int j = 0; j < NR; ++j) yp[j] = y[j * N + tid];
#pragma unroll
  for (int j = 0; j < PF; ++j) {
    const int kk = N - 1 - j;
    fcur[j] = F[(int64_t)(kk >= 0 ? kk : 0) * N + trow];
  }
  for (int k0 = N - 1; k0 >= 0; k0 -= PF) {
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      const int kk = k0 - PF - j;
      fnxt[j] = F[(int64_t)(kk >= 0 ? kk : 0) * N + trow];
    }
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      const int k = k0 - j;
      if (k >= 0) {  // uniform
        const double uk = fcur[j];  // u_{tid,k}
        if (tid == k)
          for (int c = 0; c < NR; ++c) {
            yp[c] = yp[c] / uk;
            x[c * N + k] = yp[c];
          }
        __syncthreads();
        if (tid < k)
          for (int c = 0; c < NR; ++c) yp[c] = __builtin_fma(-uk, x[c * N + k], yp[c]);
      }
    }
#pragma unroll
    for (int j = 0; j < PF; ++j) fcur[j] = fnxt[j];
  }
  __syncthreads();
}

}  // namespace rpim
