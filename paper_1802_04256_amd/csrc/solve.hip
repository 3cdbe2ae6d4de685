// Stage 3: solve of the penalty-constrained system K u = f (GeoMFree3D Sec. 2,
// stage 3, where the paper hands the sparse system to a GPU sparse solver).
// Here: conjugate gradients with the Jacobi (diagonal) preconditioner on the
// CSR matrix the assembly produced, FP64 vectors, K in FP64 or FP32 (widened
// exactly).  Every reduction has a fixed order (per-row wave sums with a fixed
// butterfly, per-workgroup trees, one final workgroup over the partials in
// index order), so two solves of the same system give the same bits.
//
// The scalars of the iteration live on the device; the host only launches.
// Every kernel first reads the `done` flag and returns once the residual test
// has passed, so launched iterations past convergence do nothing, and the host
// checks the flag every kCheck iterations.
//   r = f - K x;  z = D^-1 r;  p = z;  rz = r.z
//   repeat: q = K p;  alpha = rz / (p.q);  x += alpha p;  r -= alpha q;
//           stop when |r| <= rtol |f|;  z = D^-1 r;  beta = r.z / rz;
//           p = z + beta p
#include <cmath>
#include <type_traits>

#include "rpim_internal.h"

namespace rpim {
namespace {

constexpr int kT = 256;             // threads per workgroup
constexpr int kRowsPerBlock = kT / 64;  // SpMV: one wave per row
constexpr int kCheck = 32;          // iterations between host convergence checks

// Device scalars of the iteration.
struct CgState {
  double rz;      // r . z of the current iterate
  double pq;      // p . K p
  double rr;      // r . r
  double bnorm2;  // f . f
  double rtol2;   // (rtol |f|)^2
  int64_t iters;  // iterations done
  int32_t done;   // residual test passed (or a breakdown)
  int32_t fail;   // breakdown: p . K p <= 0 or not finite
};

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Fixed-order sum over a workgroup: wave butterflies, then wave 0 adds the
// wave totals in wave order.  Result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kT / 64; ++i) s += red[i];
  return s;
}

__global__ void __launch_bounds__(kT) k_diag_inv(const int64_t* row_ptr, const int32_t* col_idx, const void* K,
                                                 int fp32, int64_t n, double* dinv, CgState* st) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  int64_t b = row_ptr[i], e = row_ptr[i + 1];
  while (b < e) {
    const int64_t m = (b + e) >> 1;
    if (col_idx[m] < i) b = m + 1; else e = m;
  }
  double d = 0.0;
  if (b < row_ptr[i + 1] && col_idx[b] == i) d = fp32 ? (double)((const float*)K)[b] : ((const double*)K)[b];
  if (!(d > 0.0)) {  // no positive diagonal: Jacobi is undefined
    st->fail = 1;
    st->done = 1;
  }
  dinv[i] = 1.0 / d;
}

// y = K x for the rows of this workgroup (one wave per row, lanes over the
// row's entries in order), and the workgroup's partial of x . y.
template <class T>
__global__ void __launch_bounds__(kT) k_spmv_dot(const int64_t* row_ptr, const int32_t* col_idx, const T* K,
                                                 int64_t n, const double* x, double* y, double* part,
                                                 const CgState* st) {
  if (st->done) return;
  __shared__ double red[kT / 64];
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * kRowsPerBlock + (threadIdx.x >> 6);
  double xy = 0.0;
  if (row < n) {
    double s = 0.0;
    for (int64_t e = row_ptr[row] + lane; e < row_ptr[row + 1]; e += 64) s += (double)K[e] * x[col_idx[e]];
    s = wave_sum(s);
    if (lane == 0) {
      y[row] = s;
      xy = x[row] * s;
    }
  }
  const double b = block_sum(xy, red);
  if (threadIdx.x == 0) part[blockIdx.x] = b;
}

// One workgroup: sum of the partials in index order, into *out.
__global__ void __launch_bounds__(kT) k_reduce(const double* part, int64_t np, double* out, const CgState* st) {
  if (st->done) return;
  __shared__ double red[kT / 64];
  double s = 0.0;
  // thread t adds partials t, t + kT, ... in order; the tree over threads is fixed
  for (int64_t i = threadIdx.x; i < np; i += kT) s += part[i];
  const double b = block_sum(s, red);
  if (threadIdx.x == 0) *out = b;
}

// x += alpha p, r -= alpha q, z = D^-1 r; partials of r . z and r . r.
__global__ void __launch_bounds__(kT) k_update(int64_t n, const double* p, const double* q, const double* dinv,
                                               double* x, double* r, double* z, double* part_rz, double* part_rr,
                                               CgState* st) {
  if (st->done) return;
  __shared__ double red[kT / 64];
  const double alpha = st->rz / st->pq;
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  double rz = 0.0, rr = 0.0;
  if (i < n) {
    x[i] = __builtin_fma(alpha, p[i], x[i]);
    const double ri = __builtin_fma(-alpha, q[i], r[i]);
    r[i] = ri;
    const double zi = dinv[i] * ri;
    z[i] = zi;
    rz = ri * zi;
    rr = ri * ri;
  }
  const double a = block_sum(rz, red);
  __syncthreads();
  const double b = block_sum(rr, red);
  if (threadIdx.x == 0) {
    part_rz[blockIdx.x] = a;
    part_rr[blockIdx.x] = b;
  }
}

// One workgroup: finish r . z and r . r, test the residual, form beta.
__global__ void __launch_bounds__(kT) k_step_scalars(const double* part_rz, const double* part_rr, int64_t np,
                                                     double* beta, CgState* st) {
  if (st->done) return;
  __shared__ double red[kT / 64];
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < np; i += kT) {
    a += part_rz[i];
    b += part_rr[i];
  }
  a = block_sum(a, red);
  __syncthreads();
  b = block_sum(b, red);
  if (threadIdx.x == 0) {
    st->iters += 1;
    st->rr = b;
    *beta = a / st->rz;
    st->rz = a;
    if (b <= st->rtol2) st->done = 1;
  }
}

// p = z + beta p
__global__ void __launch_bounds__(kT) k_direction(int64_t n, const double* z, const double* beta, double* p,
                                                  const CgState* st) {
  if (st->done) return;
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i < n) p[i] = __builtin_fma(*beta, p[i], z[i]);
}

// After the first K x: r = f - K x, z = D^-1 r, p = z; partials of r . z, r . r, f . f.
__global__ void __launch_bounds__(kT) k_start(int64_t n, const double* f, const double* Kx, const double* dinv,
                                              double* r, double* z, double* p, double* part_rz, double* part_rr,
                                              double* part_ff, const CgState* st) {
  if (st->done) return;
  __shared__ double red[kT / 64];
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  double rz = 0.0, rr = 0.0, ff = 0.0;
  if (i < n) {
    const double ri = f[i] - Kx[i];
    const double zi = dinv[i] * ri;
    r[i] = ri;
    z[i] = zi;
    p[i] = zi;
    rz = ri * zi;
    rr = ri * ri;
    ff = f[i] * f[i];
  }
  const double a = block_sum(rz, red);
  __syncthreads();
  const double b = block_sum(rr, red);
  __syncthreads();
  const double c = block_sum(ff, red);
  if (threadIdx.x == 0) {
    part_rz[blockIdx.x] = a;
    part_rr[blockIdx.x] = b;
    part_ff[blockIdx.x] = c;
  }
}

__global__ void __launch_bounds__(kT) k_start_scalars(const double* part_rz, const double* part_rr,
                                                      const double* part_ff, int64_t np, double rtol, CgState* st) {
  __shared__ double red[kT / 64];
  double a = 0.0, b = 0.0, c = 0.0;
  for (int64_t i = threadIdx.x; i < np; i += kT) {
    a += part_rz[i];
    b += part_rr[i];
    c += part_ff[i];
  }
  a = block_sum(a, red);
  __syncthreads();
  b = block_sum(b, red);
  __syncthreads();
  c = block_sum(c, red);
  if (threadIdx.x == 0) {
    st->rz = a;
    st->rr = b;
    st->bnorm2 = c;
    st->rtol2 = (rtol * rtol) * c;
    st->iters = 0;
    if (!st->fail) st->done = (b <= st->rtol2) ? 1 : 0;
  }
}

// A breakdown (p . K p not positive or not finite) ends the iteration.
__global__ void k_check_pq(CgState* st) {
  if (st->done) return;
  if (!(st->pq > 0.0) || !std::isfinite(st->pq)) {
    st->fail = 1;
    st->done = 1;
  }
}

__global__ void k_init_state(CgState* st) {
  st->rz = st->pq = st->rr = st->bnorm2 = st->rtol2 = 0.0;
  st->iters = 0;
  st->done = 0;
  st->fail = 0;
}

inline int64_t nblocks(int64_t n, int t) { return (n + t - 1) / t; }

struct CgWs {
  CgState* st;
  double *r, *z, *p, *q, *dinv, *beta, *part_a, *part_b, *part_c;
  int64_t np_vec, np_spmv;
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t cg_layout(int64_t n, CgWs* w, void* base) {
  char* b = static_cast<char*>(base);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    void* q = b ? b + off : nullptr;
    off += align256(bytes);
    return q;
  };
  const int64_t npv = nblocks(n, kT), nps = nblocks(n, kRowsPerBlock);
  CgWs t;
  t.st = (CgState*)take(sizeof(CgState));
  t.r = (double*)take(8 * (size_t)n);
  t.z = (double*)take(8 * (size_t)n);
  t.p = (double*)take(8 * (size_t)n);
  t.q = (double*)take(8 * (size_t)n);
  t.dinv = (double*)take(8 * (size_t)n);
  t.beta = (double*)take(8);
  t.part_a = (double*)take(8 * (size_t)std::max(npv, nps));
  t.part_b = (double*)take(8 * (size_t)npv);
  t.part_c = (double*)take(8 * (size_t)npv);
  t.np_vec = npv;
  t.np_spmv = nps;
  if (w) *w = t;
  return off;
}

template <class T>
rpim_status cg_run(const int64_t* row_ptr, const int32_t* col_idx, const T* K, int64_t n, const double* f, double* x,
                   double rtol, int64_t max_iter, const CgWs& w, hipStream_t s, int64_t* iters, double* relres) {
  const dim3 tb(kT);
  const dim3 gv((unsigned)w.np_vec), gs((unsigned)w.np_spmv);
  hipLaunchKernelGGL(k_init_state, dim3(1), dim3(1), 0, s, w.st);
  hipLaunchKernelGGL(k_diag_inv, gv, tb, 0, s, row_ptr, col_idx, (const void*)K, (int)std::is_same<T, float>::value,
                     n, w.dinv, w.st);
  hipLaunchKernelGGL(k_spmv_dot<T>, gs, tb, 0, s, row_ptr, col_idx, K, n, (const double*)x, w.q, w.part_a,
                     (const CgState*)w.st);
  hipLaunchKernelGGL(k_start, gv, tb, 0, s, n, f, (const double*)w.q, (const double*)w.dinv, w.r, w.z, w.p,
                     w.part_a, w.part_b, w.part_c, (const CgState*)w.st);
  hipLaunchKernelGGL(k_start_scalars, dim3(1), tb, 0, s, (const double*)w.part_a, (const double*)w.part_b,
                     (const double*)w.part_c, w.np_vec, rtol, w.st);
  RPIM_HIP(hipGetLastError());
  CgState h = {};
  for (int64_t it = 0; it < max_iter; ++it) {
    hipLaunchKernelGGL(k_spmv_dot<T>, gs, tb, 0, s, row_ptr, col_idx, K, n, (const double*)w.p, w.q, w.part_a,
                       (const CgState*)w.st);
    hipLaunchKernelGGL(k_reduce, dim3(1), tb, 0, s, (const double*)w.part_a, w.np_spmv, &w.st->pq,
                       (const CgState*)w.st);
    hipLaunchKernelGGL(k_check_pq, dim3(1), dim3(1), 0, s, w.st);
    hipLaunchKernelGGL(k_update, gv, tb, 0, s, n, (const double*)w.p, (const double*)w.q, (const double*)w.dinv, x,
                       w.r, w.z, w.part_a, w.part_b, w.st);
    hipLaunchKernelGGL(k_step_scalars, dim3(1), tb, 0, s, (const double*)w.part_a, (const double*)w.part_b,
                       w.np_vec, w.beta, w.st);
    hipLaunchKernelGGL(k_direction, gv, tb, 0, s, n, (const double*)w.z, (const double*)w.beta, w.p,
                       (const CgState*)w.st);
    if ((it + 1) % kCheck == 0 || it + 1 == max_iter) {
      RPIM_HIP(hipGetLastError());
      RPIM_HIP(hipMemcpyAsync(&h, w.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
      RPIM_HIP(hipStreamSynchronize(s));
      if (h.done) break;
    }
  }
  RPIM_HIP(hipGetLastError());
  RPIM_HIP(hipMemcpyAsync(&h, w.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
  RPIM_HIP(hipStreamSynchronize(s));
  if (iters) *iters = h.iters;
  if (relres) *relres = h.bnorm2 > 0 ? std::sqrt(h.rr / h.bnorm2) : std::sqrt(h.rr);
  if (h.fail) return RPIM_E_SINGULAR;
  return h.done ? RPIM_OK : RPIM_E_CONVERGENCE;
}

}  // namespace

size_t pcg_workspace_bytes(int64_t n) { return cg_layout(n, nullptr, nullptr); }

rpim_status solve_pcg(const int64_t* row_ptr, const int32_t* col_idx, const void* K, int precision, int64_t n,
                      const double* f, double* x, double rtol, int64_t max_iter, void* ws, size_t ws_bytes,
                      int64_t* iters, double* relres, hipStream_t s) {
  if (!ws || ws_bytes < pcg_workspace_bytes(n) || (reinterpret_cast<uintptr_t>(ws) & 255u)) return RPIM_E_ARG;
  CgWs w;
  cg_layout(n, &w, ws);
  if (precision == RPIM_FP64)
    return cg_run(row_ptr, col_idx, (const double*)K, n, f, x, rtol, max_iter, w, s, iters, relres);
  return cg_run(row_ptr, col_idx, (const float*)K, n, f, x, rtol, max_iter, w, s, iters, relres);
}

}  // namespace rpim
