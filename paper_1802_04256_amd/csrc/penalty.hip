// Stage 2: penalty enforcement of prescribed displacements (GeoMFree3D
// Sec. 2: one GPU thread per constrained degree of freedom).
//   alpha = factor * max_i K_ii   (max over every diagonal, before the update)
//   K_dd += alpha,  rhs_d += alpha * u_bar_d   for each fixed dof d.
// The max is an exact, order-independent reduction; fixed dofs are unique so
// the update needs no atomics.
#include <cfloat>
#include <cmath>

#include "rpim_internal.h"

namespace rpim {
namespace {

constexpr int kT = 256;

__device__ __forceinline__ int64_t diag_pos(const int64_t* row_ptr, const int32_t* col_idx, int64_t d) {
  int64_t b = row_ptr[d], e = row_ptr[d + 1];
  while (b < e) {
    const int64_t m = (b + e) >> 1;
    if (col_idx[m] < d) b = m + 1; else e = m;
  }
  return (b < row_ptr[d + 1] && col_idx[b] == d) ? b : -1;
}

__global__ void k_check_fixed(const int32_t* fixed, int64_t n_fixed, int64_t n_dof, unsigned* bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_fixed) return;
  const int32_t d = fixed[i];
  if (d < 0 || d >= n_dof || (i > 0 && fixed[i - 1] >= d)) atomicOr(bad, 1u);
}

template <class T>
__global__ void __launch_bounds__(kT) k_diag_max(const int64_t* row_ptr, const int32_t* col_idx, const T* K,
                                                 int64_t n_dof, double* part, unsigned* bad) {
  double m = -INFINITY;
  for (int64_t d = (int64_t)blockIdx.x * kT + threadIdx.x; d < n_dof; d += (int64_t)gridDim.x * kT) {
    const int64_t p = diag_pos(row_ptr, col_idx, d);
    if (p < 0) atomicOr(bad, 2u);
    else m = fmax(m, (double)K[p]);
  }
  __shared__ double red[kT];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = kT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(kT) k_alpha(const double* part, int nparts, double factor, double* alpha) {
  double m = -INFINITY;
  for (int i = threadIdx.x; i < nparts; i += kT) m = fmax(m, part[i]);
  __shared__ double red[kT];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = kT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *alpha = factor * red[0];
}

template <class T>
__global__ void k_apply(const int64_t* row_ptr, const int32_t* col_idx, T* K, const int32_t* fixed,
                        const double* ubar, int64_t n_fixed, const double* alpha_p, double* rhs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_fixed) return;
  const double alpha = *alpha_p;
  const int32_t d = fixed[i];
  const int64_t p = diag_pos(row_ptr, col_idx, d);
  if (p < 0) return;
  K[p] = K[p] + (T)alpha;
  if (rhs) rhs[d] = rhs[d] + alpha * (ubar ? ubar[i] : 0.0);
}

}  // namespace

rpim_status launch_penalty(const int64_t* row_ptr, const int32_t* col_idx, void* K, int precision, int64_t n_dof,
                           const int32_t* fixed, const double* ubar, int64_t n_fixed, double factor, double* rhs,
                           double* alpha_out, hipStream_t s) {
  const int nparts = (int)std::min<int64_t>((n_dof + kT - 1) / kT, 1024);
  void* scratch = nullptr;
  const size_t bytes = sizeof(double) * (nparts + 1) + 2 * sizeof(unsigned);
  RPIM_HIP(hipMallocAsync(&scratch, bytes, s));
  double* part = (double*)scratch;
  double* alpha = part + nparts;
  unsigned* bad = (unsigned*)(alpha + 1);
  RPIM_HIP(hipMemsetAsync(bad, 0, sizeof(unsigned), s));
  if (n_fixed > 0)
    hipLaunchKernelGGL(k_check_fixed, dim3((unsigned)((n_fixed + kT - 1) / kT)), dim3(kT), 0, s, fixed, n_fixed,
                       n_dof, bad);
  if (precision == RPIM_FP64)
    hipLaunchKernelGGL(k_diag_max<double>, dim3(nparts), dim3(kT), 0, s, row_ptr, col_idx, (const double*)K, n_dof,
                       part, bad);
  else
    hipLaunchKernelGGL(k_diag_max<float>, dim3(nparts), dim3(kT), 0, s, row_ptr, col_idx, (const float*)K, n_dof,
                       part, bad);
  RPIM_HIP(hipGetLastError());
  unsigned hbad = 0;
  RPIM_HIP(hipMemcpyAsync(&hbad, bad, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  RPIM_HIP(hipStreamSynchronize(s));
  if (hbad) {
    RPIM_HIP(hipFreeAsync(scratch, s));
    return RPIM_E_ARG;
  }
  hipLaunchKernelGGL(k_alpha, dim3(1), dim3(kT), 0, s, (const double*)part, nparts, factor, alpha);
  if (n_fixed > 0) {
    const dim3 grid((unsigned)((n_fixed + kT - 1) / kT));
    if (precision == RPIM_FP64)
      hipLaunchKernelGGL(k_apply<double>, grid, dim3(kT), 0, s, row_ptr, col_idx, (double*)K, fixed, ubar, n_fixed,
                         (const double*)alpha, rhs);
    else
      hipLaunchKernelGGL(k_apply<float>, grid, dim3(kT), 0, s, row_ptr, col_idx, (float*)K, fixed, ubar, n_fixed,
                         (const double*)alpha, rhs);
  }
  RPIM_HIP(hipGetLastError());
  if (alpha_out) {
    RPIM_HIP(hipMemcpyAsync(alpha_out, alpha, sizeof(double), hipMemcpyDeviceToHost, s));
    RPIM_HIP(hipStreamSynchronize(s));
  }
  RPIM_HIP(hipFreeAsync(scratch, s));
  return RPIM_OK;
}

}  // namespace rpim
