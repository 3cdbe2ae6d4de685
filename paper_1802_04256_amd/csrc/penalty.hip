// Stage 2: penalty enforcement of prescribed displacements (GeoMFree3D
// Sec. 2: one GPU thread per constrained degree of freedom).
//   alpha = factor * max_i K_ii   (max over every diagonal, before the update)
//   K_dd += alpha,  rhs_d += alpha * u_bar_d   for each fixed dof d.
// The max is an exact, order-independent reduction; fixed dofs are unique so
// the update needs no atomics.  Every step is a kernel on the caller's stream
// (no host synchronisation, no memset, no allocation), so the call can be
// recorded into a graph; the argument check runs on the device and, when it
// fails, leaves K and rhs untouched and reports through a device status word.
//
// Workspace layout (device bytes, from rpim_penalty_workspace_bytes):
//   [0, 8)            check flags (bit 0: fixed dofs not strictly ascending in
//                     [0, n_dof); bit 1: a needed diagonal is missing)
//   [8, 16)           alpha
//   [16, 16 + 8 P)    partial maxima, P = number of diag-max workgroups
//   then 8 n_fixed    diagonal position of each fixed dof
#include <cfloat>
#include <climits>
#include <cmath>
#include <mutex>

#include "rpim_internal.h"

namespace rpim {
namespace {

constexpr int kT = 256;
constexpr int kMaxParts = 1024;  // workgroups of the diagonal max (grid-stride beyond)
constexpr int kCheckT = 1024;    // the single workgroup of the argument check

struct PenaltyWs {
  unsigned* flags;
  double* alpha;
  double* part;
  int64_t* pos;
  int nparts;
};

int parts_for(int64_t n_dof) { return (int)std::min<int64_t>((n_dof + kT - 1) / kT, kMaxParts); }

size_t ws_bytes(int64_t n_dof, int64_t n_fixed) {
  return 16 + sizeof(double) * (size_t)parts_for(n_dof) + sizeof(int64_t) * (size_t)std::max<int64_t>(n_fixed, 0);
}

PenaltyWs carve(void* ws, int64_t n_dof) {
  PenaltyWs w;
  char* b = static_cast<char*>(ws);
  w.flags = reinterpret_cast<unsigned*>(b);
  w.alpha = reinterpret_cast<double*>(b + 8);
  w.part = reinterpret_cast<double*>(b + 16);
  w.nparts = parts_for(n_dof);
  w.pos = reinterpret_cast<int64_t*>(w.part + w.nparts);
  return w;
}

__device__ __forceinline__ int64_t diag_pos(const int64_t* row_ptr, const int32_t* col_idx, int64_t d) {
  int64_t b = row_ptr[d], e = row_ptr[d + 1];
  while (b < e) {
    const int64_t m = (b + e) >> 1;
    if (col_idx[m] < d) b = m + 1; else e = m;
  }
  return (b < row_ptr[d + 1] && col_idx[b] == d) ? b : -1;
}

// One workgroup: checks the fixed dofs, finds their diagonal positions and
// writes the flag word afresh (so nothing has to be cleared beforehand).
__global__ void __launch_bounds__(kCheckT) k_check_fixed(const int64_t* row_ptr, const int32_t* col_idx,
                                                         const int32_t* fixed, int64_t n_fixed, int64_t n_dof,
                                                         unsigned* flags, int64_t* pos) {
  unsigned bad = 0;
  for (int64_t i = threadIdx.x; i < n_fixed; i += kCheckT) {
    const int32_t d = fixed[i];
    if (d < 0 || d >= n_dof || (i > 0 && fixed[i - 1] >= d)) {
      bad |= 1u;
      pos[i] = -1;
      continue;
    }
    const int64_t p = diag_pos(row_ptr, col_idx, d);
    if (p < 0) bad |= 2u;
    pos[i] = p;
  }
  __shared__ unsigned red[kCheckT / 64];
  for (int o = 32; o > 0; o >>= 1) bad |= __shfl_xor(bad, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = bad;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned f = 0;
    for (int i = 0; i < kCheckT / 64; ++i) f |= red[i];
    *flags = f;
  }
}

template <class T>
__global__ void __launch_bounds__(kT) k_diag_max(const int64_t* row_ptr, const int32_t* col_idx, const T* K,
                                                 int64_t n_dof, double* part, unsigned* flags) {
  double m = -INFINITY;
  bool missing = false;
  for (int64_t d = (int64_t)blockIdx.x * kT + threadIdx.x; d < n_dof; d += (int64_t)gridDim.x * kT) {
    const int64_t p = diag_pos(row_ptr, col_idx, d);
    if (p < 0) missing = true;
    else m = fmax(m, (double)K[p]);
  }
  if (missing) atomicOr(flags, 2u);  // an OR: the same result in any order
  __shared__ double red[kT];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = kT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(kT) k_alpha(const double* part, int nparts, double factor, const unsigned* flags,
                                              double* alpha_ws, double* alpha_out, int32_t* status_out) {
  double m = -INFINITY;
  for (int i = threadIdx.x; i < nparts; i += kT) m = fmax(m, part[i]);
  __shared__ double red[kT];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = kT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double a = factor * red[0];
    *alpha_ws = a;
    if (alpha_out) *alpha_out = a;
    if (status_out) *status_out = *flags ? (int32_t)RPIM_E_ARG : (int32_t)RPIM_OK;
  }
}

template <class T>
__global__ void k_apply(T* K, const int32_t* fixed, const int64_t* pos, const double* ubar, int64_t n_fixed,
                        const double* alpha_p, const unsigned* flags, double* rhs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_fixed || *flags) return;  // a failed check leaves K and rhs as they were
  const double alpha = *alpha_p;
  const int64_t p = pos[i];
  K[p] = K[p] + (T)alpha;
  if (rhs) {
    const int32_t d = fixed[i];
    rhs[d] = rhs[d] + alpha * (ubar ? ubar[i] : 0.0);
  }
}

// The launch sequence shared by both entry points; ws holds ws_bytes(n_dof, n_fixed) bytes.
rpim_status penalty_launch(const int64_t* row_ptr, const int32_t* col_idx, void* K, int precision, int64_t n_dof,
                           const int32_t* fixed, const double* ubar, int64_t n_fixed, double factor, double* rhs,
                           double* alpha_out, int32_t* status_out, void* ws, hipStream_t s) {
  const PenaltyWs w = carve(ws, n_dof);
  hipLaunchKernelGGL(k_check_fixed, dim3(1), dim3(kCheckT), 0, s, row_ptr, col_idx, fixed, n_fixed, n_dof, w.flags,
                     w.pos);
  if (precision == RPIM_FP64)
    hipLaunchKernelGGL(k_diag_max<double>, dim3(w.nparts), dim3(kT), 0, s, row_ptr, col_idx, (const double*)K,
                       n_dof, w.part, w.flags);
  else
    hipLaunchKernelGGL(k_diag_max<float>, dim3(w.nparts), dim3(kT), 0, s, row_ptr, col_idx, (const float*)K, n_dof,
                       w.part, w.flags);
  hipLaunchKernelGGL(k_alpha, dim3(1), dim3(kT), 0, s, (const double*)w.part, w.nparts, factor,
                     (const unsigned*)w.flags, w.alpha, alpha_out, status_out);
  if (n_fixed > 0) {
    const dim3 grid((unsigned)((n_fixed + kT - 1) / kT));
    if (precision == RPIM_FP64)
      hipLaunchKernelGGL(k_apply<double>, grid, dim3(kT), 0, s, (double*)K, fixed, (const int64_t*)w.pos, ubar,
                         n_fixed, (const double*)w.alpha, (const unsigned*)w.flags, rhs);
    else
      hipLaunchKernelGGL(k_apply<float>, grid, dim3(kT), 0, s, (float*)K, fixed, (const int64_t*)w.pos, ubar,
                         n_fixed, (const double*)w.alpha, (const unsigned*)w.flags, rhs);
  }
  RPIM_HIP(hipGetLastError());
  return RPIM_OK;
}

// ---- library-owned scratch for callers that cannot allocate -----------------
// One copy per GPU, held until the process ends.  Host code never uses the
// array's name as an address: the device address of each GPU's copy comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr int64_t kNoallocMaxFixed = RPIM_PENALTY_NOALLOC_MAX_FIXED;
constexpr size_t kNoallocBytes = 16 + sizeof(double) * kMaxParts + sizeof(int64_t) * kNoallocMaxFixed;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

rpim_status scratch_for_current_device(void** out) {
  int dev = 0;
  RPIM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return RPIM_E_RANGE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    RPIM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return RPIM_E_HIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return RPIM_OK;
}

}  // namespace

size_t penalty_workspace_bytes(int64_t n_dof, int64_t n_fixed) { return ws_bytes(n_dof, n_fixed); }

rpim_status launch_penalty(const int64_t* row_ptr, const int32_t* col_idx, void* K, int precision, int64_t n_dof,
                           const int32_t* fixed, const double* ubar, int64_t n_fixed, double factor, double* rhs,
                           double* alpha_out, int32_t* status_out, void* ws, size_t ws_size, hipStream_t s) {
  if (!ws || ws_size < ws_bytes(n_dof, n_fixed) || (reinterpret_cast<uintptr_t>(ws) & 7u)) return RPIM_E_ARG;
  return penalty_launch(row_ptr, col_idx, K, precision, n_dof, fixed, ubar, n_fixed, factor, rhs, alpha_out,
                        status_out, ws, s);
}

rpim_status launch_penalty_noalloc(const int64_t* row_ptr, const int32_t* col_idx, void* K, int precision,
                                   int64_t n_dof, const int32_t* fixed, const double* ubar, int64_t n_fixed,
                                   double factor, double* rhs, double* alpha_out, int32_t* status_out,
                                   hipStream_t s) {
  if (n_fixed > kNoallocMaxFixed) return RPIM_E_RANGE;
  void* ws = nullptr;
  if (rpim_status st = scratch_for_current_device(&ws)) return st;
  return penalty_launch(row_ptr, col_idx, K, precision, n_dof, fixed, ubar, n_fixed, factor, rhs, alpha_out,
                        status_out, ws, s);
}

}  // namespace rpim
