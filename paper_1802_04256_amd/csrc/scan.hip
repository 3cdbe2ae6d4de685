// Exclusive prefix sums (int32 or int64 values -> int64 offsets[n+1]) in three passes:
// per-tile totals, a scan of the totals (recursively), then each tile rescans
// and adds its base.  Used to size supports, inverse lists, bins and rows.
#include "rpim_internal.h"

namespace rpim {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;  // items per thread
constexpr int kTile = kScanThreads * kScanPer;

// Exclusive scan of one value per thread across the block; *total = block sum.
__device__ int64_t block_exclusive(int64_t v, int64_t* total) {
  __shared__ int64_t warp_sums[kScanThreads / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int64_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    int64_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) warp_sums[wid] = x;
  __syncthreads();
  int64_t base = 0, tot = 0;
  for (int w = 0; w < kScanThreads / 64; ++w) {
    if (w < wid) base += warp_sums[w];
    tot += warp_sums[w];
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

template <class T>
__global__ void __launch_bounds__(kScanThreads) k_tile_sums(const T* in, int64_t n, int64_t* sums) {
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kScanPer;
  int64_t s = 0;
  for (int i = 0; i < kScanPer; ++i)
    if (base + i < n) s += (int64_t)in[base + i];
  int64_t tot;
  block_exclusive(s, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// out[i] = base + exclusive prefix; the thread holding element n-1 also
// writes out[n] (the grand total).
template <class T>
__global__ void __launch_bounds__(kScanThreads) k_tile_scan(const T* in, int64_t n, const int64_t* tile_base,
                                                            int64_t* out) {
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kScanPer;
  int64_t v[kScanPer];
  int64_t s = 0;
  for (int i = 0; i < kScanPer; ++i) {
    v[i] = (base + i < n) ? (int64_t)in[base + i] : 0;
    s += v[i];
  }
  int64_t tot;
  int64_t run = block_exclusive(s, &tot) + (tile_base ? tile_base[blockIdx.x] : 0);
  for (int i = 0; i < kScanPer; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
    if (base + i == n - 1) out[n] = run;
  }
}

template <class T>
rpim_status scan_impl(const T* in, int64_t n, int64_t* out, hipStream_t s) {
  if (n <= 0) {
    RPIM_HIP(hipMemsetAsync(out, 0, sizeof(int64_t), s));
    return RPIM_OK;
  }
  const int64_t tiles = (n + kTile - 1) / kTile;
  int64_t* sums = nullptr;
  int64_t* bases = nullptr;
  if (tiles > 1) {
    RPIM_HIP(hipMallocAsync((void**)&sums, sizeof(int64_t) * tiles, s));
    RPIM_HIP(hipMallocAsync((void**)&bases, sizeof(int64_t) * (tiles + 1), s));
    hipLaunchKernelGGL(k_tile_sums<T>, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, in, n, sums);
    RPIM_HIP(hipGetLastError());
    rpim_status st = scan_impl<int64_t>(sums, tiles, bases, s);
    if (st != RPIM_OK) return st;
  }
  hipLaunchKernelGGL(k_tile_scan<T>, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, in, n,
                     (const int64_t*)bases, out);
  RPIM_HIP(hipGetLastError());
  if (sums) RPIM_HIP(hipFreeAsync(sums, s));
  if (bases) RPIM_HIP(hipFreeAsync(bases, s));
  return RPIM_OK;
}

}  // namespace

rpim_status exclusive_scan(const int32_t* counts, int64_t n, int64_t* out, hipStream_t s) {
  return scan_impl<int32_t>(counts, n, out, s);
}

rpim_status exclusive_scan64(const int64_t* values, int64_t n, int64_t* out, hipStream_t s) {
  return scan_impl<int64_t>(values, n, out, s);
}

}  // namespace rpim
