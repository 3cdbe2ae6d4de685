// Support search and sparsity pattern (one-time per geometry).
//
// 1. Nodes of each model are binned on a uniform grid with edge slightly
//    above the support radius, so a Gauss point's support lies in the 3x3x3
//    bins around it; bins are sorted so the result is independent of launch
//    order.
// 2. One wavefront per Gauss point tests the candidates with the canonical
//    squared distance s = fma(dz,dz, fma(dy,dy, dx*dx)) <= fl(d_s*d_s),
//    compacts hits by ballot into LDS and writes them sorted by node id
//    (rank = number of smaller hits).  A count pass sizes the lists first.
// 3. Inverse lists node -> (Gauss point, local index), filled by integer
//    atomics, then each node's list is sorted in LDS (bitonic) so it is in
//    ascending Gauss-point order.
// 4. Node-block rows: for node I the union of the supports containing I,
//    formed as a bitmap over the node-id window of I's neighbourhood in LDS,
//    counted, scanned and enumerated in ascending order.
// 5. Expansion to the scalar CSR (dof = 3*node + component).
#include <algorithm>
#include <climits>
#include <cmath>

#include "rpim_internal.h"

namespace rpim {
namespace {

__device__ __forceinline__ int model_of(const int64_t* off, int n_models, int64_t i) {
  int lo = 0, hi = n_models - 1;  // largest m with off[m] <= i
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ void flag_error(DevStatus* st, unsigned flag, int64_t g) {
  atomicOr(&st->flags, flag);
  atomicMin(&st->first_bad, (unsigned long long)g);
}

// ---- 0. bounding box per model --------------------------------------------
__global__ void __launch_bounds__(256) k_bbox(const double* X, const int64_t* node_off, double* out) {
  const int m = blockIdx.x;
  const int64_t b = node_off[m], e = node_off[m + 1];
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x)
    for (int k = 0; k < 3; ++k) {
      double v = X[3 * i + k];
      lo[k] = fmin(lo[k], v);
      hi[k] = fmax(hi[k], v);
    }
  __shared__ double red[6][256];
  for (int k = 0; k < 3; ++k) { red[k][threadIdx.x] = lo[k]; red[3 + k][threadIdx.x] = hi[k]; }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < 3; ++k) {
        red[k][threadIdx.x] = fmin(red[k][threadIdx.x], red[k][threadIdx.x + w]);
        red[3 + k][threadIdx.x] = fmax(red[3 + k][threadIdx.x], red[3 + k][threadIdx.x + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) out[6 * m + threadIdx.x] = red[threadIdx.x][0];
}

__device__ __forceinline__ void bin_coords(const BinGrid& gr, double x, double y, double z, int* ix, int* iy,
                                           int* iz) {
  int a = (int)floor((x - gr.ox) / gr.h), b = (int)floor((y - gr.oy) / gr.h), c = (int)floor((z - gr.oz) / gr.h);
  *ix = min(max(a, 0), gr.nx - 1);
  *iy = min(max(b, 0), gr.ny - 1);
  *iz = min(max(c, 0), gr.nz - 1);
}

// ---- 1. binning -------------------------------------------------------------
__global__ void k_bin_count(const double* X, int64_t N, const int64_t* node_off, int n_models,
                            const BinGrid* grids, int32_t* node_bin, int32_t* bin_cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const BinGrid gr = grids[model_of(node_off, n_models, i)];
  int ix, iy, iz;
  bin_coords(gr, X[3 * i], X[3 * i + 1], X[3 * i + 2], &ix, &iy, &iz);
  const int64_t bin = gr.bin0 + ((int64_t)ix * gr.ny + iy) * gr.nz + iz;
  node_bin[i] = (int32_t)bin;
  atomicAdd(&bin_cnt[bin], 1);
}

__global__ void k_bin_fill(int64_t N, const int32_t* node_bin, const int64_t* bin_start, int32_t* cursor,
                           int32_t* bin_nodes) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int32_t b = node_bin[i];
  const int slot = atomicAdd(&cursor[b], 1);
  bin_nodes[bin_start[b] + slot] = (int32_t)i;
}

__global__ void k_bin_sort(int64_t nbins, const int64_t* bin_start, int32_t* bin_nodes, const double* X,
                           double* bxyz) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  const int64_t s = bin_start[b], e = bin_start[b + 1];
  for (int64_t i = s + 1; i < e; ++i) {  // insertion sort: bins hold a handful of nodes
    int32_t v = bin_nodes[i];
    int64_t j = i - 1;
    while (j >= s && bin_nodes[j] > v) { bin_nodes[j + 1] = bin_nodes[j]; --j; }
    bin_nodes[j + 1] = v;
  }
  for (int64_t i = s; i < e; ++i)
    for (int k = 0; k < 3; ++k) bxyz[3 * i + k] = X[3 * (int64_t)bin_nodes[i] + k];
}

// ---- 2. support search: one wavefront per Gauss point -----------------------
template <bool kFill>
__global__ void __launch_bounds__(256) k_support(int64_t G, const int64_t* gp_off, int n_models,
                                                 const BinGrid* grids, const int64_t* bin_start,
                                                 const int32_t* bin_nodes, const double* bxyz,
                                                 const double* gp_xyz, int32_t* counts, const int64_t* gp_ptr,
                                                 int32_t* gp_nbr, DevStatus* st) {
  __shared__ int32_t hits[4][kMaxSupport];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * 4 + w;
  if (g >= G) return;
  const BinGrid gr = grids[model_of(gp_off, n_models, g)];
  const double xg = gp_xyz[3 * g], yg = gp_xyz[3 * g + 1], zg = gp_xyz[3 * g + 2];
  int ix, iy, iz;
  bin_coords(gr, xg, yg, zg, &ix, &iy, &iz);
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int n = 0;
  for (int ax = max(ix - 1, 0); ax <= min(ix + 1, gr.nx - 1); ++ax)
    for (int ay = max(iy - 1, 0); ay <= min(iy + 1, gr.ny - 1); ++ay) {
      const int64_t row = gr.bin0 + ((int64_t)ax * gr.ny + ay) * gr.nz;
      const int64_t j0 = bin_start[row + max(iz - 1, 0)];
      const int64_t j1 = bin_start[row + min(iz + 1, gr.nz - 1) + 1];
      for (int64_t base = j0; base < j1; base += 64) {
        const int64_t j = base + lane;
        bool hit = false;
        if (j < j1) {
          const double dx = bxyz[3 * j] - xg, dy = bxyz[3 * j + 1] - yg, dz = bxyz[3 * j + 2] - zg;
          const double s = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
          hit = s <= gr.r2;
        }
        const unsigned long long mask = __ballot(hit);
        if (kFill && hit) {
          const int pos = n + __popcll(mask & below);
          if (pos < kMaxSupport) hits[w][pos] = bin_nodes[j];
        }
        n += __popcll(mask);
      }
    }
  if (!kFill) {
    if (lane == 0) {
      counts[g] = n;
      if (n < 5) flag_error(st, kFlagSupport, g);
      if (n > kMaxSupport) flag_error(st, kFlagRange, g);
    }
    return;
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const int nn = min(n, kMaxSupport);
  int32_t* out = gp_nbr + gp_ptr[g];
  for (int i = lane; i < nn; i += 64) {
    const int32_t v = hits[w][i];
    int r = 0;
    for (int k = 0; k < nn; ++k) r += hits[w][k] < v;
    out[r] = v;
  }
}

// ---- 3. inverse lists -------------------------------------------------------
__global__ void k_inv_count(int64_t sum_n, const int32_t* gp_nbr, int32_t* cnt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < sum_n) atomicAdd(&cnt[gp_nbr[e]], 1);
}

__global__ void k_inv_fill(int64_t G, const int64_t* gp_ptr, const int32_t* gp_nbr, const int64_t* inv_ptr,
                           int32_t* cursor, uint64_t* inv_key) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  const int64_t b = gp_ptr[g], n = gp_ptr[g + 1] - b;
  for (int a = 0; a < n; ++a) {
    const int32_t I = gp_nbr[b + a];
    const int slot = atomicAdd(&cursor[I], 1);
    inv_key[inv_ptr[I] + slot] = ((uint64_t)g << 8) | (uint64_t)a;
  }
}

// Bitonic sort of each node's inverse list in LDS (P = power of two >= longest).
__global__ void __launch_bounds__(1024) k_inv_sort(const int64_t* inv_ptr, uint64_t* inv_key, int P) {
  extern __shared__ uint64_t keys[];
  const int64_t I = blockIdx.x;
  const int64_t b = inv_ptr[I];
  const int n = (int)(inv_ptr[I + 1] - b);
  for (int i = threadIdx.x; i < P; i += blockDim.x) keys[i] = i < n ? inv_key[b + i] : ~0ull;
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += blockDim.x) {
        const int l = i ^ j;
        if (l > i) {
          const uint64_t x = keys[i], y = keys[l];
          const bool up = (i & k) == 0;
          if ((x > y) == up) { keys[i] = y; keys[l] = x; }
        }
      }
      __syncthreads();
    }
  for (int i = threadIdx.x; i < n; i += blockDim.x) inv_key[b + i] = keys[i];
}

// ---- 4. node-block rows -------------------------------------------------------
__global__ void __launch_bounds__(256) k_window(int64_t N, const int64_t* inv_ptr, const uint64_t* inv_key,
                                                const int64_t* gp_ptr, const int32_t* gp_nbr, int32_t* win_lo,
                                                int32_t* win_len) {
  const int64_t I = blockIdx.x;
  int lo = INT_MAX, hi = -1;
  for (int64_t e = inv_ptr[I] + threadIdx.x; e < inv_ptr[I + 1]; e += blockDim.x) {
    const int64_t g = (int64_t)(inv_key[e] >> 8);
    lo = min(lo, gp_nbr[gp_ptr[g]]);
    hi = max(hi, gp_nbr[gp_ptr[g + 1] - 1]);
  }
  __shared__ int rlo[256], rhi[256];
  rlo[threadIdx.x] = lo;
  rhi[threadIdx.x] = hi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      rlo[threadIdx.x] = min(rlo[threadIdx.x], rlo[threadIdx.x + w]);
      rhi[threadIdx.x] = max(rhi[threadIdx.x], rhi[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    win_lo[I] = rlo[0];
    win_len[I] = rhi[0] >= rlo[0] ? rhi[0] - rlo[0] + 1 : 0;
  }
}

// Union of the supports of every Gauss point whose support holds node I, as a
// bitmap over I's node-id window: the words go to I's rank-bitmap slots (bits
// only; the prefix counts follow in k_blocks_fill) and the set-bit count to
// blk_cnt[I].
__global__ void __launch_bounds__(256) k_blocks_union(const int64_t* inv_ptr, const uint64_t* inv_key,
                                                      const int64_t* gp_ptr, const int32_t* gp_nbr,
                                                      const int32_t* win_lo, const int32_t* win_len,
                                                      int32_t* blk_cnt, const int64_t* rbm_off, uint2* rbm) {
  extern __shared__ unsigned bm[];
  const int64_t I = blockIdx.x;
  const int lo = win_lo[I];
  const int nw = (win_len[I] + 31) >> 5;
  for (int i = threadIdx.x; i < nw; i += blockDim.x) bm[i] = 0u;
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int64_t e = inv_ptr[I] + w; e < inv_ptr[I + 1]; e += 4) {
    const int64_t g = (int64_t)(inv_key[e] >> 8);
    const int64_t b = gp_ptr[g], n = gp_ptr[g + 1] - b;
    for (int64_t a = lane; a < n; a += 64) {
      const int r = gp_nbr[b + a] - lo;
      atomicOr(&bm[r >> 5], 1u << (r & 31));
    }
  }
  __syncthreads();
  int cnt = 0;
  const int64_t w_beg = rbm_off[I];
  for (int i = threadIdx.x; i < nw; i += blockDim.x) {
    rbm[w_beg + i] = make_uint2(bm[i], 0u);
    cnt += __popc(bm[i]);
  }
  __shared__ int part[256];
  part[threadIdx.x] = cnt;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) blk_cnt[I] = part[0];
}

// Expand row I's bitmap into its sorted columns and set each word's prefix
// count (position of J in row I = prefix + popc(bits below J)); upper[I] gets
// the number of columns J >= I.
__global__ void __launch_bounds__(256) k_blocks_fill(const int32_t* win_lo, const int64_t* blk_ptr, int32_t* blk_col,
                                                     int32_t* blk_row, const int64_t* rbm_off, uint2* rbm,
                                                     int32_t* upper) {
  const int64_t I = blockIdx.x;
  const int lo = win_lo[I];
  const int64_t w_beg = rbm_off[I];
  const int nw = (int)(rbm_off[I + 1] - w_beg);
  // each thread owns a contiguous run of words
  const int per = (nw + blockDim.x - 1) / blockDim.x;
  const int w0 = threadIdx.x * per, w1 = min(w0 + per, nw);
  int cnt = 0;
  for (int i = w0; i < w1; ++i) cnt += __popc(rbm[w_beg + i].x);
  __shared__ int part[256];
  part[threadIdx.x] = cnt;
  __syncthreads();
  int pos = 0;
  for (int t = 0; t < (int)threadIdx.x; ++t) pos += part[t];
  const int64_t out = blk_ptr[I] + pos;
  const int rI = (int)I - lo, wI = rI >> 5;
  if (nw == 0 && threadIdx.x == 0) upper[I] = 0;  // empty row
  int k = 0;
  for (int i = w0; i < w1; ++i) {
    unsigned v = rbm[w_beg + i].x;
    rbm[w_beg + i].y = (unsigned)(pos + k);
    if (i == wI) upper[I] = (int32_t)(blk_ptr[I + 1] - blk_ptr[I]) - (pos + k + __popc(v & ((1u << (rI & 31)) - 1u)));
    while (v) {
      const int bit = __ffs(v) - 1;
      v &= v - 1;
      blk_col[out + k] = lo + (i << 5) + bit;
      blk_row[out + k] = (int32_t)I;
      ++k;
    }
  }
}

// ---- 5. scalar CSR ------------------------------------------------------------
__global__ void k_expand_rows(int64_t N, const int64_t* blk_ptr, int64_t* row_ptr) {
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= N) return;
  const int64_t b = blk_ptr[I], L = blk_ptr[I + 1] - b;
  for (int al = 0; al < 3; ++al) row_ptr[3 * I + al] = 9 * b + 3 * al * L;
  if (I == N - 1) row_ptr[3 * N] = 9 * blk_ptr[N];
}

__global__ void k_expand_cols(int64_t nblk, const int64_t* blk_ptr, const int32_t* blk_row,
                              const int32_t* blk_col, int32_t* col_idx) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nblk) return;
  const int32_t I = blk_row[e];
  const int64_t b = blk_ptr[I], L = blk_ptr[I + 1] - b, pos = e - b;
  const int32_t J = blk_col[e];
  for (int al = 0; al < 3; ++al)
    for (int be = 0; be < 3; ++be) col_idx[9 * b + 3 * al * L + 3 * pos + be] = 3 * J + be;
}

inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Device temporaries of one pattern build, freed on every exit path (the
// stream is synchronised first, so no kernel still uses them).
class Scratch {
 public:
  explicit Scratch(hipStream_t s) : s_(s) {}
  ~Scratch() {
    if (ptrs_.empty()) return;
    (void)hipStreamSynchronize(s_);
    for (void* q : ptrs_) (void)hipFree(q);
  }
  template <class T>
  rpim_status alloc(T** out, int64_t count) {
    *out = nullptr;
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, sizeof(T) * (size_t)std::max<int64_t>(count, 1));
    if (e != hipSuccess) return hip_ok(e);
    ptrs_.push_back(q);
    *out = static_cast<T*>(q);
    return RPIM_OK;
  }
  // hand a temporary over to the plan (not freed here)
  template <class T>
  void release(T* q) {
    for (size_t i = 0; i < ptrs_.size(); ++i)
      if (ptrs_[i] == (void*)q) {
        ptrs_.erase(ptrs_.begin() + (long)i);
        return;
      }
  }

 private:
  hipStream_t s_;
  std::vector<void*> ptrs_;
};

template <class T>
void dfree(T*& q) {
  if (q) (void)hipFree(q);
  q = nullptr;
}

}  // namespace

void free_pattern(rpim_plan* p) {
  dfree(p->gp_ptr); dfree(p->gp_nbr); dfree(p->inv_ptr); dfree(p->inv_key); dfree(p->blk_ptr);
  dfree(p->blk_col); dfree(p->blk_row); dfree(p->gp_order); dfree(p->lu_off);
  dfree(p->cell_ptr); dfree(p->cell_gp); dfree(p->row_lo); dfree(p->rbm_off); dfree(p->rbm);
  p->built = false;
  p->buckets.clear();
}

rpim_status build_pattern_device(rpim_plan* p, const double* X, hipStream_t s) {
  const int M = p->n_models;
  const int64_t N = p->N, G = p->G;
  RPIM_HIP(hipStreamSynchronize(s));
  free_pattern(p);  // arrays of an earlier (possibly failed) build
  Scratch tmp(s);
  rpim_status st = RPIM_OK;
#define RPIM_TRY(x)                   \
  do {                                \
    if ((st = (x)) != RPIM_OK) return st; \
  } while (0)
  // bounding boxes -> bin grids (host)
  double* d_bb = nullptr;
  RPIM_TRY(tmp.alloc(&d_bb, 6 * M));
  hipLaunchKernelGGL(k_bbox, dim3(M), dim3(256), 0, s, X, (const int64_t*)p->d_node_off, d_bb);
  RPIM_HIP(hipGetLastError());
  std::vector<double> bb(6 * M);
  RPIM_HIP(hipMemcpyAsync(bb.data(), d_bb, sizeof(double) * 6 * M, hipMemcpyDeviceToHost, s));
  RPIM_HIP(hipStreamSynchronize(s));
  std::vector<BinGrid> grids(M);
  int64_t nbins = 0;
  for (int m = 0; m < M; ++m) {
    for (int k = 0; k < 6; ++k)
      if (!std::isfinite(bb[6 * m + k])) return RPIM_E_ARG;
    BinGrid& gr = grids[m];
    const double r = p->radius[m];
    gr.h = r * 1.001;
    gr.r2 = r * r;
    gr.ox = bb[6 * m];
    gr.oy = bb[6 * m + 1];
    gr.oz = bb[6 * m + 2];
    const double ext[3] = {bb[6 * m + 3] - gr.ox, bb[6 * m + 4] - gr.oy, bb[6 * m + 5] - gr.oz};
    int64_t dims[3];
    for (int k = 0; k < 3; ++k) dims[k] = (int64_t)std::floor(ext[k] / gr.h) + 1;
    if (dims[0] * dims[1] * dims[2] > (int64_t)1 << 28) return RPIM_E_RANGE;
    gr.nx = (int)dims[0];
    gr.ny = (int)dims[1];
    gr.nz = (int)dims[2];
    gr.pad = 0;
    gr.bin0 = nbins;
    nbins += dims[0] * dims[1] * dims[2];
  }
  if (nbins >= INT32_MAX) return RPIM_E_RANGE;
  BinGrid* d_grids = nullptr;
  int32_t *node_bin = nullptr, *bin_cnt = nullptr, *bin_nodes = nullptr, *counts = nullptr;
  int64_t* bin_start = nullptr;
  double* bxyz = nullptr;
  RPIM_TRY(tmp.alloc(&d_grids, M));
  RPIM_HIP(hipMemcpyAsync(d_grids, grids.data(), sizeof(BinGrid) * M, hipMemcpyHostToDevice, s));
  RPIM_TRY(tmp.alloc(&node_bin, N));
  RPIM_TRY(tmp.alloc(&bin_cnt, nbins));
  RPIM_TRY(tmp.alloc(&bin_start, nbins + 1));
  RPIM_TRY(tmp.alloc(&bin_nodes, N));
  RPIM_TRY(tmp.alloc(&bxyz, 3 * N));
  RPIM_HIP(hipMemsetAsync(bin_cnt, 0, sizeof(int32_t) * nbins, s));
  hipLaunchKernelGGL(k_bin_count, dim3(nblocks(N, 256)), dim3(256), 0, s, X, N, (const int64_t*)p->d_node_off,
                     M, (const BinGrid*)d_grids, node_bin, bin_cnt);
  RPIM_HIP(hipGetLastError());
  RPIM_TRY(exclusive_scan(bin_cnt, nbins, bin_start, s));
  RPIM_HIP(hipMemsetAsync(bin_cnt, 0, sizeof(int32_t) * nbins, s));
  hipLaunchKernelGGL(k_bin_fill, dim3(nblocks(N, 256)), dim3(256), 0, s, N, (const int32_t*)node_bin,
                     (const int64_t*)bin_start, bin_cnt, bin_nodes);
  hipLaunchKernelGGL(k_bin_sort, dim3(nblocks(nbins, 256)), dim3(256), 0, s, nbins, (const int64_t*)bin_start,
                     bin_nodes, X, bxyz);
  RPIM_HIP(hipGetLastError());

  // supports: count, scan, fill
  RPIM_TRY(tmp.alloc(&counts, std::max<int64_t>(G, N)));
  RPIM_HIP(hipMalloc((void**)&p->gp_ptr, sizeof(int64_t) * (G + 1)));
  hipLaunchKernelGGL(k_support<false>, dim3(nblocks(G, 4)), dim3(256), 0, s, G, (const int64_t*)p->d_gp_off, M,
                     (const BinGrid*)d_grids, (const int64_t*)bin_start, (const int32_t*)bin_nodes,
                     (const double*)bxyz, (const double*)p->gp_xyz, counts, (const int64_t*)nullptr,
                     (int32_t*)nullptr, p->status);
  RPIM_HIP(hipGetLastError());
  DevStatus hst;
  RPIM_HIP(hipMemcpyAsync(&hst, p->status, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
  RPIM_HIP(hipStreamSynchronize(s));
  if (hst.flags & kFlagRange) return RPIM_E_RANGE;
  if (hst.flags & kFlagSupport) return RPIM_E_SUPPORT;
  RPIM_TRY(exclusive_scan(counts, G, p->gp_ptr, s));
  std::vector<int64_t> gp_ptr_h(G + 1);
  RPIM_HIP(hipMemcpyAsync(gp_ptr_h.data(), p->gp_ptr, sizeof(int64_t) * (G + 1), hipMemcpyDeviceToHost, s));
  RPIM_HIP(hipStreamSynchronize(s));
  p->sum_n = gp_ptr_h[G];
  if (p->sum_n >= INT32_MAX) return RPIM_E_RANGE;
  RPIM_HIP(hipMalloc((void**)&p->gp_nbr, sizeof(int32_t) * p->sum_n));
  hipLaunchKernelGGL(k_support<true>, dim3(nblocks(G, 4)), dim3(256), 0, s, G, (const int64_t*)p->d_gp_off, M,
                     (const BinGrid*)d_grids, (const int64_t*)bin_start, (const int32_t*)bin_nodes,
                     (const double*)bxyz, (const double*)p->gp_xyz, counts, (const int64_t*)p->gp_ptr,
                     p->gp_nbr, p->status);
  RPIM_HIP(hipGetLastError());

  // inverse lists
  int32_t *cursor = nullptr, *inv_cnt = nullptr;
  RPIM_TRY(tmp.alloc(&inv_cnt, N));
  RPIM_TRY(tmp.alloc(&cursor, N));
  RPIM_HIP(hipMemsetAsync(inv_cnt, 0, sizeof(int32_t) * N, s));
  hipLaunchKernelGGL(k_inv_count, dim3(nblocks(p->sum_n, 256)), dim3(256), 0, s, p->sum_n,
                     (const int32_t*)p->gp_nbr, inv_cnt);
  RPIM_HIP(hipMalloc((void**)&p->inv_ptr, sizeof(int64_t) * (N + 1)));
  RPIM_TRY(exclusive_scan(inv_cnt, N, p->inv_ptr, s));
  std::vector<int32_t> cnt_h(N);
  RPIM_HIP(hipMemcpyAsync(cnt_h.data(), inv_cnt, sizeof(int32_t) * N, hipMemcpyDeviceToHost, s));
  RPIM_HIP(hipMemsetAsync(cursor, 0, sizeof(int32_t) * N, s));
  RPIM_HIP(hipMalloc((void**)&p->inv_key, sizeof(uint64_t) * p->sum_n));
  hipLaunchKernelGGL(k_inv_fill, dim3(nblocks(G, 256)), dim3(256), 0, s, G, (const int64_t*)p->gp_ptr,
                     (const int32_t*)p->gp_nbr, (const int64_t*)p->inv_ptr, cursor, p->inv_key);
  RPIM_HIP(hipGetLastError());
  RPIM_HIP(hipStreamSynchronize(s));
  int64_t max_inv = 0;
  for (int64_t i = 0; i < N; ++i) max_inv = std::max<int64_t>(max_inv, cnt_h[i]);
  if (max_inv > kMaxInverse) return RPIM_E_RANGE;
  p->max_inverse = max_inv;
  int P = 2;
  while (P < max_inv) P <<= 1;
  hipLaunchKernelGGL(k_inv_sort, dim3((unsigned)N), dim3(1024), sizeof(uint64_t) * P, s,
                     (const int64_t*)p->inv_ptr, p->inv_key, P);
  RPIM_HIP(hipGetLastError());

  // node-block rows
  int32_t *win_lo = nullptr, *win_len = nullptr, *blk_cnt = nullptr;
  RPIM_HIP(hipMalloc((void**)&win_lo, sizeof(int32_t) * N));
  p->row_lo = win_lo;  // plan-owned from here (the window start of each row)
  RPIM_TRY(tmp.alloc(&win_len, N));
  hipLaunchKernelGGL(k_window, dim3((unsigned)N), dim3(256), 0, s, N, (const int64_t*)p->inv_ptr,
                     (const uint64_t*)p->inv_key, (const int64_t*)p->gp_ptr, (const int32_t*)p->gp_nbr, win_lo,
                     win_len);
  RPIM_HIP(hipGetLastError());
  RPIM_HIP(hipMemcpyAsync(cnt_h.data(), win_len, sizeof(int32_t) * N, hipMemcpyDeviceToHost, s));
  RPIM_HIP(hipStreamSynchronize(s));
  int64_t max_win = 0;
  for (int64_t i = 0; i < N; ++i) max_win = std::max<int64_t>(max_win, cnt_h[i]);
  if (max_win > kMaxWindow) return RPIM_E_RANGE;
  const int words = (int)((max_win + 31) / 32);
  blk_cnt = counts;  // reuse (size >= N)
  // per-row rank bitmaps: word offsets from the window lengths
  {
    std::vector<int64_t> off(N + 1, 0);
    int32_t mw = 0;
    for (int64_t i = 0; i < N; ++i) {
      const int32_t nw = (cnt_h[i] + 31) / 32;
      off[i + 1] = off[i] + nw;
      mw = std::max(mw, nw);
    }
    p->rbm_words = off[N];
    p->max_row_words = mw;
    RPIM_HIP(hipMalloc((void**)&p->rbm_off, sizeof(int64_t) * (N + 1)));
    RPIM_HIP(hipMalloc((void**)&p->rbm, sizeof(uint2) * std::max<int64_t>(off[N], 1)));
    RPIM_HIP(hipMemcpyAsync(p->rbm_off, off.data(), sizeof(int64_t) * (N + 1), hipMemcpyHostToDevice, s));
  }
  hipLaunchKernelGGL(k_blocks_union, dim3((unsigned)N), dim3(256), sizeof(unsigned) * std::max(words, 1), s,
                     (const int64_t*)p->inv_ptr, (const uint64_t*)p->inv_key, (const int64_t*)p->gp_ptr,
                     (const int32_t*)p->gp_nbr, (const int32_t*)win_lo, (const int32_t*)win_len, blk_cnt,
                     (const int64_t*)p->rbm_off, p->rbm);
  RPIM_HIP(hipGetLastError());
  RPIM_HIP(hipMalloc((void**)&p->blk_ptr, sizeof(int64_t) * (N + 1)));
  RPIM_TRY(exclusive_scan(blk_cnt, N, p->blk_ptr, s));
  RPIM_HIP(hipMemcpyAsync(cnt_h.data(), blk_cnt, sizeof(int32_t) * N, hipMemcpyDeviceToHost, s));
  int64_t nblk = 0;
  RPIM_HIP(hipMemcpyAsync(&nblk, p->blk_ptr + N, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  RPIM_HIP(hipStreamSynchronize(s));
  p->nblk = nblk;
  p->nnz = 9 * nblk;
  p->max_row_blocks = 0;
  for (int64_t i = 0; i < N; ++i) p->max_row_blocks = std::max<int64_t>(p->max_row_blocks, cnt_h[i]);
  RPIM_HIP(hipMalloc((void**)&p->blk_col, sizeof(int32_t) * nblk));
  RPIM_HIP(hipMalloc((void**)&p->blk_row, sizeof(int32_t) * nblk));
  int32_t* upper = inv_cnt;  // reuse (size N): columns J >= I of each row
  hipLaunchKernelGGL(k_blocks_fill, dim3((unsigned)N), dim3(256), 0, s, (const int32_t*)win_lo,
                     (const int64_t*)p->blk_ptr, p->blk_col, p->blk_row, (const int64_t*)p->rbm_off, p->rbm, upper);
  RPIM_HIP(hipGetLastError());
  RPIM_HIP(hipMemcpyAsync(cnt_h.data(), upper, sizeof(int32_t) * N, hipMemcpyDeviceToHost, s));
  RPIM_HIP(hipStreamSynchronize(s));
  p->max_row_upper = 0;
  for (int64_t i = 0; i < N; ++i) p->max_row_upper = std::max<int64_t>(p->max_row_upper, cnt_h[i]);

  // buckets by padded moment-matrix size, and LU offsets (host, from gp_ptr)
  p->min_n = INT32_MAX;
  p->max_n = 0;
  const int nb = (kMaxSupport + 4) / kBucketStep + 1;
  std::vector<int64_t> bcount(nb, 0);
  std::vector<int64_t> lu_off_h(G + 1, 0);
  for (int64_t g = 0; g < G; ++g) {
    const int n = (int)(gp_ptr_h[g + 1] - gp_ptr_h[g]);
    p->min_n = std::min(p->min_n, n);
    p->max_n = std::max(p->max_n, n);
    bcount[(n + 4 + kBucketStep - 1) / kBucketStep]++;
    lu_off_h[g + 1] = lu_off_h[g] + (int64_t)(n + 4) * (n + 4);  // packed multipliers and U
  }
  p->lu_doubles = lu_off_h[G];
  p->buckets.clear();
  std::vector<int64_t> bstart(nb, 0);
  int64_t acc = 0;
  for (int b = 0; b < nb; ++b) {
    bstart[b] = acc;
    if (bcount[b]) p->buckets.push_back(Bucket{b * kBucketStep, acc, bcount[b]});
    acc += bcount[b];
  }
  std::vector<int32_t> order(G);
  for (int64_t g = 0; g < G; ++g) {
    const int n = (int)(gp_ptr_h[g + 1] - gp_ptr_h[g]);
    order[bstart[(n + 4 + kBucketStep - 1) / kBucketStep]++] = (int32_t)g;
  }
  RPIM_HIP(hipMalloc((void**)&p->gp_order, sizeof(int32_t) * std::max<int64_t>(G, 1)));
  RPIM_HIP(hipMemcpyAsync(p->gp_order, order.data(), sizeof(int32_t) * G, hipMemcpyHostToDevice, s));
  // cell -> Gauss point lists (ascending g) for the deterministic dE reduction
  {
    std::vector<int32_t> cell_h(G);
    RPIM_HIP(hipMemcpyAsync(cell_h.data(), p->gp_cell, sizeof(int32_t) * G, hipMemcpyDeviceToHost, s));
    RPIM_HIP(hipStreamSynchronize(s));
    std::vector<int64_t> cptr(p->C + 1, 0);
    for (int64_t g = 0; g < G; ++g) {
      if (cell_h[g] < 0 || cell_h[g] >= p->C) return RPIM_E_ARG;
      cptr[cell_h[g] + 1]++;
    }
    for (int64_t c = 0; c < p->C; ++c) cptr[c + 1] += cptr[c];
    std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
    std::vector<int32_t> cgp(std::max<int64_t>(G, 1));
    for (int64_t g = 0; g < G; ++g) cgp[fill[cell_h[g]]++] = (int32_t)g;
    RPIM_HIP(hipMalloc((void**)&p->cell_ptr, sizeof(int64_t) * (p->C + 1)));
    RPIM_HIP(hipMalloc((void**)&p->cell_gp, sizeof(int32_t) * std::max<int64_t>(G, 1)));
    RPIM_HIP(hipMemcpyAsync(p->cell_ptr, cptr.data(), sizeof(int64_t) * (p->C + 1), hipMemcpyHostToDevice, s));
    RPIM_HIP(hipMemcpyAsync(p->cell_gp, cgp.data(), sizeof(int32_t) * G, hipMemcpyHostToDevice, s));
    RPIM_HIP(hipStreamSynchronize(s));
  }
  RPIM_HIP(hipMalloc((void**)&p->lu_off, sizeof(int64_t) * (G + 1)));
  RPIM_HIP(hipMemcpyAsync(p->lu_off, lu_off_h.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s));
  RPIM_HIP(hipStreamSynchronize(s));
#undef RPIM_TRY
  p->built = true;
  return RPIM_OK;
}

rpim_status expand_pattern(const rpim_plan* p, int64_t* row_ptr, int32_t* col_idx, hipStream_t s) {
  hipLaunchKernelGGL(k_expand_rows, dim3(nblocks(p->N, 256)), dim3(256), 0, s, p->N, (const int64_t*)p->blk_ptr,
                     row_ptr);
  hipLaunchKernelGGL(k_expand_cols, dim3(nblocks(p->nblk, 256)), dim3(256), 0, s, p->nblk,
                     (const int64_t*)p->blk_ptr, (const int32_t*)p->blk_row, (const int32_t*)p->blk_col, col_idx);
  RPIM_HIP(hipGetLastError());
  return RPIM_OK;
}

}  // namespace rpim
