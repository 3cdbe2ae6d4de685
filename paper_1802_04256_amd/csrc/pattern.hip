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
  int bad = 0;  // a non-finite coordinate makes the box NaN, which the host rejects
  for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x)
    for (int k = 0; k < 3; ++k) {
      double v = X[3 * i + k];
      bad |= !isfinite(v);
      lo[k] = fmin(lo[k], v);
      hi[k] = fmax(hi[k], v);
    }
  bad = __syncthreads_or(bad);
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
  if (threadIdx.x < 6) out[6 * m + threadIdx.x] = bad ? NAN : red[threadIdx.x][0];
}

// Bin of a point, clamped to the grid in floating point before the integer
// conversion (a point outside the grid, or NaN, lands in a valid bin and then
// simply finds no node within the radius).
__device__ __forceinline__ int bin_index(double f, int n) {
  return f >= 0.0 ? (f < (double)n ? (int)f : n - 1) : 0;
}

__device__ __forceinline__ void bin_coords(const BinGrid& gr, double x, double y, double z, int* ix, int* iy,
                                           int* iz) {
  *ix = bin_index(floor((x - gr.ox) / gr.h), gr.nx);
  *iy = bin_index(floor((y - gr.oy) / gr.h), gr.ny);
  *iz = bin_index(floor((z - gr.oz) / gr.h), gr.nz);
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

// Bitonic sort of each node's inverse list in LDS, at the list's own power of
// two (the LDS holds P >= the longest list).
__global__ void __launch_bounds__(1024) k_inv_sort(const int64_t* inv_ptr, uint64_t* inv_key, int P) {
  extern __shared__ uint64_t keys[];
  const int64_t I = blockIdx.x;
  const int64_t b = inv_ptr[I];
  const int n = (int)(inv_ptr[I + 1] - b);
  int Q = 2;
  while (Q < n) Q <<= 1;  // <= P
  for (int i = threadIdx.x; i < Q; i += blockDim.x) keys[i] = i < n ? inv_key[b + i] : ~0ull;
  __syncthreads();
  for (int k = 2; k <= Q; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < Q; i += blockDim.x) {
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
  // Each wave takes every fourth point of I's list.  The support ranges of
  // 64 of its points are loaded at once, one point per lane (the key ->
  // point -> range loads run once per 64 points), and taken by readlane;
  // each point's ids are loaded kAhead points before they are entered.
  constexpr int kAhead = 8;  // divides 64
  const int64_t e0 = inv_ptr[I] + w, e1 = inv_ptr[I + 1];
  const int64_t cnt_w = e0 < e1 ? (e1 - e0 + 3) / 4 : 0;  // this wave's points: e0 + 4 k
  struct Ids {
    int32_t id0, id1;  // support entries lane and lane + 64 (clamped to the last)
  };
  auto load_batch = [&](int64_t k0, int64_t& b, int& n) {  // lane l: point k0 + l (past the end: the last)
    const int64_t k = k0 + lane < cnt_w ? k0 + lane : cnt_w - 1;
    const int64_t g = (int64_t)(inv_key[e0 + 4 * k] >> 8);
    b = gp_ptr[g];
    n = (int)(gp_ptr[g + 1] - b);
  };
  auto ids = [&](int64_t b, int n) {
    Ids r;
    r.id0 = gp_nbr[b + (lane < n ? lane : n - 1)];
    r.id1 = gp_nbr[b + (lane + 64 < n ? lane + 64 : n - 1)];
    return r;
  };
  if (cnt_w > 0) {
    int64_t bc = 0, bx = 0;
    int nc = 0, nx = 0;
    load_batch(0, bc, nc);
    bx = bc;
    nx = nc;
    if (cnt_w > 64) load_batch(64, bx, nx);
    Ids ring[kAhead];
#pragma unroll
    for (int u = 0; u < kAhead; ++u) {
      const int j = u < cnt_w ? u : (int)cnt_w - 1;
      ring[u] = ids(readlane_i64(bc, j), __builtin_amdgcn_readlane(nc, j));
    }
    for (int64_t k0 = 0; k0 < cnt_w; k0 += kAhead) {
      if (k0 > 0 && (k0 & 63) == 0) {  // next batch (uniform)
        bc = bx;
        nc = nx;
        if (k0 + 64 < cnt_w) load_batch(k0 + 64, bx, nx);
      }
#pragma unroll
      for (int u = 0; u < kAhead; ++u) {
        const int64_t k = k0 + u;
        if (k < cnt_w) {  // uniform
          const int j = (int)(k & 63);
          const int64_t b = readlane_i64(bc, j);
          const int n = __builtin_amdgcn_readlane(nc, j);
          const Ids r = ring[u];
          if (lane < n) {
            const int rr = r.id0 - lo;
            atomicOr(&bm[rr >> 5], 1u << (rr & 31));
          }
          if (lane + 64 < n) {
            const int rr = r.id1 - lo;
            atomicOr(&bm[rr >> 5], 1u << (rr & 31));
          }
          for (int64_t a = lane + 128; a < n; a += 64) {  // supports above 128 nodes
            const int rr = gp_nbr[b + a] - lo;
            atomicOr(&bm[rr >> 5], 1u << (rr & 31));
          }
          // refill with point k + kAhead (past the end: the last point again)
          const int64_t kp = k + kAhead < cnt_w ? k + kAhead : cnt_w - 1;
          const int jp = (int)(kp & 63);
          if ((kp >> 6) == (k0 >> 6))
            ring[u] = ids(readlane_i64(bc, jp), __builtin_amdgcn_readlane(nc, jp));
          else
            ring[u] = ids(readlane_i64(bx, jp), __builtin_amdgcn_readlane(nx, jp));
        }
      }
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

// ---- buckets and packed-factor offsets (every rebuild) ------------------------
// Bucket of each Gauss point (N = n + 4 rounded up to kBucketStep), its packed
// factor size N^2, the bucket sizes and the smallest and largest support
// (integer atomics: the totals do not depend on the order).
// Counted in LDS per block first, then one global atomic per bucket and block.
__global__ void __launch_bounds__(256) k_point_sizes(int64_t G, const int64_t* gp_ptr, int32_t* bkt, int64_t* nsq,
                                                     unsigned long long* bcount, int* nrange) {
  __shared__ unsigned c[kMaxBuckets];
  __shared__ int lo, hi;
  for (int i = threadIdx.x; i < kMaxBuckets; i += blockDim.x) c[i] = 0;
  if (threadIdx.x == 0) {
    lo = INT_MAX;
    hi = 0;
  }
  __syncthreads();
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < G) {
    const int n = (int)(gp_ptr[g + 1] - gp_ptr[g]);
    const int b = (n + 4 + kBucketStep - 1) / kBucketStep;
    bkt[g] = b;
    nsq[g] = (int64_t)(n + 4) * (n + 4);
    atomicAdd(&c[b], 1u);
    atomicMin(&lo, n);
    atomicMax(&hi, n);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kMaxBuckets; i += blockDim.x)
    if (c[i]) atomicAdd(&bcount[i], (unsigned long long)c[i]);
  if (threadIdx.x == 0 && hi > 0) {
    atomicMin(&nrange[0], lo);
    atomicMax(&nrange[1], hi);
  }
}

constexpr int kOrderTile = 1024;  // Gauss points per tile of the bucket grouping

// Points of tile t in each bucket, bucket-major: cnt[b * tiles + t].
__global__ void __launch_bounds__(256) k_order_count(int64_t G, const int32_t* bkt, int64_t tiles, int32_t* cnt) {
  __shared__ int c[kMaxBuckets];
  for (int i = threadIdx.x; i < kMaxBuckets; i += blockDim.x) c[i] = 0;
  __syncthreads();
  const int64_t t0 = (int64_t)blockIdx.x * kOrderTile;
  for (int i = threadIdx.x; i < kOrderTile; i += blockDim.x)
    if (t0 + i < G) atomicAdd(&c[bkt[t0 + i]], 1);
  __syncthreads();
  for (int b = threadIdx.x; b < kMaxBuckets; b += blockDim.x) cnt[(int64_t)b * tiles + blockIdx.x] = c[b];
}

// One wave per tile: the tile's points, in ascending g, go to their bucket's
// range from the tile's offset on, so each bucket lists its points in
// ascending g.  Lane b < kMaxBuckets carries bucket b's next free slot.
__global__ void __launch_bounds__(64) k_order_fill(int64_t G, const int32_t* bkt, int64_t tiles, const int64_t* off,
                                                   int32_t* order) {
  static_assert(kMaxBuckets <= 64, "one lane per bucket");
  const int lane = threadIdx.x;
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  long long mine = lane < kMaxBuckets ? off[(int64_t)lane * tiles + blockIdx.x] : 0;
  const int64_t t0 = (int64_t)blockIdx.x * kOrderTile;
  for (int r = 0; r < kOrderTile; r += 64) {
    const int64_t g = t0 + r + lane;
    const int b = g < G ? bkt[g] : -1;
    for (int bb = 0; bb < kMaxBuckets; ++bb) {
      const unsigned long long m = __ballot(b == bb);
      if (m == 0) continue;  // uniform
      const long long base = __shfl(mine, bb);
      if (b == bb) order[base + __popcll(m & below)] = (int32_t)g;
      if (lane == bb) mine += __popcll(m);
    }
  }
}

inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

inline size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// The temporaries of one pattern build, carved from one plan-owned buffer that
// every rebuild reuses (no allocation or free on the rebuild path once sized).
class Arena {
 public:
  Arena(char* base, size_t cap) : base_(base), cap_(cap) {}
  template <class T>
  T* take(int64_t count) {
    const size_t b = bytes<T>(count);
    if (used_ + b > cap_) return nullptr;
    T* q = reinterpret_cast<T*>(base_ + used_);
    used_ += b;
    return q;
  }
  template <class T>
  static size_t bytes(int64_t count) {
    return round256(sizeof(T) * (size_t)std::max<int64_t>(count, 1));
  }

 private:
  char* base_;
  size_t cap_;
  size_t used_ = 0;
};

rpim_status ensure_bytes(void** q, size_t* cap, size_t need) {
  if (*q && *cap >= need) return RPIM_OK;
  if (*q) (void)hipFree(*q);
  *q = nullptr;
  *cap = 0;
  RPIM_HIP(hipMalloc(q, need));
  *cap = need;
  return RPIM_OK;
}

// Plan arrays whose size depends on the geometry: kept while large enough.
template <class T>
rpim_status reserve(T** q, int64_t* cap, int64_t count) {
  if (*q && *cap >= count) return RPIM_OK;
  if (*q) (void)hipFree(*q);
  *q = nullptr;
  *cap = 0;
  RPIM_HIP(hipMalloc((void**)q, sizeof(T) * (size_t)std::max<int64_t>(count, 1)));
  *cap = count;
  return RPIM_OK;
}

// Plan arrays of fixed size (nodes or Gauss points): allocated once.
template <class T>
rpim_status once(T** q, int64_t count) {
  if (*q) return RPIM_OK;
  RPIM_HIP(hipMalloc((void**)q, sizeof(T) * (size_t)std::max<int64_t>(count, 1)));
  return RPIM_OK;
}

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
  if (p->pat_scratch) (void)hipFree(p->pat_scratch);
  p->pat_scratch = nullptr;
  p->cap_pat_scratch = 0;
  p->cap_gp_nbr = p->cap_inv_key = p->cap_blk = p->cap_rbm = 0;
  p->built = false;
  p->buckets.clear();
}

rpim_status build_pattern_device(rpim_plan* p, const double* X, hipStream_t s) {
  const int M = p->n_models;
  const int64_t N = p->N, G = p->G;
  RPIM_HIP(hipStreamSynchronize(s));
  p->built = false;
  p->buckets.clear();
  rpim_status st = RPIM_OK;
#define RPIM_TRY(x)                   \
  do {                                \
    if ((st = (x)) != RPIM_OK) return st; \
  } while (0)
  // bounding boxes -> bin grids (host)
  RPIM_TRY(ensure_bytes(&p->pat_scratch, &p->cap_pat_scratch, Arena::bytes<double>(6 * M)));
  double* d_bb = Arena((char*)p->pat_scratch, p->cap_pat_scratch).take<double>(6 * M);
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
  // every temporary of this build in one buffer (the bounding boxes are consumed)
  const int64_t tiles = (G + kOrderTile - 1) / kOrderTile;
  const size_t need = Arena::bytes<BinGrid>(M) + Arena::bytes<int32_t>(N) + Arena::bytes<int32_t>(nbins) +
                      Arena::bytes<int64_t>(nbins + 1) + Arena::bytes<int32_t>(N) + Arena::bytes<double>(3 * N) +
                      Arena::bytes<int32_t>(std::max<int64_t>(G, N)) + 3 * Arena::bytes<int32_t>(N) +
                      Arena::bytes<int32_t>(G) + Arena::bytes<int64_t>(G) +
                      Arena::bytes<int32_t>(kMaxBuckets * tiles) + Arena::bytes<int64_t>(kMaxBuckets * tiles + 1) +
                      Arena::bytes<unsigned long long>(kMaxBuckets) + Arena::bytes<int>(2);
  RPIM_TRY(ensure_bytes(&p->pat_scratch, &p->cap_pat_scratch, need));
  Arena tmp((char*)p->pat_scratch, p->cap_pat_scratch);
  BinGrid* d_grids = tmp.take<BinGrid>(M);
  int32_t* node_bin = tmp.take<int32_t>(N);
  int32_t* bin_cnt = tmp.take<int32_t>(nbins);
  int64_t* bin_start = tmp.take<int64_t>(nbins + 1);
  int32_t* bin_nodes = tmp.take<int32_t>(N);
  double* bxyz = tmp.take<double>(3 * N);
  int32_t* counts = tmp.take<int32_t>(std::max<int64_t>(G, N));
  int32_t* inv_cnt = tmp.take<int32_t>(N);
  int32_t* cursor = tmp.take<int32_t>(N);
  int32_t* win_len = tmp.take<int32_t>(N);
  int32_t* bkt = tmp.take<int32_t>(G);
  int64_t* nsq = tmp.take<int64_t>(G);
  int32_t* ocnt = tmp.take<int32_t>(kMaxBuckets * tiles);
  int64_t* ooff = tmp.take<int64_t>(kMaxBuckets * tiles + 1);
  unsigned long long* bcount = tmp.take<unsigned long long>(kMaxBuckets);
  int* nrange = tmp.take<int>(2);
  if (!nrange) return RPIM_E_STATE;  // the sizes above and the carving disagree (never)
  RPIM_HIP(hipMemcpyAsync(d_grids, grids.data(), sizeof(BinGrid) * M, hipMemcpyHostToDevice, s));
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
  RPIM_TRY(once(&p->gp_ptr, G + 1));
  hipLaunchKernelGGL(k_support<false>, dim3(nblocks(G, 4)), dim3(256), 0, s, G, (const int64_t*)p->d_gp_off, M,
                     (const BinGrid*)d_grids, (const int64_t*)bin_start, (const int32_t*)bin_nodes,
                     (const double*)bxyz, (const double*)p->gp_xyz, counts, (const int64_t*)nullptr,
                     (int32_t*)nullptr, p->status);
  RPIM_HIP(hipGetLastError());
  RPIM_TRY(exclusive_scan(counts, G, p->gp_ptr, s));
  DevStatus hst;
  int64_t sum_n = 0;
  RPIM_HIP(hipMemcpyAsync(&hst, p->status, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
  RPIM_HIP(hipMemcpyAsync(&sum_n, p->gp_ptr + G, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  RPIM_HIP(hipStreamSynchronize(s));
  if (hst.flags & kFlagRange) return RPIM_E_RANGE;
  if (hst.flags & kFlagSupport) return RPIM_E_SUPPORT;
  p->sum_n = sum_n;
  if (p->sum_n >= INT32_MAX) return RPIM_E_RANGE;
  RPIM_TRY(reserve(&p->gp_nbr, &p->cap_gp_nbr, p->sum_n));
  hipLaunchKernelGGL(k_support<true>, dim3(nblocks(G, 4)), dim3(256), 0, s, G, (const int64_t*)p->d_gp_off, M,
                     (const BinGrid*)d_grids, (const int64_t*)bin_start, (const int32_t*)bin_nodes,
                     (const double*)bxyz, (const double*)p->gp_xyz, counts, (const int64_t*)p->gp_ptr,
                     p->gp_nbr, p->status);
  RPIM_HIP(hipGetLastError());

  // inverse lists
  RPIM_HIP(hipMemsetAsync(inv_cnt, 0, sizeof(int32_t) * N, s));
  hipLaunchKernelGGL(k_inv_count, dim3(nblocks(p->sum_n, 256)), dim3(256), 0, s, p->sum_n,
                     (const int32_t*)p->gp_nbr, inv_cnt);
  RPIM_TRY(once(&p->inv_ptr, N + 1));
  RPIM_TRY(exclusive_scan(inv_cnt, N, p->inv_ptr, s));
  std::vector<int32_t> cnt_h(N);
  RPIM_HIP(hipMemcpyAsync(cnt_h.data(), inv_cnt, sizeof(int32_t) * N, hipMemcpyDeviceToHost, s));
  RPIM_HIP(hipMemsetAsync(cursor, 0, sizeof(int32_t) * N, s));
  RPIM_TRY(reserve(&p->inv_key, &p->cap_inv_key, p->sum_n));
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
  RPIM_TRY(once(&p->row_lo, N));  // the window start of each row
  hipLaunchKernelGGL(k_window, dim3((unsigned)N), dim3(256), 0, s, N, (const int64_t*)p->inv_ptr,
                     (const uint64_t*)p->inv_key, (const int64_t*)p->gp_ptr, (const int32_t*)p->gp_nbr, p->row_lo,
                     win_len);
  RPIM_HIP(hipGetLastError());
  RPIM_HIP(hipMemcpyAsync(cnt_h.data(), win_len, sizeof(int32_t) * N, hipMemcpyDeviceToHost, s));
  RPIM_HIP(hipStreamSynchronize(s));
  int64_t max_win = 0;
  for (int64_t i = 0; i < N; ++i) max_win = std::max<int64_t>(max_win, cnt_h[i]);
  if (max_win > kMaxWindow) return RPIM_E_RANGE;
  const int words = (int)((max_win + 31) / 32);
  int32_t* blk_cnt = counts;  // reuse (size >= N)
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
    RPIM_TRY(once(&p->rbm_off, N + 1));
    RPIM_TRY(reserve(&p->rbm, &p->cap_rbm, std::max<int64_t>(off[N], 1)));
    RPIM_HIP(hipMemcpyAsync(p->rbm_off, off.data(), sizeof(int64_t) * (N + 1), hipMemcpyHostToDevice, s));
    RPIM_HIP(hipStreamSynchronize(s));  // off is a host temporary
  }
  hipLaunchKernelGGL(k_blocks_union, dim3((unsigned)N), dim3(256), sizeof(unsigned) * std::max(words, 1), s,
                     (const int64_t*)p->inv_ptr, (const uint64_t*)p->inv_key, (const int64_t*)p->gp_ptr,
                     (const int32_t*)p->gp_nbr, (const int32_t*)p->row_lo, (const int32_t*)win_len, blk_cnt,
                     (const int64_t*)p->rbm_off, p->rbm);
  RPIM_HIP(hipGetLastError());
  RPIM_TRY(once(&p->blk_ptr, N + 1));
  RPIM_TRY(exclusive_scan(blk_cnt, N, p->blk_ptr, s));
  RPIM_HIP(hipMemcpyAsync(cnt_h.data(), blk_cnt, sizeof(int32_t) * N, hipMemcpyDeviceToHost, s));
  int64_t nblk = 0;
  RPIM_HIP(hipMemcpyAsync(&nblk, p->blk_ptr + N, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  RPIM_HIP(hipStreamSynchronize(s));
  p->nblk = nblk;
  p->nnz = 9 * nblk;
  p->max_row_blocks = 0;
  for (int64_t i = 0; i < N; ++i) p->max_row_blocks = std::max<int64_t>(p->max_row_blocks, cnt_h[i]);
  if (p->cap_blk < nblk || !p->blk_col || !p->blk_row) {  // blk_col and blk_row share one capacity
    dfree(p->blk_col);
    dfree(p->blk_row);
    p->cap_blk = 0;
    RPIM_TRY(once(&p->blk_col, nblk));
    RPIM_TRY(once(&p->blk_row, nblk));
    p->cap_blk = nblk;
  }
  int32_t* upper = inv_cnt;  // reuse (size N): columns J >= I of each row
  hipLaunchKernelGGL(k_blocks_fill, dim3((unsigned)N), dim3(256), 0, s, (const int32_t*)p->row_lo,
                     (const int64_t*)p->blk_ptr, p->blk_col, p->blk_row, (const int64_t*)p->rbm_off, p->rbm, upper);
  RPIM_HIP(hipGetLastError());

  // buckets by padded moment-matrix size, packed-factor offsets and the
  // bucket-grouped point order, on the device
  static const int kNrangeInit[2] = {INT_MAX, 0};
  RPIM_HIP(hipMemsetAsync(bcount, 0, sizeof(unsigned long long) * kMaxBuckets, s));
  RPIM_HIP(hipMemcpyAsync(nrange, kNrangeInit, sizeof(kNrangeInit), hipMemcpyHostToDevice, s));
  RPIM_TRY(once(&p->lu_off, G + 1));
  RPIM_TRY(once(&p->gp_order, G));
  if (G > 0) {
    hipLaunchKernelGGL(k_point_sizes, dim3(nblocks(G, 256)), dim3(256), 0, s, G, (const int64_t*)p->gp_ptr, bkt, nsq,
                       bcount, nrange);
    RPIM_HIP(hipGetLastError());
    RPIM_TRY(exclusive_scan64(nsq, G, p->lu_off, s));
    hipLaunchKernelGGL(k_order_count, dim3((unsigned)tiles), dim3(256), 0, s, G, (const int32_t*)bkt, tiles, ocnt);
    RPIM_HIP(hipGetLastError());
    RPIM_TRY(exclusive_scan(ocnt, kMaxBuckets * tiles, ooff, s));
    hipLaunchKernelGGL(k_order_fill, dim3((unsigned)tiles), dim3(64), 0, s, G, (const int32_t*)bkt, tiles,
                       (const int64_t*)ooff, p->gp_order);
    RPIM_HIP(hipGetLastError());
  } else {
    RPIM_HIP(hipMemsetAsync(p->lu_off, 0, sizeof(int64_t), s));
  }
  // the host needs the bucket sizes (one launch per bucket) and the widest rows
  unsigned long long bc[kMaxBuckets];
  int nr[2];
  int64_t lu_total = 0;
  RPIM_HIP(hipMemcpyAsync(cnt_h.data(), upper, sizeof(int32_t) * N, hipMemcpyDeviceToHost, s));
  RPIM_HIP(hipMemcpyAsync(bc, bcount, sizeof(bc), hipMemcpyDeviceToHost, s));
  RPIM_HIP(hipMemcpyAsync(nr, nrange, sizeof(nr), hipMemcpyDeviceToHost, s));
  RPIM_HIP(hipMemcpyAsync(&lu_total, p->lu_off + G, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  RPIM_HIP(hipStreamSynchronize(s));
  p->max_row_upper = 0;
  for (int64_t i = 0; i < N; ++i) p->max_row_upper = std::max<int64_t>(p->max_row_upper, cnt_h[i]);
  p->min_n = G > 0 ? nr[0] : 0;
  p->max_n = G > 0 ? nr[1] : 0;
  p->lu_doubles = lu_total;
  int64_t acc = 0;
  for (int b = 0; b < kMaxBuckets; ++b) {
    if (bc[b]) p->buckets.push_back(Bucket{b * kBucketStep, acc, (int64_t)bc[b]});
    acc += (int64_t)bc[b];
  }
  // cell -> Gauss point lists (ascending g) for the deterministic dE reduction:
  // they depend on the cells only, so the first build makes them for good
  if (!p->cell_ptr) {
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
    RPIM_TRY(once(&p->cell_ptr, p->C + 1));
    RPIM_TRY(once(&p->cell_gp, G));
    RPIM_HIP(hipMemcpyAsync(p->cell_ptr, cptr.data(), sizeof(int64_t) * (p->C + 1), hipMemcpyHostToDevice, s));
    RPIM_HIP(hipMemcpyAsync(p->cell_gp, cgp.data(), sizeof(int32_t) * G, hipMemcpyHostToDevice, s));
    RPIM_HIP(hipStreamSynchronize(s));
  }
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
