// Internal state and launcher declarations of the RPIM library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/rpim.h"

namespace rpim {

// Limits (documented in rpim.h).
constexpr int kMaxSupport = 132;        // nodes per support (N = n + 4 <= 136 fits the LDS solver)
constexpr int kMaxInverse = 8192;       // supports containing one node
constexpr int64_t kMaxWindow = 1 << 18; // node-id span of a node's neighbourhood
constexpr int kBucketStep = 8;          // support-size buckets: padded N in steps of 8
constexpr int kMaxBuckets = (kMaxSupport + 4) / kBucketStep + 1;

// Device-side error record: smallest failing Gauss point and kinds seen.
struct DevStatus {
  unsigned long long first_bad;  // ULLONG_MAX when clean
  unsigned int flags;            // bit set of kFlag*
  unsigned int pad;
};
constexpr unsigned kFlagSupport = 1u, kFlagSingular = 2u, kFlagPow = 4u, kFlagRange = 8u;

// Uniform bin grid of one model for the support search.
struct BinGrid {
  double ox, oy, oz;  // origin
  double h;           // bin edge (>= support radius)
  double r2;          // fl(d_s * d_s)
  int nx, ny, nz;     // bins per axis
  int pad;
  int64_t bin0;       // first global bin id of this model
};

// Gauss points with the same padded moment-matrix size share a bucket.
// Position of column J in node-block row I through the row's rank bitmap.
__device__ __forceinline__ int64_t block_pos(const int64_t* blk_ptr, const int32_t* row_lo, const int64_t* rbm_off,
                                             const uint2* rbm, int32_t I, int32_t J) {
  const int r = J - row_lo[I];
  const uint2 w = rbm[rbm_off[I] + (r >> 5)];
  return blk_ptr[I] + (int64_t)w.y + __popc(w.x & ((1u << (r & 31)) - 1u));
}

// 64-bit readlanes: lane L's value of x (L wave-uniform).
__device__ __forceinline__ double readlane_f64(double x, int L) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, L);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), L);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ int64_t readlane_i64(int64_t x, int L) {
  const int lo = __builtin_amdgcn_readlane((int)x, L);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), L);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

struct Bucket {
  int nmax;        // largest N = n + 4 in the bucket
  int64_t begin;   // range in gp_order
  int64_t count;
};

}  // namespace rpim

struct rpim_plan {
  int device = 0;
  int32_t n_models = 0;
  int64_t N = 0, G = 0, C = 0;
  double alpha_c = 0, d_c = 0, q = 0;
  std::vector<int64_t> node_off, gp_off;
  std::vector<double> radius;

  // plan-owned device copies of the Gauss-point description
  double* node_xyz0 = nullptr;   // [N][3] build-time node coordinates
  double* gp_xyz = nullptr;
  double* gp_wdet = nullptr;
  int32_t* gp_cell = nullptr;
  int64_t* d_gp_off = nullptr;   // [n_models+1]
  int64_t* d_node_off = nullptr; // [n_models+1]

  // pattern (built by rpim_build_pattern)
  bool built = false;
  int64_t sum_n = 0, nblk = 0, nnz = 0;
  int32_t min_n = 0, max_n = 0;
  int64_t* gp_ptr = nullptr;     // [G+1]
  int32_t* gp_nbr = nullptr;     // [sum_n]
  int64_t* inv_ptr = nullptr;    // [N+1]
  uint64_t* inv_key = nullptr;   // [sum_n]  (g << 8) | local index, ascending g per node
  int64_t* blk_ptr = nullptr;    // [N+1]
  int32_t* blk_col = nullptr;    // [nblk]
  int32_t* blk_row = nullptr;    // [nblk]
  // rank structure of each node-block row over its node-id window:
  // word i of row I covers ids lo_I + 32 i ... + 31; .x = bits, .y = set bits in words < i.
  // position of column J in row I = blk_ptr[I] + y + popc(x & ((1 << b) - 1)).
  int32_t* row_lo = nullptr;     // [N]   first id of the window (= smallest column)
  int64_t* rbm_off = nullptr;    // [N+1] word offsets
  uint2* rbm = nullptr;          // [rbm_off[N]]
  int64_t rbm_words = 0;
  int32_t max_row_words = 0;
  int64_t max_row_blocks = 0;    // longest node-block row
  int64_t max_row_upper = 0;     // most blocks J >= I in a row I
  int64_t max_inverse = 0;       // longest inverse list
  std::vector<rpim::Bucket> buckets;
  // solver kernel per bucket (index nmax / kBucketStep): RPIM_SOLVER_* from rpim.h
  int8_t solver_kind[rpim::kMaxBuckets] = {};
  int shape_kind = 0;  // RPIM_SHAPE_* from rpim.h
  int32_t* gp_order = nullptr;   // [G] Gauss points grouped by bucket
  // rebuild reuse: capacities of the pattern arrays whose size follows the
  // geometry, and one buffer for the temporaries of a build
  int64_t cap_gp_nbr = 0, cap_inv_key = 0, cap_blk = 0, cap_rbm = 0;
  void* pat_scratch = nullptr;
  size_t cap_pat_scratch = 0;

  // assembly workspace
  double* R = nullptr;           // [nblk] radial basis per node pair
  double* dphi = nullptr;        // [sum_n][3]
  float* dphi32 = nullptr;       // [sum_n][3] (mixed precision)

  // kept factors (keep_factors = 1)
  // per point, N^2 doubles at lu_off[g], column-major F[c*N + p]: for p <= c the
  // U entry u_pc (rows by position), for p > c the multiplier applied at step c to
  // the row that held position p after step c's interchange; piv[k] holds the
  // position the pivot of step k held before that interchange (>= k).
  int64_t* lu_off = nullptr;     // [G+1]
  int64_t lu_doubles = 0;
  double* lu = nullptr;          // [lu_doubles]
  int32_t* piv = nullptr;        // [sum_n + 4G] per point at 4g + gp_ptr[g]
  double* gam = nullptr;         // [3 * (sum_n + 4G)] full solutions gamma_k per point
  bool have_factors = false;
  int64_t factor_gen = 0;        // bumped whenever kept factors are written or invalidated

  // backward scratch and cell -> Gauss point lists
  double* msym = nullptr;        // [nnz]        dK + dK^T on the pattern
  double* pbar = nullptr;        // [sum_n][3]   dL/dphi per support entry
  double* dEs = nullptr;         // [sum_n]      dL/dE share per support entry (row of the entry)
  double* dEg = nullptr;         // [G]          dL/dE contribution per Gauss point
  double* dXs = nullptr;         // [sum_n][3]   dL/dx contribution per support entry
  int64_t* cell_ptr = nullptr;   // [C+1]
  int32_t* cell_gp = nullptr;    // [G] Gauss points of each cell, ascending

  rpim::DevStatus* status = nullptr;

  // launch configurations chosen by rpim_autotune (defaults until then)
  int gather_waves[2] = {1, 1};  // row-gather waves per node row: [FP64, mixed]

  // capacities (elements) of the workspaces above, so a rebuilt pattern can reuse them
  int64_t cap_R = 0, cap_dphi = 0, cap_dphi32 = 0, cap_lu = 0, cap_piv = 0, cap_gam = 0;
  int64_t cap_msym = 0, cap_pbar = 0, cap_dEs = 0, cap_dEg = 0, cap_dXs = 0;

  // optional per-phase timing with HIP events on the call's stream
  bool profiling = false;
  hipEvent_t ev[2 * RPIM_N_PHASES] = {};
  float phase_ms[RPIM_N_PHASES] = {};
  bool phase_recorded[RPIM_N_PHASES] = {};
};

namespace rpim {

// phase timing helpers (api.hip)
void phase_begin(rpim_plan* p, int phase, hipStream_t s);
void phase_end(rpim_plan* p, int phase, hipStream_t s);

// --- helpers (api.hip) -----------------------------------------------------
rpim_status hip_ok(hipError_t e);
// Raise a kernel's dynamic-LDS limit on `device` when a launch needs more than
// was set before; once a plan has run eagerly, launches recorded into a graph
// make no attribute calls.  Thread-safe; limits are per kernel and device.
rpim_status raise_lds_limit(const void* fn, size_t lds, int device);
// (Re)allocate *p to hold at least `count` elements; *cap tracks its capacity.
rpim_status ensure_alloc(void** p, int64_t* cap, int64_t count, size_t elem);
template <class T>
inline rpim_status ensure(T** p, int64_t* cap, int64_t count) {
  return ensure_alloc((void**)p, cap, count, sizeof(T));
}
#define RPIM_HIP(x)                                 \
  do {                                              \
    hipError_t e_ = (x);                            \
    if (e_ != hipSuccess) return rpim::hip_ok(e_);  \
  } while (0)

// --- scan.hip ----------------------------------------------------------------
// Exclusive prefix sum of n int32 counts into int64 offsets out[n+1].
rpim_status exclusive_scan(const int32_t* counts, int64_t n, int64_t* out, hipStream_t s);
rpim_status exclusive_scan64(const int64_t* values, int64_t n, int64_t* out, hipStream_t s);

// --- pattern.hip -------------------------------------------------------------
// Builds supports, pattern, buckets and lists into the plan; frees the plan's
// pattern arrays first and every temporary on each exit path.
rpim_status build_pattern_device(rpim_plan* p, const double* node_xyz, hipStream_t s);
void free_pattern(rpim_plan* p);
rpim_status expand_pattern(const rpim_plan* p, int64_t* row_ptr, int32_t* col_idx, hipStream_t s);

// --- assemble.hip ------------------------------------------------------------
rpim_status launch_pair_table(rpim_plan* p, const double* X, hipStream_t s);
// dphi32 (may be null): also write the gradients rounded to float, for the mixed-precision gather
rpim_status launch_shape(rpim_plan* p, const double* X, int keep, float* dphi32, hipStream_t s);
rpim_status launch_shape_bucket(rpim_plan* p, const Bucket& b, const double* X, int keep, float* dphi32,
                                hipStream_t s);
// gather_waves: waves per row of the gather (1 to 4), 0 = the plan's tuned choice
rpim_status launch_rowgather(rpim_plan* p, const double* E, double nu, int precision, void* K, hipStream_t s,
                             int gather_waves = 0);
int gather_waves_valid(int gw);
int shape_reg_max();
rpim_status launch_shape_reg(rpim_plan* p, const Bucket& b, const double* X, double C2, int keep, float* dphi32,
                             hipStream_t s);
int shape_panel_max();
rpim_status launch_shape_panel(rpim_plan* p, const Bucket& b, const double* X, double C2, int keep, float* dphi32,
                               hipStream_t s);
rpim_status launch_pow_test(const double* x, double q, double* y, int64_t n, hipStream_t s);

// --- backward.hip ------------------------------------------------------------
rpim_status launch_backward(rpim_plan* p, const double* X, const double* E, double nu,
                            const double* dK, double* dE, double* dX, hipStream_t s);

// --- post.hip ----------------------------------------------------------------
rpim_status launch_shape_values(rpim_plan* p, const double* X, double* phi, hipStream_t s);
rpim_status launch_mls(rpim_plan* p, const double* X, double* dphi, float* dphi32, double* phi, hipStream_t s);
rpim_status launch_body_force(rpim_plan* p, const double* phi, const double* gp_force, double* f, hipStream_t s);
rpim_status launch_gauss_stress(rpim_plan* p, const double* E, double nu, const double* u, double* sigma,
                                hipStream_t s);

// --- solve.hip ---------------------------------------------------------------
size_t pcg_workspace_bytes(int64_t n);
rpim_status solve_pcg(const int64_t* row_ptr, const int32_t* col_idx, const void* K, int precision, int64_t n,
                      const double* f, double* x, double rtol, int64_t max_iter, void* ws, size_t ws_bytes,
                      int64_t* iters, double* relres, hipStream_t s);

// --- penalty.hip -------------------------------------------------------------
size_t penalty_workspace_bytes(int64_t n_dof, int64_t n_fixed);
rpim_status launch_penalty(const int64_t* row_ptr, const int32_t* col_idx, void* K, int precision, int64_t n_dof,
                           const int32_t* fixed, const double* ubar, int64_t n_fixed, double factor, double* rhs,
                           double* alpha_out, int32_t* status_out, void* ws, size_t ws_size, hipStream_t s);
rpim_status launch_penalty_noalloc(const int64_t* row_ptr, const int32_t* col_idx, void* K, int precision,
                                   int64_t n_dof, const int32_t* fixed, const double* ubar, int64_t n_fixed,
                                   double factor, double* rhs, double* alpha_out, int32_t* status_out,
                                   hipStream_t s);

}  // namespace rpim
