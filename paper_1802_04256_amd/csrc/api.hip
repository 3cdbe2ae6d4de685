// C ABI: argument validation, plan memory, and the launch sequence of each
// call.  Every numerical step runs in the kernels of pattern.hip,
// assemble.hip, backward.hip and penalty.hip.
#include <climits>
#include <cmath>
#include <cstring>
#include <cstdio>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rpim_internal.h"

namespace rpim {

rpim_status hip_ok(hipError_t e) {
  if (e == hipSuccess) return RPIM_OK;
  if (e == hipErrorOutOfMemory) return RPIM_E_NOMEM;
  return RPIM_E_HIP;
}

rpim_status ensure_alloc(void** p, int64_t* cap, int64_t count, size_t elem) {
  if (count <= 0) count = 1;
  if (*p && *cap >= count) return RPIM_OK;
  if (*p) {
    hipError_t e = hipFree(*p);
    *p = nullptr;
    *cap = 0;
    if (e != hipSuccess) return hip_ok(e);
  }
  hipError_t e = hipMalloc(p, elem * (size_t)count);
  if (e != hipSuccess) {
    *p = nullptr;
    return hip_ok(e);
  }
  *cap = count;
  return RPIM_OK;
}

rpim_status raise_lds_limit(const void* fn, size_t lds, int device) {
  struct Entry {
    const void* fn;
    int device;
    size_t lds;
  };
  static std::mutex mu;
  static std::vector<Entry> set;
  std::lock_guard<std::mutex> lock(mu);
  Entry* e = nullptr;
  for (Entry& x : set)
    if (x.fn == fn && x.device == device) e = &x;
  if (e && lds <= e->lds) return RPIM_OK;
  RPIM_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  if (e) e->lds = lds;
  else set.push_back(Entry{fn, device, lds});
  return RPIM_OK;
}

void phase_begin(rpim_plan* p, int phase, hipStream_t s) {
  if (!p->profiling) return;
  if (!p->ev[2 * phase]) {
    (void)hipEventCreate(&p->ev[2 * phase]);
    (void)hipEventCreate(&p->ev[2 * phase + 1]);
  }
  (void)hipEventRecord(p->ev[2 * phase], s);
}

void phase_end(rpim_plan* p, int phase, hipStream_t s) {
  if (!p->profiling || !p->ev[2 * phase]) return;
  (void)hipEventRecord(p->ev[2 * phase + 1], s);
  p->phase_recorded[phase] = true;
}

namespace {

template <class T>
rpim_status dalloc(T** p, int64_t count) {
  if (*p) return RPIM_OK;
  if (count <= 0) count = 1;
  hipError_t e = hipMalloc((void**)p, sizeof(T) * (size_t)count);
  if (e != hipSuccess) {
    *p = nullptr;
    return hip_ok(e);
  }
  return RPIM_OK;
}

template <class T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

rpim_status reset_status(rpim_plan* p, hipStream_t s) {
  DevStatus clean;
  clean.first_bad = ULLONG_MAX;
  clean.flags = 0;
  clean.pad = 0;
  RPIM_HIP(hipMemcpyAsync(p->status, &clean, sizeof(DevStatus), hipMemcpyHostToDevice, s));
  return RPIM_OK;
}

}  // namespace
}  // namespace rpim

using namespace rpim;

extern "C" {

const char* rpim_status_string(rpim_status st) {
  switch (st) {
    case RPIM_OK: return "ok";
    case RPIM_E_ARG: return "invalid argument";
    case RPIM_E_NOMEM: return "device allocation failed";
    case RPIM_E_HIP: return "HIP runtime error";
    case RPIM_E_SUPPORT: return "support has fewer than 5 nodes";
    case RPIM_E_SINGULAR: return "singular moment matrix";
    case RPIM_E_RANGE: return "size exceeds a documented limit";
    case RPIM_E_POW: return "power not correctly roundable";
    case RPIM_E_STATE: return "call order violated";
    case RPIM_E_CONVERGENCE: return "iteration limit reached before the tolerance";
  }
  return "unknown status";
}

rpim_status rpim_plan_create(const rpim_problem* pb, rpim_plan** out) {
  if (!pb || !out) return RPIM_E_ARG;
  *out = nullptr;
  if (pb->n_models < 1 || !pb->node_off || !pb->gp_off || !pb->support_radius || !pb->node_xyz || !pb->gp_xyz ||
      !pb->gp_wdet || !pb->gp_cell || pb->n_cells < 1)
    return RPIM_E_ARG;
  if (!(pb->alpha_c > 0) || !(pb->d_c > 0) || !(pb->q > 0) || !std::isfinite(pb->alpha_c) ||
      !std::isfinite(pb->d_c) || !std::isfinite(pb->q))
    return RPIM_E_ARG;
  const int M = pb->n_models;
  if (pb->node_off[0] != 0 || pb->gp_off[0] != 0) return RPIM_E_ARG;
  for (int m = 0; m < M; ++m) {
    if (pb->node_off[m + 1] <= pb->node_off[m] || pb->gp_off[m + 1] < pb->gp_off[m]) return RPIM_E_ARG;
    if (!(pb->support_radius[m] > 0) || !std::isfinite(pb->support_radius[m])) return RPIM_E_ARG;
  }
  const int64_t N = pb->node_off[M], G = pb->gp_off[M];
  if (N >= INT32_MAX / 3 || G >= ((int64_t)1 << 55)) return RPIM_E_RANGE;
  rpim_plan* p = new (std::nothrow) rpim_plan;
  if (!p) return RPIM_E_NOMEM;
  (void)hipGetDevice(&p->device);
  p->n_models = M;
  p->N = N;
  p->G = G;
  p->C = pb->n_cells;
  p->alpha_c = pb->alpha_c;
  p->d_c = pb->d_c;
  p->q = pb->q;
  p->node_off.assign(pb->node_off, pb->node_off + M + 1);
  p->gp_off.assign(pb->gp_off, pb->gp_off + M + 1);
  p->radius.assign(pb->support_radius, pb->support_radius + M);
  rpim_status st = RPIM_OK;
  if ((st = dalloc(&p->node_xyz0, 3 * N)) || (st = dalloc(&p->gp_xyz, 3 * G)) || (st = dalloc(&p->gp_wdet, G)) ||
      (st = dalloc(&p->gp_cell, G)) || (st = dalloc(&p->d_gp_off, M + 1)) || (st = dalloc(&p->d_node_off, M + 1)) ||
      (st = dalloc(&p->status, 1))) {
    rpim_plan_destroy(p);
    return st;
  }
  hipError_t e = hipMemcpy(p->node_xyz0, pb->node_xyz, sizeof(double) * 3 * N, hipMemcpyDeviceToDevice);
  if (G > 0) {
    if (e == hipSuccess) e = hipMemcpy(p->gp_xyz, pb->gp_xyz, sizeof(double) * 3 * G, hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->gp_wdet, pb->gp_wdet, sizeof(double) * G, hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->gp_cell, pb->gp_cell, sizeof(int32_t) * G, hipMemcpyDeviceToDevice);
  }
  if (e == hipSuccess) e = hipMemcpy(p->d_gp_off, pb->gp_off, sizeof(int64_t) * (M + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_node_off, pb->node_off, sizeof(int64_t) * (M + 1), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    rpim_plan_destroy(p);
    return hip_ok(e);
  }
  if ((st = reset_status(p, nullptr)) != RPIM_OK) {
    rpim_plan_destroy(p);
    return st;
  }
  *out = p;
  return RPIM_OK;
}

void rpim_plan_destroy(rpim_plan* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  dfree(p->node_xyz0); dfree(p->gp_xyz); dfree(p->gp_wdet); dfree(p->gp_cell); dfree(p->d_gp_off); dfree(p->d_node_off);
  free_pattern(p);
  dfree(p->R); dfree(p->dphi); dfree(p->dphi32);
  dfree(p->lu); dfree(p->piv); dfree(p->gam); dfree(p->msym); dfree(p->pbar); dfree(p->dEs); dfree(p->dEg); dfree(p->dXs);
  dfree(p->status);
  for (int i = 0; i < 2 * RPIM_N_PHASES; ++i)
    if (p->ev[i]) (void)hipEventDestroy(p->ev[i]);
  delete p;
}

rpim_status rpim_build_pattern(rpim_plan* p, int64_t* row_ptr, int32_t* col_idx, int64_t* nnz, void* stream) {
  if (!p || !nnz) return RPIM_E_ARG;
  if ((row_ptr == nullptr) != (col_idx == nullptr)) return RPIM_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (!p->built) {
    phase_begin(p, RPIM_PHASE_PATTERN, s);
    rpim_status st = build_pattern_device(p, p->node_xyz0, s);
    phase_end(p, RPIM_PHASE_PATTERN, s);
    if (st != RPIM_OK) return st;
  }
  *nnz = p->nnz;
  if (row_ptr) {
    rpim_status st = expand_pattern(p, row_ptr, col_idx, s);
    if (st != RPIM_OK) return st;
  }
  return RPIM_OK;
}

rpim_status rpim_rebuild_pattern(rpim_plan* p, const double* node_xyz, int64_t* row_ptr, int32_t* col_idx,
                                 int64_t* nnz, void* stream) {
  if (!p || !node_xyz || !nnz) return RPIM_E_ARG;
  if ((row_ptr == nullptr) != (col_idx == nullptr)) return RPIM_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  RPIM_HIP(hipStreamSynchronize(s));
  p->built = false;  // the pattern arrays are rebuilt in place
  p->have_factors = false;
  ++p->factor_gen;
  RPIM_HIP(hipMemcpyAsync(p->node_xyz0, node_xyz, sizeof(double) * 3 * p->N, hipMemcpyDeviceToDevice, s));
  return rpim_build_pattern(p, row_ptr, col_idx, nnz, stream);
}

rpim_status rpim_profile_enable(rpim_plan* p, int enable) {
  if (!p) return RPIM_E_ARG;
  p->profiling = enable != 0;
  for (int i = 0; i < RPIM_N_PHASES; ++i) p->phase_recorded[i] = false;
  return RPIM_OK;
}

rpim_status rpim_profile_read(rpim_plan* p, double* ms) {
  if (!p || !ms) return RPIM_E_ARG;
  for (int i = 0; i < RPIM_N_PHASES; ++i) {
    ms[i] = -1.0;
    if (!p->phase_recorded[i]) continue;
    RPIM_HIP(hipEventSynchronize(p->ev[2 * i + 1]));
    float t = 0.f;
    RPIM_HIP(hipEventElapsedTime(&t, p->ev[2 * i], p->ev[2 * i + 1]));
    ms[i] = t;
  }
  return RPIM_OK;
}

rpim_status rpim_assemble(rpim_plan* p, const double* node_xyz, const double* cell_E, double nu, int precision,
                          int keep_factors, void* K_vals, void* stream) {
  if (!p || !node_xyz || !cell_E || !K_vals) return RPIM_E_ARG;
  if (!p->built) return RPIM_E_STATE;
  if (precision != RPIM_FP64 && precision != RPIM_MIXED) return RPIM_E_ARG;
  if (!(nu > -1.0 && nu < 0.5)) return RPIM_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  rpim_status st;
  if ((st = ensure(&p->R, &p->cap_R, p->nblk)) || (st = ensure(&p->dphi, &p->cap_dphi, 3 * p->sum_n))) return st;
  if (precision == RPIM_MIXED && (st = ensure(&p->dphi32, &p->cap_dphi32, 3 * p->sum_n))) return st;
  if (keep_factors && p->shape_kind == RPIM_SHAPE_RPIM) {
    if ((st = ensure(&p->lu, &p->cap_lu, p->lu_doubles)) || (st = ensure(&p->piv, &p->cap_piv, p->sum_n + 4 * p->G)) ||
        (st = ensure(&p->gam, &p->cap_gam, 3 * (p->sum_n + 4 * p->G))))
      return st;
  }
  if (p->have_factors) ++p->factor_gen;
  p->have_factors = false;
  if (p->shape_kind != RPIM_SHAPE_RPIM) {  // moving least squares: gradients, then the same gather
    phase_begin(p, RPIM_PHASE_SHAPE, s);
    if ((st = launch_mls(p, node_xyz, p->dphi, precision == RPIM_MIXED ? p->dphi32 : nullptr, nullptr, s)) !=
        RPIM_OK)
      return st;
    phase_end(p, RPIM_PHASE_SHAPE, s);
    phase_begin(p, RPIM_PHASE_GATHER, s);
    if ((st = launch_rowgather(p, cell_E, nu, precision, K_vals, s)) != RPIM_OK) return st;
    phase_end(p, RPIM_PHASE_GATHER, s);
    return RPIM_OK;
  }
  phase_begin(p, RPIM_PHASE_PAIRS, s);
  if ((st = launch_pair_table(p, node_xyz, s)) != RPIM_OK) return st;
  phase_end(p, RPIM_PHASE_PAIRS, s);
  phase_begin(p, RPIM_PHASE_SHAPE, s);
  if ((st = launch_shape(p, node_xyz, keep_factors ? 1 : 0, precision == RPIM_MIXED ? p->dphi32 : nullptr, s)) !=
      RPIM_OK)
    return st;
  phase_end(p, RPIM_PHASE_SHAPE, s);
  phase_begin(p, RPIM_PHASE_GATHER, s);
  if ((st = launch_rowgather(p, cell_E, nu, precision, K_vals, s)) != RPIM_OK) return st;
  phase_end(p, RPIM_PHASE_GATHER, s);
  p->have_factors = keep_factors != 0;
  if (p->have_factors) ++p->factor_gen;
  return RPIM_OK;
}

rpim_status rpim_assemble_backward(rpim_plan* p, const double* node_xyz, const double* cell_E, double nu,
                                   const double* dK_vals, double* dE_cell, double* dX_node, void* stream) {
  if (!p || !node_xyz || !cell_E || !dK_vals || !dE_cell || !dX_node) return RPIM_E_ARG;
  if (!p->built || !p->have_factors || p->shape_kind != RPIM_SHAPE_RPIM) return RPIM_E_STATE;
  if (!(nu > -1.0 && nu < 0.5)) return RPIM_E_ARG;
  return launch_backward(p, node_xyz, cell_E, nu, dK_vals, dE_cell, dX_node, (hipStream_t)stream);
}

// ---- launch-configuration tuning --------------------------------------------
// Choices are cached per process, keyed by (GPU architecture, precision,
// bucket size) for the solver kernel and (architecture, precision) for the
// row gather, and can be saved to / loaded from a text file.
namespace {

std::mutex g_tune_mu;
std::map<std::string, int> g_tune_cache;

std::string arch_name(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);  // gfx950 (target features dropped)
}

std::string tune_key(const std::string& arch, int precision, const char* what, int nmax) {
  return arch + " " + (precision == RPIM_MIXED ? "mixed" : "fp64") + " " + what + " " + std::to_string(nmax);
}

bool cache_get(const std::string& k, int* v) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune_cache.find(k);
  if (it == g_tune_cache.end()) return false;
  *v = it->second;
  return true;
}

void cache_put(const std::string& k, int v) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune_cache[k] = v;
}

}  // namespace

rpim_status rpim_autotune(rpim_plan* p, const double* node_xyz, const double* cell_E, double nu, int precision,
                          void* K_vals, void* stream, rpim_tuning* out) {
  if (!p || !node_xyz || !cell_E || !K_vals) return RPIM_E_ARG;
  if (!p->built) return RPIM_E_STATE;
  if (precision != RPIM_FP64 && precision != RPIM_MIXED) return RPIM_E_ARG;
  if (!(nu > -1.0 && nu < 0.5)) return RPIM_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  rpim_tuning t = {};
  const std::string arch = arch_name(p->device);
  // everything cached for this architecture and precision: apply, time nothing
  {
    bool all = true;
    int gw = 0;
    all = cache_get(tune_key(arch, precision, "gather", 0), &gw);
    std::vector<int> kinds;
    for (const Bucket& b : p->buckets) {
      int k = 0;
      if (!all || !cache_get(tune_key(arch, precision, "solver", b.nmax), &k)) {
        all = false;
        break;
      }
      kinds.push_back(k);
    }
    if (all) {
      p->gather_waves[precision == RPIM_MIXED ? 1 : 0] = gw;
      int nb = 0;
      for (size_t i = 0; i < p->buckets.size(); ++i) {
        const Bucket& b = p->buckets[i];
        p->solver_kind[b.nmax / kBucketStep] = (int8_t)kinds[i];
        if (nb < RPIM_TUNING_MAX_BUCKETS) {
          t.bucket_nmax[nb] = b.nmax;
          t.bucket_points[nb] = b.count;
          t.bucket_solver[nb] = kinds[i];
          t.bucket_ms[nb] = t.bucket_ms_window[nb] = t.bucket_ms_panel[nb] = -1.f;
          ++nb;
        }
      }
      t.n_buckets = nb;
      t.gather_waves = gw;
      t.gather_ms[0] = t.gather_ms[1] = t.gather_ms[2] = t.gather_ms[3] = -1.f;
      t.from_cache = 1;
      if (out) *out = t;
      return RPIM_OK;
    }
  }
  rpim_status st;
  if ((st = ensure(&p->R, &p->cap_R, p->nblk)) || (st = ensure(&p->dphi, &p->cap_dphi, 3 * p->sum_n))) return st;
  if (precision == RPIM_MIXED && (st = ensure(&p->dphi32, &p->cap_dphi32, 3 * p->sum_n))) return st;
  float* d32 = precision == RPIM_MIXED ? p->dphi32 : nullptr;
  // the runs below rewrite the pair table and the gradients that kept factors belong to
  if (p->have_factors) ++p->factor_gen;
  p->have_factors = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  RPIM_HIP(hipEventCreate(&e0));
  if (hip_ok(hipEventCreate(&e1)) != RPIM_OK) {
    (void)hipEventDestroy(e0);
    return RPIM_E_HIP;
  }
  auto timed = [&](auto&& launch, float* ms) -> rpim_status {
    hipError_t e = hipEventRecord(e0, s);
    rpim_status r = e == hipSuccess ? launch() : hip_ok(e);
    if (r == RPIM_OK) r = hip_ok(hipEventRecord(e1, s));
    if (r == RPIM_OK) r = hip_ok(hipEventSynchronize(e1));
    if (r == RPIM_OK) r = hip_ok(hipEventElapsedTime(ms, e0, e1));
    return r;
  };
  // best of two runs (the first also loads the kernel code)
  auto best_of_two = [&](auto&& launch, float* ms) -> rpim_status {
    float a = 0.f, b2 = 0.f;
    rpim_status r = timed(launch, &a);
    if (r == RPIM_OK) r = timed(launch, &b2);
    *ms = a < b2 ? a : b2;
    return r;
  };
  st = launch_pair_table(p, node_xyz, s);
  int nb = 0;
  for (const Bucket& b : p->buckets) {
    if (st != RPIM_OK) break;
    int8_t& kind = p->solver_kind[b.nmax / kBucketStep];
    float ms_w = -1.f, ms_p = -1.f;
    if (b.nmax <= shape_reg_max()) {
      kind = RPIM_SOLVER_WINDOW;
      st = best_of_two([&] { return launch_shape_bucket(p, b, node_xyz, 0, d32, s); }, &ms_w);
    }
    if (st == RPIM_OK && b.nmax <= shape_panel_max()) {
      kind = RPIM_SOLVER_PANEL;
      st = best_of_two([&] { return launch_shape_bucket(p, b, node_xyz, 0, d32, s); }, &ms_p);
    }
    float ms = 0.f;
    if (ms_w < 0.f && ms_p < 0.f) {
      kind = RPIM_SOLVER_LDS;
      if (st == RPIM_OK) st = best_of_two([&] { return launch_shape_bucket(p, b, node_xyz, 0, d32, s); }, &ms);
    } else if (ms_p >= 0.f && (ms_w < 0.f || ms_p < ms_w)) {
      kind = RPIM_SOLVER_PANEL;
      ms = ms_p;
    } else {
      kind = RPIM_SOLVER_WINDOW;
      ms = ms_w;
    }
    cache_put(tune_key(arch, precision, "solver", b.nmax), kind);
    if (nb < RPIM_TUNING_MAX_BUCKETS) {
      t.bucket_nmax[nb] = b.nmax;
      t.bucket_points[nb] = b.count;
      t.bucket_ms[nb] = ms;
      t.bucket_solver[nb] = kind;
      t.bucket_ms_window[nb] = ms_w;
      t.bucket_ms_panel[nb] = ms_p;
      ++nb;
    }
  }
  t.n_buckets = nb;
  // the gradients with the chosen kernels (every kernel gives the same bits)
  if (st == RPIM_OK) st = launch_shape(p, node_xyz, 0, d32, s);
  int best = 0;
  for (int i = 0; i < 4 && st == RPIM_OK; ++i) {
    const int gw = 1 + i;
    float ms = 0.f, best_ms = 0.f;
    for (int rep = 0; rep < 3 && st == RPIM_OK; ++rep) {  // first run warms caches and sets LDS limits
      st = timed([&] { return launch_rowgather(p, cell_E, nu, precision, K_vals, s, gw); }, &ms);
      if (rep == 1 || (rep > 1 && ms < best_ms)) best_ms = ms;
    }
    t.gather_ms[i] = best_ms;
    if (best_ms < t.gather_ms[best]) best = i;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != RPIM_OK) return st;
  t.gather_waves = 1 + best;
  p->gather_waves[precision == RPIM_MIXED ? 1 : 0] = t.gather_waves;
  cache_put(tune_key(arch, precision, "gather", 0), t.gather_waves);
  if (out) *out = t;
  return RPIM_OK;
}

rpim_status rpim_tuning_cache_save(const char* path) {
  if (!path) return RPIM_E_ARG;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  FILE* f = std::fopen(path, "w");
  if (!f) return RPIM_E_ARG;
  std::fprintf(f, "# rpim tuning cache: arch precision what nmax value\n");
  for (const auto& kv : g_tune_cache) std::fprintf(f, "%s %d\n", kv.first.c_str(), kv.second);
  return std::fclose(f) == 0 ? RPIM_OK : RPIM_E_ARG;
}

rpim_status rpim_tuning_cache_load(const char* path) {
  if (!path) return RPIM_E_ARG;
  FILE* f = std::fopen(path, "r");
  if (!f) return RPIM_E_ARG;
  char arch[64], prec[16], what[16];
  int nmax = 0, value = 0;
  char line[256];
  rpim_status st = RPIM_OK;
  while (std::fgets(line, sizeof(line), f)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    if (std::sscanf(line, "%63s %15s %15s %d %d", arch, prec, what, &nmax, &value) != 5) {
      st = RPIM_E_ARG;
      break;
    }
    const std::string w = what, pr = prec;
    const bool ok = (pr == "fp64" || pr == "mixed") &&
                    ((w == "solver" && value >= RPIM_SOLVER_AUTO && value <= RPIM_SOLVER_PANEL) ||
                     (w == "gather" && gather_waves_valid(value)));
    if (!ok) {
      st = RPIM_E_ARG;
      break;
    }
    cache_put(std::string(arch) + " " + pr + " " + w + " " + std::to_string(nmax), value);
  }
  std::fclose(f);
  return st;
}

void rpim_tuning_cache_clear(void) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune_cache.clear();
}

rpim_status rpim_set_gather_waves(rpim_plan* p, int precision, int waves) {
  if (!p || (precision != RPIM_FP64 && precision != RPIM_MIXED) || !gather_waves_valid(waves)) return RPIM_E_ARG;
  p->gather_waves[precision == RPIM_MIXED ? 1 : 0] = waves;
  return RPIM_OK;
}

size_t rpim_penalty_workspace_bytes(int64_t n_dof, int64_t n_fixed) {
  if (n_dof <= 0 || n_fixed < 0) return 0;
  return penalty_workspace_bytes(n_dof, n_fixed);
}

rpim_status rpim_apply_penalty_bc(const int64_t* row_ptr, const int32_t* col_idx, void* K_vals, int precision,
                                  int64_t n_dof, const int32_t* fixed_dof, const double* u_bar, int64_t n_fixed,
                                  double factor, double* rhs, double* alpha, int32_t* status, void* workspace,
                                  size_t workspace_bytes, void* stream) {
  if (!row_ptr || !col_idx || !K_vals || n_dof <= 0 || n_fixed < 0 || (n_fixed > 0 && !fixed_dof)) return RPIM_E_ARG;
  if (n_dof > INT32_MAX) return RPIM_E_RANGE;
  if (precision != RPIM_FP64 && precision != RPIM_MIXED) return RPIM_E_ARG;
  if (!(factor > 0) || !std::isfinite(factor)) return RPIM_E_ARG;
  return launch_penalty(row_ptr, col_idx, K_vals, precision, n_dof, fixed_dof, u_bar, n_fixed, factor, rhs, alpha,
                        status, workspace, workspace_bytes, (hipStream_t)stream);
}

rpim_status rpim_apply_penalty_bc_noalloc(const int64_t* row_ptr, const int32_t* col_idx, void* K_vals,
                                          int precision, int64_t n_dof, const int32_t* fixed_dof,
                                          const double* u_bar, int64_t n_fixed, double factor, double* rhs,
                                          double* alpha, int32_t* status, void* stream) {
  if (!row_ptr || !col_idx || !K_vals || n_dof <= 0 || n_fixed < 0 || (n_fixed > 0 && !fixed_dof)) return RPIM_E_ARG;
  if (n_dof > INT32_MAX) return RPIM_E_RANGE;
  if (precision != RPIM_FP64 && precision != RPIM_MIXED) return RPIM_E_ARG;
  if (!(factor > 0) || !std::isfinite(factor)) return RPIM_E_ARG;
  return launch_penalty_noalloc(row_ptr, col_idx, K_vals, precision, n_dof, fixed_dof, u_bar, n_fixed, factor, rhs,
                                alpha, status, (hipStream_t)stream);
}

rpim_status rpim_shape_values(rpim_plan* p, const double* node_xyz, double* phi, void* stream) {
  if (!p || !node_xyz || !phi) return RPIM_E_ARG;
  if (!p->built) return RPIM_E_STATE;
  if (p->shape_kind != RPIM_SHAPE_RPIM) return launch_mls(p, node_xyz, nullptr, nullptr, phi, (hipStream_t)stream);
  if (!p->have_factors) return RPIM_E_STATE;
  return launch_shape_values(p, node_xyz, phi, (hipStream_t)stream);
}

rpim_status rpim_body_force(rpim_plan* p, const double* phi, const double* gp_force, double* f, void* stream) {
  if (!p || !phi || !gp_force || !f) return RPIM_E_ARG;
  if (!p->built) return RPIM_E_STATE;
  return launch_body_force(p, phi, gp_force, f, (hipStream_t)stream);
}

rpim_status rpim_gauss_stress(rpim_plan* p, const double* cell_E, double nu, const double* u, double* sigma,
                              void* stream) {
  if (!p || !cell_E || !u || !sigma) return RPIM_E_ARG;
  if (!p->built || !p->dphi) return RPIM_E_STATE;
  if (!(nu > -1.0 && nu < 0.5)) return RPIM_E_ARG;
  return launch_gauss_stress(p, cell_E, nu, u, sigma, (hipStream_t)stream);
}

size_t rpim_pcg_workspace_bytes(int64_t n_dof) {
  if (n_dof <= 0) return 0;
  return pcg_workspace_bytes(n_dof);
}

rpim_status rpim_solve_pcg(const int64_t* row_ptr, const int32_t* col_idx, const void* K_vals, int precision,
                           int64_t n_dof, const double* rhs, double* x, double rtol, int64_t max_iter,
                           void* workspace, size_t workspace_bytes, int64_t* iterations, double* rel_residual,
                           void* stream) {
  if (!row_ptr || !col_idx || !K_vals || !rhs || !x || n_dof <= 0 || max_iter < 0) return RPIM_E_ARG;
  if (precision != RPIM_FP64 && precision != RPIM_MIXED) return RPIM_E_ARG;
  if (!(rtol >= 0) || !std::isfinite(rtol)) return RPIM_E_ARG;
  if (n_dof > INT32_MAX) return RPIM_E_RANGE;
  return solve_pcg(row_ptr, col_idx, K_vals, precision, n_dof, rhs, x, rtol, max_iter, workspace, workspace_bytes,
                   iterations, rel_residual, (hipStream_t)stream);
}

rpim_status rpim_set_solver(rpim_plan* p, int nmax, int kind) {
  if (!p || nmax < 0 || nmax > kMaxSupport + 4) return RPIM_E_ARG;
  if (kind != RPIM_SOLVER_AUTO && kind != RPIM_SOLVER_LDS && kind != RPIM_SOLVER_WINDOW && kind != RPIM_SOLVER_PANEL)
    return RPIM_E_ARG;
  for (int b = 0; b < kMaxBuckets; ++b)
    if (nmax == 0 || b == (nmax + kBucketStep - 1) / kBucketStep) p->solver_kind[b] = (int8_t)kind;
  return RPIM_OK;
}

rpim_status rpim_set_shape_functions(rpim_plan* p, int kind) {
  if (!p) return RPIM_E_ARG;
  if (kind != RPIM_SHAPE_RPIM && kind != RPIM_SHAPE_MLS && kind != RPIM_SHAPE_SHEPARD) return RPIM_E_ARG;
  if (kind != p->shape_kind) {
    if (p->have_factors) ++p->factor_gen;
    p->have_factors = false;
    p->shape_kind = kind;
  }
  return RPIM_OK;
}

rpim_status rpim_factor_generation(const rpim_plan* p, int64_t* gen) {
  if (!p || !gen) return RPIM_E_ARG;
  *gen = p->have_factors ? p->factor_gen : 0;
  return RPIM_OK;
}

rpim_status rpim_get_status(rpim_plan* p, void* stream, int64_t* first_bad_gp) {
  if (!p) return RPIM_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  DevStatus h;
  RPIM_HIP(hipMemcpyAsync(&h, p->status, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
  RPIM_HIP(hipStreamSynchronize(s));
  rpim_status st = reset_status(p, s);
  if (st != RPIM_OK) return st;
  RPIM_HIP(hipStreamSynchronize(s));
  if (first_bad_gp) *first_bad_gp = h.first_bad == ULLONG_MAX ? -1 : (int64_t)h.first_bad;
  if (h.flags & kFlagSupport) return RPIM_E_SUPPORT;
  if (h.flags & kFlagSingular) return RPIM_E_SINGULAR;
  if (h.flags & kFlagRange) return RPIM_E_RANGE;
  if (h.flags & kFlagPow) return RPIM_E_POW;
  return RPIM_OK;
}

rpim_status rpim_plan_info(const rpim_plan* p, rpim_info* info) {
  if (!p || !info) return RPIM_E_ARG;
  std::memset(info, 0, sizeof(*info));
  info->n_nodes = p->N;
  info->n_gp = p->G;
  info->n_cells = p->C;
  info->n_models = p->n_models;
  info->sum_n = p->sum_n;
  info->nnz = p->nnz;
  info->n_blocks = p->nblk;
  info->min_n = p->min_n;
  info->max_n = p->max_n;
  info->lu_doubles = p->lu_doubles;
  info->n_buckets = (int32_t)p->buckets.size();
  return RPIM_OK;
}

rpim_status rpim_get_support(const rpim_plan* p, int64_t* gp_ptr, int32_t* gp_nbr, void* stream) {
  if (!p || !gp_ptr || !gp_nbr) return RPIM_E_ARG;
  if (!p->built) return RPIM_E_STATE;
  hipStream_t s = (hipStream_t)stream;
  RPIM_HIP(hipMemcpyAsync(gp_ptr, p->gp_ptr, sizeof(int64_t) * (p->G + 1), hipMemcpyDeviceToDevice, s));
  if (p->sum_n > 0)
    RPIM_HIP(hipMemcpyAsync(gp_nbr, p->gp_nbr, sizeof(int32_t) * p->sum_n, hipMemcpyDeviceToDevice, s));
  return RPIM_OK;
}

rpim_status rpim_get_dphi(const rpim_plan* p, double* dphi, void* stream) {
  if (!p || !dphi) return RPIM_E_ARG;
  if (!p->dphi) return RPIM_E_STATE;
  RPIM_HIP(hipMemcpyAsync(dphi, p->dphi, sizeof(double) * 3 * p->sum_n, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return RPIM_OK;
}

rpim_status rpim_pow_cr(const double* x, double q, double* y, int64_t n, void* stream) {
  if ((!x || !y) && n > 0) return RPIM_E_ARG;
  if (n < 0 || !(q > 0)) return RPIM_E_ARG;
  return launch_pow_test(x, q, y, n, (hipStream_t)stream);
}

}  // extern "C"
