/*
 * rpim.h -- C ABI of the MI355X RPIM global-stiffness assembly library.
 *
 * The library assembles the global stiffness matrix K of 3D linear elasticity
 * with the radial point interpolation method, point by point over background
 * Gauss points (GeoMFree3D, Sec. 2, stage 1), and enforces displacement
 * boundary conditions by the penalty method (Sec. 2, stage 2).  The paper
 * prints no formulas; the method is Liu's polynomial-augmented RPIM cited in
 * Sec. 1, written out here:
 *
 *   for each Gauss point g at x_g with weight w_g (Gauss weight * |J|) in cell c:
 *     S_g  = { i : |x_i - x_g|^2 <= d_s^2 }, sorted by node id          (support)
 *     G_g  = [[R, P], [P^T, 0]],  R_ab = (|x_a - x_b|^2 + (alpha_c d_c)^2)^q,
 *            P_a = [1, x_a - x_g]                                       (moment matrix)
 *     G_g gamma_k = d/dx_k [R(x); 1, x - x_g] at x_g,  dphi_a/dx_k = gamma_k[a]
 *     k^g_ab = w_g E_c [lam phi_a phi_b^T + mu phi_b phi_a^T + mu (phi_a . phi_b) I3]
 *            (= B_a^T D B_b for isotropic D; lam, mu for E = 1 and the given nu)
 *   K = sum_g scatter(k^g) into a CSR matrix over dof = 3*node + component.
 *
 * Conventions shared by every call
 *   - Pointers are DEVICE pointers unless marked [host].  All arrays are
 *     C-contiguous.  The caller owns every buffer it passes; the library never
 *     frees them.  A plan owns the device memory it allocates itself.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *   - Errors in arguments are returned synchronously.  Errors found on the
 *     device (a support with fewer than 5 nodes, a singular moment matrix, a
 *     power too close to a rounding boundary to round correctly) are recorded
 *     in the plan with the smallest failing Gauss-point id and reported by
 *     rpim_get_status(); K values of failing points are then undefined.
 *   - Every output is a deterministic function of the inputs: no floating
 *     point atomics, every K entry is summed over contributing Gauss points in
 *     ascending Gauss-point id.  On the FP64 path the result is bitwise equal
 *     to a serial evaluation in the same operation order (correctly rounded
 *     power, IEEE division, explicit fma, no other contraction).
 */
#ifndef RPIM_H
#define RPIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RPIM_OK = 0,
  RPIM_E_ARG = -1,      /* invalid argument                                     */
  RPIM_E_NOMEM = -2,    /* device allocation failed                             */
  RPIM_E_HIP = -3,      /* HIP runtime error                                    */
  RPIM_E_SUPPORT = -4,  /* a Gauss point has fewer than 5 support nodes         */
  RPIM_E_SINGULAR = -5, /* |u_kk| <= N * eps * max|G| during the LU             */
  RPIM_E_RANGE = -6,    /* a size exceeds a documented limit                    */
  RPIM_E_POW = -7,      /* a power could not be rounded correctly (never seen)  */
  RPIM_E_STATE = -8,    /* call order violated (e.g. backward before assemble)  */
  RPIM_E_CONVERGENCE = -9 /* an iteration limit was reached before its tolerance */
} rpim_status;

typedef enum {
  RPIM_FP64 = 0,  /* K is double[nnz]; everything FP64                         */
  RPIM_MIXED = 1  /* K is float[nnz]: FP64 moment matrix + LU, FP32 B^T D B,
                     each entry a compensated (Kahan) FP32 sum in ascending g  */
} rpim_precision;

/* One model, or a block-diagonal batch of independent models.
 * Node, Gauss-point and cell ids are global over the batch; model m owns
 * nodes [node_off[m], node_off[m+1]) and Gauss points [gp_off[m], gp_off[m+1]),
 * and its Gauss points search only its own nodes. */
typedef struct {
  int32_t n_models;             /* >= 1                                              */
  const int64_t* node_off;      /* [host] n_models + 1 prefix offsets (node_off[0] = 0) */
  const int64_t* gp_off;        /* [host] n_models + 1                                */
  int64_t n_cells;              /* number of cells (length of cell_E)                 */
  const double* support_radius; /* [host] d_s per model, > 0                          */
  const double* node_xyz;       /* [N][3] build-time node coordinates                 */
  const double* gp_xyz;         /* [G][3] Gauss-point coordinates                     */
  const double* gp_wdet;        /* [G] Gauss weight * |J| (> 0)                       */
  const int32_t* gp_cell;       /* [G] cell id of each Gauss point, in [0, n_cells)   */
  double alpha_c, d_c, q;       /* MQ basis (r^2 + (alpha_c d_c)^2)^q; all > 0        */
} rpim_problem;

typedef struct rpim_plan rpim_plan; /* opaque; owns device memory for supports etc. */

/* Phases reported by rpim_profile_read (milliseconds of the most recent call
 * that ran the phase, from HIP events recorded on that call's stream). */
enum {
  RPIM_PHASE_PATTERN = 0,    /* support search + pattern (build or rebuild)        */
  RPIM_PHASE_PAIRS = 1,      /* radial basis on node pairs                         */
  RPIM_PHASE_SHAPE = 2,      /* moment matrices, LU, solves (all buckets)          */
  RPIM_PHASE_GATHER = 3,     /* B^T D B reduction into K                           */
  RPIM_PHASE_BWD_ROWS = 4,   /* adjoint: symmetrise dK + row gather                */
  RPIM_PHASE_BWD_GP = 5,     /* adjoint: per-point solves and chain rule           */
  RPIM_PHASE_BWD_REDUCE = 6, /* adjoint: slot reductions to nodes and cells        */
  RPIM_N_PHASES = 7
};

/* Sizes of a built plan (filled by rpim_plan_info). */
typedef struct {
  int64_t n_nodes, n_gp, n_cells, n_models;
  int64_t sum_n;       /* total support entries sum_g |S_g|                       */
  int64_t nnz;         /* scalar nonzeros of K (9 x node-block nonzeros)          */
  int64_t n_blocks;    /* node-block nonzeros                                     */
  int32_t min_n, max_n;/* support sizes                                           */
  int64_t lu_doubles;  /* doubles needed to keep LU factors (keep_factors = 1)    */
  int32_t n_buckets;   /* support-size buckets used by the solver kernels         */
} rpim_info;

/* Create a plan: validates the problem and copies the Gauss-point arrays to
 * plan-owned device memory (so the caller may free theirs).  No kernels run.
 * Returns RPIM_E_ARG for NULL pointers, non-positive sizes or parameters, or
 * offsets that are not non-decreasing and consistent. */
rpim_status rpim_plan_create(const rpim_problem* problem, rpim_plan** plan);

/* Support search and sparsity pattern (one-time per geometry; synchronous).
 *   S_g = { i in model(g) : s_ig <= fl(d_s * d_s) },
 *   s_ig = fma(dz, dz, fma(dy, dy, dx * dx)), d = x_i - x_g per component,
 *   sorted by node id; the node-block pattern is the union of S_g x S_g over g
 *   (symmetric, diagonal included), expanded to scalar CSR with columns sorted.
 * The first call builds the plan's supports and pattern and writes *nnz.
 * When row_ptr and col_idx are non-NULL they are filled:
 *   row_ptr int64[3N + 1], col_idx int32[nnz] (device).
 * Typical use: call once with NULLs to learn nnz, allocate, call again.
 * RPIM_E_SUPPORT if some |S_g| < 5 (rpim_get_status gives the first such g);
 * RPIM_E_RANGE if a support exceeds 132 nodes, a node lies in more than 8192
 * supports, or the node ids in a node's neighbourhood span more than 2^18. */
rpim_status rpim_build_pattern(rpim_plan* plan, int64_t* row_ptr, int32_t* col_idx, int64_t* nnz,
                               void* stream);

/* Re-run the support search and pattern for new node coordinates node_xyz
 * [N][3] (e.g. after the nodes have moved), replacing the plan's supports and
 * pattern and keeping its workspaces where they are large enough.  Same
 * contract, limits and synchronisation as rpim_build_pattern; kept LU factors
 * are invalidated. */
rpim_status rpim_rebuild_pattern(rpim_plan* plan, const double* node_xyz, int64_t* row_ptr, int32_t* col_idx,
                                 int64_t* nnz, void* stream);

/* Stage 1, forward (asynchronous).  node_xyz [N][3] may differ from the
 * build-time coordinates: supports and pattern stay frozen.  cell_E [n_cells],
 * 0 < nu < 0.5 (nu > -1 accepted).  K_vals: double[nnz] (RPIM_FP64) or
 * float[nnz] (RPIM_MIXED), fully overwritten.  keep_factors = 1 keeps the LU
 * factors, pivots and solutions of every Gauss point in plan memory for
 * rpim_assemble_backward (rpim_info.lu_doubles doubles). */
rpim_status rpim_assemble(rpim_plan* plan, const double* node_xyz, const double* cell_E, double nu,
                          int precision, int keep_factors, void* K_vals, void* stream);

/* Adjoint of rpim_assemble (asynchronous).  dK_vals double[nnz] = dL/dK on the
 * pattern (any values, not necessarily symmetric).  Writes dE_cell [n_cells] =
 * dL/dE_c and dX_node [N][3] = dL/dx_i, with Gauss points, weights and supports
 * held fixed.  Reuses the LU factors kept by the last rpim_assemble call with
 * keep_factors = 1 (RPIM_E_STATE otherwise); node_xyz, cell_E and nu must be
 * the ones that call used. */
rpim_status rpim_assemble_backward(rpim_plan* plan, const double* node_xyz, const double* cell_E,
                                   double nu, const double* dK_vals, double* dE_cell, double* dX_node,
                                   void* stream);

/* Stage 2: penalty boundary conditions (GeoMFree3D Sec. 2, stage 2: the
 * constraints are imposed by a penalty on the assembled system, one GPU
 * thread per fixed dof).  alpha = factor * max_i K_ii over all n_dof
 * diagonals (before the update); K_dd += alpha and, if rhs != NULL,
 * rhs_d += alpha * u_bar_d (u_bar may be NULL = zero) for each fixed dof d.
 * K_vals is double or float per `precision`; for float, K_dd += (float)alpha.
 *   fixed_dof int32[n_fixed]: strictly ascending, in [0, n_dof), each with a
 *             diagonal entry in the pattern.  Checked on the device: if the
 *             check fails, K and rhs are left unchanged and *status gets
 *             RPIM_E_ARG (RPIM_OK otherwise).
 *   alpha     device double receiving alpha, or NULL.
 *   status    device int32 receiving the check's result, or NULL.
 *   workspace caller-owned device memory of at least
 *             rpim_penalty_workspace_bytes(n_dof, n_fixed) bytes (8-byte
 *             aligned); it may be reused once the call's kernels are done.
 * Asynchronous: kernels only (no host synchronisation, allocation or memset),
 * so the call can be recorded into a graph.  Argument errors found on the host
 * (NULL pointers, n_dof <= 0, a non-positive factor, a short workspace) return
 * RPIM_E_ARG before anything runs; n_dof > 2^31 - 1 returns RPIM_E_RANGE. */
size_t rpim_penalty_workspace_bytes(int64_t n_dof, int64_t n_fixed);
rpim_status rpim_apply_penalty_bc(const int64_t* row_ptr, const int32_t* col_idx, void* K_vals,
                                  int precision, int64_t n_dof, const int32_t* fixed_dof,
                                  const double* u_bar, int64_t n_fixed, double factor, double* rhs,
                                  double* alpha, int32_t* status, void* workspace, size_t workspace_bytes,
                                  void* stream);

/* After the solve (GeoMFree3D Sec. 2: displacements first, then the stresses;
 * Sec. 3, Example 1: a cube loaded by its own weight).  Asynchronous.
 *
 * rpim_shape_values: phi double[sum_n], entry gp_ptr[g] + a = phi_a(x_g) for
 *   support node a of point g, the first n entries of G_g^-1 [R(x_g); 1, 0, 0, 0]
 *   (the value right-hand side of the moment system), from the LU factors
 *   kept by the last rpim_assemble with keep_factors = 1 (RPIM_E_STATE
 *   otherwise); node_xyz must be the coordinates of that call.
 * rpim_body_force: f double[3N] = sum_g w_g phi_I(x_g) b_g per node I and
 *   component, b_g = gp_force[3g .. 3g+2] the force per unit volume at point g
 *   (device), summed in ascending g; phi from rpim_shape_values.
 * rpim_gauss_stress: sigma double[G][6] = E_c D(nu) eps(u) at every Gauss point
 *   in the order [xx, yy, zz, yz, xz, xy], eps the symmetric gradient of the
 *   nodal displacements u double[3N] through the shape-function gradients of
 *   the last rpim_assemble (RPIM_E_STATE before any). */
rpim_status rpim_shape_values(rpim_plan* plan, const double* node_xyz, double* phi, void* stream);
rpim_status rpim_body_force(rpim_plan* plan, const double* phi, const double* gp_force, double* f, void* stream);
rpim_status rpim_gauss_stress(rpim_plan* plan, const double* cell_E, double nu, const double* u, double* sigma,
                              void* stream);

/* Stage 3: solve K x = rhs (GeoMFree3D Sec. 2, stage 3: the assembled sparse
 * system is solved on the GPU) by conjugate gradients with the Jacobi
 * (diagonal) preconditioner; K symmetric positive definite, e.g. an assembled
 * stiffness after rpim_apply_penalty_bc.
 *   row_ptr int64[n_dof + 1], col_idx int32[nnz] (sorted per row, every row
 *   with a positive diagonal), K_vals double or float per `precision` (float
 *   values are widened exactly); rhs double[n_dof]; x double[n_dof], the
 *   initial guess on entry and the solution on return.
 *   Stops when |rhs - K x| <= rtol |rhs| (2-norms) or after max_iter
 *   iterations.  *iterations and *rel_residual (host, may be NULL) receive the
 *   count and |rhs - K x| / |rhs| of the recursively updated residual.
 *   workspace: caller-owned device memory of rpim_pcg_workspace_bytes(n_dof)
 *   bytes, 256-byte aligned.
 * All vector arithmetic is FP64 and every reduction has a fixed order, so a
 * solve is deterministic.  Synchronous: the host tests convergence every 32
 * iterations.  Returns RPIM_E_CONVERGENCE when max_iter is reached first,
 * RPIM_E_SINGULAR when a diagonal is not positive or p.Kp <= 0 (x then holds
 * the last iterate), RPIM_E_ARG for bad arguments. */
size_t rpim_pcg_workspace_bytes(int64_t n_dof);
rpim_status rpim_solve_pcg(const int64_t* row_ptr, const int32_t* col_idx, const void* K_vals, int precision,
                           int64_t n_dof, const double* rhs, double* x, double rtol, int64_t max_iter,
                           void* workspace, size_t workspace_bytes, int64_t* iterations, double* rel_residual,
                           void* stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): rpim_apply_penalty_bc
 * with the library's own device scratch in place of the workspace; the same
 * kernels, arguments, outputs and device-side check.  The scratch is a static
 * array of about 2 MB per GPU (held until the process ends), so n_fixed may be
 * at most RPIM_PENALTY_NOALLOC_MAX_FIXED (RPIM_E_RANGE beyond, before anything
 * runs).  Every call on one GPU uses that GPU's scratch: calls that overlap on
 * one GPU (other streams, other threads) race and must be serialised by the
 * caller.  Nothing in the scratch needs clearing between calls. */
#define RPIM_PENALTY_NOALLOC_MAX_FIXED (1 << 18)
rpim_status rpim_apply_penalty_bc_noalloc(const int64_t* row_ptr, const int32_t* col_idx, void* K_vals,
                                          int precision, int64_t n_dof, const int32_t* fixed_dof,
                                          const double* u_bar, int64_t n_fixed, double factor, double* rhs,
                                          double* alpha, int32_t* status, void* stream);

/* Launch-configuration tuning (synchronous).  Kept LU factors are invalidated.
 * For every support-size bucket it times the moment-matrix solver kernels
 * that can hold the bucket (RPIM_SOLVER_WINDOW, RPIM_SOLVER_PANEL; the LDS
 * kernel beyond them) and keeps the fastest for the bucket; then it times the
 * row gather of `precision` with 1, 2, 3 and 4 waves per node row and keeps
 * the fastest.  Every configuration computes the same bits; only speed differs.
 * K_vals (nnz values of the precision's type) serves as scratch and is
 * overwritten.  The choices go to a process-wide cache keyed by (GPU
 * architecture, precision, bucket size) and (architecture, precision); when
 * the cache already holds every choice this plan needs, they are applied and
 * nothing is timed (from_cache = 1).  `out` may be NULL.  Supports and pattern
 * must be built (RPIM_E_STATE otherwise). */
#define RPIM_TUNING_MAX_BUCKETS 32
typedef struct {
  int32_t gather_waves;                          /* chosen: 1, 2, 3 or 4           */
  float gather_ms[4];                            /* row gather with 1 to 4 waves   */
  int32_t n_buckets;                             /* buckets reported (<= 32)       */
  int32_t bucket_nmax[RPIM_TUNING_MAX_BUCKETS];  /* padded size N of each bucket   */
  int64_t bucket_points[RPIM_TUNING_MAX_BUCKETS];
  float bucket_ms[RPIM_TUNING_MAX_BUCKETS];      /* solver time, chosen kernel     */
  int32_t bucket_solver[RPIM_TUNING_MAX_BUCKETS];   /* chosen RPIM_SOLVER_*        */
  float bucket_ms_window[RPIM_TUNING_MAX_BUCKETS];  /* each candidate (-1: not run) */
  float bucket_ms_panel[RPIM_TUNING_MAX_BUCKETS];
  int32_t from_cache;                            /* 1: choices from the cache      */
} rpim_tuning;
rpim_status rpim_autotune(rpim_plan* plan, const double* node_xyz, const double* cell_E, double nu, int precision,
                          void* K_vals, void* stream, rpim_tuning* out);
/* The tuning cache as text lines "arch precision what nmax value" (what =
 * solver or gather).  Loading adds to the cache (RPIM_E_ARG for an unreadable
 * file or a malformed line); clearing empties it. */
rpim_status rpim_tuning_cache_save(const char* path);
rpim_status rpim_tuning_cache_load(const char* path);
void rpim_tuning_cache_clear(void);
/* Set the row-gather configuration (1, 2, 3 or 4 waves per node row) for
 * `precision` by hand, as rpim_autotune would; RPIM_E_ARG otherwise. */
rpim_status rpim_set_gather_waves(rpim_plan* plan, int precision, int waves);

/* Moment-matrix solver kernel of the support-size bucket holding padded size
 * nmax = n + 4 (nmax = 0: every bucket).  Every kernel computes the same bits
 * (the elimination order of the arithmetic contract); only speed differs.
 *   RPIM_SOLVER_AUTO   the library's choice (default)
 *   RPIM_SOLVER_LDS    the whole augmented matrix in LDS (any size up to 136)
 *   RPIM_SOLVER_WINDOW one matrix row per thread in registers, eliminated one
 *                      pivot step at a time (N <= 104)
 *   RPIM_SOLVER_PANEL  rows in registers, blocked elimination: sixteen pivot
 *                      steps on a panel, then one trailing update (N <= 96)
 * Buckets a kernel cannot hold fall back to the window kernel, then to the
 * LDS kernel.  RPIM_E_ARG for an unknown kind or nmax outside [0, 136]. */
enum { RPIM_SOLVER_AUTO = 0, RPIM_SOLVER_LDS = 1, RPIM_SOLVER_WINDOW = 2, RPIM_SOLVER_PANEL = 3 };
rpim_status rpim_set_solver(rpim_plan* plan, int nmax, int kind);

/* Shape functions of the plan (GeoMFree3D Sec. 4 names moving least squares
 * as the package's next shape functions):
 *   RPIM_SHAPE_RPIM     radial point interpolation (default; the path above)
 *   RPIM_SHAPE_MLS      moving least squares, linear basis [1, x - x_g]
 *   RPIM_SHAPE_SHEPARD  Shepard's functions (moving least squares with the
 *                       constant basis)
 * Both moving-least-squares kinds use the cubic-spline weight over the
 * support radius (one radius for the whole plan, else RPIM_E_ARG from
 * rpim_assemble) and the supports of the plan; rpim_assemble then forms the
 * gradients with one 4 x 4 (or 1 x 1) moment matrix per Gauss point instead
 * of the RPIM solve, and assembles K from them exactly as for RPIM.  With
 * these kinds keep_factors has no effect, rpim_assemble_backward returns
 * RPIM_E_STATE, and rpim_shape_values evaluates the values directly (no kept
 * factors needed).  Changing the kind drops kept factors.  RPIM_E_ARG for an
 * unknown kind. */
enum { RPIM_SHAPE_RPIM = 0, RPIM_SHAPE_MLS = 1, RPIM_SHAPE_SHEPARD = 2 };
rpim_status rpim_set_shape_functions(rpim_plan* plan, int kind);

/* Identifier of the LU factors the plan currently keeps for the backward: a
 * new positive value after each rpim_assemble with keep_factors = 1, 0 once
 * they are gone (an assembly without keep_factors, rpim_autotune or
 * rpim_rebuild_pattern overwrite the state they belong to).  A caller that
 * saves it at the forward can check, before rpim_assemble_backward, that the
 * factors still belong to that forward. */
rpim_status rpim_factor_generation(const rpim_plan* plan, int64_t* gen);

/* Synchronise `stream` and report device-side errors of the plan's last calls:
 * the most severe status and the smallest failing Gauss-point id (-1 if none).
 * Clears the record. */
rpim_status rpim_get_status(rpim_plan* plan, void* stream, int64_t* first_bad_gp);

rpim_status rpim_plan_info(const rpim_plan* plan, rpim_info* info);

/* Enable (1) or disable (0) per-phase event timing for later calls on this
 * plan; rpim_profile_read synchronises on the recorded events and writes
 * RPIM_N_PHASES values in milliseconds to ms (host), -1 for phases not run
 * since timing was enabled. */
rpim_status rpim_profile_enable(rpim_plan* plan, int enable);
rpim_status rpim_profile_read(rpim_plan* plan, double* ms);

/* Copies of plan state for inspection and tests (device outputs, async):
 * supports gp_ptr int64[G+1], gp_nbr int32[sum_n]; shape-function gradients
 * of the last assembly dphi double[sum_n][3]. */
rpim_status rpim_get_support(const rpim_plan* plan, int64_t* gp_ptr, int32_t* gp_nbr, void* stream);
rpim_status rpim_get_dphi(const rpim_plan* plan, double* dphi, void* stream);

/* Correctly rounded x^q for n device doubles x > 0 (the kernel the assembly
 * uses for the radial basis), for tests of the rounding contract. */
rpim_status rpim_pow_cr(const double* x, double q, double* y, int64_t n, void* stream);

void rpim_plan_destroy(rpim_plan* plan);
const char* rpim_status_string(rpim_status status);

#ifdef __cplusplus
}
#endif
#endif /* RPIM_H */
