#!/usr/bin/env python3
"""Benchmark of the RPIM stiffness-assembly hot path on one MI355X.

A step is one pass of the whole path over the jittered slope workload
(40 x 20 x 20 m trapezoidal prism, 18,081 nodes, 432,000 Gauss points,
lognormal E), inputs resident in HBM:
  support search + pattern (rebuilt every step), FP64 assembly of K with the
  LU factors kept, penalty boundary conditions on the base, and the adjoint
  dL/dK -> dL/dE, dL/dx for L = sum_v 0.5 v^T K v (8 probe vectors).
value = Gauss points per second over the step.  Extra fields report the
per-phase times (HIP events recorded by the library on the launch stream),
assembly-only throughput in FP64 and mixed precision, the backward/forward
ratio, the roofline of the dominant kernel and the CPU oracle on a bounded
sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps 5] [--warmup 2]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gauss pts assembled/s + HBM GB/s, plain FP64 vs mixed/batched; bwd/fwd time"
PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector (and matrix) peak
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E

# HBM bytes moved by all moment-matrix kernel launches (k_shape*) of one step: FETCH_SIZE and WRITE_SIZE
# counter runs of this script, each scaled by what the same counter reads for one streaming kernel that
# reads and writes 1 GiB (fetch x2.000, write x1.000).  The summary and its commands are in profiles/.  The figure belongs to
# the kernel sources it was measured on: any change to them reports traffic as null until re-measured.
SHAPE_SOURCES = ("paper_1802_04256_amd/csrc/shape_reg.hip", "paper_1802_04256_amd/csrc/shape_panel.hip",
                 "paper_1802_04256_amd/csrc/shape_common.h", "paper_1802_04256_amd/csrc/assemble.hip",
                 "paper_1802_04256_amd/csrc/dd_pow.h", "paper_1802_04256_amd/csrc/rpim_internal.h")
SHAPE_TRAFFIC = {"sources_sha256": "90b710f08be523e5b1f00673ce29976ca79023937c17c25562ef6d457a5018f4", "bytes_per_step": 3.4496e10}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def shape_flops(n):
    """Algorithmic FP64 flops of the per-point moment solve: LU (2/3 N^3) + 3 RHS solves (6 N^2), N = n + 4."""
    import numpy as np
    N = n.astype(np.float64) + 4.0
    return float(np.sum(2.0 / 3.0 * N ** 3 + 6.0 * N ** 2))


def shape_traffic():
    """Measured HBM bytes per step of the moment-matrix kernels, or None if their sources changed since."""
    import hashlib
    h = hashlib.sha256()
    for f in SHAPE_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return SHAPE_TRAFFIC["bytes_per_step"] if h.hexdigest() == SHAPE_TRAFFIC["sources_sha256"] else None


def displacement_error(prob, row_ptr, col_idx, K64, K32, factor=1e8):
    """Relative displacement error of the mixed-precision K after a solve.

    Base nodes fixed by the penalty method (as in the benchmark step), a unit
    downward force on every node of the top surface.  u64 solves K64 u = f;
    since K32 u32 = f, u32 - u64 = K32^-1 (K64 - K32) u64 exactly, which is
    solved directly (its accuracy then does not depend on how far u64 is
    converged).  Both solves are the library's Jacobi-preconditioned CG on the
    GPU.  K64 and K32 are modified in place by the penalty update."""
    import numpy as np
    import torch
    import paper_1802_04256_amd as rp
    dev = K64.device
    X = prob.node_xyz
    base = np.where(X[:, 2] == X[:, 2].min())[0]
    fixed = torch.from_numpy(np.sort((3 * base[:, None] + np.arange(3)).ravel()).astype(np.int32)).to(dev)
    rp.apply_penalty_bc(row_ptr, col_idx, K64, fixed, factor=factor)
    rp.apply_penalty_bc(row_ptr, col_idx, K32, fixed, factor=factor)
    top = np.where(X[:, 2] == X[:, 2].max())[0]
    f = torch.zeros(3 * prob.n_nodes, dtype=torch.float64, device=dev)
    f[torch.from_numpy(3 * top + 2).to(dev)] = -1.0
    t0 = time.perf_counter()
    u64, it64, res64 = rp.solve_pcg(row_ptr, col_idx, K64, f, rtol=1e-10)
    t_solve = time.perf_counter() - t0
    n = 3 * prob.n_nodes
    A64 = torch.sparse_csr_tensor(row_ptr, col_idx.long(), K64, size=(n, n))
    A32 = torch.sparse_csr_tensor(row_ptr, col_idx.long(), K32.double(), size=(n, n))
    d = torch.mv(A64, u64) - torch.mv(A32, u64)
    del A64, A32
    du, it32, res32 = rp.solve_pcg(row_ptr, col_idx, K32, d, rtol=1e-6)
    return {"u_rel_err": float(torch.linalg.norm(du) / torch.linalg.norm(u64)), "cg_iters": [it64, it32],
            "cg_rel_residual": [res64, res32], "solve_s": t_solve,
            "load": "unit downward force on each top-surface node; base fixed by penalty 1e8 x max diag",
            "solver": "rpim_solve_pcg (Jacobi-preconditioned CG, FP64 vectors)"}


def graph_timing(fn, reps=5):
    """Capture fn once in a HIP graph (after an eager call), replay it reps times; median, min, max in seconds."""
    import numpy as np
    import torch
    fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    g.replay()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = time.perf_counter()
        g.replay()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - a)
    del g
    return float(np.median(ts)), float(min(ts)), float(max(ts))


def batched_leg():
    """64 independent jittered slopes (log-uniform 1k-30k nodes) in one plan, launch configuration tuned on
    it: the whole assembly (pair table, one launch per support-size bucket, row gather) captured in one HIP
    graph and replayed, in mixed precision and in FP64 on the same batch and in the same launch mode."""
    import torch

    import paper_1802_04256_amd as rp
    import workloads as W
    dev = torch.device("cuda:0")
    prob = W.named("batch64")
    log(f"batched: models={prob.n_models} nodes={prob.n_nodes} gps={prob.n_gp}")
    plan = rp.Plan.from_problem(prob, device=dev)
    plan.build_pattern()
    info = plan.info()
    X = torch.from_numpy(prob.node_xyz).to(dev)
    E = torch.from_numpy(prob.cell_E).to(dev)
    K32 = torch.empty(plan.nnz, dtype=torch.float32, device=dev)
    K64 = torch.empty(plan.nnz, dtype=torch.float64, device=dev)
    tuned = {"mixed": plan.autotune(X, E, prob.nu, rp.MIXED, out=K32)["gather_waves"],
             "fp64": plan.autotune(X, E, prob.nu, rp.FP64, out=K64)["gather_waves"]}
    t32 = graph_timing(lambda: plan.assemble(X, E, prob.nu, rp.MIXED, out=K32))
    t64 = graph_timing(lambda: plan.assemble(X, E, prob.nu, rp.FP64, out=K64))
    plan.status()
    err = float(torch.linalg.norm(K32.double() - K64) / torch.linalg.norm(K64))
    res = {"workload": "64 jittered slopes, log-uniform 1k-30k nodes (seed 4), lognormal E, one block-diagonal plan",
           "n_models": prob.n_models, "n_nodes": prob.n_nodes, "n_gp": prob.n_gp, "nnz": info["nnz"],
           "sum_n": info["sum_n"], "buckets": info["n_buckets"], "launch": "one HIP graph per precision, replayed",
           "ms": {"mixed": t32[0] * 1e3, "fp64": t64[0] * 1e3},
           "ms_min_max": {"mixed": [t32[1] * 1e3, t32[2] * 1e3], "fp64": [t64[1] * 1e3, t64[2] * 1e3]},
           "gp_per_s": {"mixed": prob.n_gp / t32[0], "fp64": prob.n_gp / t64[0]},
           "mixed_vs_fp64_same_batch": t64[0] / t32[0],
           "mixed_rel_fro_err": err, "gather_waves": tuned}
    log(f"batched: mixed {t32[0] * 1e3:.1f} ms [{t32[1] * 1e3:.1f}, {t32[2] * 1e3:.1f}], fp64 {t64[0] * 1e3:.1f} ms "
        f"[{t64[1] * 1e3:.1f}, {t64[2] * 1e3:.1f}], err {err:.2e}")
    return res


def large_leg():
    """The 3-layer slope at 250k nodes (100 x 50 x 50 m, 262,701 nodes, 6,750,000 Gauss points): assembly
    throughput in FP64 and mixed precision (HIP graph replays), the mixed K error, and the displacement
    error of the mixed K after a GPU solve."""
    import torch

    import paper_1802_04256_amd as rp
    import workloads as W
    dev = torch.device("cuda:0")
    prob = W.named("slope_large")
    log(f"large: nodes={prob.n_nodes} gps={prob.n_gp}")
    plan = rp.Plan.from_problem(prob, device=dev)
    t0 = time.perf_counter()
    plan.build_pattern()
    t_pat = time.perf_counter() - t0
    info = plan.info()
    X = torch.from_numpy(prob.node_xyz).to(dev)
    E = torch.from_numpy(prob.cell_E).to(dev)
    K32 = torch.empty(plan.nnz, dtype=torch.float32, device=dev)
    K64 = torch.empty(plan.nnz, dtype=torch.float64, device=dev)
    plan.autotune(X, E, prob.nu, rp.MIXED, out=K32)
    plan.autotune(X, E, prob.nu, rp.FP64, out=K64)
    t32 = graph_timing(lambda: plan.assemble(X, E, prob.nu, rp.MIXED, out=K32), reps=3)
    t64 = graph_timing(lambda: plan.assemble(X, E, prob.nu, rp.FP64, out=K64), reps=3)
    plan.status()
    err = float(torch.linalg.norm(K32.double() - K64) / torch.linalg.norm(K64))
    log(f"large: mixed {t32[0] * 1e3:.1f} ms, fp64 {t64[0] * 1e3:.1f} ms, K err {err:.2e}; solving ...")
    disp = displacement_error(prob, plan.row_ptr, plan.col_idx, K64, K32)
    log(f"large: displacement error {disp['u_rel_err']:.2e} (CG iterations {disp['cg_iters']})")
    return {"workload": "3-layer jittered slope 100x50x50 m (E = 300 / 80 / 20 MPa), 262,701 nodes, 6,750,000 "
                        "Gauss points", "n_gp": prob.n_gp, "nnz": info["nnz"], "sum_n": info["sum_n"],
            "pattern_s": t_pat, "ms": {"mixed": t32[0] * 1e3, "fp64": t64[0] * 1e3},
            "ms_min_max": {"mixed": [t32[1] * 1e3, t32[2] * 1e3], "fp64": [t64[1] * 1e3, t64[2] * 1e3]},
            "gp_per_s": {"mixed": prob.n_gp / t32[0], "fp64": prob.n_gp / t64[0]},
            "mixed_vs_fp64": t64[0] / t32[0], "mixed_rel_fro_err": err, "mixed_displacement": disp}


def host_info():
    """CPU model, logical CPUs and the CPUs this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "cpus_available": avail}


def software_info():
    import torch
    return {"torch": torch.__version__, "hip": getattr(torch.version, "hip", None), "python": sys.version.split()[0]}


def cpu_baseline(prob, cell_stride, n_vec=8):
    """Oracle (serial, one core) on the Gauss points of every cell_stride-th cell of the workload,
    spread over the whole domain: support search, pattern, FP64 assembly and adjoint, scaled to Gauss
    points per second."""
    import numpy as np

    import oracle
    import workloads as W
    cells = np.arange(0, prob.n_cells, cell_stride)
    gps = np.nonzero(np.isin(prob.gp_cell, cells))[0]
    sub = W.Problem(name="sample", node_xyz=prob.node_xyz, gp_xyz=prob.gp_xyz[gps], gp_wdet=prob.gp_wdet[gps],
                    gp_cell=prob.gp_cell[gps], cell_E=prob.cell_E, nu=prob.nu,
                    support_radius=prob.support_radius, alpha_c=prob.alpha_c, d_c=prob.d_c, q=prob.q)
    oracle.lib()
    t0 = time.perf_counter()
    m = oracle.OracleModel(sub)
    m.build_pattern()
    m.assemble()
    rp_, ci = m.pattern()
    V = W.probe_vectors(3 * prob.n_nodes, n_vec, 5)
    rows = np.repeat(np.arange(len(rp_) - 1), np.diff(rp_))
    Kb = 0.5 * np.einsum("vi,vi->i", V[:, rows], V[:, ci])
    m.backward(Kb)
    dt = time.perf_counter() - t0
    gp_ptr, _ = m.support()
    n = np.diff(gp_ptr)
    return {"value": len(gps) / dt, "unit": "GP/s", "cores": 1, "kind": "oracle", **host_info(),
            "sample": f"the {len(gps)} Gauss points of every {cell_stride}th cell ({len(cells)} cells spread over the "
                      f"slope; mean support {n.mean():.1f} nodes against {prob.meta.get('mean_support', 'n/a')} over "
                      f"the whole slope): oracle support search + pattern + FP64 assembly + adjoint, {dt:.1f} s "
                      f"serial on one core (the O(dofs) penalty update is left out)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-cell-stride", type=int, default=157,
                    help="the oracle's timed sample: the Gauss points of every N-th cell")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the assembly-only / mixed measurements")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-model batched assembly")
    ap.add_argument("--no-large", action="store_true", help="skip the 250k-node slope")
    ap.add_argument("--solver-probe", default="", metavar="KINDS",
                    help="profiling aid: one FP64 assembly of the workload per solver kernel in this comma-separated "
                         "list (window, panel, lds), then exit without timing")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MiB",
                    help="before the steps, run one device fill and one device copy of this many MiB "
                         "(a known-size reference for the HBM byte counters of a profiler)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this library runs each model (or batch of models) on a single "
              "MI355X; multi-GPU sharding is a design note, not a measured path. Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1802_04256_amd as rp
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    prob = W.slope()
    log(f"workload slope: nodes={prob.n_nodes} gps={prob.n_gp} cells={prob.n_cells}")
    X = torch.from_numpy(prob.node_xyz).to(dev)
    E = torch.from_numpy(prob.cell_E).to(dev)
    plan = rp.Plan.from_problem(prob, device=dev)
    row_ptr, col_idx = plan.build_pattern()
    info = plan.info()
    log(f"pattern: nnz={info['nnz']} sum_n={info['sum_n']} n={info['min_n']}..{info['max_n']} "
        f"buckets={info['n_buckets']}")
    if args.solver_probe:
        Kp = torch.empty(plan.nnz, dtype=torch.float64, device=dev)
        for kind in args.solver_probe.split(","):
            plan.set_solver(kind)
            plan.assemble(X, E, prob.nu, rp.FP64, out=Kp)
            torch.cuda.synchronize()
            log(f"solver probe: {kind} assembly done")
        plan.status()
        return
    # probe-vector adjoint seed on the pattern: dL/dK_ij = 0.5 sum_v v_i v_j
    V = torch.from_numpy(W.probe_vectors(3 * prob.n_nodes, 8, 5)).to(dev)
    rows = torch.repeat_interleave(torch.arange(3 * prob.n_nodes, device=dev), torch.diff(row_ptr))
    dK = 0.5 * (V[:, rows] * V[:, col_idx.long()]).sum(0)
    del rows
    # launch-configuration tuning on this plan (setup, untimed; results are unchanged by it)
    Ktmp = torch.empty(plan.nnz, dtype=torch.float64, device=dev)
    tuning = {"fp64": plan.autotune(X, E, prob.nu, rp.FP64, out=Ktmp)}
    tuning["mixed"] = plan.autotune(X, E, prob.nu, rp.MIXED, out=torch.empty(plan.nnz, dtype=torch.float32,
                                                                               device=dev))
    del Ktmp
    log(f"autotune: gather waves fp64 {tuning['fp64']['gather_waves']} {tuning['fp64']['gather_ms']}, "
        f"mixed {tuning['mixed']['gather_waves']} {tuning['mixed']['gather_ms']}")
    Xh = prob.node_xyz
    fixed = np.where(Xh[:, 2] == Xh[:, 2].min())[0]
    fixed = torch.from_numpy(np.sort((3 * fixed[:, None] + np.arange(3)).ravel()).astype(np.int32)).to(dev)

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        # one streaming kernel that reads and writes nbytes each (negation: a kernel name of its own)
        src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
        log(f"copy calibration: neg kernel reads {nbytes} B, writes {nbytes} B")

    def step():
        plan.rebuild_pattern(X)
        K = plan.assemble(X, E, prob.nu, rp.FP64, keep_factors=True)
        rp.apply_penalty_bc(plan.row_ptr, plan.col_idx, K, fixed, factor=1e8, check=False)
        plan.assemble_backward(X, E, prob.nu, dK)
        return K

    for i in range(args.warmup):
        step()
        log(f"warmup step {i + 1}/{args.warmup} done")
    plan.status()
    plan.profile(True)
    phase_sum = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        for k, v in plan.profile_read().items():
            phase_sum[k] = phase_sum.get(k, 0.0) + v
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.profile(False)
    plan.status()
    ms_step = (t1 - t0) * 1e3 / args.steps
    phases = {k: v / args.steps for k, v in phase_sum.items()}
    log(f"timed {args.steps} steps: {ms_step:.2f} ms/step; phases {json.dumps({k: round(v, 3) for k, v in phases.items()})}")

    gp_ptr, _ = plan.support()
    n = np.diff(gp_ptr.cpu().numpy())
    flops = shape_flops(n)
    shape_ms = phases["shape"]
    achieved = flops / (shape_ms * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": prob.n_gp / (ms_step * 1e-3),
        "unit": "GP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "jittered slope 40x20x20 m, 1 m spacing, 18,081 nodes, 432,000 Gauss points "
                               "(3^3 per cell), lognormal E, d_s = 2.5 m, MQ alpha_c = 4, q = 1.03",
                   "n_nodes": prob.n_nodes, "n_gp": prob.n_gp, "nnz": info["nnz"], "sum_n": info["sum_n"],
                   "step": "pattern + FP64 assembly (factors kept) + penalty BCs + adjoint"},
        "phases_ms": {k: round(v, 4) for k, v in phases.items()},
        "tuning": {k: {"gather_waves": v["gather_waves"], "gather_ms": v["gather_ms"],
                       "solver_ms_by_bucket": {b["nmax"]: round(b["ms"], 3) for b in v["buckets"]}}
                   for k, v in tuning.items()},
        "roofline": {"kernel": "k_shape (moment matrix + LU + 3 solves, all buckets)", "bound": "alu",
                     "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": shape_traffic(),
                     "flops_per_step": flops, "launches_per_step": info["n_buckets"],
                     "ms_per_step": shape_ms},
        "software": software_info(),
    }

    if not args.no_extras:
        def timed(fn, reps=3):
            fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                torch.cuda.synchronize()
                a = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - a)
            return float(np.median(ts))
        Kout = torch.empty(plan.nnz, dtype=torch.float64, device=dev)
        K32 = torch.empty(plan.nnz, dtype=torch.float32, device=dev)
        t_fp64 = timed(lambda: plan.assemble(X, E, prob.nu, rp.FP64, out=Kout))
        t_mixed = timed(lambda: plan.assemble(X, E, prob.nu, rp.MIXED, out=K32))
        t_fwd_keep = timed(lambda: plan.assemble(X, E, prob.nu, rp.FP64, keep_factors=True, out=Kout))
        t_bwd = timed(lambda: plan.assemble_backward(X, E, prob.nu, dK))
        t_pat = timed(lambda: plan.rebuild_pattern(X), reps=2)
        err32 = float(torch.linalg.norm(K32.double() - Kout) / torch.linalg.norm(Kout))
        out["assemble_gp_per_s"] = {"fp64": prob.n_gp / t_fp64, "mixed": prob.n_gp / t_mixed}
        out["assemble_ms"] = {"fp64": t_fp64 * 1e3, "mixed": t_mixed * 1e3, "fp64_keep_factors": t_fwd_keep * 1e3,
                              "backward": t_bwd * 1e3, "pattern": t_pat * 1e3}
        out["bwd_fwd"] = t_bwd / t_fwd_keep
        out["mixed_rel_fro_err"] = err32
        plan.assemble(X, E, prob.nu, rp.FP64, out=Kout)
        out["mixed_displacement"] = displacement_error(prob, plan.row_ptr, plan.col_idx, Kout, K32)
        log(f"mixed displacement error {out['mixed_displacement']['u_rel_err']:.3e} "
            f"(CG iterations {out['mixed_displacement']['cg_iters']})")
        # algorithmic HBM bytes of one FP64 assembly: K values written once, dphi written
        # and read once, supports / inverse lists / pattern read once
        sum_n = info["sum_n"]
        alg_bytes = info["nnz"] * 8 + sum_n * 24 * 2 + sum_n * (4 + 8) + info["n_blocks"] * 4 * 2
        out["hbm_gbps_fp64_assembly"] = alg_bytes / t_fp64 / 1e9
        log(f"assemble fp64 {t_fp64 * 1e3:.2f} ms, mixed {t_mixed * 1e3:.2f} ms (err {err32:.2e}), "
            f"bwd {t_bwd * 1e3:.2f} ms, bwd/fwd {out['bwd_fwd']:.2f}")
        # the same slope with moving-least-squares and Shepard shape functions (same supports, same
        # gather); the gradient kernel's algorithmic bytes: per support entry the node id, its
        # coordinates and the gradient written, per point its support range and coordinates
        shapes = {}
        mls_bytes = sum_n * (4 + 24 + 24) + prob.n_gp * (16 + 24)
        plan.profile(True)
        for kind in ("mls", "shepard"):
            plan.set_shape_functions(kind)
            t64 = timed(lambda: plan.assemble(X, E, prob.nu, rp.FP64, out=Kout))
            kshape = plan.profile_read()["shape"]
            t32 = timed(lambda: plan.assemble(X, E, prob.nu, rp.MIXED, out=K32))
            shapes[kind] = {"assemble_ms": {"fp64": t64 * 1e3, "mixed": t32 * 1e3},
                            "assemble_gp_per_s": {"fp64": prob.n_gp / t64, "mixed": prob.n_gp / t32},
                            "gradient_kernel_ms": kshape,
                            "gradient_kernel_gbps": mls_bytes / (kshape * 1e-3) / 1e9,
                            "mixed_rel_fro_err": float(torch.linalg.norm(K32.double() - Kout.double()) /
                                                       torch.linalg.norm(Kout))}
            log(f"{kind}: assemble fp64 {t64 * 1e3:.2f} ms, gradients {kshape:.3f} ms")
        plan.profile(False)
        plan.set_shape_functions("rpim")
        out["shape_functions"] = shapes

    if not args.no_extras and not args.no_batched:
        out["batched"] = batched_leg()
    if not args.no_extras and not args.no_large:
        out["large"] = large_leg()

    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        prob.meta["mean_support"] = round(float(info["sum_n"]) / prob.n_gp, 1)
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_cell_stride)
        log(f"cpu baseline {out['cpu_baseline']['value']:.1f} GP/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
