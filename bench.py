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
# counter runs of this script, each scaled by what the same counter reads for a plain 1 GiB device copy
# (fetch x2.000, write x1.000).  The summary and its commands are in profiles/.  The figure belongs to
# the kernel sources it was measured on: any change to them reports traffic as null until re-measured.
SHAPE_SOURCES = ("paper_1802_04256_amd/csrc/shape_reg.hip", "paper_1802_04256_amd/csrc/assemble.hip",
                 "paper_1802_04256_amd/csrc/dd_pow.h", "paper_1802_04256_amd/csrc/rpim_internal.h")
SHAPE_TRAFFIC = {"sources_sha256": "3cdd9b187e9f4577b3e909845dd5c40721d78f462ff639176c2fc55c40b49cd8", "bytes_per_step": 3.903e10}


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


def csr_operator(row_ptr, col_idx, vals):
    """x -> K x for a CSR matrix on the GPU, in float64 (float32 values are widened exactly)."""
    import torch
    n = row_ptr.numel() - 1
    A = torch.sparse_csr_tensor(row_ptr, col_idx.to(torch.int64), vals.to(torch.float64), size=(n, n))
    return lambda x: torch.mv(A, x)


def pcg(A, b, dinv, rtol, maxit=50000):
    """Jacobi-preconditioned conjugate gradients; returns (x, iterations, relative residual)."""
    import torch
    x = torch.zeros_like(b)
    r = b.clone()
    z = dinv * r
    p = z.clone()
    rz = torch.dot(r, z)
    bn = float(torch.linalg.norm(b))
    it, rel = 0, 1.0
    for it in range(1, maxit + 1):
        Ap = A(p)
        alpha = rz / torch.dot(p, Ap)
        x += alpha * p
        r -= alpha * Ap
        rel = float(torch.linalg.norm(r)) / bn
        if rel <= rtol:
            break
        z = dinv * r
        rz_new = torch.dot(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, rel


def displacement_error(prob, row_ptr, col_idx, K64, K32, factor=1e8):
    """Relative displacement error of the mixed-precision K after a solve.

    Base nodes fixed by the penalty method (as in the benchmark step), a unit
    downward force on every node of the top surface.  u64 solves K64 u = f;
    since K32 u32 = f, u32 - u64 = K32^-1 (K64 - K32) u64 exactly, which is
    solved directly (its accuracy then does not depend on how far u64 is
    converged).  K64 and K32 are modified in place by the penalty update."""
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
    rows = torch.repeat_interleave(torch.arange(3 * prob.n_nodes, device=dev), torch.diff(row_ptr))
    diag = torch.zeros_like(f).index_add_(0, rows, torch.where(rows == col_idx.long(), K64, 0.0))
    del rows
    A64 = csr_operator(row_ptr, col_idx, K64)
    A32 = csr_operator(row_ptr, col_idx, K32)
    u64, it64, res64 = pcg(A64, f, 1.0 / diag, 1e-10)
    d = A64(u64) - A32(u64)
    du, it32, res32 = pcg(A32, d, 1.0 / diag, 1e-6)
    return {"u_rel_err": float(torch.linalg.norm(du) / torch.linalg.norm(u64)), "cg_iters": [it64, it32],
            "cg_rel_residual": [res64, res32],
            "load": "unit downward force on each top-surface node; base fixed by penalty 1e8 x max diag"}


def batched_leg(plain_fp64_gp_s):
    """64 independent jittered slopes (log-uniform 1k-30k nodes) in one plan, launch configuration tuned on
    it: one HIP graph holding the whole mixed-precision assembly (pair table, one launch per support-size
    bucket, row gather), replayed; the same batch assembled eagerly in FP64 beside it."""
    import numpy as np
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
    tuned = plan.autotune(X, E, prob.nu, rp.MIXED, out=K32)
    plan.assemble(X, E, prob.nu, rp.MIXED, out=K32)
    torch.cuda.synchronize()
    plan.status()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.assemble(X, E, prob.nu, rp.MIXED, out=K32)

    def timed(fn, reps=3):
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            a = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - a)
        return float(np.median(ts))
    t_graph = timed(graph.replay)
    del graph
    K64 = torch.empty(plan.nnz, dtype=torch.float64, device=dev)
    plan.autotune(X, E, prob.nu, rp.FP64, out=K64)
    plan.assemble(X, E, prob.nu, rp.FP64, out=K64)
    t_fp64 = timed(lambda: plan.assemble(X, E, prob.nu, rp.FP64, out=K64))
    plan.assemble(X, E, prob.nu, rp.MIXED, out=K32)
    err = float(torch.linalg.norm(K32.double() - K64) / torch.linalg.norm(K64))
    plan.status()
    res = {"workload": "64 jittered slopes, log-uniform 1k-30k nodes (seed 4), lognormal E, one block-diagonal plan",
           "n_models": prob.n_models, "n_nodes": prob.n_nodes, "n_gp": prob.n_gp, "nnz": info["nnz"],
           "sum_n": info["sum_n"], "buckets": info["n_buckets"],
           "ms": {"mixed_graph": t_graph * 1e3, "fp64_eager": t_fp64 * 1e3},
           "gp_per_s": {"mixed_graph": prob.n_gp / t_graph, "fp64_eager": prob.n_gp / t_fp64},
           "mixed_rel_fro_err": err, "gather_waves_mixed": tuned["gather_waves"]}
    if plain_fp64_gp_s:
        res["mixed_graph_vs_plain_fp64_slope"] = res["gp_per_s"]["mixed_graph"] / plain_fp64_gp_s
    log(f"batched: mixed graph {t_graph * 1e3:.1f} ms, fp64 {t_fp64 * 1e3:.1f} ms, err {err:.2e}")
    return res


def cpu_baseline(prob, n_sample, n_vec=8):
    """Oracle (serial, one core) on the first n_sample Gauss points of the workload:
    pattern, FP64 assembly, penalty and adjoint, scaled to Gauss points per second."""
    import numpy as np

    import oracle
    import workloads as W
    sub = W.Problem(name="sample", node_xyz=prob.node_xyz, gp_xyz=prob.gp_xyz[:n_sample],
                    gp_wdet=prob.gp_wdet[:n_sample], gp_cell=prob.gp_cell[:n_sample], cell_E=prob.cell_E,
                    nu=prob.nu, support_radius=prob.support_radius, alpha_c=prob.alpha_c, d_c=prob.d_c,
                    q=prob.q)
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
    return {"value": n_sample / dt, "unit": "GP/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_sample} Gauss points ({n_sample // 27} cells) of the same slope: "
                      f"oracle support search + pattern + FP64 assembly + adjoint, {dt:.1f} s serial (the penalty "
                      f"update, O(dofs), is left out: nodes outside the sample have empty rows)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-sample", type=int, default=2700, help="Gauss points in the oracle's timed sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the assembly-only / mixed measurements")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-model batched assembly")
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
        src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"copy calibration: fill {nbytes} B, copy {nbytes} B -> {nbytes} B")

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

    if not args.no_extras and not args.no_batched:
        out["batched"] = batched_leg(out.get("assemble_gp_per_s", {}).get("fp64"))

    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_sample)
        log(f"cpu baseline {out['cpu_baseline']['value']:.1f} GP/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
