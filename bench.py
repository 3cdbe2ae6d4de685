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
SHAPE_TRAFFIC = {"sources_sha256": "8abb461089a2b3d64f891d1dc3930d6e0f31e805df4bd2b5ff7d257230abc6e5", "bytes_per_step": 3.926e10}


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
        rp.apply_penalty_bc(plan.row_ptr, plan.col_idx, K, fixed, factor=1e8)
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
        # algorithmic HBM bytes of one FP64 assembly: K values written once, dphi written
        # and read once, supports / inverse lists / pattern read once
        sum_n = info["sum_n"]
        alg_bytes = info["nnz"] * 8 + sum_n * 24 * 2 + sum_n * (4 + 8) + info["n_blocks"] * 4 * 2
        out["hbm_gbps_fp64_assembly"] = alg_bytes / t_fp64 / 1e9
        log(f"assemble fp64 {t_fp64 * 1e3:.2f} ms, mixed {t_mixed * 1e3:.2f} ms (err {err32:.2e}), "
            f"bwd {t_bwd * 1e3:.2f} ms, bwd/fwd {out['bwd_fwd']:.2f}")

    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_sample)
        log(f"cpu baseline {out['cpu_baseline']['value']:.1f} GP/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
