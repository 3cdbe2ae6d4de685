#!/usr/bin/env python3
"""Write the stored expected values of the full-size GPU parity tests.

Every value comes from the serial CPU oracle (oracle/) on the seeded
workloads (workloads/); nothing is taken from the HIP library.  The GPU
tests compare against these files instead of running the oracle on the GPU
machine, which would take hours at these sizes.

  slope_K_sha256.json       jittered slope, 18,081 nodes, 432,000 Gauss points:
                            SHA-256 of the CSR pattern and of the FP64 and the
                            mixed-precision (Kahan) K, in chunks of node rows.
                            Rows are complete because each worker assembles every
                            Gauss point whose support touches its slab of nodes.
  slope_adjoint.json        the same slope, loss L = sum over 8 probe vectors v
                            (seed 5) of 0.5 v^T K v: dL/dE on 16 sampled cells and
                            dL/dx on 16 sampled nodes (oracle FP64 adjoint over
                            the Gauss points that reach them), and 32 central
                            finite differences of L (h = 1e-6) in __float128 with
                            supports frozen, at seeded (node, axis) samples.
  batch64_rows.json         the 64-model batch: SHA-256 of the three scalar rows
                            of sampled nodes in 4 models, FP64 and mixed, each
                            model assembled on its own (the batch is block
                            diagonal, so its rows carry the same values).

Usage: python tests/golden/make_fixtures.py [--only slope_K|slope_adjoint|batch64] [--jobs 8]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

CHUNK_ROWS = 1024        # node rows per K hash chunk
FD_H = 1.0e-6            # central-difference step on a node coordinate (times d_c = 1 m)
TMP = os.environ.get("FIXTURE_TMP", "/tmp/rpim_fixtures")


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def _model(prob):
    m = oracle.OracleModel(prob)
    m.build_pattern()
    return m


def _touching(gp_ptr, gp_nbr, n_gp, nodes):
    """Ascending Gauss points whose support holds any of `nodes`."""
    owner = np.repeat(np.arange(n_gp, dtype=np.int64), np.diff(gp_ptr))
    return np.unique(owner[np.isin(gp_nbr, nodes)])


# ---- slope K --------------------------------------------------------------------
def _slab_rows(args):
    prec, lo, hi = args
    prob = W.slope()
    m = _model(prob)
    gp_ptr, gp_nbr = m.support()
    gps = _touching(gp_ptr, gp_nbr, prob.n_gp, np.arange(lo, hi))
    t = time.time()
    K = m.assemble(gps=gps, precision=prec)
    row_ptr, _ = m.pattern()
    out = K[row_ptr[3 * lo]:row_ptr[3 * hi]].copy()
    print(f"  slab [{lo},{hi}) precision {prec}: {len(gps)} points, {time.time() - t:.0f} s", flush=True)
    return out


def slope_K(jobs):
    prob = W.slope()
    m = _model(prob)
    row_ptr, col_idx = m.pattern()
    N = prob.n_nodes
    bounds = np.linspace(0, N, jobs + 1).round().astype(int)
    res = {"workload": "jittered slope 40x20x20 m (W.slope()), 18,081 nodes, 432,000 Gauss points, lognormal E",
           "source": "oracle/rpim_oracle.cpp (orcl_assemble) via tests/golden/make_fixtures.py",
           "n_nodes": N, "nnz": int(m.nnz), "chunk_node_rows": CHUNK_ROWS,
           "row_ptr_sha256": sha(row_ptr), "col_idx_sha256": sha(col_idx)}
    for prec, name in ((0, "fp64"), (1, "mixed")):
        with ProcessPoolExecutor(jobs) as ex:
            parts = list(ex.map(_slab_rows, [(prec, int(bounds[i]), int(bounds[i + 1])) for i in range(jobs)]))
        K = np.concatenate(parts)
        assert len(K) == m.nnz
        chunks = []
        for a in range(0, N, CHUNK_ROWS):
            b = min(N, a + CHUNK_ROWS)
            chunks.append(sha(K[row_ptr[3 * a]:row_ptr[3 * b]]))
        res[name] = {"dtype": str(K.dtype), "sha256": sha(K), "chunks": chunks,
                     "fro_norm": float(np.linalg.norm(K.astype(np.float64)))}
        print(f"slope K {name}: sha256 {res[name]['sha256'][:16]}...", flush=True)
    return res


# ---- slope adjoint ------------------------------------------------------------------
def _kbar_path():
    return os.path.join(TMP, "slope_kbar.npy")


def _make_kbar(m, prob):
    """dL/dK on the pattern for L = sum_v 0.5 v^T K v: 0.5 sum_v v_i v_j (row-chunked)."""
    os.makedirs(TMP, exist_ok=True)
    row_ptr, col_idx = m.pattern()
    V = W.probe_vectors(3 * prob.n_nodes, 8, 5)
    Kb = np.empty(m.nnz)
    n = 3 * prob.n_nodes
    for a in range(0, n, 6000):
        b = min(n, a + 6000)
        rows = np.repeat(np.arange(a, b), np.diff(row_ptr[a:b + 1]))
        s, e = row_ptr[a], row_ptr[b]
        Kb[s:e] = 0.5 * np.einsum("vi,vi->i", V[:, rows], V[:, col_idx[s:e]])
    np.save(_kbar_path(), Kb)


def _adjoint_task(args):
    kind, item = args
    prob = W.slope()
    m = _model(prob)
    gp_ptr, gp_nbr = m.support()
    Kb = np.load(_kbar_path(), mmap_mode="r")
    t = time.time()
    if kind == "node":
        gps = _touching(gp_ptr, gp_nbr, prob.n_gp, [item])
        _, dX = m.backward(np.asarray(Kb), gps=gps)
        out = [float(v) for v in dX[item]]
    elif kind == "cells":
        cells = np.asarray(item)
        gps = np.nonzero(np.isin(prob.gp_cell, cells))[0].astype(np.int64)
        dE, _ = m.backward(np.asarray(Kb), gps=gps)
        out = [float(dE[c]) for c in cells]
    else:  # central difference of L in __float128 at (node, axis), supports frozen
        node, axis = item
        gps = _touching(gp_ptr, gp_nbr, prob.n_gp, [node])
        vals = []
        for sgn in (1.0, -1.0):
            X = prob.node_xyz.copy()
            X[node, axis] += sgn * FD_H * prob.d_c
            vals.append(m.dot_q(np.asarray(Kb), gps, node_xyz=X))
        # (L+ - L-) / 2h from the double-double results: the high parts nearly cancel exactly
        dl = (vals[0][0] - vals[1][0]) + (vals[0][1] - vals[1][1])
        out = dl / (2.0 * FD_H * prob.d_c)
    print(f"  {kind} {item}: {len(gps) if kind != 'cells' else ''} {time.time() - t:.0f} s", flush=True)
    return out


def slope_adjoint(jobs):
    prob = W.slope()
    m = _model(prob)
    _make_kbar(m, prob)
    rng = np.random.default_rng(81)
    nodes = np.concatenate([[0, prob.n_nodes - 1], rng.choice(prob.n_nodes, 14, replace=False)]).astype(int)
    cells = np.concatenate([[0, prob.n_cells - 1], rng.choice(prob.n_cells, 14, replace=False)]).astype(int)
    rng6 = np.random.default_rng(6)  # finite-difference samples
    fd = [(int(a), int(b)) for a, b in zip(rng6.choice(prob.n_nodes, 32, replace=False), rng6.integers(0, 3, 32))]
    tasks = [("node", int(i)) for i in nodes] + [("cells", [int(c) for c in cells])] + [("fd", s) for s in fd]
    with ProcessPoolExecutor(jobs) as ex:
        out = list(ex.map(_adjoint_task, tasks))
    res = {"workload": "jittered slope (W.slope()); L = sum_v 0.5 v^T K v, 8 probe vectors "
                       "W.probe_vectors(3N, 8, 5); supports, Gauss points and weights frozen",
           "source": "oracle/rpim_oracle.cpp (orcl_assemble_backward, orcl_dot_q) via tests/golden/make_fixtures.py",
           "nodes": [int(i) for i in nodes], "dX": out[:len(nodes)],
           "cells": [int(c) for c in cells], "dE": out[len(nodes)],
           "fd_h": FD_H, "fd_samples": [list(s) for s in fd], "fd_dX": out[len(nodes) + 1:]}
    os.remove(_kbar_path())
    return res


# ---- batch rows -------------------------------------------------------------------------
def _batch_task(args):
    m_id, nodes = args
    prob = W.batched_slopes()[m_id]
    m = _model(prob)
    gp_ptr, gp_nbr = m.support()
    row_ptr, col_idx = m.pattern()
    rows = []
    for i in nodes:
        gps = _touching(gp_ptr, gp_nbr, prob.n_gp, [i])
        a, b = row_ptr[3 * i], row_ptr[3 * i + 3]
        K64 = m.assemble(gps=gps, precision=0)
        K32 = m.assemble(gps=gps, precision=1)
        rows.append({"node": int(i), "row_ptr": [int(row_ptr[3 * i + k]) - int(a) for k in range(4)],
                     "col_sha256": sha(col_idx[a:b]), "fp64_sha256": sha(K64[a:b]), "mixed_sha256": sha(K32[a:b]),
                     "fp64_first": float(K64[a]), "mixed_first": float(K32[a])})
    print(f"  model {m_id}: {prob.n_nodes} nodes", flush=True)
    return {"model": m_id, "n_nodes": prob.n_nodes, "rows": rows}


def batch64(jobs):
    models = W.batched_slopes()
    sizes = np.array([p.n_nodes for p in models])
    rng = np.random.default_rng(83)
    pick = [int(np.argmin(sizes)), int(np.argmax(sizes))]
    pick += [int(x) for x in rng.choice([i for i in range(len(models)) if i not in pick], 2, replace=False)]
    tasks = []
    for mi in pick:
        n = models[mi].n_nodes
        tasks.append((mi, [0, n - 1, int(rng.integers(0, n))]))
    with ProcessPoolExecutor(jobs) as ex:
        out = list(ex.map(_batch_task, tasks))
    return {"workload": "64 jittered slopes (W.batch(W.batched_slopes())), each model assembled alone",
            "source": "oracle/rpim_oracle.cpp (orcl_assemble) via tests/golden/make_fixtures.py",
            "models": out}


JOBS = {"slope_K": ("slope_K_sha256.json", slope_K), "slope_adjoint": ("slope_adjoint.json", slope_adjoint),
        "batch64": ("batch64_rows.json", batch64)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", choices=sorted(JOBS))
    ap.add_argument("--jobs", type=int, default=8)
    args = ap.parse_args()
    oracle.lib()
    for name, (fname, fn) in JOBS.items():
        if args.only and name != args.only:
            continue
        t = time.time()
        res = fn(args.jobs)
        with open(os.path.join(HERE, fname), "w") as f:
            json.dump(res, f, indent=1)
        print(f"{name}: wrote {fname} in {time.time() - t:.0f} s", flush=True)


if __name__ == "__main__":
    main()
