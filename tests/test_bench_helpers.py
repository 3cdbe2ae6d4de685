"""CPU checks of bench.py's own helpers: the CSR operator and the
Jacobi-preconditioned CG used to state the mixed-precision displacement
error (against SciPy's direct solve on the oracle's penalty-constrained
cantilever), and the single-GPU contract of the command line."""
import os
import subprocess
import sys

import numpy as np

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_pcg_matches_direct_solve(oracle_mod):
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    import torch
    sys.path.insert(0, ROOT)
    import bench
    prob = W.cantilever()
    m = oracle_mod.OracleModel(prob)
    m.build_pattern()
    K = m.assemble()
    rp_, ci = m.pattern()
    X = prob.node_xyz
    fixed = np.where(X[:, 0] == X[:, 0].min())[0]
    fd = np.sort((3 * fixed[:, None] + np.arange(3)).ravel())
    oracle_mod.penalty(rp_, ci, K, fd)
    n = 3 * prob.n_nodes
    f = np.zeros(n)
    top = np.where(X[:, 2] == X[:, 2].max())[0]
    f[3 * top + 2] = -1.0
    S = sp.csr_matrix((K, ci, rp_), shape=(n, n))
    u_ref = spl.spsolve(S.tocsc(), f)
    A = bench.csr_operator(torch.from_numpy(rp_), torch.from_numpy(ci.astype(np.int64)), torch.from_numpy(K))
    u, it, res = bench.pcg(A, torch.from_numpy(f), torch.from_numpy(1.0 / S.diagonal()), 1e-12)
    assert res <= 1e-12 and it < 2000
    assert np.linalg.norm(u.numpy() - u_ref) / np.linalg.norm(u_ref) < 1e-10


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_solver_traffic_matches_committed_profile():
    # the bench's recorded solver bytes per step are the figure the committed
    # rocprofv3 summary derives from its FETCH_SIZE / WRITE_SIZE runs
    import os
    import re
    import bench
    text = open(os.path.join(bench.ROOT, "profiles", "slope_step_kernels.md")).read()
    m = re.search(r"\*\*([0-9.]+e\+[0-9]+) scaled HBM bytes\*\* per step for all `k_shape\*` launches", text)
    assert m, "profile summary lacks the per-step solver traffic line"
    assert float(m.group(1)) == bench.SHAPE_TRAFFIC["bytes_per_step"]
