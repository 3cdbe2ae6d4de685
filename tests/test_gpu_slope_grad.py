"""GPU adjoint at full size: the jittered slope (18,081 nodes, 432,000 Gauss
points) with the probe loss L = sum over 8 seeded N(0,1) vectors v of
0.5 v^T K v, so dL/dK_ij = 0.5 sum_v v_i v_j on the pattern.

Expected values were written on the CPU by tests/golden/make_fixtures.py
from the oracle only: its FP64 adjoint for 16 sampled cells (dL/dE) and 16
sampled nodes (dL/dx), each over the Gauss points that reach it, and 32
central finite differences of L in __float128 with supports frozen
(h = 1e-6 m).  Error metric for gradients: |g - g_ref| / max(|g_ref|,
1e-3 max|g|).  Also checked: Euler homogeneity sum_c E_c dL/dE_c = L, which
holds at any size because K is linear in E.
"""
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "slope_adjoint.json")


@pytest.fixture(scope="module")
def grads():
    import torch
    import paper_1802_04256_amd as rp
    assert torch.cuda.is_available()
    prob = W.slope()
    print(f"[gpu case] slope adjoint: nodes={prob.n_nodes} gps={prob.n_gp}", flush=True)
    dev = torch.device("cuda:0")
    plan = rp.Plan.from_problem(prob, device=dev)
    row_ptr, col_idx = plan.build_pattern()
    X = torch.from_numpy(prob.node_xyz).to(dev)
    E = torch.from_numpy(prob.cell_E).to(dev)
    K = plan.assemble(X, E, prob.nu, keep_factors=True)
    V = torch.from_numpy(W.probe_vectors(3 * prob.n_nodes, 8, 5)).to(dev)
    rows = torch.repeat_interleave(torch.arange(3 * prob.n_nodes, device=dev), torch.diff(row_ptr))
    dK = torch.zeros_like(K)
    for v in V:  # 0.5 sum_v v_i v_j, one probe vector at a time
        dK += 0.5 * v[rows] * v[col_idx.long()]
    A = torch.sparse_csr_tensor(row_ptr, col_idx.long(), K, size=(3 * prob.n_nodes,) * 2)
    L = float(sum(0.5 * torch.dot(v, torch.mv(A, v)) for v in V))
    del rows, A
    dE, dX = plan.assemble_backward(X, E, prob.nu, dK)
    plan.status()
    return prob, dE.cpu().numpy(), dX.cpu().numpy(), L


def _err(g, ref, scale):
    return np.abs(g - ref) / np.maximum(np.abs(ref), 1e-3 * scale)


def test_full_adjoint_vs_oracle(grads):
    prob, dE, dX, _ = grads
    ref = json.load(open(GOLD))
    cells, nodes = np.array(ref["cells"]), np.array(ref["nodes"])
    eE = _err(dE[cells], np.array(ref["dE"]), np.abs(dE).max())
    eX = _err(dX[nodes], np.array(ref["dX"]), np.abs(dX).max())
    print(f"max rel err dE {eE.max():.2e}, dX {eX.max():.2e}")
    assert eE.max() <= 1e-10
    assert eX.max() <= 1e-6


def test_full_adjoint_vs_quad_fd(grads):
    prob, dE, dX, _ = grads
    ref = json.load(open(GOLD))
    s = np.array(ref["fd_samples"])
    assert len(s) >= 32
    e = _err(dX[s[:, 0], s[:, 1]], np.array(ref["fd_dX"]), np.abs(dX).max())
    print(f"max rel err vs __float128 FD over {len(s)} samples: {e.max():.2e}")
    assert e.max() <= 1e-6


def test_full_adjoint_euler_homogeneity(grads):
    prob, dE, dX, L = grads
    lhs = float(np.dot(prob.cell_E, dE))
    assert abs(lhs - L) <= 1e-10 * abs(L), (lhs, L)
