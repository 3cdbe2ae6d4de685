"""Assembly captured in a HIP graph: a batch of independent models (different
support-size buckets in one plan), captured once per precision and replayed
several times with other eager work and synchronisations in between; every
replay must equal the eager result bit for bit."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _batch():
    return W.batch([W.cantilever(), W.box(n=6), W.slope(L=10.0, W=6.0, H=5.0, x_c=2.5), W.box(n=5, jitter_seed=3)])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replay_matches_eager(precision):
    import torch
    import paper_1802_04256_amd as rp
    prob = _batch()
    print(f"[gpu case] graph replay {precision}: models={prob.n_models} gps={prob.n_gp}", flush=True)
    dev = torch.device("cuda:0")
    plan = rp.Plan.from_problem(prob, device=dev)
    plan.build_pattern()
    X = torch.from_numpy(prob.node_xyz).to(dev)
    E = torch.from_numpy(prob.cell_E).to(dev)
    dt = torch.float64 if precision == "fp64" else torch.float32
    K_eager = torch.empty(plan.nnz, dtype=dt, device=dev)
    K_graph = torch.empty(plan.nnz, dtype=dt, device=dev)
    K_other = torch.empty(plan.nnz, dtype=dt, device=dev)
    plan.assemble(X, E, prob.nu, precision, out=K_eager)  # eager call first: workspaces exist before capture
    torch.cuda.synchronize()
    plan.status()
    ref = K_eager.cpu().numpy()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.assemble(X, E, prob.nu, precision, out=K_graph)
    for rep in range(3):
        K_graph.fill_(-1.0)
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(K_graph.cpu().numpy(), ref), rep
        # eager work on the same plan between replays (other output buffer, other E)
        plan.assemble(X, E * (2.0 + rep), prob.nu, precision, out=K_other)
        torch.cuda.synchronize()
    plan.status()


def test_graph_penalty_matches_eager():
    # the penalty call records kernels only (no memset, no synchronisation): capture it with a copy of the
    # assembled K in front, replay with eager work in between, compare K, rhs and alpha with an eager call
    import torch
    import paper_1802_04256_amd as rp
    prob = W.cantilever()
    print(f"[gpu case] graph penalty: gps={prob.n_gp}", flush=True)
    dev = torch.device("cuda:0")
    plan = rp.Plan.from_problem(prob, device=dev)
    row_ptr, col_idx = plan.build_pattern()
    K0 = plan.assemble(cell_E=prob.cell_E, nu=prob.nu)
    X = prob.node_xyz
    fixed = np.sort((3 * np.where(X[:, 0] == 0.0)[0][:, None] + np.arange(3)).ravel()).astype(np.int32)
    ub = np.linspace(-1.0, 1.0, len(fixed))
    K_ref, rhs_ref = K0.clone(), torch.zeros(3 * prob.n_nodes, dtype=torch.float64, device=dev)
    alpha_ref = rp.apply_penalty_bc(row_ptr, col_idx, K_ref, fixed, u_bar=ub, rhs=rhs_ref)
    fx = torch.from_numpy(fixed).to(dev)
    ubt = torch.from_numpy(ub).to(dev)
    K, rhs = torch.empty_like(K0), torch.empty_like(rhs_ref)
    rp.apply_penalty_bc(row_ptr, col_idx, K0.clone(), fx, u_bar=ubt, rhs=rhs.zero_(), check=False)  # warm
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        K.copy_(K0)
        rhs.zero_()
        alpha, status = rp.apply_penalty_bc(row_ptr, col_idx, K, fx, u_bar=ubt, rhs=rhs, check=False)
    for rep in range(3):
        K.fill_(-1.0)
        g.replay()
        torch.cuda.synchronize()
        assert int(status.item()) == 0 and float(alpha.item()) == alpha_ref, rep
        assert torch.equal(K, K_ref) and torch.equal(rhs, rhs_ref), rep
        rp.apply_penalty_bc(row_ptr, col_idx, K0.clone(), fixed, factor=3.0)  # eager work between replays
        torch.cuda.synchronize()
