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
