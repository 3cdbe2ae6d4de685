"""GPU checks on the 250k-node slope (100 x 50 x 50 m, 262,701 nodes,
6,750,000 Gauss points, three horizontal layers E = 300 / 80 / 20 MPa): the
mixed-precision configuration.

The oracle cannot assemble the whole model in test time, so K is compared
on sampled rows: for a sampled node the oracle gets a sub-model with every
node and every Gauss point within the support radius of that node (ids kept
in ascending order), which makes that node's three rows complete; FP64 rows
must match bit for bit and mixed rows must match the oracle's own mixed
evaluation bit for bit.  Over the whole matrix: the mixed K is within 1e-6
relative Frobenius of the FP64 K, rigid motions lie in the null space of
the FP64 K, and the displacement error of the mixed K after a solve is
measured (and bounded loosely).
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def large():
    import torch
    import paper_1802_04256_amd as rp
    assert torch.cuda.is_available()
    prob = W.named("slope_large")
    print(f"[gpu case] slope_large: nodes={prob.n_nodes} gps={prob.n_gp}", flush=True)
    plan = rp.Plan.from_problem(prob)
    plan.build_pattern()
    K64 = plan.assemble(cell_E=prob.cell_E, nu=prob.nu, precision="fp64")
    K32 = plan.assemble(cell_E=prob.cell_E, nu=prob.nu, precision="mixed")
    plan.status()
    info = plan.info()
    print(f"nnz={info['nnz']} sum_n={info['sum_n']} n={info['min_n']}..{info['max_n']}", flush=True)
    return prob, plan, K64, K32


def _submodel(prob, node):
    """Every Gauss point within (slightly more than) the support radius of `node`, all nodes."""
    d2 = ((prob.gp_xyz - prob.node_xyz[node]) ** 2).sum(1)
    gps = np.nonzero(d2 <= (prob.support_radius * (1 + 1e-9)) ** 2)[0]
    sub = W.Problem(name="sub", node_xyz=prob.node_xyz, gp_xyz=prob.gp_xyz[gps], gp_wdet=prob.gp_wdet[gps],
                    gp_cell=prob.gp_cell[gps], cell_E=prob.cell_E, nu=prob.nu,
                    support_radius=prob.support_radius, alpha_c=prob.alpha_c, d_c=prob.d_c, q=prob.q)
    return sub


def test_large_sampled_rows(large, oracle_mod):
    prob, plan, K64, K32 = large
    row_ptr = plan.row_ptr.cpu().numpy()
    col_idx = plan.col_idx.cpu().numpy()
    k64 = K64.cpu().numpy()
    k32 = K32.cpu().numpy()
    rng = np.random.default_rng(91)
    nodes = np.concatenate([[0, prob.n_nodes - 1, prob.n_nodes // 2], rng.integers(0, prob.n_nodes, 2)])
    for I in nodes:
        m = oracle_mod.OracleModel(_submodel(prob, int(I)))
        m.build_pattern()
        orp, oci = m.pattern()
        a, b = row_ptr[3 * I], row_ptr[3 * I + 3]
        oa, ob = orp[3 * I], orp[3 * I + 3]
        assert np.array_equal(col_idx[a:b], oci[oa:ob]), I
        assert np.array_equal(k64[a:b], m.assemble()[oa:ob]), I
        assert np.array_equal(k32[a:b], m.assemble(precision=1)[oa:ob]), I


def test_large_mixed_error_and_rigid_modes(large):
    import torch
    prob, plan, K64, K32 = large
    err = float(torch.linalg.norm(K32.double() - K64) / torch.linalg.norm(K64))
    print(f"mixed relative Frobenius error {err:.3e}")
    assert err <= 1e-6
    n = 3 * prob.n_nodes
    S = torch.sparse_csr_tensor(plan.row_ptr, plan.col_idx.long(), K64, size=(n, n))
    A = lambda v: torch.mv(S, v)  # noqa: E731
    X = torch.from_numpy(prob.node_xyz).to(K64.device)
    Knorm = float(torch.linalg.norm(K64))
    for mode in range(6):
        u = torch.zeros(n, dtype=torch.float64, device=K64.device)
        if mode < 3:
            u[mode::3] = 1.0
        else:
            i, j = [(0, 1), (1, 2), (2, 0)][mode - 3]
            u[i::3], u[j::3] = -X[:, j], X[:, i]
        res = float(torch.linalg.norm(A(u))) / (Knorm * float(torch.linalg.norm(u)))
        assert res < 1e-11, (mode, res)


def test_large_mixed_displacement_error(large):
    import bench
    prob, plan, K64, K32 = large
    out = bench.displacement_error(prob, plan.row_ptr, plan.col_idx, K64.clone(), K32.clone())
    print(f"mixed displacement error {out}")
    assert out["cg_rel_residual"][0] <= 1e-10 and out["cg_rel_residual"][1] <= 1e-6
    assert out["u_rel_err"] < 1e-4
