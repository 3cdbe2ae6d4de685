"""Moving-least-squares and Shepard shape functions on the GPU (GeoMFree3D
Sec. 4 names moving least squares as the package's next shape functions):
gradients, values, FP64 and mixed K, body force and Gauss-point stresses bit
for bit against the oracle's evaluation in the same operation order, through
the C ABI."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

CASES = {
    "cantilever": lambda: W.cantilever(),
    "jbox4": lambda: W.box(n=4, p=2, jitter=0.3, jitter_seed=17, E_seed=18),
    "slope_small": lambda: W.slope(L=12.0, W=6.0, H=6.0, x_c=3.0, jitter_seed=5, E_seed=6),
}


@pytest.fixture(scope="module", params=[(c, k) for c in CASES for k in ("mls", "shepard")],
                ids=lambda ck: f"{ck[0]}-{ck[1]}")
def case(request, oracle_mod):
    import paper_1802_04256_amd as rp
    name, kind = request.param
    prob = CASES[name]()
    print(f"[gpu case] {kind} {name}: gps={prob.n_gp}", flush=True)
    m = oracle_mod.OracleModel(prob, kind)
    m.build_pattern()
    plan = rp.Plan.from_problem(prob)
    plan.build_pattern()
    plan.set_shape_functions(kind)
    return name, kind, prob, m, plan


def test_gradients_values_and_K_equal_oracle(case):
    import torch
    name, kind, prob, m, plan = case
    E = torch.from_numpy(prob.cell_E).cuda()
    K = plan.assemble(cell_E=E, nu=prob.nu).cpu().numpy()
    plan.status()
    gp_ptr, _ = m.support()
    d = plan.dphi().cpu().numpy()
    ref = [m.shape(g) for g in range(prob.n_gp)]
    assert np.array_equal(d, np.concatenate([r[1] for r in ref]))
    assert np.array_equal(plan.shape_values().cpu().numpy(), np.concatenate([r[0] for r in ref]))
    assert np.array_equal(K, m.assemble())
    K32 = plan.assemble(cell_E=E, nu=prob.nu, precision="mixed").cpu().numpy()
    plan.status()
    assert np.array_equal(K32, m.assemble(precision=1))


def test_body_force_and_stress_equal_oracle(case):
    import torch
    name, kind, prob, m, plan = case
    E = torch.from_numpy(prob.cell_E).cuda()
    plan.assemble(cell_E=E, nu=prob.nu)
    phi = plan.shape_values()
    rng = np.random.default_rng(29)
    b = rng.standard_normal((prob.n_gp, 3))
    f = plan.body_force(phi, torch.from_numpy(b).cuda())
    assert np.array_equal(f.cpu().numpy(), m.body_force(b))
    u = rng.standard_normal((prob.n_nodes, 3)) * 1e-3
    sig = plan.gauss_stress(torch.from_numpy(u).cuda(), E, prob.nu)
    plan.status()
    assert np.array_equal(sig.cpu().numpy(), m.gauss_stress(u))


def test_no_adjoint_and_back_to_rpim(oracle_mod):
    import torch
    import paper_1802_04256_amd as rp
    prob = W.cantilever()
    plan = rp.Plan.from_problem(prob)
    plan.build_pattern()
    E = torch.from_numpy(prob.cell_E).cuda()
    K_rpim = plan.assemble(cell_E=E, nu=prob.nu, keep_factors=True).clone()
    plan.set_shape_functions("mls")
    plan.assemble(cell_E=E, nu=prob.nu, keep_factors=True)
    with pytest.raises(rp.RpimError) as ei:  # the adjoint goes through kept RPIM factors only
        plan.assemble_backward(prob.node_xyz, E, prob.nu, np.zeros(plan.nnz))
    assert ei.value.code == -8
    plan.set_shape_functions("rpim")
    assert torch.equal(plan.assemble(cell_E=E, nu=prob.nu), K_rpim)
    with pytest.raises(rp.RpimError):
        plan.set_shape_functions(7)
