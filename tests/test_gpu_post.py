"""Post-solve quantities on the GPU through the C ABI (GeoMFree3D Sec. 2:
displacements, then stresses; Sec. 3, Example 1: a cube under its own
weight): shape-function values from the kept factors, the body-force vector
and the Gauss-point stresses, bit for bit against the oracle; and the whole
chain on the GPU (assembly, penalty, body force, CG solve, stress) for a
gravity column with rollers against the uniaxial-strain closed form."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

CASES = {
    "cantilever": lambda: W.cantilever(),
    "jbox4": lambda: W.box(n=4, p=2, jitter=0.3, jitter_seed=17, E_seed=18),
    "slope_small": lambda: W.slope(L=12.0, W=6.0, H=6.0, x_c=3.0, jitter_seed=5, E_seed=6),
}


@pytest.mark.parametrize("name", list(CASES))
def test_values_body_force_stress_equal_oracle(name, oracle_mod):
    import torch
    import paper_1802_04256_amd as rp
    prob = CASES[name]()
    print(f"[gpu case] post {name}: gps={prob.n_gp}", flush=True)
    plan = rp.Plan.from_problem(prob)
    plan.build_pattern()
    E = torch.from_numpy(prob.cell_E).cuda()
    plan.assemble(cell_E=E, nu=prob.nu, keep_factors=True)
    phi = plan.shape_values()
    plan.status()
    m = oracle_mod.OracleModel(prob)
    m.build_pattern()
    gp_ptr, _ = m.support()
    ref_phi = np.concatenate([m.shape(g)[0] for g in range(prob.n_gp)])
    assert np.array_equal(phi.cpu().numpy(), ref_phi)
    rng = np.random.default_rng(23)
    b = rng.standard_normal((prob.n_gp, 3))
    f = plan.body_force(phi, torch.from_numpy(b).cuda())
    assert np.array_equal(f.cpu().numpy(), m.body_force(b))
    u = rng.standard_normal((prob.n_nodes, 3)) * 1e-3
    sig = plan.gauss_stress(torch.from_numpy(u).cuda(), E, prob.nu)
    plan.status()
    assert np.array_equal(sig.cpu().numpy(), m.gauss_stress(u))


def test_shape_values_need_kept_factors():
    import paper_1802_04256_amd as rp
    prob = W.cantilever()
    plan = rp.Plan.from_problem(prob)
    plan.build_pattern()
    plan.assemble(cell_E=prob.cell_E, nu=prob.nu)
    with pytest.raises(rp.RpimError) as ei:
        plan.shape_values()
    assert ei.value.code == -8


def test_gravity_column_on_gpu():
    # Example 1's load: a 100 m cube under its own weight (rho = 2600 kg/m^3, g = 9.8 m/s^2); rollers on
    # the four sides and the base make the exact state uniaxial strain, sigma_zz = -rho g (H - z), so the
    # base carries rho g H = 2.548 MPa (the paper reports 2.376 MPa from its own discretisation).
    import torch
    import paper_1802_04256_amd as rp
    H, n = 100.0, 8
    prob = W.box(n=n, h=H / n, p=3, jitter=0.0, jitter_seed=1, E_seed=2)
    prob.cell_E[:] = 1.0e9
    print(f"[gpu case] gravity column: nodes={prob.n_nodes} gps={prob.n_gp}", flush=True)
    plan = rp.Plan.from_problem(prob)
    row_ptr, col_idx = plan.build_pattern()
    E = torch.from_numpy(prob.cell_E).cuda()
    K = plan.assemble(cell_E=E, nu=prob.nu, keep_factors=True)
    phi = plan.shape_values()
    rho, g = 2600.0, 9.8
    f = plan.body_force(phi, torch.tensor([0.0, 0.0, -rho * g], dtype=torch.float64))
    X = prob.node_xyz
    fixed = np.sort(np.concatenate([3 * np.where((X[:, 0] == 0) | (X[:, 0] == H))[0],
                                    3 * np.where((X[:, 1] == 0) | (X[:, 1] == H))[0] + 1,
                                    3 * np.where(X[:, 2] == 0)[0] + 2])).astype(np.int32)
    rp.apply_penalty_bc(row_ptr, col_idx, K, fixed, factor=1e8)
    u, it, res = rp.solve_pcg(row_ptr, col_idx, K, f.reshape(-1), rtol=1e-10)
    sig = plan.gauss_stress(u, E, prob.nu).cpu().numpy()
    plan.status()
    assert abs(float(f[:, 2].sum()) / (-rho * g * H ** 3) - 1) <= 1e-12
    nu = prob.nu
    M = 1.0e9 * (1 - nu) / ((1 + nu) * (1 - 2 * nu))
    uu = u.reshape(-1, 3).cpu().numpy()
    top = X[:, 2] == H
    settle = -rho * g * H ** 2 / (2 * M)
    mean = (prob.gp_wdet @ sig[:, 2]) / prob.gp_wdet.sum()
    zb = prob.gp_xyz[:, 2].min()
    base = np.isclose(prob.gp_xyz[:, 2], zb)
    print(f"CG {it} iterations; top settlement {uu[top, 2].mean():.5e} (closed form {settle:.5e}); "
          f"mean sigma_zz {mean:.4e} (closed form {-rho * g * H / 2:.4e}); lowest Gauss layer z = {zb:.3f}: "
          f"sigma_zz {sig[base, 2].mean():.4e} (closed form {-rho * g * (H - zb):.4e})")
    assert abs(uu[top, 2].mean() / settle - 1) <= 1e-2
    assert abs(mean / (-rho * g * H / 2) - 1) <= 0.02
    assert abs(sig[base, 2].mean() / (-rho * g * (H - zb)) - 1) <= 0.10
