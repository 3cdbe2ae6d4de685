"""GPU parity: the HIP path through the C ABI against the CPU oracle.

The FP64 path follows the same operation order as the oracle, so supports,
pattern, shape-function gradients and K are compared bit for bit; the
relative Frobenius bar for K is 1e-12.  The mixed path is compared with the
oracle's own mixed evaluation and with FP64 (<= 1e-6).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rp():
    import torch
    import paper_1802_04256_amd as rp
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    rp.lib()
    return rp


def _both(prob, oracle_mod, rp):
    m = oracle_mod.OracleModel(prob)
    m.build_pattern()
    plan = rp.Plan.from_problem(prob)
    plan.build_pattern()
    return m, plan


def rel_fro(a, b):
    return float(np.linalg.norm(a.astype(np.float64) - b) / np.linalg.norm(b))


SMALL = {
    "cantilever": lambda: W.cantilever(),
    "jbox6": lambda: W.box(n=6, p=3, jitter=0.3, jitter_seed=31, E_seed=32),
    "slope_small": lambda: W.slope(L=12.0, W=6.0, H=6.0, x_c=3.0, jitter_seed=5, E_seed=6),
}


_ORACLE_K = {}  # (case, precision) -> the oracle's K: several tests compare against the same one


def oracle_K(name, m, precision=0):
    if (name, precision) not in _ORACLE_K:
        _ORACLE_K[(name, precision)] = m.assemble(precision=precision)
    return _ORACLE_K[(name, precision)].copy()


@pytest.fixture(scope="module", params=list(SMALL))
def case(request, oracle_mod, rp):
    prob = SMALL[request.param]()
    print(f"[gpu case] {request.param}: nodes={prob.n_nodes} gps={prob.n_gp}", flush=True)
    m, plan = _both(prob, oracle_mod, rp)
    return request.param, prob, m, plan


def test_pow_bitwise(rp, oracle_mod):
    import torch
    rng = np.random.default_rng(123)
    x = np.concatenate([rng.uniform(16.0, 60.0, 200000), np.arange(16.0, 60.0, 0.125)])
    y = rp.pow_cr(torch.from_numpy(x).cuda(), 1.03).cpu().numpy()
    ref = np.array([oracle_mod.pow_cr(v, 1.03) for v in x])
    assert np.array_equal(y, ref)


def test_support_and_pattern_bitwise(case):
    name, prob, m, plan = case
    gp_ptr, gp_nbr = m.support()
    g_ptr, g_nbr = plan.support()
    assert np.array_equal(g_ptr.cpu().numpy(), gp_ptr)
    assert np.array_equal(g_nbr.cpu().numpy(), gp_nbr)
    row_ptr, col_idx = m.pattern()
    assert plan.nnz == m.nnz
    assert np.array_equal(plan.row_ptr.cpu().numpy(), row_ptr)
    assert np.array_equal(plan.col_idx.cpu().numpy(), col_idx)


def test_dphi_bitwise(case):
    name, prob, m, plan = case
    plan.assemble(cell_E=prob.cell_E, nu=prob.nu)
    plan.status()
    d = plan.dphi().cpu().numpy()
    gp_ptr, _ = m.support()
    for g in range(0, prob.n_gp, max(1, prob.n_gp // 64)):
        _, dphi = m.shape(g)
        assert np.array_equal(d[gp_ptr[g]:gp_ptr[g + 1]], dphi), g


def test_K_fp64_bitwise(case):
    name, prob, m, plan = case
    K = plan.assemble(cell_E=prob.cell_E, nu=prob.nu).cpu().numpy()
    plan.status()
    Ko = oracle_K(name, m)
    err = rel_fro(K, Ko)
    print(f"[{name}] FP64 K rel Frobenius error {err:.3e}")
    assert err <= 1e-12
    assert np.array_equal(K, Ko)


def test_K_mixed(case):
    name, prob, m, plan = case
    K32 = plan.assemble(cell_E=prob.cell_E, nu=prob.nu, precision="mixed").cpu().numpy()
    plan.status()
    Ko32 = oracle_K(name, m, 1)
    Ko64 = oracle_K(name, m)
    assert K32.dtype == np.float32
    assert np.array_equal(K32, Ko32)
    err = rel_fro(K32, Ko64)
    print(f"[{name}] mixed K rel Frobenius error vs FP64 {err:.3e}")
    assert err <= 1e-6


def test_deterministic_repeat(case):
    name, prob, m, plan = case
    a = plan.assemble(cell_E=prob.cell_E, nu=prob.nu).cpu().numpy()
    b = plan.assemble(cell_E=prob.cell_E, nu=prob.nu).cpu().numpy()
    assert np.array_equal(a, b)


def test_penalty_matches_oracle(case, oracle_mod):
    import torch
    name, prob, m, plan = case
    K = plan.assemble(cell_E=prob.cell_E, nu=prob.nu)
    X = prob.node_xyz
    nodes = np.where(X[:, 0] == X[:, 0].min())[0]
    fixed = np.sort((3 * nodes[:, None] + np.arange(3)).ravel()).astype(np.int32)
    ub = np.linspace(-1e-3, 1e-3, len(fixed))
    rhs = torch.zeros(3 * prob.n_nodes, dtype=torch.float64, device="cuda")
    alpha = rp_apply(plan, K, fixed, ub, rhs)
    Ko = oracle_K(name, m)
    rhs_o = np.zeros(3 * prob.n_nodes)
    rp_o, ci_o = m.pattern()
    alpha_o = oracle_mod.penalty(rp_o, ci_o, Ko, fixed, u_bar=ub, factor=1e8, rhs=rhs_o)
    assert alpha == alpha_o
    assert np.array_equal(K.cpu().numpy(), Ko)
    assert np.array_equal(rhs.cpu().numpy(), rhs_o)


def rp_apply(plan, K, fixed, ub, rhs):
    import paper_1802_04256_amd as rp
    return rp.apply_penalty_bc(plan.row_ptr, plan.col_idx, K, fixed, u_bar=ub, factor=1e8, rhs=rhs)


def test_penalty_rejects_bad_fixed(rp):
    import torch
    Kd = np.diag([4.0, 5.0, 6.0])
    S = sp.csr_matrix(Kd)
    row_ptr = torch.from_numpy(S.indptr.astype(np.int64)).cuda()
    col_idx = torch.from_numpy(S.indices.astype(np.int32)).cuda()
    K = torch.from_numpy(S.data.copy()).cuda()
    rhs = torch.ones(3, dtype=torch.float64, device="cuda")
    with pytest.raises(rp.RpimError) as ei:
        rp.apply_penalty_bc(row_ptr, col_idx, K, np.array([2, 1], np.int32), u_bar=np.ones(2), rhs=rhs)
    assert ei.value.code == -1
    with pytest.raises(rp.RpimError):
        rp.apply_penalty_bc(row_ptr, col_idx, K, np.array([3], np.int32), rhs=rhs)
    # a rejected call leaves K and rhs untouched; without the check nothing synchronises and the
    # status word carries the result
    assert np.array_equal(K.cpu().numpy(), [4.0, 5.0, 6.0]) and np.array_equal(rhs.cpu().numpy(), [1.0, 1.0, 1.0])
    alpha, status = rp.apply_penalty_bc(row_ptr, col_idx, K, np.array([-1], np.int32), check=False)
    assert int(status.item()) == -1 and np.array_equal(K.cpu().numpy(), [4.0, 5.0, 6.0])
    alpha, status = rp.apply_penalty_bc(row_ptr, col_idx, K, np.array([0, 2], np.int32), factor=2.0, check=False)
    assert int(status.item()) == 0 and float(alpha.item()) == 12.0
    assert np.array_equal(K.cpu().numpy(), [16.0, 5.0, 18.0])


def test_cantilever_tip_deflection_from_gpu_K(rp):
    import torch
    prob = W.cantilever()
    plan = rp.Plan.from_problem(prob)
    plan.build_pattern()
    K = plan.assemble(cell_E=prob.cell_E, nu=prob.nu)
    X = prob.node_xyz
    fixed = np.sort((3 * np.where(X[:, 0] == 0.0)[0][:, None] + np.arange(3)).ravel()).astype(np.int32)
    rp.apply_penalty_bc(plan.row_ptr, plan.col_idx, K, fixed, factor=1e8)
    n = 3 * prob.n_nodes
    D = sp.csr_matrix((K.cpu().numpy(), plan.col_idx.cpu().numpy(), plan.row_ptr.cpu().numpy()), shape=(n, n))
    f = np.zeros(n)
    tip = np.where(X[:, 0] == 8.0)[0]
    for i in tip:
        wy = 0.5 if X[i, 1] in (0.0, 2.0) else 1.0
        wz = 0.5 if X[i, 2] in (0.0, 2.0) else 1.0
        f[3 * i + 2] = -wy * wz / 4.0
    u = np.linalg.solve(D.toarray(), f)
    mid = np.where((X[:, 0] == 8.0) & (X[:, 1] == 1.0) & (X[:, 2] == 1.0))[0][0]
    I = 16.0 / 12.0
    dT = 8.0 ** 3 / (3 * 3e7 * I) + (4 + 5 * 0.3) * 8.0 * 4.0 / (24 * 3e7 * I)
    assert 0.95 <= -u[3 * mid + 2] / dT <= 1.05


def test_support_error_reported(rp):
    prob = W.cantilever()
    prob.support_radius = 0.6
    plan = rp.Plan.from_problem(prob)
    with pytest.raises(rp.RpimError) as ei:
        plan.build_pattern()
    assert ei.value.code == -4


def test_singular_moment_matrix_reported(rp):
    # all nodes and Gauss points in the plane z = 0: the z column of the
    # polynomial block vanishes and the moment matrix is singular
    xs, ys = np.meshgrid(np.arange(6.0), np.arange(6.0), indexing="ij")
    nodes = np.stack([xs.ravel(), ys.ravel(), np.zeros(36)], axis=1)
    gps = np.array([[2.3, 2.6, 0.0], [1.1, 3.2, 0.0]])
    plan = rp.Plan(nodes, gps, np.ones(2), np.zeros(2, np.int32), 1, 2.5)
    plan.build_pattern()
    plan.assemble(cell_E=np.ones(1), nu=0.3)
    st, bad = plan.status(raise_on_error=False)
    assert st == -5
    assert bad == 0


def test_batched_models_equal_individual(rp):
    models = [W.box(n=3, p=2, jitter_seed=40 + i, E_seed=50 + i) for i in range(2)] + [W.cantilever(4, 2, 2)]
    batch = W.batch(models)
    plan = rp.Plan.from_problem(batch)
    plan.build_pattern()
    Kb = plan.assemble(cell_E=batch.cell_E, nu=batch.nu).cpu().numpy()
    rpb = plan.row_ptr.cpu().numpy()
    for i, mdl in enumerate(models):
        pl = rp.Plan.from_problem(mdl)
        pl.build_pattern()
        Ki = pl.assemble(cell_E=mdl.cell_E, nu=mdl.nu).cpu().numpy()
        r0 = 3 * batch.node_off[i]
        seg = Kb[rpb[r0]:rpb[r0 + 3 * mdl.n_nodes]]
        assert np.array_equal(seg, Ki)


def test_large_supports_lds_kernel_bitwise(rp, oracle_mod):
    # a wider support radius puts the largest supports past the register
    # kernel's 104-row limit, into the LDS kernel
    prob = W.box(n=8, p=2, jitter=0.3, jitter_seed=61, E_seed=62)
    prob.support_radius = 2.9
    print(f"[gpu case] box8 radius 2.9: nodes={prob.n_nodes} gps={prob.n_gp}", flush=True)
    m, plan = _both(prob, oracle_mod, rp)
    info = plan.info()
    assert info["max_n"] + 4 > 104, info["max_n"]
    gp_ptr, gp_nbr = m.support()
    assert np.array_equal(plan.support()[1].cpu().numpy(), gp_nbr)
    K = plan.assemble(cell_E=prob.cell_E, nu=prob.nu).cpu().numpy()
    plan.status()
    assert np.array_equal(plan.dphi().cpu().numpy(), np.concatenate([m.shape(g)[1] for g in range(prob.n_gp)]))
    assert np.array_equal(K, m.assemble())


def test_lds_kernel_equals_register_kernel(rp):
    prob = W.slope(L=12.0, W=8.0, H=6.0, x_c=3.0, jitter_seed=71, E_seed=72)
    plan = rp.Plan.from_problem(prob)
    plan.build_pattern()
    K_reg = plan.assemble(cell_E=prob.cell_E, nu=prob.nu).cpu().numpy()
    d_reg = plan.dphi().cpu().numpy()
    plan.set_solver("lds")
    K_lds = plan.assemble(cell_E=prob.cell_E, nu=prob.nu).cpu().numpy()
    d_lds = plan.dphi().cpu().numpy()
    plan.status()
    assert np.array_equal(d_reg, d_lds)
    assert np.array_equal(K_reg, K_lds)


@pytest.mark.parametrize("name", ["slope_small", "jbox6", "cantilever"])
def test_solver_kernels_agree(rp, name, oracle_mod):
    # every moment-matrix kernel gives the same bits: gradients, K, and the kept factors the adjoint uses
    # (the window kernel is compared with the oracle by the tests above)
    import torch
    prob = SMALL[name]()
    print(f"[gpu case] solver kernels {name}: gps={prob.n_gp}", flush=True)
    plan = rp.Plan.from_problem(prob)
    plan.build_pattern()
    E = torch.from_numpy(prob.cell_E).cuda()
    out = {}
    for kind in ("window", "panel", "lds"):
        plan.set_solver(kind)
        K = plan.assemble(cell_E=E, nu=prob.nu, keep_factors=True)
        plan.status()
        dK = torch.ones_like(K)
        dE, dX = plan.assemble_backward(plan.node_xyz, E, prob.nu, dK)
        out[kind] = (plan.dphi().cpu().numpy(), K.cpu().numpy(), dE.cpu().numpy(), dX.cpu().numpy())
    for kind in ("panel", "lds"):
        for a, b in zip(out["window"], out[kind]):
            assert np.array_equal(a, b), kind
    if name != "slope_small":
        m = oracle_mod.OracleModel(prob)
        m.build_pattern()
        assert np.array_equal(out["panel"][1], m.assemble())


def test_rebuild_pattern_equals_fresh_plan():
    # A plan rebuilt for moved nodes keeps its arrays where they are large
    # enough and builds buckets and factor offsets on the device: supports,
    # pattern, plan sizes, K and the kept-factor adjoint must equal those of a
    # plan built afresh on the same coordinates, over several rebuilds that
    # grow and shrink the pattern.
    import dataclasses
    import torch
    import paper_1802_04256_amd as rp
    prob = W.slope(L=12.0, W=6.0, H=6.0, x_c=3.0, jitter_seed=5, E_seed=6)
    X1 = prob.node_xyz.copy()
    rng = np.random.default_rng(31)
    X2 = X1 + rng.uniform(-0.2, 0.2, X1.shape)
    print(f"[gpu case] rebuild: nodes={prob.n_nodes} gps={prob.n_gp}", flush=True)
    E = torch.from_numpy(prob.cell_E).cuda()
    plan = rp.Plan.from_problem(prob)
    plan.build_pattern()
    for X in (X2, X1, X2):
        row_ptr, col_idx = plan.rebuild_pattern(X)
        K = plan.assemble(node_xyz=X, cell_E=E, nu=prob.nu, keep_factors=True)
        plan.status()
        fresh = rp.Plan.from_problem(dataclasses.replace(prob, node_xyz=X))
        f_row, f_col = fresh.build_pattern()
        Kf = fresh.assemble(cell_E=E, nu=prob.nu, keep_factors=True)
        fresh.status()
        assert plan.info() == fresh.info()
        for a, b in zip(plan.support(), fresh.support()):
            assert torch.equal(a, b)
        assert torch.equal(row_ptr, f_row) and torch.equal(col_idx, f_col)
        assert torch.equal(K, Kf)
        dK = torch.from_numpy(rng.standard_normal(plan.nnz)).cuda()
        a = plan.assemble_backward(X, E, prob.nu, dK)
        b = fresh.assemble_backward(X, E, prob.nu, dK)
        for u, v in zip(a, b):
            assert torch.equal(u, v)


def test_nan_coordinates_reported():
    # a NaN node coordinate is rejected before any search (bounding box);
    # a NaN Gauss point finds no support node and is reported as that point
    import paper_1802_04256_amd as rp
    prob = W.cantilever()
    prob.node_xyz[7, 1] = np.nan
    plan = rp.Plan.from_problem(prob)
    with pytest.raises(rp.RpimError) as ei:
        plan.build_pattern()
    assert ei.value.code == -1
    prob = W.cantilever()
    prob.gp_xyz[11, 2] = np.nan
    plan = rp.Plan.from_problem(prob)
    with pytest.raises(rp.RpimError) as ei:
        plan.build_pattern()
    assert ei.value.code == -4
    assert "first bad gauss point 11" in str(ei.value)
