"""GPU adjoint (rpim_assemble_backward, autograd) against the oracle's FP64
adjoint and against central finite differences evaluated in __float128.

The adjoint passes through solves with the ill-conditioned moment matrix, so
two FP64 evaluations that sum in different orders agree to ~1e-8 relative;
the bar against the oracle's adjoint is 1e-6 (scaled by the largest entry
where an entry is tiny), and against the extended-precision finite
differences 1e-6.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def rel_err(g, ref):
    scale = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    return float(np.max(np.abs(g - ref) / scale))


def probe_kbar(row_ptr, col_idx, n_dof, n_vec=8, seed=5):
    V = W.probe_vectors(n_dof, n_vec, seed)
    rows = np.repeat(np.arange(n_dof), np.diff(row_ptr))
    return 0.5 * np.einsum("vi,vi->i", V[:, rows], V[:, col_idx])


CASES = {
    "cantilever": lambda: W.cantilever(),
    "jbox4": lambda: W.box(n=4, p=2, jitter=0.3, jitter_seed=21, E_seed=22),
    "slope_small": lambda: W.slope(L=12.0, W=6.0, H=6.0, x_c=3.0, jitter_seed=5, E_seed=6),
}


_ORACLE_BWD = {}  # (case, load) -> the oracle's (dE, dX): the same load is checked twice


def oracle_backward(name, m, kind, Kb):
    if (name, kind) not in _ORACLE_BWD:
        _ORACLE_BWD[(name, kind)] = m.backward(Kb)
    return _ORACLE_BWD[(name, kind)]


@pytest.fixture(scope="module", params=list(CASES))
def case(request, oracle_mod):
    import torch
    import paper_1802_04256_amd as rp
    prob = CASES[request.param]()
    print(f"[gpu case] adjoint {request.param}: nodes={prob.n_nodes} gps={prob.n_gp}", flush=True)
    m = oracle_mod.OracleModel(prob)
    m.build_pattern()
    plan = rp.Plan.from_problem(prob)
    plan.build_pattern()
    return request.param, prob, m, plan


@pytest.mark.parametrize("kind", ["probe", "random"])
def test_backward_vs_oracle(case, kind):
    name, prob, m, plan = case
    row_ptr, col_idx = m.pattern()
    if kind == "probe":
        Kb = probe_kbar(row_ptr, col_idx, 3 * prob.n_nodes)
    else:
        Kb = np.random.default_rng(9).standard_normal(m.nnz)
    plan.assemble(cell_E=prob.cell_E, nu=prob.nu, keep_factors=True)
    dE, dX = plan.assemble_backward(prob.node_xyz, prob.cell_E, prob.nu, Kb)
    plan.status()
    dEo, dXo = oracle_backward(name, m, kind, Kb)
    eE = rel_err(dE.cpu().numpy(), dEo)
    eX = rel_err(dX.cpu().numpy(), dXo)
    print(f"[{name}/{kind}] dE rel err {eE:.2e}  dX rel err {eX:.2e}")
    assert eE < 1e-10
    assert eX < 1e-6


def test_backward_vs_quad_fd(case):
    name, prob, m, plan = case
    row_ptr, col_idx = m.pattern()
    Kb = probe_kbar(row_ptr, col_idx, 3 * prob.n_nodes)
    plan.assemble(cell_E=prob.cell_E, nu=prob.nu, keep_factors=True)
    _, dX = plan.assemble_backward(prob.node_xyz, prob.cell_E, prob.nu, Kb)
    dX = dX.cpu().numpy()
    gp_ptr, gp_nbr = m.support()
    owner = np.repeat(np.arange(prob.n_gp), np.diff(gp_ptr))
    rng = np.random.default_rng(6)
    got, ref = [], []
    # the full-size slope has 32 stored extended-precision samples; one here for the larger small case
    n_fd = 1 if name == "slope_small" else 2
    for i, k in zip(rng.integers(0, prob.n_nodes, n_fd), rng.integers(0, 3, n_fd)):
        gps = np.unique(owner[gp_nbr == i])
        h = 1e-6 * prob.d_c
        Xp, Xm = prob.node_xyz.copy(), prob.node_xyz.copy()
        Xp[i, k] += h
        Xm[i, k] -= h
        hp, lp = m.dot_q(Kb, gps, node_xyz=Xp)
        hm, lm = m.dot_q(Kb, gps, node_xyz=Xm)
        ref.append(((hp - hm) + (lp - lm)) / (Xp[i, k] - Xm[i, k]))
        got.append(dX[i, k])
    assert rel_err(np.array(got), np.array(ref)) < 1e-6


def test_autograd_function(case):
    import torch
    import paper_1802_04256_amd as rp
    name, prob, m, plan = case
    X = torch.from_numpy(prob.node_xyz.copy()).cuda().requires_grad_(True)
    E = torch.from_numpy(prob.cell_E.copy()).cuda().requires_grad_(True)
    K = rp.assemble(plan, X, E, prob.nu)
    row_ptr, col_idx = m.pattern()
    Kb = torch.from_numpy(probe_kbar(row_ptr, col_idx, 3 * prob.n_nodes)).cuda()
    L = (K * Kb).sum()
    L.backward()
    dEo, dXo = oracle_backward(name, m, "probe", Kb.cpu().numpy())
    assert rel_err(E.grad.cpu().numpy(), dEo) < 1e-10
    assert rel_err(X.grad.cpu().numpy(), dXo) < 1e-6
    # Euler homogeneity: sum_c E_c dL/dE_c = L
    assert abs(float((E.detach() * E.grad).sum()) - float(L)) <= 1e-11 * abs(float(L))


def test_backward_needs_kept_factors():
    import paper_1802_04256_amd as rp
    prob = W.cantilever()
    plan = rp.Plan.from_problem(prob)
    plan.build_pattern()
    plan.assemble(cell_E=prob.cell_E, nu=prob.nu, keep_factors=False)
    with pytest.raises(rp.RpimError) as ei:
        plan.assemble_backward(prob.node_xyz, prob.cell_E, prob.nu, np.zeros(plan.nnz))
    assert ei.value.code == -8


def test_backward_large_supports(oracle_mod):
    # supports up to 131 rows: the adjoint's per-point kernel runs two and three
    # waves, handing substitution values between waves through LDS
    import paper_1802_04256_amd as rp
    prob = W.box(n=8, p=2, jitter=0.3, jitter_seed=61, E_seed=62)
    prob.support_radius = 3.05
    print(f"[gpu case] adjoint box8 radius 3.05: nodes={prob.n_nodes} gps={prob.n_gp}", flush=True)
    m = oracle_mod.OracleModel(prob)
    m.build_pattern()
    plan = rp.Plan.from_problem(prob)
    plan.build_pattern()
    assert plan.info()["max_n"] + 4 > 128
    row_ptr, col_idx = m.pattern()
    Kb = probe_kbar(row_ptr, col_idx, 3 * prob.n_nodes)
    plan.assemble(cell_E=prob.cell_E, nu=prob.nu, keep_factors=True)
    dE, dX = plan.assemble_backward(prob.node_xyz, prob.cell_E, prob.nu, Kb)
    plan.status()
    dEo, dXo = m.backward(Kb)
    assert rel_err(dE.cpu().numpy(), dEo) < 1e-10
    assert rel_err(dX.cpu().numpy(), dXo) < 1e-6


def test_backward_of_an_older_forward_raises():
    import torch
    import paper_1802_04256_amd as rp
    prob = W.cantilever()
    plan = rp.Plan.from_problem(prob)
    plan.build_pattern()
    E = torch.from_numpy(prob.cell_E.copy()).cuda()
    X1 = torch.from_numpy(prob.node_xyz.copy()).cuda().requires_grad_(True)
    X2 = torch.from_numpy(prob.node_xyz * 1.001).cuda().requires_grad_(True)
    K1 = rp.assemble(plan, X1, E, prob.nu)
    K2 = rp.assemble(plan, X2, E, prob.nu)
    with pytest.raises(rp.RpimError) as ei:
        K1.sum().backward()
    assert ei.value.code == -8
    K2.sum().backward()  # the latest forward still differentiates
    assert X2.grad is not None and torch.isfinite(X2.grad).all()
