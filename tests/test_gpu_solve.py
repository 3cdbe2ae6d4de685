"""Stage 3 on the GPU: Jacobi-preconditioned CG (rpim_solve_pcg) on the
penalty-constrained stiffness, through the C ABI.

Checked against SciPy's direct sparse solve of the same matrix, for
determinism (two solves, same bits), against the Timoshenko closed form for
the cantilever tip deflection (the whole path on the GPU: assembly, penalty,
solve), and on its error paths (no positive diagonal, iteration limit)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

import workloads as W

pytestmark = pytest.mark.gpu


def _cantilever_system(rp, precision="fp64", prob=None):
    import torch
    prob = prob or W.cantilever()
    plan = rp.Plan.from_problem(prob)
    row_ptr, col_idx = plan.build_pattern()
    K = plan.assemble(cell_E=prob.cell_E, nu=prob.nu, precision=precision)
    X = prob.node_xyz
    fixed = np.sort((3 * np.where(X[:, 0] == 0.0)[0][:, None] + np.arange(3)).ravel()).astype(np.int32)
    rp.apply_penalty_bc(row_ptr, col_idx, K, fixed, factor=1e8)
    L = X[:, 0].max()
    f = np.zeros(3 * prob.n_nodes)
    for i in np.where(X[:, 0] == L)[0]:  # unit shear on the end face, tensor-trapezoid weights
        wy = 0.5 if X[i, 1] in (X[:, 1].min(), X[:, 1].max()) else 1.0
        wz = 0.5 if X[i, 2] in (X[:, 2].min(), X[:, 2].max()) else 1.0
        f[3 * i + 2] = -wy * wz
    f /= -f.sum()  # total load 1 N downwards
    return prob, plan, row_ptr, col_idx, K, torch.from_numpy(f).cuda()


def test_pcg_matches_direct_solve_and_is_deterministic():
    import paper_1802_04256_amd as rp
    prob, plan, row_ptr, col_idx, K, f = _cantilever_system(rp)
    print(f"[gpu case] pcg cantilever: dofs={3 * prob.n_nodes}", flush=True)
    x1, it1, res1 = rp.solve_pcg(row_ptr, col_idx, K, f, rtol=1e-12)
    x2, it2, res2 = rp.solve_pcg(row_ptr, col_idx, K, f, rtol=1e-12)
    assert it1 == it2 and res1 == res2 and np.array_equal(x1.cpu().numpy(), x2.cpu().numpy())
    assert res1 <= 1e-12
    n = 3 * prob.n_nodes
    A = sp.csr_matrix((K.cpu().numpy(), col_idx.cpu().numpy(), row_ptr.cpu().numpy()), shape=(n, n))
    ref = spl.spsolve(A.tocsc(), f.cpu().numpy())
    err = np.linalg.norm(x1.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"CG iterations {it1}, relative residual {res1:.2e}, error vs direct {err:.2e}")
    assert err <= 1e-6  # the penalty makes K ill conditioned (cond ~ 1e8 * 1e4)


def test_pcg_cantilever_tip_deflection():
    # assembly, penalty and solve all on the GPU; Timoshenko: P L^3/(3EI) + (4+5nu) P L D^2/(24 E I)
    import paper_1802_04256_amd as rp
    prob, plan, row_ptr, col_idx, K, f = _cantilever_system(rp)
    x, it, res = rp.solve_pcg(row_ptr, col_idx, K, f, rtol=1e-12)
    u = x.cpu().numpy()
    X = prob.node_xyz
    tip = np.where((X[:, 0] == 8.0) & (X[:, 1] == 1.0) & (X[:, 2] == 1.0))[0][0]
    E, nu, Lb, D, b, P = 3.0e7, 0.3, 8.0, 2.0, 2.0, 1.0
    I = b * D ** 3 / 12.0
    delta = P * Lb ** 3 / (3 * E * I) + (4 + 5 * nu) * P * Lb * D ** 2 / (24 * E * I)
    ratio = -u[3 * tip + 2] / delta
    print(f"tip deflection / Timoshenko = {ratio:.4f} ({it} iterations)")
    assert 0.95 <= ratio <= 1.05


def test_pcg_mixed_precision_K():
    import paper_1802_04256_amd as rp
    _, _, row_ptr, col_idx, K64, f = _cantilever_system(rp, "fp64")
    _, _, _, _, K32, _ = _cantilever_system(rp, "mixed")
    x64, _, _ = rp.solve_pcg(row_ptr, col_idx, K64, f, rtol=1e-12)
    x32, it, res = rp.solve_pcg(row_ptr, col_idx, K32, f, rtol=1e-12)
    err = float((x32 - x64).norm() / x64.norm())
    print(f"mixed-precision K: displacement error {err:.2e} ({it} iterations)")
    assert res <= 1e-12 and err <= 1e-4


def test_pcg_error_paths():
    import torch
    import paper_1802_04256_amd as rp
    _, _, row_ptr, col_idx, K, f = _cantilever_system(rp)
    with pytest.raises(rp.RpimError) as ei:
        rp.solve_pcg(row_ptr, col_idx, K, f, rtol=1e-14, max_iter=3)
    assert ei.value.code == -9
    x, it, res = rp.solve_pcg(row_ptr, col_idx, K, f, rtol=1e-14, max_iter=3, raise_on_error=False)
    assert it == 3 and torch.isfinite(x).all()
    # a zero diagonal (no Jacobi preconditioner)
    S = sp.csr_matrix(np.diag([2.0, 0.0, 3.0]))
    rp3 = torch.from_numpy(S.indptr.astype(np.int64)).cuda()
    ci3 = torch.from_numpy(S.indices.astype(np.int32)).cuda()
    K3 = torch.from_numpy(S.data.copy()).cuda()
    with pytest.raises(rp.RpimError) as ei:
        rp.solve_pcg(rp3, ci3, K3, np.ones(3))
    assert ei.value.code == -5
