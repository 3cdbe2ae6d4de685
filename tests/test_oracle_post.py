"""Pins of the oracle's post-solve quantities (GeoMFree3D Sec. 2: after the
solve the displacements, then the stresses; Sec. 3, Example 1: a cube under
gravity).  Body force f_I = sum_g w_g phi_I(x_g) b_g and Gauss-point stress
sigma_g = E_c D B_g u are pinned by properties the mathematics fixes:
partition of unity and linear reproduction make the total body force equal
b times the volume and its first moment equal b times the quadrature's first
moment; a linear displacement field gives the exact constant stress at every
point; and a column under gravity with rollers (uniaxial strain) has the
closed form u_z = -rho g (2 H z - z^2) / (2 M), M = E (1 - nu) /
((1 + nu)(1 - 2 nu)), sigma_zz = -rho g (H - z)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

import workloads as W


@pytest.fixture(scope="module")
def jbox(oracle_mod):
    prob = W.box(n=4, p=2, jitter=0.3, jitter_seed=17, E_seed=18)
    m = oracle_mod.OracleModel(prob)
    m.build_pattern()
    return prob, m


def test_body_force_total_and_first_moment(jbox):
    prob, m = jbox
    b = np.array([0.3, -1.7, -25480.0])
    f = m.body_force(b)
    V = prob.gp_wdet.sum()
    assert np.allclose(f.sum(0), b * V, rtol=1e-12, atol=0)
    # sum_I f_I x_I^T = b (sum_g w_g x_g)^T, because sum_a phi_a x_a = x_g
    mom = f.T @ prob.node_xyz
    ref = np.outer(b, prob.gp_wdet @ prob.gp_xyz)
    assert np.abs(mom - ref).max() <= 1e-11 * np.abs(ref).max()
    # per-point forces: the same total from different force fields adds up linearly
    f2 = m.body_force(np.tile(b, (prob.n_gp, 1)) * 2.0)
    assert np.allclose(f2, 2.0 * f, rtol=1e-15, atol=0)


def test_stress_of_a_linear_field_is_exact(jbox):
    prob, m = jbox
    rng = np.random.default_rng(19)
    A = rng.standard_normal((3, 3)) * 1e-3
    eps0 = 0.5 * (A + A.T)
    omega = 0.5 * (A - A.T)  # a rigid rotation adds no stress
    u = prob.node_xyz @ (eps0 + omega).T + np.array([0.1, -0.2, 0.3])
    sig = m.gauss_stress(u)
    lam = prob.nu / ((1 + prob.nu) * (1 - 2 * prob.nu))
    mu = 1.0 / (2 * (1 + prob.nu))
    Ec = prob.cell_E[prob.gp_cell]
    S = lam * np.trace(eps0) * np.eye(3) + 2 * mu * eps0
    ref = Ec[:, None] * np.array([S[0, 0], S[1, 1], S[2, 2], S[1, 2], S[0, 2], S[0, 1]])[None, :]
    assert np.abs(sig - ref).max() <= 1e-10 * np.abs(ref).max()


def test_gravity_column_closed_form(oracle_mod):
    # a 100 m cube, 25 m spacing, rollers on the sides, base fixed in z, gravity: uniaxial strain
    H, n = 100.0, 4
    prob = W.box(n=n, h=H / n, p=3, jitter=0.0, jitter_seed=1, E_seed=2)
    prob.cell_E[:] = 1.0e9
    m = oracle_mod.OracleModel(prob)
    m.build_pattern()
    K = m.assemble()
    row_ptr, col_idx = m.pattern()
    X = prob.node_xyz
    fixed = np.sort(np.concatenate([3 * np.where((X[:, 0] == 0) | (X[:, 0] == H))[0],
                                    3 * np.where((X[:, 1] == 0) | (X[:, 1] == H))[0] + 1,
                                    3 * np.where(X[:, 2] == 0)[0] + 2])).astype(np.int32)
    oracle_mod.penalty(row_ptr, col_idx, K, fixed, factor=1e8)
    rho, g = 2600.0, 9.8
    f = m.body_force(np.array([0.0, 0.0, -rho * g])).reshape(-1)
    nd = 3 * prob.n_nodes
    u = spl.spsolve(sp.csr_matrix((K, col_idx, row_ptr), shape=(nd, nd)).tocsc(), f).reshape(-1, 3)
    nu, E = prob.nu, 1.0e9
    M = E * (1 - nu) / ((1 + nu) * (1 - 2 * nu))
    # the coarse 5 x 5 x 5 node grid has local errors near the constrained edges; on average over the
    # top face the settlement is the closed form's
    top = X[:, 2] == H
    settle = -rho * g * H ** 2 / (2 * M)
    assert abs(u[top, 2].mean() / settle - 1) <= 5e-3
    sig = m.gauss_stress(u)
    z = prob.gp_xyz[:, 2]
    # weighted mean of sigma_zz over the volume: -rho g H / 2
    mean = (prob.gp_wdet @ sig[:, 2]) / prob.gp_wdet.sum()
    assert abs(mean / (-rho * g * H / 2) - 1) <= 0.02
    # lateral stress of uniaxial strain: sigma_xx = nu / (1 - nu) sigma_zz (median over the points)
    assert abs(np.median(sig[:, 0] / sig[:, 2]) / (nu / (1 - nu)) - 1) <= 0.05
