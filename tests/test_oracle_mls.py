"""Pins of the oracle's moving-least-squares and Shepard shape functions
(GeoMFree3D Sec. 4 names moving least squares as the package's next shape
functions).  They check reproduction properties, an independent textbook
evaluation in global coordinates, Shepard's closed form, central differences
of the values, and the stiffness the functions give: symmetry, null space,
the linear-field energy identity and the cantilever tip deflection."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from test_oracle_pins import _rigid_modes, _tip_deflection, dense


def cubic_spline(r):
    """Cubic-spline weight W(r) and W'(r), written from its piecewise definition."""
    r = np.asarray(r, float)
    w = np.where(r <= 0.5, 2 / 3 - 4 * r ** 2 + 4 * r ** 3,
                 np.where(r <= 1.0, 4 / 3 - 4 * r + 4 * r ** 2 - 4 / 3 * r ** 3, 0.0))
    dw = np.where(r <= 0.5, -8 * r + 12 * r ** 2, np.where(r <= 1.0, -4 + 8 * r - 4 * r ** 2, 0.0))
    return w, dw


def weights(X, xg, ds):
    d = xg - X                       # x_g - x_i
    r = np.sqrt((d ** 2).sum(1)) / ds
    w, dw = cubic_spline(r)
    with np.errstate(invalid="ignore", divide="ignore"):
        gw = np.where(r[:, None] > 0, (dw / (r * ds * ds))[:, None] * d, 0.0)  # dW/dx at x_g
    return w, gw


@pytest.fixture(scope="module")
def models(oracle_mod):
    out = {}
    for name, p in (("cant", W.cantilever()), ("jbox", W.box(n=4, p=2, jitter=0.3, jitter_seed=3, E_seed=4))):
        for kind in ("mls", "shepard"):
            m = oracle_mod.OracleModel(p, kind)
            m.build_pattern()
            out[(name, kind)] = (p, m)
    return out


@pytest.mark.parametrize("name", ["cant", "jbox"])
@pytest.mark.parametrize("kind", ["mls", "shepard"])
def test_reproduction(models, name, kind):
    p, m = models[(name, kind)]
    gp_ptr, gp_nbr = m.support()
    for g in range(0, p.n_gp, max(1, p.n_gp // 40)):
        phi, dphi = m.shape(g)
        X = p.node_xyz[gp_nbr[gp_ptr[g]:gp_ptr[g + 1]]]
        assert abs(phi.sum() - 1) <= 1e-13
        assert np.abs(dphi.sum(0)).max() <= 1e-13
        if kind == "mls":  # a linear basis reproduces linear fields and their gradients
            assert np.abs(phi @ X - p.gp_xyz[g]).max() <= 1e-12
            assert np.abs(dphi.T @ X - np.eye(3)).max() <= 1e-12
        else:
            assert phi.min() >= 0.0


@pytest.mark.parametrize("name", ["cant", "jbox"])
def test_mls_matches_textbook_global_basis(models, name):
    # phi = p(x_g)^T A^-1 B with the unshifted basis p(x) = [1, x, y, z];
    # dphi_k = p_k^T A^-1 B + p^T A^-1 (B_k - A_k A^-1 B), solved with numpy
    p, m = models[(name, "mls")]
    gp_ptr, gp_nbr = m.support()
    for g in range(0, p.n_gp, max(1, p.n_gp // 25)):
        phi, dphi = m.shape(g)
        X = p.node_xyz[gp_nbr[gp_ptr[g]:gp_ptr[g + 1]]]
        xg = p.gp_xyz[g]
        w, gw = weights(X, xg, p.support_radius)
        P = np.hstack([np.ones((len(X), 1)), X])
        A = (P * w[:, None]).T @ P
        B = P.T * w
        px = np.r_[1.0, xg]
        AiB = np.linalg.solve(A, B)
        ref = px @ AiB
        dref = np.zeros((len(X), 3))
        for k in range(3):
            Ak = (P * gw[:, k:k + 1]).T @ P
            Bk = P.T * gw[:, k]
            pk = np.eye(4)[k + 1]
            dref[:, k] = pk @ AiB + px @ np.linalg.solve(A, Bk - Ak @ AiB)
        scale = np.abs(ref).max()
        assert np.abs(phi - ref).max() <= 1e-10 * scale
        assert np.abs(dphi - dref).max() <= 1e-9 * np.abs(dref).max()


@pytest.mark.parametrize("name", ["cant", "jbox"])
def test_shepard_is_the_normalised_weight(models, name):
    p, m = models[(name, "shepard")]
    gp_ptr, gp_nbr = m.support()
    for g in range(0, p.n_gp, max(1, p.n_gp // 25)):
        phi, dphi = m.shape(g)
        X = p.node_xyz[gp_nbr[gp_ptr[g]:gp_ptr[g + 1]]]
        w, gw = weights(X, p.gp_xyz[g], p.support_radius)
        S, Sk = w.sum(), gw.sum(0)
        assert np.abs(phi - w / S).max() <= 1e-14
        dref = (gw * S - w[:, None] * Sk) / S ** 2
        assert np.abs(dphi - dref).max() <= 1e-12 * np.abs(dref).max()


@pytest.mark.parametrize("kind", ["mls", "shepard"])
def test_gradient_vs_central_difference(oracle_mod, kind):
    # the values at x_g +- h e_k, from one-point models, against the gradient at x_g
    p = W.box(n=4, p=2, jitter=0.3, jitter_seed=3, E_seed=4)
    h = 1e-6
    for g in (5, 60, 333):
        xg = p.gp_xyz[g]

        def values(x):
            q = dataclasses.replace(p, gp_xyz=x[None, :].copy(), gp_wdet=np.ones(1), gp_cell=np.zeros(1, np.int32),
                                    node_off=np.zeros(2, np.int64))
            mm = oracle_mod.OracleModel(q, kind)
            mm.build_pattern()
            ptr, nbr = mm.support()
            phi, dphi = mm.shape(0)
            return dict(zip(nbr.tolist(), phi)), dict(zip(nbr.tolist(), map(tuple, dphi)))

        v0, d0 = values(xg)
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            vp, _ = values(xg + e)
            vm, _ = values(xg - e)
            for i, dv in d0.items():
                fd = (vp.get(i, 0.0) - vm.get(i, 0.0)) / (2 * h)
                assert abs(fd - dv[k]) <= 1e-6 * max(1.0, abs(dv[k])), (kind, g, i, k)


def test_mls_stiffness_null_space_and_patch(models):
    p, m = models[("cant", "mls")]
    D = dense(m, m.assemble())
    assert np.array_equal(D, D.T)
    ev = np.linalg.eigvalsh(D)
    assert np.all(np.abs(ev[:6]) <= 1e-10 * ev[-1]) and ev[6] >= 1e-5 * ev[-1]
    U = _rigid_modes(p.node_xyz)
    assert (np.linalg.norm(D @ U, axis=0) / (np.linalg.norm(D, 2) * np.linalg.norm(U, axis=0))).max() < 1e-12
    # linear reproduction of gradients: the energy of u = eps x is exact
    rng = np.random.default_rng(3)
    A = rng.standard_normal((3, 3))
    eps = 0.5 * (A + A.T)
    u = (p.node_xyz @ eps.T).ravel()
    lam = p.nu / ((1 + p.nu) * (1 - 2 * p.nu))
    mu = 1 / (2 * (1 + p.nu))
    ref = np.sum(p.gp_wdet * p.cell_E[p.gp_cell]) * (lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps))
    assert abs(u @ D @ u - ref) <= 1e-11 * ref


def test_shepard_stiffness_null_space_is_the_translations(models):
    # constants are reproduced, gradients of linear fields are not: exactly three zero modes
    p, m = models[("cant", "shepard")]
    D = dense(m, m.assemble())
    assert np.array_equal(D, D.T)
    ev = np.linalg.eigvalsh(D)
    assert np.all(np.abs(ev[:3]) <= 1e-10 * ev[-1]) and ev[3] >= 1e-6 * ev[-1]
    T = _rigid_modes(p.node_xyz)[:, :3]
    assert (np.linalg.norm(D @ T, axis=0) / (np.linalg.norm(D, 2) * np.linalg.norm(T, axis=0))).max() < 1e-12


@pytest.mark.parametrize("kind,lo,hi", [("mls", 0.95, 1.10), ("shepard", 0.95, 1.15)])
def test_cantilever_tip_deflection(models, kind, lo, hi):
    p, m = models[("cant", kind)]
    E, nu, L, b = 3.0e7, 0.3, 8.0, 2.0
    I = b ** 4 / 12
    dT = L ** 3 / (3 * E * I) + (4 + 5 * nu) * L * b ** 2 / (24 * E * I)
    assert lo <= _tip_deflection(p, m, m.assemble()) / dT <= hi


def test_mls_adjoint_is_not_offered(models):
    p, m = models[("cant", "mls")]
    with pytest.raises(Exception):
        m.backward(np.zeros(m.nnz))
