"""Pins of the oracle's adjoint (dL/dE per cell, dL/dx per node) -- no GPU.

The finite differences are evaluated in __float128 with the supports frozen:
in FP64 a central difference on a node coordinate is ~1e-3 wrong because the
moment matrix has cond ~1e10, which would hide any error in the adjoint.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W


def rel_err(g, ref):
    scale = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    return float(np.max(np.abs(g - ref) / scale))


@pytest.fixture(scope="module")
def small(oracle_mod):
    p = W.box(n=4, p=2, jitter=0.3, jitter_seed=21, E_seed=22)
    m = oracle_mod.OracleModel(p)
    m.build_pattern()
    return p, m


def probe_kbar(m, p, n_vec=8, seed=5):
    """dL/dK for L = sum_v 0.5 v^T K v, restricted to the pattern."""
    rp, ci = m.pattern()
    V = W.probe_vectors(3 * p.n_nodes, n_vec, seed)
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    return 0.5 * np.einsum("vi,vi->i", V[:, rows], V[:, ci])


def random_kbar(m, seed=9):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(m.nnz)  # not symmetric


def gps_touching(m, node):
    gp_ptr, gp_nbr = m.support()
    rows = np.repeat(np.arange(len(gp_ptr) - 1), np.diff(gp_ptr))
    return np.unique(rows[gp_nbr == node])


@pytest.mark.parametrize("kind", ["probe", "random"])
def test_dE_euler_homogeneity(small, kind):
    p, m = small
    Kb = probe_kbar(m, p) if kind == "probe" else random_kbar(m)
    dE, _ = m.backward(Kb)
    K = m.assemble()
    L = float(Kb @ K)
    assert abs(float(p.cell_E @ dE) - L) <= 1e-12 * abs(L) + 1e-12 * float(np.abs(Kb) @ np.abs(K))


def test_dE_vs_central_fd(small):
    p, m = small
    Kb = probe_kbar(m, p)
    dE, _ = m.backward(Kb)
    for c in (0, 17, 63):
        gps = np.where(p.gp_cell == c)[0]
        h = 1e-6 * p.cell_E[c]
        Ep, Em = p.cell_E.copy(), p.cell_E.copy()
        Ep[c] += h
        Em[c] -= h
        hp, lp = m.dot_q(Kb, gps, cell_E=Ep)
        hm, lm = m.dot_q(Kb, gps, cell_E=Em)
        fd = ((hp - hm) + (lp - lm)) / (Ep[c] - Em[c])
        assert abs(fd - dE[c]) <= 1e-9 * abs(dE[c])


@pytest.mark.parametrize("kind", ["probe", "random"])
def test_dX_vs_extended_precision_fd(small, kind):
    p, m = small
    Kb = probe_kbar(m, p) if kind == "probe" else random_kbar(m)
    _, dX = m.backward(Kb)
    rng = np.random.default_rng(6)
    samples = [(int(i), int(k)) for i, k in zip(rng.integers(0, p.n_nodes, 2), rng.integers(0, 3, 2))]
    got, ref = [], []
    for i, k in samples:
        gps = gps_touching(m, i)
        h = 1e-6 * p.d_c
        Xp, Xm = p.node_xyz.copy(), p.node_xyz.copy()
        Xp[i, k] += h
        Xm[i, k] -= h
        hp, lp = m.dot_q(Kb, gps, node_xyz=Xp)
        hm, lm = m.dot_q(Kb, gps, node_xyz=Xm)
        fd = ((hp - hm) + (lp - lm)) / (Xp[i, k] - Xm[i, k])
        got.append(dX[i, k])
        ref.append(fd)
    assert rel_err(np.array(got), np.array(ref)) < 1e-6
