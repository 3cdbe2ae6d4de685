"""Pins of the CPU oracle against what mathematics fixes (no GPU).

Each test checks the oracle against something other than itself: a
high-precision library value, a closed form, an invariant of the method, or
an independent brute-force construction.  A plausible slip anywhere in the
oracle (a dropped term, a sign, a transposed index) fails at least one.
"""
import math

import mpmath
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.spatial import cKDTree

import workloads as W


# --------------------------------------------------------------------------
# shared small models
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def cant(oracle_mod):
    p = W.cantilever()
    m = oracle_mod.OracleModel(p)
    m.build_pattern()
    return p, m


@pytest.fixture(scope="module")
def jbox(oracle_mod):
    # jittered 5 m cube, 216 nodes, 125 cells x 8 Gauss points
    p = W.box(n=5, p=2)
    m = oracle_mod.OracleModel(p)
    m.build_pattern()
    return p, m


def dense(m, K):
    rp, ci = m.pattern()
    n = len(rp) - 1
    return sp.csr_matrix((K.astype(np.float64), ci, rp), shape=(n, n)).toarray()


# --------------------------------------------------------------------------
# correctly rounded power (contract C4): nearest double to the exact value
# --------------------------------------------------------------------------
def test_pow_correctly_rounded_vs_mpmath(oracle_mod):
    mpmath.mp.prec = 200
    rng = np.random.default_rng(11)
    xs = np.concatenate([rng.uniform(16.0, 45.0, 4000), np.arange(16.0, 42.0)])
    for q in (1.03, 0.03 + 1.0, 1.5, 0.5):
        for x in xs:
            exact = mpmath.power(mpmath.mpf(float(x)), mpmath.mpf(q))
            assert oracle_mod.pow_cr(x, q) == float(exact), (x, q)


def test_pow_quad_reference_and_fallback_used(oracle_mod):
    # the quad path agrees with mpmath to ~1e-33 relative, and the powl fast
    # path hands ambiguous cases to it (about 1 in 64 random arguments)
    mpmath.mp.prec = 200
    rng = np.random.default_rng(12)
    f0, _ = oracle_mod.pow_stats()
    for x in rng.uniform(16.0, 45.0, 2000):
        hi, lo = oracle_mod.pow_q(x, 1.03)
        exact = mpmath.power(mpmath.mpf(float(x)), mpmath.mpf(1.03))
        assert abs((mpmath.mpf(hi) + mpmath.mpf(lo)) - exact) < 1e-31 * exact
        oracle_mod.pow_cr(x, 1.03)
    f1, hard = oracle_mod.pow_stats()
    assert f1 - f0 > 5
    assert hard == 0


# --------------------------------------------------------------------------
# support search and pattern
# --------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["cant", "jbox"])
def test_support_matches_kdtree(which, request):
    p, m = request.getfixturevalue(which)
    gp_ptr, gp_nbr = m.support()
    tree = cKDTree(p.node_xyz)
    r = p.support_radius
    for g in range(p.n_gp):
        S = gp_nbr[gp_ptr[g]:gp_ptr[g + 1]]
        assert np.all(np.diff(S) > 0)  # sorted, unique (C3)
        lo = set(tree.query_ball_point(p.gp_xyz[g], r * (1 - 1e-12)))
        hi = set(tree.query_ball_point(p.gp_xyz[g], r * (1 + 1e-12)))
        assert lo <= set(S.tolist()) <= hi


@pytest.mark.parametrize("which", ["cant", "jbox"])
def test_pattern_is_incidence_product(which, request):
    p, m = request.getfixturevalue(which)
    gp_ptr, gp_nbr = m.support()
    A = sp.csr_matrix((np.ones(len(gp_nbr)), gp_nbr, gp_ptr), shape=(p.n_gp, p.n_nodes))
    AtA = (A.T @ A).tocsr()
    AtA.sort_indices()
    rp, ci = m.pattern()
    # expand the node-block pattern to scalar dofs: kron with a 3x3 block of ones
    S = sp.kron(AtA, np.ones((3, 3)), format="csr")
    S.sort_indices()
    assert np.array_equal(S.indptr, rp)
    assert np.array_equal(S.indices, ci)


def test_cantilever_support_sizes(cant):
    p, m = cant
    n = np.diff(m.support()[0])
    assert (n.min(), float(np.median(n)), n.max()) == (20, 34.5, 40)


def test_too_small_support_is_reported(oracle_mod):
    p = W.cantilever()
    p.support_radius = 0.6
    m = oracle_mod.OracleModel(p)
    with pytest.raises(oracle_mod.OracleError) as ei:
        m.build_pattern()
    assert ei.value.code == oracle_mod.E_SUPPORT


# --------------------------------------------------------------------------
# shape functions
# --------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["cant", "jbox"])
def test_partition_of_unity_and_linear_reproduction(which, request):
    p, m = request.getfixturevalue(which)
    gp_ptr, gp_nbr = m.support()
    for g in range(0, p.n_gp, 7):
        S = gp_nbr[gp_ptr[g]:gp_ptr[g + 1]]
        phi, dphi = m.shape(g)
        xa = p.node_xyz[S]
        assert abs(phi.sum() - 1.0) < 1e-13
        assert np.abs(phi @ xa - p.gp_xyz[g]).max() < 1e-12
        # derivative reproduction (patch test at the Gauss point)
        assert np.abs(dphi.sum(axis=0)).max() < 1e-12
        assert np.abs(dphi.T @ xa - np.eye(3)).max() < 1e-12


def test_kronecker_delta_at_nodes(oracle_mod):
    # Gauss points placed exactly on field nodes: phi_a(x_b) = delta_ab
    base = W.box(n=4, p=2, jitter=0.3)
    idx = np.array([31, 62, 93, 55])
    p = W.Problem(name="kd", node_xyz=base.node_xyz, gp_xyz=base.node_xyz[idx].copy(),
                  gp_wdet=np.ones(len(idx)), gp_cell=np.zeros(len(idx), np.int32),
                  cell_E=np.ones(1), support_radius=2.5)
    m = oracle_mod.OracleModel(p)
    m.build_pattern()
    gp_ptr, gp_nbr = m.support()
    for g, node in enumerate(idx):
        S = gp_nbr[gp_ptr[g]:gp_ptr[g + 1]]
        phi, _ = m.shape(g)
        expect = (S == node).astype(float)
        assert np.abs(phi - expect).max() < 1e-9


def _mp_shape(p, S, xg, digits=40):
    """Shape functions and derivatives at xg by an mpmath solve (exact-ish)."""
    mpmath.mp.dps = digits
    n = len(S)
    N = n + 4
    C2 = mpmath.mpf(p.alpha_c * p.d_c) ** 2
    q = mpmath.mpf(p.q)
    X = [[mpmath.mpf(float(v)) for v in p.node_xyz[i]] for i in S]
    xg = [mpmath.mpf(float(v)) for v in xg]
    G = mpmath.matrix(N, N)
    for a in range(n):
        for b in range(n):
            s = sum((X[a][k] - X[b][k]) ** 2 for k in range(3))
            G[a, b] = (s + C2) ** q
        G[a, n] = G[n, a] = 1
        for k in range(3):
            G[a, n + 1 + k] = G[n + 1 + k, a] = X[a][k] - xg[k]
    R = mpmath.matrix(N, 4)
    for a in range(n):
        s = sum((X[a][k] - xg[k]) ** 2 for k in range(3))
        t = s + C2
        for k in range(3):
            R[a, k] = 2 * q * t ** (q - 1) * (xg[k] - X[a][k])
        R[a, 3] = t ** q
    for k in range(3):
        R[n + 1 + k, k] = 1
    R[n, 3] = 1
    Gi = mpmath.inverse(G)
    Y = Gi * R
    dphi = np.array([[float(Y[a, k]) for k in range(3)] for a in range(n)])
    phi = np.array([float(Y[a, 3]) for a in range(n)])
    return phi, dphi


def test_shape_vs_high_precision(jbox):
    p, m = jbox
    gp_ptr, gp_nbr = m.support()
    for g in (3, 777):
        S = gp_nbr[gp_ptr[g]:gp_ptr[g + 1]]
        phi, dphi = m.shape(g)
        phi_mp, dphi_mp = _mp_shape(p, S, p.gp_xyz[g])
        # FP64 floor of the ill-conditioned moment matrix is ~1e-8 relative
        assert np.abs(dphi - dphi_mp).max() < 1e-6 * np.abs(dphi_mp).max()
        assert np.abs(phi - phi_mp).max() < 1e-6


# --------------------------------------------------------------------------
# the stiffness matrix
# --------------------------------------------------------------------------
def _voigt_B(dphi):
    n = len(dphi)
    B = np.zeros((6, 3 * n))
    for a in range(n):
        dx, dy, dz = dphi[a]
        B[0, 3 * a] = dx
        B[1, 3 * a + 1] = dy
        B[2, 3 * a + 2] = dz
        B[3, 3 * a + 1], B[3, 3 * a + 2] = dz, dy
        B[4, 3 * a], B[4, 3 * a + 2] = dz, dx
        B[5, 3 * a], B[5, 3 * a + 1] = dy, dx
    return B


def _D(E, nu):
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[[0, 1, 2], [0, 1, 2]] += 2 * mu
    D[[3, 4, 5], [3, 4, 5]] = mu
    return D


@pytest.mark.parametrize("which", ["cant", "jbox"])
def test_single_point_block_is_voigt_BtDB(which, request):
    p, m = request.getfixturevalue(which)
    gp_ptr, gp_nbr = m.support()
    for g in (0, p.n_gp // 3, p.n_gp - 1):
        S = gp_nbr[gp_ptr[g]:gp_ptr[g + 1]]
        _, dphi = m.shape(g)
        Kg = dense(m, m.assemble(gps=[g]))
        dofs = (3 * S[:, None] + np.arange(3)).ravel()
        B = _voigt_B(dphi)
        ref = p.gp_wdet[g] * B.T @ _D(p.cell_E[p.gp_cell[g]], p.nu) @ B
        sub = Kg[np.ix_(dofs, dofs)]
        assert np.abs(sub - ref).max() <= 1e-14 * np.abs(ref).max()
        # nothing lands outside the support block
        Kg[np.ix_(dofs, dofs)] = 0
        assert not Kg.any()


def test_stiffness_is_sum_over_points(jbox):
    p, m = jbox
    K = m.assemble()
    parts = [m.assemble(gps=np.arange(s, min(s + 200, p.n_gp))) for s in range(0, p.n_gp, 200)]
    ref = np.sum(parts, axis=0)
    assert np.abs(K - ref).max() <= 1e-12 * np.abs(K).max()


@pytest.mark.parametrize("which", ["cant", "jbox"])
def test_symmetry_bitwise(which, request):
    p, m = request.getfixturevalue(which)
    D = dense(m, m.assemble())
    assert np.array_equal(D, D.T)


def _rigid_modes(X):
    n = len(X)
    U = np.zeros((3 * n, 6))
    for k in range(3):
        U[k::3, k] = 1.0
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    U[0::3, 3], U[1::3, 3] = -y, x
    U[1::3, 4], U[2::3, 4] = -z, y
    U[0::3, 5], U[2::3, 5] = z, -x
    return U


@pytest.mark.parametrize("which", ["cant", "jbox"])
def test_exactly_six_rigid_modes(which, request):
    p, m = request.getfixturevalue(which)
    D = dense(m, m.assemble())
    ev = np.linalg.eigvalsh(D)
    lmax = ev[-1]
    assert np.all(np.abs(ev[:6]) <= 1e-10 * lmax)
    assert ev[6] >= 1e-6 * lmax
    U = _rigid_modes(p.node_xyz)
    res = np.linalg.norm(D @ U, axis=0) / (np.linalg.norm(D, 2) * np.linalg.norm(U, axis=0))
    assert res.max() < 1e-12


@pytest.mark.parametrize("which", ["cant", "jbox"])
def test_linear_field_energy(which, request):
    # u = eps0 x reproduced exactly by RPIM: u^T K u = sum_g w E (lam tr^2 + 2 mu eps:eps)
    p, m = request.getfixturevalue(which)
    D = dense(m, m.assemble())
    rng = np.random.default_rng(3)
    A = rng.standard_normal((3, 3))
    eps = 0.5 * (A + A.T)
    u = (p.node_xyz @ eps.T).ravel()
    lam = p.nu / ((1 + p.nu) * (1 - 2 * p.nu))
    mu = 1 / (2 * (1 + p.nu))
    dens = lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps)
    ref = np.sum(p.gp_wdet * p.cell_E[p.gp_cell]) * dens
    assert abs(u @ D @ u - ref) <= 1e-11 * ref


def test_quadrature_volume():
    for p in (W.cantilever(), W.box(n=5, p=2), W.slope(), W.cantilever(16, 4, 4, h=0.5)):
        assert abs(p.gp_wdet.sum() - p.volume) <= 1e-13 * p.volume


def test_linear_in_E_bitwise(cant, oracle_mod):
    p, m = cant
    K1 = m.assemble()
    K2 = m.assemble(cell_E=2.0 * p.cell_E)  # power-of-two scaling is exact
    assert np.array_equal(K2, 2.0 * K1)


def _tip_deflection(p, m, K):
    """Fixed end x=0 by penalty, unit total shear -z at x=L (trapezoid weights)."""
    rp, ci = m.pattern()
    X = p.node_xyz
    L = X[:, 0].max()
    fixed_nodes = np.where(X[:, 0] == 0.0)[0]
    fixed = (3 * fixed_nodes[:, None] + np.arange(3)).ravel().astype(np.int32)
    Kp = K.copy()
    import oracle
    oracle.penalty(rp, ci, Kp, fixed, factor=1e8)
    f = np.zeros(3 * p.n_nodes)
    tip = np.where(X[:, 0] == L)[0]
    ys, zs = np.unique(X[tip, 1]), np.unique(X[tip, 2])
    wy = np.ones(len(ys)); wy[[0, -1]] = 0.5
    wz = np.ones(len(zs)); wz[[0, -1]] = 0.5
    wy /= wy.sum(); wz /= wz.sum()
    for i in tip:
        f[3 * i + 2] = -np.interp(X[i, 1], ys, wy) * np.interp(X[i, 2], zs, wz)
    D = sp.csr_matrix((Kp, ci, rp), shape=(len(rp) - 1,) * 2).toarray()
    u = np.linalg.solve(D, f)
    Wd, Hd = X[:, 1].max(), X[:, 2].max()
    mid = np.where((X[:, 0] == L) & (X[:, 1] == Wd / 2) & (X[:, 2] == Hd / 2))[0][0]
    return -u[3 * mid + 2]


def test_timoshenko_cantilever(cant):
    # closed form: PL^3/(3EI) + (4+5nu) P L / (24 E I) * D^2 for a square section
    p, m = cant
    E, nu, L, b = 3.0e7, 0.3, 8.0, 2.0
    I = b ** 4 / 12
    dT = L ** 3 / (3 * E * I) + (4 + 5 * nu) * L * b ** 2 / (24 * E * I)
    assert abs(dT - 4.4500e-6) < 1e-9
    d = _tip_deflection(p, m, m.assemble())
    assert 0.95 <= d / dT <= 1.05


@pytest.mark.slow
def test_timoshenko_refined_closer(oracle_mod, cant):
    p, m = cant
    p2 = W.cantilever(16, 4, 4, h=0.5)
    m2 = oracle_mod.OracleModel(p2)
    m2.build_pattern()
    E, nu, L, b = 3.0e7, 0.3, 8.0, 2.0
    I = b ** 4 / 12
    dT = L ** 3 / (3 * E * I) + (4 + 5 * nu) * L * b ** 2 / (24 * E * I)
    e1 = abs(_tip_deflection(p, m, m.assemble()) / dT - 1)
    e2 = abs(_tip_deflection(p2, m2, m2.assemble()) / dT - 1)
    assert e2 < e1


# --------------------------------------------------------------------------
# penalty boundary conditions (stage 2)
# --------------------------------------------------------------------------
def _read_golden(name):
    """Parse a tests/golden fixture: '#' comments, a 'matrix' block, then 'key values...' lines."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    rows, fields, in_matrix = [], {}, False
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        if line == "matrix":
            in_matrix = True
            continue
        head = line.split()[0]
        if in_matrix and not head[0].isalpha():
            rows.append([float(v) for v in line.split()])
            continue
        in_matrix = False
        fields[head] = [float(v) for v in line.split()[1:]]
    return np.array(rows), fields


def test_penalty_hand_computed(oracle_mod):
    # 6x6 symmetric CSR with a full tridiagonal + corner pattern; expected values
    # are hand-computed from the definition (tests/golden/penalty_6x6.txt)
    Kd, f = _read_golden("penalty_6x6.txt")
    S = sp.csr_matrix(Kd)
    S.sort_indices()
    rp, ci = S.indptr.astype(np.int64), S.indices.astype(np.int32)
    K = S.data.copy()
    rhs = np.zeros(6)
    dofs = np.array(f["constrained"], np.int32)
    alpha = oracle_mod.penalty(rp, ci, K, dofs, u_bar=np.array(f["u_bar"]), factor=f["factor"][0], rhs=rhs)
    assert alpha == f["alpha"][0]
    expect = Kd.copy()
    np.fill_diagonal(expect, f["diag_after"])
    assert np.array_equal(sp.csr_matrix((K, ci, rp), shape=(6, 6)).toarray(), expect)
    assert np.array_equal(rhs, np.array(f["rhs_after"]))
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.penalty(rp, ci, K, np.array([2, 2], np.int32), factor=10.0)


# --------------------------------------------------------------------------
# mixed precision (contract C11) against FP64
# --------------------------------------------------------------------------
def fmaf_exact(a, b, c):
    """Correctly rounded float32 a*b + c (round to nearest even) for normal float32 arrays.

    a*b is exact in double; s = fl64(a*b + c) and its exact error err come from
    Knuth's TwoSum, so a*b + c = s + err exactly.  Rounding s to float32 is the
    correctly rounded result unless s sits exactly on a midpoint between two
    float32 values while err != 0; then the exact value lies on err's side."""
    f32, f64 = np.float32, np.float64
    p = a.astype(f64) * b.astype(f64)
    c64 = c.astype(f64)
    s = p + c64
    bb = s - p
    err = (p - (s - bb)) + (c64 - bb)
    r = s.astype(f32)
    r64 = r.astype(f64)
    other = np.nextafter(r, np.where(s > r64, np.inf, -np.inf).astype(f32))
    mid = 0.5 * (r64 + other.astype(f64))
    at_mid = (s == mid) & (err != 0)
    hi, lo = np.maximum(r, other), np.minimum(r, other)
    return np.where(at_mid, np.where(err > 0, hi, lo), r).astype(f32)


def test_fmaf_exact_emulation():
    # the helper against the exact rational value on random operands, including
    # constructed midpoint cases where a plain double evaluation rounds twice
    from fractions import Fraction
    rng = np.random.default_rng(17)
    f32 = np.float32
    a = rng.standard_normal(3000).astype(f32)
    b = rng.standard_normal(3000).astype(f32)
    c = rng.standard_normal(3000).astype(f32)
    # midpoint cases: a*b = 1 + (k+1) 2^-12 + k 2^-24 lies exactly halfway between two
    # float32 values for odd k; c = +-2^-60 moves the exact sum off the midpoint by far
    # less than half a double ulp, so a double evaluation rounds onto it and then ties
    k = np.arange(1, 200, 2, dtype=np.float64)
    a2 = (1.0 + k * 2.0 ** -12).astype(f32)
    b2 = np.full(len(k), f32(1.0 + 2.0 ** -12))
    c2 = np.where(np.arange(len(k)) % 2 == 0, 2.0 ** -60, -(2.0 ** -60)).astype(f32)
    a, b, c = np.concatenate([a, a2]), np.concatenate([b, b2]), np.concatenate([c, c2])
    got = fmaf_exact(a, b, c)

    def rn32(x):
        # nearest float32 to the rational x, ties to even
        lo = f32(float(x))
        cands = {lo, np.nextafter(lo, f32(np.inf)), np.nextafter(lo, f32(-np.inf))}
        best = sorted(cands, key=lambda v: (abs(Fraction(float(v)) - x), int(np.float32(v).view(np.int32)) & 1))
        return best[0]
    twice = 0
    for i in range(len(a)):
        exact = Fraction(float(a[i])) * Fraction(float(b[i])) + Fraction(float(c[i]))
        assert got[i] == rn32(exact), i
        twice += f32(float(a[i]) * float(b[i]) + float(c[i])) != got[i]
    assert twice > 0  # the naive double evaluation is wrong somewhere: the test can tell


def _mixed_models(p, m, gps):
    """Per entry, from the oracle's FP64 gradients: the C11 terms (float32, fmaf) summed
    (a) by the compensated float sum of C11, (b) in double and rounded once, (c) in float."""
    gp_ptr, gp_nbr = m.support()
    row_ptr, col_idx = m.pattern()
    ndof = len(row_ptr) - 1
    pos_of = -np.ones((ndof, ndof), np.int64)  # small models only
    rows = np.repeat(np.arange(ndof), np.diff(row_ptr))
    pos_of[rows, col_idx] = np.arange(len(col_idx))
    lam = p.nu / ((1 + p.nu) * (1 - 2 * p.nu))
    mu = 1 / (2 * (1 + p.nu))
    f32 = np.float32
    nnz = len(col_idx)
    ks, kc = np.zeros(nnz, f32), np.zeros(nnz, f32)
    dsum = np.zeros(nnz, np.float64)
    asum = np.zeros(nnz, np.float64)
    fsum = np.zeros(nnz, f32)
    for g in gps:
        S = gp_nbr[gp_ptr[g]:gp_ptr[g + 1]]
        n = len(S)
        _, dphi = m.shape(int(g))
        fp = dphi.astype(f32)
        c = p.gp_wdet[g] * p.cell_E[p.gp_cell[g]]
        flc, fmc = f32(c * lam), f32(c * mu)
        A = np.repeat(np.arange(n), n)
        B = np.tile(np.arange(n), n)
        fa, fb = fp[A], fp[B]
        dot = fmaf_exact(fa[:, 2], fb[:, 2], fmaf_exact(fa[:, 1], fb[:, 1], fa[:, 0] * fb[:, 0]))
        for al in range(3):
            for be in range(3):
                m1 = fa[:, al] * fb[:, be]
                m2 = fa[:, be] * fb[:, al]
                if al == be:
                    m2 = m2 + dot
                e = fmaf_exact(np.full(len(A), flc), m1, fmc * m2)
                pos = pos_of[3 * S[A] + al, 3 * S[B] + be]
                assert (pos >= 0).all()
                y = e - kc[pos]
                t = ks[pos] + y
                kc[pos] = (t - ks[pos]) - y
                ks[pos] = t
                dsum[pos] += e.astype(np.float64)
                asum[pos] += np.abs(e.astype(np.float64))
                fsum[pos] = fsum[pos] + e
    return ks, dsum, asum, fsum


def test_mixed_is_compensated_float_sum(cant):
    """C11 rebuilt in numpy from the oracle's FP64 gradients: float32 terms
    (fused multiply-adds emulated exactly), each entry a Kahan-compensated
    float32 sum in ascending point order.  The oracle's mixed K equals it bit
    for bit, and the check tells it apart from summing the same terms in
    double (rounded once) and from a plain float32 sum."""
    p, m = cant
    gps = np.arange(p.n_gp, dtype=np.int64)
    kahan, dsum, asum, flt = _mixed_models(p, m, gps)
    K32 = m.assemble(precision=1, gps=gps)
    assert K32.dtype == np.float32
    assert np.array_equal(K32, kahan)
    assert np.count_nonzero(K32 != dsum.astype(np.float32)) > 0
    assert np.count_nonzero(K32 != flt) > 0
    # compensated summation error bound: |s - sum e| <= (2u + O(n u^2)) sum |e|, u = 2^-24
    # (the double sum of the same float terms is exact to ~1e-16 sum |e|)
    u = 2.0 ** -24
    n_terms = 2 * 27
    assert np.all(np.abs(K32.astype(np.float64) - dsum) <= (2 * u + n_terms * u * u) * asum + 1e-300)
    # and a plain float32 sum of the same terms breaks that bound somewhere
    assert np.any(np.abs(flt.astype(np.float64) - dsum) > (2 * u + n_terms * u * u) * asum)
    K64 = m.assemble(gps=gps)
    assert np.linalg.norm(K32 - K64) / np.linalg.norm(K64) < 1e-6


@pytest.mark.parametrize("which", ["cant", "jbox"])
def test_mixed_within_1e6(which, request):
    p, m = request.getfixturevalue(which)
    K64 = m.assemble()
    K32 = m.assemble(precision=1)
    err = np.linalg.norm(K32.astype(np.float64) - K64) / np.linalg.norm(K64)
    assert err < 1e-6
    assert err > 0


# --------------------------------------------------------------------------
# singular moment matrices (contract C6: |u_kk| <= N eps max|G| is an error)
# --------------------------------------------------------------------------
def test_coplanar_support_is_singular_at_first_such_point(oracle_mod):
    """A 3D block of nodes plus a planar sheet far from it.  Gauss points in
    the block have full 3D supports; a Gauss point in the sheet's plane sees
    only coplanar nodes, so the z column of its polynomial block is exactly
    zero and elimination reaches an exactly zero pivot.  The first such point
    (id fixed by construction) is the one reported."""
    g3 = np.stack(np.meshgrid(*(np.arange(5.0),) * 3, indexing="ij"), -1).reshape(-1, 3)
    sx, sy = np.meshgrid(np.arange(6.0), np.arange(6.0), indexing="ij")
    sheet = np.stack([sx.ravel() + 40.0, sy.ravel(), np.full(36, 50.0)], 1)
    nodes = np.concatenate([g3, sheet])
    rng = np.random.default_rng(4)
    block_gps = 1.0 + 2.0 * rng.random((7, 3))
    sheet_gps = np.stack([42.0 + rng.random(3), 2.0 + rng.random(3), np.full(3, 50.0)], 1)
    gps = np.concatenate([block_gps, sheet_gps, block_gps[:2] + 0.1])
    first_bad = len(block_gps)
    p = W.Problem(name="coplanar", node_xyz=nodes, gp_xyz=gps, gp_wdet=np.ones(len(gps)),
                  gp_cell=np.zeros(len(gps), np.int32), cell_E=np.ones(1), support_radius=2.5)
    m = oracle_mod.OracleModel(p)
    m.build_pattern()
    gp_ptr, gp_nbr = m.support()
    for g in range(first_bad, first_bad + 3):  # the construction: sheet points see only the sheet
        S = gp_nbr[gp_ptr[g]:gp_ptr[g + 1]]
        assert len(S) >= 5 and np.all(nodes[S, 2] == 50.0)
    with pytest.raises(oracle_mod.OracleError) as ei:
        m.assemble()
    assert ei.value.code == oracle_mod.E_SINGULAR
    assert f"first bad gp {first_bad})" in str(ei.value)
    with pytest.raises(oracle_mod.OracleError) as ei:
        m.shape(first_bad + 1)
    assert ei.value.code == oracle_mod.E_SINGULAR
    # every point before it, and the block points after it, are regular
    ok = np.r_[np.arange(first_bad), np.arange(first_bad + 3, len(gps))]
    K = m.assemble(gps=ok)
    assert np.isfinite(K).all() and np.abs(K).max() > 0


# --------------------------------------------------------------------------
# adjoint over a subset of Gauss points
# --------------------------------------------------------------------------
def test_backward_subset_completes_touched_nodes_and_cells(jbox, oracle_mod):
    """The backward over the Gauss points that touch a node (or lie in a cell)
    reproduces that node's (cell's) full value bit for bit: both sums take the
    same terms in the same ascending order."""
    p, m = jbox
    rp_, ci = m.pattern()
    Kb = np.random.default_rng(19).standard_normal(m.nnz)
    dE, dX = m.backward(Kb)
    gp_ptr, gp_nbr = m.support()
    owner = np.repeat(np.arange(p.n_gp), np.diff(gp_ptr))
    for node in (0, 77, p.n_nodes - 1):
        gps = np.unique(owner[gp_nbr == node])
        _, dXs = m.backward(Kb, gps=gps)
        assert np.array_equal(dXs[node], dX[node])
    for cell in (0, 64, p.n_cells - 1):
        gps = np.where(p.gp_cell == cell)[0]
        dEs, _ = m.backward(Kb, gps=gps)
        assert dEs[cell] == dE[cell]
        assert np.count_nonzero(dEs) == 1
    # splitting the points into two halves adds up to the whole
    half = p.n_gp // 2
    a = m.backward(Kb, gps=np.arange(half))
    b = m.backward(Kb, gps=np.arange(half, p.n_gp))
    assert np.allclose(a[1] + b[1], dX, rtol=1e-12, atol=1e-12 * np.abs(dX).max())
