"""Seeded synthetic inputs for RPIM stiffness assembly.

This module only builds *inputs*: field-node coordinates, background
integration cells, Gauss points with their weight x |J|, per-cell Young's
modulus and probe vectors.  It holds none of the assembly arithmetic (no
support search, no radial basis, no moment matrix, no stiffness), so both
the CPU oracle and the GPU library can consume its arrays without sharing
any of the method's code.

Geometries follow the paper's verification workloads: a cantilever block
(Example 2) and a simplified slope discretised by regular or irregular
(jittered) field nodes (Example 3).  Sizes, jitter, material fields and
seeds are the ones stated for each named workload below.

Background cells are regular in a parameter cube (u, v, w) in [0, 1]^3 that
is mapped to physical space; Gauss points are tensor Gauss-Legendre points of
each cell pushed through the same map, and `gp_wdet` is the product of the
Gauss weights, the parameter-cell half-widths and the map's |J| at the point.
Gauss points are numbered cell-major: cell id = (ci*ny + cj)*nz + ck, then the
point's own (a*p + b)*p + c with z-like index fastest.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem", "gauss_legendre", "cantilever", "slope", "box", "batch",
    "probe_vectors", "named", "NAMED",
]


@dataclass
class Problem:
    """One model (or a block-diagonal batch of models) ready for assembly."""
    name: str
    node_xyz: np.ndarray          # f64 [N, 3]
    gp_xyz: np.ndarray            # f64 [G, 3]
    gp_wdet: np.ndarray           # f64 [G]   Gauss weight * |J| (> 0)
    gp_cell: np.ndarray           # i32 [G]   cell index of each Gauss point
    cell_E: np.ndarray            # f64 [C]   Young's modulus per cell
    nu: float = 0.3
    support_radius: float = 2.5   # d_s
    alpha_c: float = 4.0          # MQ shape parameter
    d_c: float = 1.0              # characteristic nodal spacing
    q: float = 1.03               # MQ exponent
    volume: float = 0.0           # exact domain volume (for the quadrature pin)
    # batch bookkeeping (n_models == 1 for a single model)
    node_off: np.ndarray = field(default_factory=lambda: np.zeros(2, np.int64))
    gp_off: np.ndarray = field(default_factory=lambda: np.zeros(2, np.int64))
    cell_off: np.ndarray = field(default_factory=lambda: np.zeros(2, np.int64))
    meta: dict = field(default_factory=dict)

    def __post_init__(self):
        if self.node_off[-1] == 0:
            self.node_off = np.array([0, len(self.node_xyz)], np.int64)
            self.gp_off = np.array([0, len(self.gp_xyz)], np.int64)
            self.cell_off = np.array([0, len(self.cell_E)], np.int64)

    @property
    def n_nodes(self) -> int:
        return int(self.node_xyz.shape[0])

    @property
    def n_gp(self) -> int:
        return int(self.gp_xyz.shape[0])

    @property
    def n_cells(self) -> int:
        return int(self.cell_E.shape[0])

    @property
    def n_models(self) -> int:
        return int(len(self.node_off) - 1)


def gauss_legendre(p: int):
    """Abscissae and weights of the p-point Gauss-Legendre rule on [-1, 1]."""
    if p == 1:
        return np.array([0.0]), np.array([2.0])
    if p == 2:
        a = 1.0 / math.sqrt(3.0)
        return np.array([-a, a]), np.array([1.0, 1.0])
    if p == 3:
        a = math.sqrt(3.0 / 5.0)
        return np.array([-a, 0.0, a]), np.array([5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0])
    x, w = np.polynomial.legendre.leggauss(p)
    return x, w


def _structured(nx, ny, nz, mapping, jac, p, jitter, jitter_seed, h):
    """Nodes on the (nx+1)(ny+1)(nz+1) parameter lattice and p^3 Gauss points per cell.

    mapping(u, v, w) -> (x, y, z) arrays; jac(u, v, w) -> |J| of the map.
    Interior nodes (not on any face) are moved by U(-jitter, +jitter) * h per
    coordinate when jitter > 0; boundary nodes stay on the faces.
    """
    i, j, k = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    u = (i / nx).ravel()
    v = (j / ny).ravel()
    w = (k / nz).ravel()
    x, y, z = mapping(u, v, w)
    node = np.stack([x, y, z], axis=1).astype(np.float64)
    if jitter > 0.0:
        rng = np.random.default_rng(jitter_seed)
        d = rng.uniform(-jitter, jitter, size=node.shape) * h
        interior = ((i > 0) & (i < nx) & (j > 0) & (j < ny) & (k > 0) & (k < nz)).ravel()
        node[interior] += d[interior]

    xi, wq = gauss_legendre(p)
    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    a, b, c = np.meshgrid(np.arange(p), np.arange(p), np.arange(p), indexing="ij")
    a, b, c = a.ravel(), b.ravel(), c.ravel()
    # cell-major: [cell, point]
    gu = (ci[:, None] + 0.5 * (1.0 + xi[a][None, :])) / nx
    gv = (cj[:, None] + 0.5 * (1.0 + xi[b][None, :])) / ny
    gw = (ck[:, None] + 0.5 * (1.0 + xi[c][None, :])) / nz
    gx, gy, gz = mapping(gu, gv, gw)
    gp = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1).astype(np.float64)
    wts = (wq[a] * wq[b] * wq[c])[None, :] / (8.0 * nx * ny * nz)
    wdet = (wts * jac(gu, gv, gw)).ravel().astype(np.float64)
    n_cells = nx * ny * nz
    gcell = np.repeat(np.arange(n_cells, dtype=np.int32), p ** 3)
    centre_w = (ck + 0.5) / nz
    return node, gp, wdet, gcell, centre_w


def cantilever(nx=8, ny=2, nz=2, h=1.0, p=2, E=3.0e7, nu=0.3) -> Problem:
    """Cantilever block nx*h x ny*h x nz*h on a regular grid (no randomness).

    Default: 8 x 2 x 2 m, 9 x 3 x 3 = 81 nodes, 32 cells with 2^3 Gauss points,
    E = 30 MPa, nu = 0.3, MQ alpha_c = 4, q = 1.03, d_s = 2.5 h.
    Node id = (i*(ny+1) + j)*(nz+1) + k, z fastest.
    """
    L, W, H = nx * h, ny * h, nz * h
    mapping = lambda u, v, w: (L * u, W * v, H * w)
    jac = lambda u, v, w: np.full(np.shape(u), L * W * H)
    node, gp, wdet, gcell, _ = _structured(nx, ny, nz, mapping, jac, p, 0.0, 0, h)
    C = nx * ny * nz
    return Problem(
        name=f"cantilever_{nx}x{ny}x{nz}_h{h:g}", node_xyz=node, gp_xyz=gp, gp_wdet=wdet,
        gp_cell=gcell, cell_E=np.full(C, E), nu=nu, support_radius=2.5 * h,
        alpha_c=4.0, d_c=h, q=1.03, volume=L * W * H,
        meta=dict(nx=nx, ny=ny, nz=nz, h=h, L=L, W=W, H=H, p=p),
    )


def slope(L=40.0, W=20.0, H=20.0, x_c=None, h=1.0, p=3, jitter=0.3, jitter_seed=0,
          E_mode="lognormal", E_seed=1, E_median=5.0e7, E_sigma=0.5,
          layers=(300.0e6, 80.0e6, 20.0e6), nu=0.3) -> Problem:
    """Trapezoidal-prism slope: parameter cube mapped by
    (u, v, w) -> (x_c*w + u*(L - x_c*w), W*v, H*w), |J| = (L - x_c*w)*W*H.

    The base is L long, the crest L - x_c.  Cells follow the parameter lattice
    (L/h x W/h x H/h), so x-spacing is h at the base and (L - x_c)/L * h at
    the crest.  E per cell is lognormal (median E_median, log-sd E_sigma,
    seed E_seed) or three horizontal layers by cell-centre height
    (bottom third layers[0], middle layers[1], top layers[2]).
    """
    if x_c is None:
        x_c = L / 4.0
    nx, ny, nz = int(round(L / h)), int(round(W / h)), int(round(H / h))
    mapping = lambda u, v, w: (x_c * w + u * (L - x_c * w), W * v, H * w)
    jac = lambda u, v, w: (L - x_c * w) * W * H
    node, gp, wdet, gcell, centre_w = _structured(nx, ny, nz, mapping, jac, p, jitter, jitter_seed, h)
    C = nx * ny * nz
    if E_mode == "lognormal":
        rng = np.random.default_rng(E_seed)
        cell_E = np.exp(rng.normal(math.log(E_median), E_sigma, size=C))
    elif E_mode == "layers":
        zc = centre_w * H
        cell_E = np.where(zc < H / 3.0, layers[0], np.where(zc < 2.0 * H / 3.0, layers[1], layers[2]))
    else:
        raise ValueError(E_mode)
    volume = W * H * (L - 0.5 * x_c)
    return Problem(
        name=f"slope_{nx}x{ny}x{nz}", node_xyz=node, gp_xyz=gp, gp_wdet=wdet, gp_cell=gcell,
        cell_E=cell_E.astype(np.float64), nu=nu, support_radius=2.5 * h, alpha_c=4.0,
        d_c=h, q=1.03, volume=volume,
        meta=dict(nx=nx, ny=ny, nz=nz, h=h, L=L, W=W, H=H, x_c=x_c, p=p, jitter=jitter),
    )


def box(n=8, h=1.0, p=2, jitter=0.3, jitter_seed=7, E_seed=8, nu=0.3) -> Problem:
    """Small jittered cube n*h on a side (test size): (n+1)^3 nodes, n^3 cells."""
    return slope(L=n * h, W=n * h, H=n * h, x_c=0.0, h=h, p=p, jitter=jitter,
                 jitter_seed=jitter_seed, E_seed=E_seed, nu=nu)


def batch(problems) -> Problem:
    """Concatenate independent models into one block-diagonal batch.

    Node, Gauss-point and cell indices are offset per model; node_off /
    gp_off / cell_off give the prefix offsets.  All models must share nu and
    the RBF parameters; the support radius may differ but is stored per model
    in meta['support_radius'].
    """
    nodes, gps, wd, gc, Es = [], [], [], [], []
    noff, goff, coff = [0], [0], [0]
    for pr in problems:
        nodes.append(pr.node_xyz)
        gps.append(pr.gp_xyz)
        wd.append(pr.gp_wdet)
        gc.append(pr.gp_cell + coff[-1])
        Es.append(pr.cell_E)
        noff.append(noff[-1] + pr.n_nodes)
        goff.append(goff[-1] + pr.n_gp)
        coff.append(coff[-1] + pr.n_cells)
    p0 = problems[0]
    return Problem(
        name=f"batch{len(problems)}", node_xyz=np.concatenate(nodes), gp_xyz=np.concatenate(gps),
        gp_wdet=np.concatenate(wd), gp_cell=np.concatenate(gc).astype(np.int32),
        cell_E=np.concatenate(Es), nu=p0.nu, support_radius=p0.support_radius,
        alpha_c=p0.alpha_c, d_c=p0.d_c, q=p0.q, volume=sum(pr.volume for pr in problems),
        node_off=np.array(noff, np.int64), gp_off=np.array(goff, np.int64),
        cell_off=np.array(coff, np.int64),
        meta=dict(support_radius=np.array([pr.support_radius for pr in problems]),
                  models=[pr.name for pr in problems]),
    )


def batched_slopes(n_models=64, size_seed=4, lo=1.0e3, hi=3.0e4):
    """Independent jittered slope models of uneven size (log-uniform node count).

    Model m: N_target = exp(U(ln lo, ln hi)) (seed size_seed), s = (N_target/18081)^(1/3),
    nx = max(4, round(40 s)), ny = nz = max(2, round(20 s)), x_c = nx/4 (1 m spacing),
    jitter seed 1000+m, lognormal E seed 2000+m.
    """
    rng = np.random.default_rng(size_seed)
    targets = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_models))
    models = []
    for m, nt in enumerate(targets):
        s = (nt / 18081.0) ** (1.0 / 3.0)
        nx = max(4, int(round(40 * s)))
        ny = nz = max(2, int(round(20 * s)))
        models.append(slope(L=float(nx), W=float(ny), H=float(nz), x_c=nx / 4.0, h=1.0, p=3,
                            jitter=0.3, jitter_seed=1000 + m, E_seed=2000 + m))
    return models


def probe_vectors(n_dof: int, n_vec: int = 8, seed: int = 5) -> np.ndarray:
    """n_vec seeded N(0,1) probe vectors of length n_dof, shape [n_vec, n_dof]."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n_vec, n_dof))


# Named workloads: the configurations this library is measured and tested on.
NAMED = {
    "cantilever": "cantilever 8x2x2 m, 81 nodes, 256 Gauss points, FP64",
    "slope": "jittered slope 40x20x20 m, 18,081 nodes, 432,000 Gauss points, lognormal E, FP64",
    "slope_large": "3-layer jittered slope 100x50x50 m, 262,701 nodes, 6,750,000 Gauss points, mixed",
    "batch64": "64 jittered slopes (1k-30k nodes each), one batched launch, mixed",
    "slope_grad": "slope geometry + 8 probe vectors, adjoint to dE and dX",
}


def named(name: str):
    if name == "cantilever":
        return cantilever()
    if name == "cantilever_h2":
        return cantilever(nx=16, ny=4, nz=4, h=0.5)
    if name == "slope":
        return slope()
    if name == "slope_large":
        return slope(L=100.0, W=50.0, H=50.0, x_c=25.0, E_mode="layers")
    if name == "batch64":
        return batch(batched_slopes())
    if name == "slope_grad":
        return slope()
    if name == "box":
        return box()
    raise KeyError(name)
