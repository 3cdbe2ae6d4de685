"""Python access to the serial CPU oracle (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It drives `librpim_oracle.so`, built from `rpim_oracle.cpp`
with gcc (no GPU code, nothing shared with the HIP library).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rpim_oracle.cpp")
LIB = os.path.join(HERE, "librpim_oracle.so")

OK, E_ARG, E_SUPPORT, E_SINGULAR, E_RANGE, E_POW, E_STATE = 0, -1, -4, -5, -6, -7, -8


def build(force: bool = True) -> str:
    """Compile the oracle with contraction off and hardware fma for std::fma."""
    if force or not os.path.exists(LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-mfma", "-fno-fast-math",
               "-fPIC", "-shared", "-Wall", SRC, "-o", LIB + ".tmp", "-lquadmath"]
        subprocess.check_call(cmd)
        os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        vp, i64, i32p, i64p, dp, d = C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double
        L.orcl_model_create.restype = vp
        L.orcl_model_create.argtypes = [i64, dp, i64, dp, dp, i32p, i64, d, d, d, d]
        L.orcl_model_destroy.argtypes = [vp]
        L.orcl_build_pattern.argtypes = [vp, i64p, i64p, i64p]
        L.orcl_get_support.argtypes = [vp, i64p, i32p]
        L.orcl_get_pattern.argtypes = [vp, i64p, i32p]
        L.orcl_shape.argtypes = [vp, i64, dp, dp, dp]
        L.orcl_assemble.argtypes = [vp, dp, dp, d, C.c_int, vp, i64p, i64, i64p]
        L.orcl_penalty.argtypes = [i64p, i32p, vp, C.c_int, i64, i32p, dp, i64, d, dp, dp]
        L.orcl_assemble_backward.argtypes = [vp, dp, dp, d, dp, i64p, i64, dp, dp]
        L.orcl_dot_q.argtypes = [vp, dp, dp, d, dp, i64p, i64, dp]
        L.orcl_body_force.argtypes = [vp, dp, dp, dp]
        L.orcl_gauss_stress.argtypes = [vp, dp, dp, d, dp, dp]
        L.orcl_set_shape.argtypes = [vp, C.c_int]
        L.orcl_pow_cr.restype = d
        L.orcl_pow_cr.argtypes = [d, d]
        L.orcl_pow_fallbacks.restype = C.c_long
        L.orcl_pow_hard_cases.restype = C.c_long
        L.orcl_pow_q.argtypes = [d, d, dp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def _check(st, what):
    if st != OK:
        raise OracleError(st, what)


class OracleModel:
    """Serial FP64 RPIM assembly of one model (or a block-diagonal batch)."""

    SHAPES = {"rpim": 0, "mls": 1, "shepard": 2}

    def __init__(self, prob, shape="rpim"):
        self.prob = prob
        L = lib()
        self._keep = [np.ascontiguousarray(prob.node_xyz, np.float64),
                      np.ascontiguousarray(prob.gp_xyz, np.float64),
                      np.ascontiguousarray(prob.gp_wdet, np.float64),
                      np.ascontiguousarray(prob.gp_cell, np.int32)]
        X, P, Wd, Cc = self._keep
        self.h = L.orcl_model_create(len(X), _p(X), len(P), _p(P), _p(Wd), _p(Cc), prob.n_cells,
                                     prob.support_radius, prob.alpha_c, prob.d_c, prob.q)
        if not self.h:
            raise OracleError(E_ARG, "create")
        _check(L.orcl_set_shape(self.h, self.SHAPES[shape]), "set_shape")
        self.nnz = None
        self.sum_n = None

    def __del__(self):
        h = getattr(self, "h", None)
        if h and lib is not None:  # module globals may already be gone at interpreter exit
            lib().orcl_model_destroy(h)
            self.h = None

    def build_pattern(self):
        nnz, sn, bad = C.c_int64(), C.c_int64(), C.c_int64()
        st = lib().orcl_build_pattern(self.h, C.byref(nnz), C.byref(sn), C.byref(bad))
        if st != OK:
            raise OracleError(st, f"build_pattern (first bad gp {bad.value})")
        self.nnz, self.sum_n = nnz.value, sn.value
        return self.nnz

    def support(self):
        gp_ptr = np.empty(self.prob.n_gp + 1, np.int64)
        gp_nbr = np.empty(self.sum_n, np.int32)
        _check(lib().orcl_get_support(self.h, _p(gp_ptr), _p(gp_nbr)), "get_support")
        return gp_ptr, gp_nbr

    def pattern(self):
        row_ptr = np.empty(3 * self.prob.n_nodes + 1, np.int64)
        col_idx = np.empty(self.nnz, np.int32)
        _check(lib().orcl_get_pattern(self.h, _p(row_ptr), _p(col_idx)), "get_pattern")
        return row_ptr, col_idx

    def shape(self, g, node_xyz=None):
        gp_ptr = self._gp_ptr()
        n = int(gp_ptr[g + 1] - gp_ptr[g])
        phi = np.empty(n)
        dphi = np.empty((n, 3))
        X = None if node_xyz is None else np.ascontiguousarray(node_xyz, np.float64)
        _check(lib().orcl_shape(self.h, g, _p(X), _p(phi), _p(dphi)), f"shape({g})")
        return phi, dphi

    def _gp_ptr(self):
        if not hasattr(self, "_gpp"):
            self._gpp = self.support()[0]
        return self._gpp

    def assemble(self, cell_E=None, nu=None, precision=0, node_xyz=None, gps=None):
        E = np.ascontiguousarray(self.prob.cell_E if cell_E is None else cell_E, np.float64)
        X = None if node_xyz is None else np.ascontiguousarray(node_xyz, np.float64)
        K = np.empty(self.nnz, np.float64 if precision == 0 else np.float32)
        g = None if gps is None else np.ascontiguousarray(gps, np.int64)
        bad = C.c_int64()
        st = lib().orcl_assemble(self.h, _p(X), _p(E), self.prob.nu if nu is None else nu, precision,
                                 _p(K), _p(g), 0 if g is None else len(g), C.byref(bad))
        if st != OK:
            raise OracleError(st, f"assemble (first bad gp {bad.value})")
        return K

    def backward(self, Kbar, cell_E=None, nu=None, node_xyz=None, gps=None):
        """dL/dE per cell and dL/dx per node, summed over `gps` (ascending; all points when None)."""
        E = np.ascontiguousarray(self.prob.cell_E if cell_E is None else cell_E, np.float64)
        X = None if node_xyz is None else np.ascontiguousarray(node_xyz, np.float64)
        Kb = np.ascontiguousarray(Kbar, np.float64)
        g = None if gps is None else np.ascontiguousarray(gps, np.int64)
        dE = np.empty(self.prob.n_cells)
        dX = np.empty((self.prob.n_nodes, 3))
        _check(lib().orcl_assemble_backward(self.h, _p(X), _p(E), self.prob.nu if nu is None else nu,
                                            _p(Kb), _p(g), 0 if g is None else len(g), _p(dE), _p(dX)),
               "assemble_backward")
        return dE, dX

    def body_force(self, gp_force, node_xyz=None):
        """f_I = sum_g w_g phi_I(x_g) b_g for b_g = gp_force[g] (force per unit volume), shape [N, 3]."""
        X = None if node_xyz is None else np.ascontiguousarray(node_xyz, np.float64)
        b = np.ascontiguousarray(np.broadcast_to(gp_force, (self.prob.n_gp, 3)), np.float64)
        f = np.empty((self.prob.n_nodes, 3))
        _check(lib().orcl_body_force(self.h, _p(X), _p(b), _p(f)), "body_force")
        return f

    def gauss_stress(self, u, cell_E=None, nu=None, node_xyz=None):
        """Stress [xx, yy, zz, yz, xz, xy] at every Gauss point for nodal displacements u [N, 3]."""
        E = np.ascontiguousarray(self.prob.cell_E if cell_E is None else cell_E, np.float64)
        X = None if node_xyz is None else np.ascontiguousarray(node_xyz, np.float64)
        uu = np.ascontiguousarray(u, np.float64).reshape(-1)
        sig = np.empty((self.prob.n_gp, 6))
        _check(lib().orcl_gauss_stress(self.h, _p(X), _p(E), self.prob.nu if nu is None else nu, _p(uu), _p(sig)),
               "gauss_stress")
        return sig

    def dot_q(self, Kbar, gps, node_xyz=None, cell_E=None, nu=None):
        """<Kbar, sum_{g in gps} k^g> in __float128 (frozen supports) -> (hi, lo)."""
        E = np.ascontiguousarray(self.prob.cell_E if cell_E is None else cell_E, np.float64)
        X = np.ascontiguousarray(self.prob.node_xyz if node_xyz is None else node_xyz, np.float64)
        Kb = np.ascontiguousarray(Kbar, np.float64)
        g = np.ascontiguousarray(gps, np.int64)
        out = np.empty(2)
        _check(lib().orcl_dot_q(self.h, _p(X), _p(E), self.prob.nu if nu is None else nu, _p(Kb),
                                _p(g), len(g), _p(out)), "dot_q")
        return out[0], out[1]


def penalty(row_ptr, col_idx, K, fixed_dof, u_bar=None, factor=1e8, rhs=None):
    """Penalty BCs in place on K (float64 or float32); returns alpha."""
    prec = 0 if K.dtype == np.float64 else 1
    fx = np.ascontiguousarray(fixed_dof, np.int32)
    ub = None if u_bar is None else np.ascontiguousarray(u_bar, np.float64)
    alpha = np.empty(1)
    _check(lib().orcl_penalty(_p(row_ptr), _p(col_idx), _p(K), prec, len(row_ptr) - 1, _p(fx), _p(ub),
                              len(fx), factor, _p(rhs), _p(alpha)), "penalty")
    return float(alpha[0])


def pow_cr(x: float, q: float) -> float:
    return lib().orcl_pow_cr(float(x), float(q))


def pow_q(x: float, q: float):
    out = np.empty(2)
    lib().orcl_pow_q(float(x), float(q), _p(out))
    return out[0], out[1]


def pow_stats():
    return lib().orcl_pow_fallbacks(), lib().orcl_pow_hard_cases()
