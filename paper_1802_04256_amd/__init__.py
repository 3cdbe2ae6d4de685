"""MI355X RPIM global-stiffness assembly: Python binding of librpim.so.

Argument marshalling only: torch tensors provide device memory and the
current HIP stream; every numerical step runs in the library's HIP kernels.
Importing works without a GPU, but any call needs the built library and a
GPU; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

__all__ = ["Plan", "assemble", "apply_penalty_bc", "solve_pcg", "pow_cr", "RpimError", "library_path", "FP64",
           "MIXED"]

FP64, MIXED = 0, 1
PENALTY_NOALLOC_MAX_FIXED = 1 << 18  # RPIM_PENALTY_NOALLOC_MAX_FIXED in rpim.h
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "librpim.so")

_STATUS = {0: "RPIM_OK", -1: "RPIM_E_ARG", -2: "RPIM_E_NOMEM", -3: "RPIM_E_HIP", -4: "RPIM_E_SUPPORT",
           -5: "RPIM_E_SINGULAR", -6: "RPIM_E_RANGE", -7: "RPIM_E_POW", -8: "RPIM_E_STATE",
           -9: "RPIM_E_CONVERGENCE"}


class RpimError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str = ""):
        self.code = code
        self.name = _STATUS.get(code, str(code))
        super().__init__(f"{what}: {self.name}{(' ' + detail) if detail else ''}")


class _Problem(C.Structure):
    _fields_ = [("n_models", C.c_int32), ("node_off", C.POINTER(C.c_int64)), ("gp_off", C.POINTER(C.c_int64)),
                ("n_cells", C.c_int64), ("support_radius", C.POINTER(C.c_double)), ("node_xyz", C.c_void_p),
                ("gp_xyz", C.c_void_p), ("gp_wdet", C.c_void_p), ("gp_cell", C.c_void_p),
                ("alpha_c", C.c_double), ("d_c", C.c_double), ("q", C.c_double)]


_TUNING_MAX = 32


class _Tuning(C.Structure):
    _fields_ = [("gather_waves", C.c_int32), ("gather_ms", C.c_float * 4), ("n_buckets", C.c_int32),
                ("bucket_nmax", C.c_int32 * _TUNING_MAX), ("bucket_points", C.c_int64 * _TUNING_MAX),
                ("bucket_ms", C.c_float * _TUNING_MAX), ("bucket_solver", C.c_int32 * _TUNING_MAX),
                ("bucket_ms_window", C.c_float * _TUNING_MAX), ("bucket_ms_panel", C.c_float * _TUNING_MAX),
                ("from_cache", C.c_int32)]


class _Info(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_gp", C.c_int64), ("n_cells", C.c_int64), ("n_models", C.c_int64),
                ("sum_n", C.c_int64), ("nnz", C.c_int64), ("n_blocks", C.c_int64), ("min_n", C.c_int32),
                ("max_n", C.c_int32), ("lu_doubles", C.c_int64), ("n_buckets", C.c_int32)]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Load librpim.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RpimError(-3, "load", f"{_LIB_PATH} is missing; build it with __graft_entry__.build()")
        L = C.CDLL(_LIB_PATH)
        vp, i64, i32, d = C.c_void_p, C.c_int64, C.c_int, C.c_double
        L.rpim_plan_create.argtypes = [C.POINTER(_Problem), C.POINTER(vp)]
        L.rpim_build_pattern.argtypes = [vp, vp, vp, C.POINTER(i64), vp]
        L.rpim_assemble.argtypes = [vp, vp, vp, d, i32, i32, vp, vp]
        L.rpim_assemble_backward.argtypes = [vp, vp, vp, d, vp, vp, vp, vp]
        L.rpim_apply_penalty_bc.argtypes = [vp, vp, vp, i32, i64, vp, vp, i64, d, vp, vp, vp, vp, C.c_size_t, vp]
        L.rpim_apply_penalty_bc_noalloc.argtypes = [vp, vp, vp, i32, i64, vp, vp, i64, d, vp, vp, vp, vp]
        L.rpim_penalty_workspace_bytes.argtypes = [i64, i64]
        L.rpim_pcg_workspace_bytes.argtypes = [i64]
        L.rpim_pcg_workspace_bytes.restype = C.c_size_t
        L.rpim_solve_pcg.argtypes = [vp, vp, vp, i32, i64, vp, vp, d, i64, vp, C.c_size_t, C.POINTER(i64),
                                     C.POINTER(d), vp]
        L.rpim_penalty_workspace_bytes.restype = C.c_size_t
        L.rpim_get_status.argtypes = [vp, vp, C.POINTER(i64)]
        L.rpim_plan_info.argtypes = [vp, C.POINTER(_Info)]
        L.rpim_get_support.argtypes = [vp, vp, vp, vp]
        L.rpim_get_dphi.argtypes = [vp, vp, vp]
        L.rpim_pow_cr.argtypes = [vp, d, vp, i64, vp]
        L.rpim_rebuild_pattern.argtypes = [vp, vp, vp, vp, C.POINTER(i64), vp]
        L.rpim_profile_enable.argtypes = [vp, i32]
        L.rpim_profile_read.argtypes = [vp, C.POINTER(d)]
        L.rpim_autotune.argtypes = [vp, vp, vp, d, i32, vp, vp, C.POINTER(_Tuning)]
        L.rpim_set_gather_waves.argtypes = [vp, i32, i32]
        L.rpim_set_solver.argtypes = [vp, i32, i32]
        L.rpim_set_shape_functions.argtypes = [vp, i32]
        L.rpim_shape_values.argtypes = [vp, vp, vp, vp]
        L.rpim_body_force.argtypes = [vp, vp, vp, vp, vp]
        L.rpim_gauss_stress.argtypes = [vp, vp, d, vp, vp, vp]
        L.rpim_tuning_cache_save.argtypes = [C.c_char_p]
        L.rpim_tuning_cache_load.argtypes = [C.c_char_p]
        L.rpim_tuning_cache_clear.restype = None
        L.rpim_factor_generation.argtypes = [vp, C.POINTER(i64)]
        L.rpim_plan_destroy.argtypes = [vp]
        L.rpim_plan_destroy.restype = None
        L.rpim_status_string.restype = C.c_char_p
        for f in ("rpim_plan_create", "rpim_build_pattern", "rpim_assemble", "rpim_assemble_backward",
                  "rpim_apply_penalty_bc", "rpim_get_status", "rpim_plan_info", "rpim_get_support",
                  "rpim_get_dphi", "rpim_pow_cr", "rpim_rebuild_pattern", "rpim_profile_enable",
                  "rpim_profile_read", "rpim_autotune", "rpim_set_gather_waves", "rpim_set_solver",
                  "rpim_factor_generation", "rpim_apply_penalty_bc_noalloc",
                  "rpim_solve_pcg", "rpim_tuning_cache_save", "rpim_tuning_cache_load",
                  "rpim_shape_values", "rpim_body_force", "rpim_gauss_stress", "rpim_set_shape_functions"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check(code, what):
    if code != 0:
        raise RpimError(code, what)


def _dev(t, dtype, device):
    torch = _torch()
    if isinstance(t, np.ndarray):
        t = torch.from_numpy(np.ascontiguousarray(t))
    return t.to(device=device, dtype=dtype).contiguous()


class Plan:
    """Supports, pattern and workspaces of one model or a block-diagonal batch."""

    def __init__(self, node_xyz, gp_xyz, gp_wdet, gp_cell, n_cells, support_radius, alpha_c=4.0, d_c=1.0,
                 q=1.03, node_off=None, gp_off=None, device="cuda"):
        torch = _torch()
        self.device = torch.device(device)
        self.node_xyz = _dev(node_xyz, torch.float64, self.device)
        self.gp_xyz = _dev(gp_xyz, torch.float64, self.device)
        self.gp_wdet = _dev(gp_wdet, torch.float64, self.device)
        self.gp_cell = _dev(gp_cell, torch.int32, self.device)
        self.n_nodes = int(self.node_xyz.shape[0])
        self.n_gp = int(self.gp_xyz.shape[0])
        self.n_cells = int(n_cells)
        node_off = np.array([0, self.n_nodes] if node_off is None else node_off, np.int64)
        gp_off = np.array([0, self.n_gp] if gp_off is None else gp_off, np.int64)
        radius = np.atleast_1d(np.asarray(support_radius, np.float64))
        if radius.size == 1 and len(node_off) > 2:
            radius = np.full(len(node_off) - 1, float(radius[0]))
        self._node_off, self._gp_off, self._radius = node_off, gp_off, radius
        pb = _Problem()
        pb.n_models = len(node_off) - 1
        pb.node_off = node_off.ctypes.data_as(C.POINTER(C.c_int64))
        pb.gp_off = gp_off.ctypes.data_as(C.POINTER(C.c_int64))
        pb.n_cells = self.n_cells
        pb.support_radius = radius.ctypes.data_as(C.POINTER(C.c_double))
        pb.node_xyz = self.node_xyz.data_ptr()
        pb.gp_xyz = self.gp_xyz.data_ptr()
        pb.gp_wdet = self.gp_wdet.data_ptr()
        pb.gp_cell = self.gp_cell.data_ptr()
        pb.alpha_c, pb.d_c, pb.q = float(alpha_c), float(d_c), float(q)
        h = C.c_void_p()
        _check(lib().rpim_plan_create(C.byref(pb), C.byref(h)), "rpim_plan_create")
        self._h = h
        self.nnz = None
        self.row_ptr = None
        self.col_idx = None

    @classmethod
    def from_problem(cls, prob, device="cuda"):
        radius = prob.meta.get("support_radius", prob.support_radius) if prob.n_models > 1 else prob.support_radius
        return cls(prob.node_xyz, prob.gp_xyz, prob.gp_wdet, prob.gp_cell, prob.n_cells, radius,
                   prob.alpha_c, prob.d_c, prob.q, prob.node_off, prob.gp_off, device)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.rpim_plan_destroy(h)
            self._h = None

    # -- pattern ------------------------------------------------------------
    def build_pattern(self):
        """Supports and CSR pattern (synchronous); returns (row_ptr int64, col_idx int32)."""
        torch = _torch()
        nnz = C.c_int64()
        st = lib().rpim_build_pattern(self._h, None, None, C.byref(nnz), _stream())
        if st != 0:
            bad = C.c_int64()
            lib().rpim_get_status(self._h, _stream(), C.byref(bad))
            raise RpimError(st, "rpim_build_pattern", f"(first bad gauss point {bad.value})")
        self.nnz = nnz.value
        self.row_ptr = torch.empty(3 * self.n_nodes + 1, dtype=torch.int64, device=self.device)
        self.col_idx = torch.empty(self.nnz, dtype=torch.int32, device=self.device)
        _check(lib().rpim_build_pattern(self._h, _ptr(self.row_ptr), _ptr(self.col_idx), C.byref(nnz), _stream()),
               "rpim_build_pattern")
        return self.row_ptr, self.col_idx

    def rebuild_pattern(self, node_xyz):
        """Re-run support search and pattern for moved nodes (synchronous)."""
        torch = _torch()
        X = _dev(node_xyz, torch.float64, self.device)
        nnz = C.c_int64()
        _check(lib().rpim_rebuild_pattern(self._h, _ptr(X), None, None, C.byref(nnz), _stream()),
               "rpim_rebuild_pattern")
        if nnz.value != self.nnz:
            self.nnz = nnz.value
            self.col_idx = torch.empty(self.nnz, dtype=torch.int32, device=self.device)
        _check(lib().rpim_build_pattern(self._h, _ptr(self.row_ptr), _ptr(self.col_idx), C.byref(nnz), _stream()),
               "rpim_build_pattern")
        self.node_xyz = X
        return self.row_ptr, self.col_idx

    PHASES = ("pattern", "pairs", "shape", "gather", "bwd_rows", "bwd_gp", "bwd_reduce")

    def profile(self, enable: bool = True):
        _check(lib().rpim_profile_enable(self._h, int(bool(enable))), "rpim_profile_enable")

    def profile_read(self) -> dict:
        out = (C.c_double * len(self.PHASES))()
        _check(lib().rpim_profile_read(self._h, out), "rpim_profile_read")
        return {k: out[i] for i, k in enumerate(self.PHASES) if out[i] >= 0}

    def info(self) -> dict:
        inf = _Info()
        _check(lib().rpim_plan_info(self._h, C.byref(inf)), "rpim_plan_info")
        return {k: getattr(inf, k) for k, _ in _Info._fields_}

    def autotune(self, node_xyz=None, cell_E=None, nu=0.3, precision=FP64, out=None) -> dict:
        """Choose the row-gather launch configuration for `precision` by timing the candidates on
        this plan (synchronous; `out`, or a temporary K buffer, is overwritten).  Returns the timings."""
        torch = _torch()
        if self.nnz is None:
            self.build_pattern()
        X = self.node_xyz if node_xyz is None else _dev(node_xyz, torch.float64, self.device)
        E = _dev(cell_E, torch.float64, self.device)
        prec = _precision(precision)
        if out is None:
            out = torch.empty(self.nnz, dtype=torch.float64 if prec == FP64 else torch.float32, device=self.device)
        t = _Tuning()
        _check(lib().rpim_autotune(self._h, _ptr(X), _ptr(E), float(nu), prec, _ptr(out), _stream(), C.byref(t)),
               "rpim_autotune")
        n = t.n_buckets
        kinds = {v: k for k, v in self.SOLVERS.items()}
        return {"gather_waves": t.gather_waves, "from_cache": bool(t.from_cache),
                "gather_ms": {w: t.gather_ms[w - 1] for w in (1, 2, 3, 4)},
                "buckets": [{"nmax": t.bucket_nmax[i], "points": t.bucket_points[i], "ms": t.bucket_ms[i],
                             "solver": kinds.get(t.bucket_solver[i], t.bucket_solver[i]),
                             "ms_window": t.bucket_ms_window[i], "ms_panel": t.bucket_ms_panel[i]}
                            for i in range(n)]}

    def set_gather_waves(self, precision, waves: int):
        _check(lib().rpim_set_gather_waves(self._h, _precision(precision), int(waves)), "rpim_set_gather_waves")

    SOLVERS = {"auto": 0, "lds": 1, "window": 2, "panel": 3}
    SHAPES = {"rpim": 0, "mls": 1, "shepard": 2}

    def set_shape_functions(self, kind):
        """'rpim' (default), 'mls' (linear basis) or 'shepard': the shape functions of later assemblies."""
        k = self.SHAPES[kind] if isinstance(kind, str) else int(kind)
        _check(lib().rpim_set_shape_functions(self._h, k), "rpim_set_shape_functions")

    def set_solver(self, kind, nmax: int = 0):
        """Moment-matrix solver kernel for the bucket of padded size nmax (0: all buckets)."""
        k = self.SOLVERS[kind] if isinstance(kind, str) else int(kind)
        _check(lib().rpim_set_solver(self._h, int(nmax), k), "rpim_set_solver")

    def factor_generation(self) -> int:
        """Identifier of the kept LU factors (0: none)."""
        g = C.c_int64()
        _check(lib().rpim_factor_generation(self._h, C.byref(g)), "rpim_factor_generation")
        return g.value

    # -- forward / backward ----------------------------------------------------
    def assemble(self, node_xyz=None, cell_E=None, nu=0.3, precision=FP64, keep_factors=False, out=None):
        torch = _torch()
        if self.nnz is None:
            self.build_pattern()
        X = self.node_xyz if node_xyz is None else _dev(node_xyz, torch.float64, self.device)
        E = _dev(cell_E, torch.float64, self.device)
        prec = _precision(precision)
        dt = torch.float64 if prec == FP64 else torch.float32
        K = out if out is not None else torch.empty(self.nnz, dtype=dt, device=self.device)
        if K.dtype != dt or K.numel() != self.nnz or not K.is_contiguous():
            raise RpimError(-1, "rpim_assemble", "output has wrong dtype/size")
        _check(lib().rpim_assemble(self._h, _ptr(X), _ptr(E), float(nu), prec, int(bool(keep_factors)), _ptr(K),
                                   _stream()), "rpim_assemble")
        return K

    def assemble_backward(self, node_xyz, cell_E, nu, dK):
        torch = _torch()
        X = _dev(node_xyz, torch.float64, self.device)
        E = _dev(cell_E, torch.float64, self.device)
        dK = _dev(dK, torch.float64, self.device)
        dE = torch.empty(self.n_cells, dtype=torch.float64, device=self.device)
        dX = torch.empty(self.n_nodes, 3, dtype=torch.float64, device=self.device)
        _check(lib().rpim_assemble_backward(self._h, _ptr(X), _ptr(E), float(nu), _ptr(dK), _ptr(dE), _ptr(dX),
                                            _stream()), "rpim_assemble_backward")
        return dE, dX

    def shape_values(self, node_xyz=None):
        """phi_a(x_g) for every support entry [sum_n], from the factors kept by the last
        assemble(keep_factors=True) at these coordinates."""
        torch = _torch()
        X = self.node_xyz if node_xyz is None else _dev(node_xyz, torch.float64, self.device)
        phi = torch.empty(self.info()["sum_n"], dtype=torch.float64, device=self.device)
        _check(lib().rpim_shape_values(self._h, _ptr(X), _ptr(phi), _stream()), "rpim_shape_values")
        return phi

    def body_force(self, phi, gp_force):
        """Nodal body force [N, 3] from force per unit volume at each Gauss point ([3] or [G, 3])."""
        torch = _torch()
        b = _dev(gp_force, torch.float64, self.device)
        b = b.expand(self.n_gp, 3).contiguous() if b.dim() == 1 else b.contiguous()
        f = torch.empty(self.n_nodes, 3, dtype=torch.float64, device=self.device)
        _check(lib().rpim_body_force(self._h, _ptr(phi), _ptr(b), _ptr(f), _stream()), "rpim_body_force")
        return f

    def gauss_stress(self, u, cell_E, nu=0.3):
        """Stress [G, 6] (xx, yy, zz, yz, xz, xy) from nodal displacements u ([N, 3] or [3N])."""
        torch = _torch()
        uu = _dev(u, torch.float64, self.device).reshape(-1).contiguous()
        E = _dev(cell_E, torch.float64, self.device)
        sig = torch.empty(self.n_gp, 6, dtype=torch.float64, device=self.device)
        _check(lib().rpim_gauss_stress(self._h, _ptr(E), float(nu), _ptr(uu), _ptr(sig), _stream()),
               "rpim_gauss_stress")
        return sig

    def status(self, raise_on_error=True):
        bad = C.c_int64()
        st = lib().rpim_get_status(self._h, _stream(), C.byref(bad))
        if st != 0 and raise_on_error:
            raise RpimError(st, "device status", f"(first bad gauss point {bad.value})")
        return st, bad.value

    def support(self):
        torch = _torch()
        inf = self.info()
        gp_ptr = torch.empty(self.n_gp + 1, dtype=torch.int64, device=self.device)
        gp_nbr = torch.empty(inf["sum_n"], dtype=torch.int32, device=self.device)
        _check(lib().rpim_get_support(self._h, _ptr(gp_ptr), _ptr(gp_nbr), _stream()), "rpim_get_support")
        return gp_ptr, gp_nbr

    def dphi(self):
        torch = _torch()
        inf = self.info()
        out = torch.empty(inf["sum_n"], 3, dtype=torch.float64, device=self.device)
        _check(lib().rpim_get_dphi(self._h, _ptr(out), _stream()), "rpim_get_dphi")
        return out


def _precision(p):
    if p in (FP64, "fp64", "f64", "double"):
        return FP64
    if p in (MIXED, "mixed", "fp32", "f32"):
        return MIXED
    raise ValueError(f"unknown precision {p!r}")


def apply_penalty_bc(row_ptr, col_idx, K, fixed_dof, u_bar=None, factor=1e8, rhs=None, check=True):
    """Penalty BCs in place on K (float64 or float32) and rhs, on the current stream.

    With check=True (default) the call synchronises, raises RpimError(RPIM_E_ARG) if the device check of
    the fixed dofs failed (K and rhs are then unchanged) and returns alpha as a float.  With check=False
    nothing synchronises and (alpha, status) come back as one-element device tensors."""
    torch = _torch()
    prec = FP64 if K.dtype == torch.float64 else MIXED
    fx = _dev(fixed_dof, torch.int32, K.device)
    ub = None if u_bar is None else _dev(u_bar, torch.float64, K.device)
    n_dof = int(row_ptr.numel() - 1)
    nbytes = lib().rpim_penalty_workspace_bytes(n_dof, int(fx.numel()))
    ws = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=K.device)
    alpha = torch.empty(1, dtype=torch.float64, device=K.device)
    status = torch.empty(1, dtype=torch.int32, device=K.device)
    _check(lib().rpim_apply_penalty_bc(_ptr(row_ptr), _ptr(col_idx), _ptr(K), prec, n_dof, _ptr(fx), _ptr(ub),
                                       int(fx.numel()), float(factor), _ptr(rhs), _ptr(alpha), _ptr(status),
                                       _ptr(ws), nbytes, _stream()), "rpim_apply_penalty_bc")
    if not check:
        return alpha, status
    code = int(status.item())
    if code != 0:
        raise RpimError(code, "rpim_apply_penalty_bc", "(fixed dofs not strictly ascending in range, or a "
                                                       "diagonal missing; K left unchanged)")
    return float(alpha.item())


def tuning_cache(save=None, load=None, clear=False):
    """Save the process-wide tuning cache to a file, load one into it, or clear it."""
    if clear:
        lib().rpim_tuning_cache_clear()
    if load is not None:
        _check(lib().rpim_tuning_cache_load(os.fsencode(load)), "rpim_tuning_cache_load")
    if save is not None:
        _check(lib().rpim_tuning_cache_save(os.fsencode(save)), "rpim_tuning_cache_save")


def solve_pcg(row_ptr, col_idx, K, rhs, x0=None, rtol=1e-10, max_iter=200000, raise_on_error=True):
    """Jacobi-preconditioned CG on the GPU for K x = rhs (K float64 or float32 on the CSR pattern).

    Returns (x, iterations, relative residual).  With raise_on_error=False a breakdown or the iteration
    limit returns the last iterate instead of raising."""
    torch = _torch()
    prec = FP64 if K.dtype == torch.float64 else MIXED
    n = int(row_ptr.numel() - 1)
    b = _dev(rhs, torch.float64, K.device)
    x = torch.zeros(n, dtype=torch.float64, device=K.device) if x0 is None else _dev(x0, torch.float64, K.device).clone()
    nbytes = lib().rpim_pcg_workspace_bytes(n)
    ws = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=K.device)
    iters, rel = C.c_int64(), C.c_double()
    st = lib().rpim_solve_pcg(_ptr(row_ptr), _ptr(col_idx), _ptr(K), prec, n, _ptr(b), _ptr(x), float(rtol),
                              int(max_iter), _ptr(ws), nbytes, C.byref(iters), C.byref(rel), _stream())
    if st != 0 and raise_on_error:
        raise RpimError(st, "rpim_solve_pcg", f"(after {iters.value} iterations, relative residual {rel.value:.3e})")
    return x, iters.value, rel.value


def pow_cr(x, q):
    """Correctly rounded x**q on the GPU (elementwise, float64)."""
    torch = _torch()
    x = x.contiguous()
    y = torch.empty_like(x)
    _check(lib().rpim_pow_cr(_ptr(x), float(q), _ptr(y), int(x.numel()), _stream()), "rpim_pow_cr")
    return y


def _make_fn():
    torch = _torch()

    class AssembleFn(torch.autograd.Function):
        """K = assemble(node_xyz, cell_E); backward maps dL/dK to dL/dE and dL/dx."""

        @staticmethod
        def forward(ctx, node_xyz, cell_E, plan, nu, precision):
            keep = bool(ctx.needs_input_grad[0] or ctx.needs_input_grad[1])
            K = plan.assemble(node_xyz.detach(), cell_E.detach(), nu, precision, keep_factors=keep)
            ctx.plan, ctx.nu = plan, nu
            ctx.factor_gen = plan.factor_generation() if keep else 0
            ctx.save_for_backward(node_xyz, cell_E)
            return K

        @staticmethod
        def backward(ctx, dK):
            X, E = ctx.saved_tensors
            _check_factors(ctx.plan, ctx.factor_gen)
            dE, dX = ctx.plan.assemble_backward(X.detach(), E.detach(), ctx.nu, dK.detach().double().contiguous())
            return (dX if ctx.needs_input_grad[0] else None, dE if ctx.needs_input_grad[1] else None,
                    None, None, None)

    return AssembleFn


_AssembleFn = None


def _check_factors(plan, gen):
    """The backward reuses the LU factors its forward kept; raise if the plan has replaced them since."""
    if gen == 0 or plan.factor_generation() != gen:
        raise RpimError(-8, "assemble backward",
                        "(the plan's kept factors belong to another forward: run the forward again)")


def assemble(plan: Plan, node_xyz, cell_E, nu=0.3, precision=FP64):
    """Differentiable stiffness assembly: K values on plan's CSR pattern."""
    global _AssembleFn
    if _AssembleFn is None:
        _AssembleFn = _make_fn()
    return _AssembleFn.apply(node_xyz, cell_E, plan, nu, precision)
