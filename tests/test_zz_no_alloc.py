"""The allocation-free penalty entry point (library-owned static scratch) gives
the same K, rhs, alpha and status as rpim_apply_penalty_bc with a caller
workspace, through the C ABI, on two calls in a row (the second with a
smaller system and fewer fixed dofs, so the scratch holds the first call's
contents), on a rejected call, and on an oversized request."""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _penalty_both(rp, row_ptr, col_idx, K0, fixed, ub, factor):
    """Run both entry points on copies of K0 (and zero rhs); return their (K, rhs, alpha, status)."""
    import torch
    lib = rp.lib()
    dev = K0.device
    prec = rp.FP64 if K0.dtype == torch.float64 else rp.MIXED
    n_dof = int(row_ptr.numel() - 1)
    fx = torch.from_numpy(np.ascontiguousarray(fixed, np.int32)).to(dev)
    ubt = torch.from_numpy(np.ascontiguousarray(ub, np.float64)).to(dev)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    out = []
    for variant in ("workspace", "noalloc"):
        K = K0.clone()
        rhs = torch.zeros(n_dof, dtype=torch.float64, device=dev)
        alpha = torch.full((1,), -7.0, dtype=torch.float64, device=dev)
        status = torch.full((1,), 99, dtype=torch.int32, device=dev)
        args = [C.c_void_p(row_ptr.data_ptr()), C.c_void_p(col_idx.data_ptr()), C.c_void_p(K.data_ptr()), prec,
                n_dof, C.c_void_p(fx.data_ptr()), C.c_void_p(ubt.data_ptr()), int(fx.numel()), float(factor),
                C.c_void_p(rhs.data_ptr()), C.c_void_p(alpha.data_ptr()), C.c_void_p(status.data_ptr())]
        if variant == "workspace":
            nbytes = lib.rpim_penalty_workspace_bytes(n_dof, int(fx.numel()))
            ws = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=dev)
            st = lib.rpim_apply_penalty_bc(*args, C.c_void_p(ws.data_ptr()), nbytes, stream)
        else:
            st = lib.rpim_apply_penalty_bc_noalloc(*args, stream)
        assert st == 0, (variant, st)
        torch.cuda.synchronize()
        out.append((K.cpu().numpy(), rhs.cpu().numpy(), float(alpha.item()), int(status.item())))
    return out


def test_noalloc_penalty_matches_workspace_entry():
    import torch
    import paper_1802_04256_amd as rp
    dev = torch.device("cuda:0")
    cases = [("slope", W.slope(L=10.0, W=6.0, H=5.0, x_c=2.5), torch.float64),
             ("cantilever", W.cantilever(), torch.float32)]  # second call: smaller system, fewer fixed dofs
    for name, prob, dt in cases:
        print(f"[gpu case] noalloc penalty {name}: nodes={prob.n_nodes} dtype={dt}", flush=True)
        plan = rp.Plan.from_problem(prob, device=dev)
        row_ptr, col_idx = plan.build_pattern()
        K0 = plan.assemble(cell_E=prob.cell_E, nu=prob.nu, precision="fp64" if dt == torch.float64 else "mixed")
        plan.status()
        X = prob.node_xyz
        side = np.where(X[:, 0] == X[:, 0].min())[0]
        fixed = np.sort((3 * side[:, None] + np.arange(3)).ravel()).astype(np.int32)
        ub = np.linspace(-1.0, 1.0, len(fixed))
        (Kw, rw, aw, sw), (Kn, rn, an, sn) = _penalty_both(rp, row_ptr, col_idx, K0, fixed, ub, 1e8)
        assert sw == 0 and sn == 0
        assert aw == an and aw > 0
        assert np.array_equal(Kw, Kn) and np.array_equal(rw, rn)
        assert not np.array_equal(Kw, K0.cpu().numpy())
        # a rejected call (fixed dofs out of order): both report RPIM_E_ARG and leave K as it was
        bad = fixed[::-1].copy()
        (Kw, _, _, sw), (Kn, _, _, sn) = _penalty_both(rp, row_ptr, col_idx, K0, bad, ub, 1e8)
        assert sw == -1 and sn == -1
        assert np.array_equal(Kw, K0.cpu().numpy()) and np.array_equal(Kn, K0.cpu().numpy())


def test_noalloc_penalty_rejects_oversized_request():
    import torch
    import paper_1802_04256_amd as rp
    lib = rp.lib()
    n = rp.PENALTY_NOALLOC_MAX_FIXED + 1
    dev = torch.device("cuda:0")
    row_ptr = torch.arange(n + 1, dtype=torch.int64, device=dev)
    col_idx = torch.arange(n, dtype=torch.int32, device=dev)
    K = torch.ones(n, dtype=torch.float64, device=dev)
    fx = torch.arange(n, dtype=torch.int32, device=dev)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = lib.rpim_apply_penalty_bc_noalloc(C.c_void_p(row_ptr.data_ptr()), C.c_void_p(col_idx.data_ptr()),
                                           C.c_void_p(K.data_ptr()), rp.FP64, n, C.c_void_p(fx.data_ptr()), None,
                                           n, 1e8, None, None, None, stream)
    assert st == -6  # RPIM_E_RANGE, before any kernel runs
    torch.cuda.synchronize()
    assert bool((K == 1.0).all())
