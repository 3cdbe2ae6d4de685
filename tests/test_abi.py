"""C ABI surface checks that need no GPU: the library loads and exports every
function that include/rpim.h declares; the oracle library loads too."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "rpim.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rpim_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for required in ("rpim_build_pattern", "rpim_assemble", "rpim_assemble_backward", "rpim_apply_penalty_bc"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_1802_04256_amd as rp
    if not os.path.exists(rp.library_path()):
        pytest.fail("librpim.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(rp.library_path())
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings():
    import paper_1802_04256_amd as rp
    lib = rp.lib()
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8, -9):
        s = lib.rpim_status_string(code)
        assert s and s != b"unknown status"


def test_plan_create_rejects_bad_arguments():
    import paper_1802_04256_amd as rp
    lib = rp.lib()
    # NULL problem / NULL out pointer are rejected before any device call
    assert lib.rpim_plan_create(None, None) == -1
    assert lib.rpim_plan_info(None, None) == -1
    assert lib.rpim_get_status(None, None, None) == -1
    assert lib.rpim_assemble(None, None, None, ctypes.c_double(0.3), 0, 0, None, None) == -1
    assert lib.rpim_apply_penalty_bc(None, None, None, 0, 0, None, None, 0, ctypes.c_double(1.0), None, None,
                                     None, None, 0, None) == -1
    assert lib.rpim_penalty_workspace_bytes(0, 0) == 0
    assert lib.rpim_penalty_workspace_bytes(100, 10) >= 16 + 8 + 80
    assert lib.rpim_set_solver(None, 0, 0) == -1
    assert lib.rpim_pcg_workspace_bytes(0) == 0 and lib.rpim_pcg_workspace_bytes(1000) >= 5 * 8 * 1000
    assert lib.rpim_solve_pcg(None, None, None, 0, 10, None, None, ctypes.c_double(1e-8), 10, None, 0, None, None,
                              None) == -1
    assert lib.rpim_factor_generation(None, None) == -1
    assert lib.rpim_autotune(None, None, None, ctypes.c_double(0.3), 0, None, None, None) == -1


def test_tuning_struct_matches_header():
    # the binding's ctypes mirror of rpim_tuning must agree with the header's layout
    import paper_1802_04256_amd as rp
    src = open(os.path.join(ROOT, "include", "rpim.h")).read()
    end = src.index("} rpim_tuning;")
    body = src[src.rindex("typedef struct {", 0, end):end]
    fields = re.findall(r"\b(int32_t|int64_t|float)\s+(\w+)(\[[A-Z_0-9]+\])?;", body)
    names = [f[1] for f in fields]
    assert names == [f[0] for f in rp._Tuning._fields_]
    assert int(re.search(r"#define RPIM_TUNING_MAX_BUCKETS (\d+)", src).group(1)) == rp._TUNING_MAX


def test_package_has_no_cpu_fallback():
    import paper_1802_04256_amd as rp
    src = open(os.path.join(os.path.dirname(rp.__file__), "__init__.py")).read()
    assert "import oracle" not in src and "from oracle" not in src


def test_backward_refuses_factors_of_another_forward():
    # the autograd backward reuses the factors its forward kept; once a later
    # forward (or a rebuild, or autotune) has replaced them it must refuse
    import paper_1802_04256_amd as rp

    class Plan:
        def __init__(self, gen):
            self.gen = gen

        def factor_generation(self):
            return self.gen

    rp._check_factors(Plan(3), 3)
    with pytest.raises(rp.RpimError) as ei:
        rp._check_factors(Plan(4), 3)
    assert ei.value.code == -8
    with pytest.raises(rp.RpimError):
        rp._check_factors(Plan(3), 0)  # the forward kept nothing


def test_tuning_cache_file_round_trip_and_validation(tmp_path):
    # host-only: the text cache keeps solver and gather choices; gather
    # configurations are 1 to 4 waves per row, solver kinds 0 to 3
    import paper_1802_04256_amd as rp
    good = tmp_path / "good.txt"
    good.write_text("# comment\ngfx950 fp64 gather 0 1\ngfx950 mixed gather 0 4\ngfx950 fp64 solver 80 2\n")
    rp.tuning_cache(clear=True)
    try:
        rp.tuning_cache(load=str(good))
        out = tmp_path / "out.txt"
        rp.tuning_cache(save=str(out))
        lines = sorted(l for l in out.read_text().splitlines() if not l.startswith("#"))
        assert lines == ["gfx950 fp64 gather 0 1", "gfx950 fp64 solver 80 2", "gfx950 mixed gather 0 4"]
        for bad in ("gfx950 fp64 gather 0 0", "gfx950 fp64 gather 0 5", "gfx950 fp32 gather 0 1",
                    "gfx950 fp64 solver 80 9", "gfx950 fp64 other 0 1", "gfx950 fp64 gather"):
            f = tmp_path / "bad.txt"
            f.write_text(bad + "\n")
            with pytest.raises(rp.RpimError) as ei:
                rp.tuning_cache(load=str(f))
            assert ei.value.code == -1, bad
        with pytest.raises(rp.RpimError):
            rp.tuning_cache(load=str(tmp_path / "missing.txt"))
    finally:
        rp.tuning_cache(clear=True)
