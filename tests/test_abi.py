"""The C-ABI library loads on the CPU and exports every entry point include/cgp.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "cgp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cgp_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_five_hot_path_calls():
    names = declared_functions()
    for fn in ("cgp_restrict", "cgp_poisson_solve", "cgp_prolong", "cgp_lorentz_force", "cgp_mesh_upload"):
        assert fn in names


def test_library_exports_every_declared_symbol():
    import paper_2003_00082_amd as cgp
    if not os.path.exists(cgp.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(cgp.LIB_PATH)
    for fn in declared_functions():
        assert hasattr(lib, fn), fn
    # and the binding marshals every one of them
    assert sorted(cgp.exported_symbols()) == declared_functions()


def test_binding_fails_loudly_without_the_library(tmp_path):
    import paper_2003_00082_amd as cgp
    saved = cgp._lib
    try:
        cgp._lib = None
        with pytest.raises(ImportError):
            cgp.load(str(tmp_path / "missing.so"))
    finally:
        cgp._lib = saved


def test_struct_layouts_match_the_header():
    import paper_2003_00082_amd as cgp
    assert ctypes.sizeof(cgp.SolveStats) == 32
    assert ctypes.sizeof(cgp.SolveOpts) == 56
    # cgp_momentum_stats: int32 iters[2], int32 status[2], double rel_res[2]
    assert ctypes.sizeof(cgp.MomentumStats) == 32
    assert cgp.MomentumStats.rel_res.offset == 16
