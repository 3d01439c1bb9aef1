"""The C-ABI library loads and exports every symbol include/wf.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wf.h")
LIB = os.path.join(ROOT, "paper_1810_00503_amd", "libwf.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([A-Za-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["map_wf_solve", "sim_fisher", "bandpower_qe", "wf_forward", "wf_adjoint", "wf_chi2_grad",
                 "wf_hvp", "wf_band_E", "wf_simulate", "wf_create", "wf_destroy", "wf_last_error"]:
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libwf.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libwf.so not built")
def test_binding_matches_exports():
    from paper_1810_00503_amd import _lib
    names = _declared()
    assert sorted(_lib.EXPORTS) == names
    lib = _lib.load()
    assert lib.wf_kernel_kinds() == 11
    assert lib.wf_kernel_kind_name(10) == b"catalog"
    assert lib.wf_kernel_kind_name(9) == b"simulate"
    assert lib.wf_kernel_kind_name(8) == b"cg_dir"
    assert lib.wf_kernel_kind_name(3) == b"passA"
    o = _lib.WfLbfgsOpts()
    lib.wf_lbfgs_default(ctypes.byref(o))
    assert o.m == 10 and o.rel_grad_tol == 1e-6 and o.use_graph == 1 and o.method == 0
    assert o.refine == 0 and o.refine_tol == 1e-10


def test_struct_layouts_match_header():
    from paper_1810_00503_amd import _lib
    assert ctypes.sizeof(_lib.WfProblem) == 4 * 4 + 5 * 8
    assert ctypes.sizeof(_lib.WfLbfgsOpts) == 4 * 2 + 8 * 2 + 4 * 6 + 8
    assert ctypes.sizeof(_lib.WfSolveStats) == 4 * 4 + 8 * 2
