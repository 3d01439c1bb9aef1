"""ctypes declarations of libwf's C-ABI (include/wf.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwf.so")

WF_OK, WF_NOT_CONVERGED = 0, 1
WF_EINVAL, WF_ESHAPE, WF_ENOMEM, WF_EHIP, WF_ENONFINITE = -1, -2, -3, -4, -5
WF_F32, WF_F64 = 0, 1
WF_SOLVE_CONVERGED, WF_SOLVE_MAXITER, WF_SOLVE_NONFINITE = 0, 1, 2
WF_ADJ_METRIC, WF_ADJ_GRAD, WF_MASK = 0, 1, 2
WF_METHOD_LBFGS, WF_METHOD_CG = 0, 1
WF_NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024

EXPORTS = [
    "wf_create", "wf_destroy", "wf_last_error", "wf_lbfgs_default", "map_wf_solve", "wf_simulate",
    "sim_fisher", "sim_fisher_rows", "bandpower_qe", "bandpower_qe_batch", "bandpower_iterate", "bmode_leakage_qe", "posterior_error", "convergence_by_band", "wf_forward", "wf_adjoint", "wf_chi2_grad", "wf_hvp", "wf_hvp_noalloc", "wf_band_E", "wf_chi2_dtheta",
    "wf_set_profiling", "wf_kernel_kinds", "wf_kernel_kind_name", "wf_get_kernel_stats",
    "wf_reset_kernel_stats", "wf_set_chain_tiles", "wf_get_chain_tiles", "wf_copy_bandwidth",
    "map_wf_solve_catalog", "wf_catalog_forward", "wf_catalog_adjoint",
]


class WfProblem(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("ncomp", C.c_int32), ("dtype", C.c_int32), ("nbands", C.c_int32),
        ("d", C.c_void_p), ("w", C.c_void_p), ("pshape", C.c_void_p), ("band", C.c_void_p),
        ("theta", C.POINTER(C.c_double)),
    ]


class WfCatalog(C.Structure):
    _fields_ = [("ngal", C.c_int32), ("pos", C.c_void_p), ("e", C.c_void_p), ("wgt", C.c_void_p)]


class WfLbfgsOpts(C.Structure):
    _fields_ = [
        ("m", C.c_int32), ("max_iter", C.c_int32), ("rel_grad_tol", C.c_double), ("dchi2_tol", C.c_double),
        ("refresh_every", C.c_int32), ("iters_per_poll", C.c_int32), ("use_graph", C.c_int32),
        ("precond", C.c_int32), ("method", C.c_int32), ("refine", C.c_int32), ("refine_tol", C.c_double),
    ]


class WfSolveStats(C.Structure):
    _fields_ = [
        ("iters", C.c_int32), ("status", C.c_int32), ("ngrad", C.c_int32), ("reserved", C.c_int32),
        ("chi2", C.c_double), ("rel_grad", C.c_double),
    ]


_lib = None


def load(path: str | None = None):
    """Load libwf.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libwf.so not found at {p}: build it with `python -m paper_1810_00503_amd.build`")
    L = C.CDLL(p)
    vp, i32, dp = C.c_void_p, C.c_int32, C.POINTER(C.c_double)
    L.wf_create.argtypes = [C.POINTER(vp), C.c_int]
    L.wf_destroy.argtypes = [vp]
    L.wf_destroy.restype = None
    L.wf_last_error.argtypes = [vp]
    L.wf_last_error.restype = C.c_char_p
    L.wf_lbfgs_default.argtypes = [C.POINTER(WfLbfgsOpts)]
    L.wf_lbfgs_default.restype = None
    L.map_wf_solve.argtypes = [vp, C.POINTER(WfProblem), i32, C.POINTER(WfLbfgsOpts), C.POINTER(vp),
                               C.POINTER(vp), C.POINTER(WfSolveStats), vp]
    L.map_wf_solve_catalog.argtypes = [vp, C.POINTER(WfProblem), C.POINTER(WfCatalog), i32, C.POINTER(WfLbfgsOpts),
                                       C.POINTER(vp), C.POINTER(WfSolveStats), vp]
    L.wf_catalog_forward.argtypes = [vp, C.POINTER(WfProblem), C.POINTER(WfCatalog), vp, vp, vp]
    L.wf_catalog_adjoint.argtypes = [vp, C.POINTER(WfProblem), C.POINTER(WfCatalog), vp, vp, i32, vp]
    L.wf_simulate.argtypes = [vp, C.POINTER(WfProblem), i32, C.c_uint64, i32, vp, dp, i32, C.c_double, vp, vp]
    L.sim_fisher.argtypes = [vp, C.POINTER(WfProblem), i32, C.c_uint64, vp, C.POINTER(WfLbfgsOpts), dp, dp, dp, dp,
                             vp]
    L.bandpower_qe.argtypes = [vp, C.POINTER(WfProblem), i32, C.c_uint64, vp, C.POINTER(WfLbfgsOpts), dp, dp, dp,
                               dp, vp]
    ip = C.POINTER(i32)
    L.bandpower_qe_batch.argtypes = [vp, C.POINTER(WfProblem), i32, i32, C.c_uint64, C.POINTER(WfLbfgsOpts),
                                     C.POINTER(dp), C.POINTER(dp), C.POINTER(dp), C.POINTER(dp), vp]
    L.wf_copy_bandwidth.argtypes = [vp, vp, vp, C.c_uint64, i32, dp]
    L.sim_fisher_rows.argtypes = [vp, C.POINTER(WfProblem), i32, C.c_uint64, vp, C.POINTER(WfLbfgsOpts), ip, i32, ip,
                                  dp, dp, dp, vp]
    L.bandpower_iterate.argtypes = [vp, C.POINTER(WfProblem), i32, C.c_uint64, vp, C.POINTER(WfLbfgsOpts), ip, i32,
                                    ip, i32, C.c_double, C.c_double, dp, dp, ip, dp, dp, dp, vp]
    L.bmode_leakage_qe.argtypes = [vp, C.POINTER(WfProblem), i32, C.c_uint64, vp, C.POINTER(WfLbfgsOpts),
                                   C.POINTER(i32), i32, dp, dp, dp, dp, vp]
    L.posterior_error.argtypes = [vp, C.POINTER(WfProblem), i32, C.c_uint64, vp, C.POINTER(WfLbfgsOpts), vp, vp, vp]
    L.convergence_by_band.argtypes = [vp, C.POINTER(WfProblem), i32, dp, C.POINTER(WfLbfgsOpts), dp, dp, dp,
                                      C.POINTER(i32), C.POINTER(vp), vp]
    L.wf_forward.argtypes = [vp, C.POINTER(WfProblem), i32, vp, vp, i32, vp]
    L.wf_adjoint.argtypes = [vp, C.POINTER(WfProblem), i32, vp, vp, i32, vp]
    L.wf_chi2_grad.argtypes = [vp, C.POINTER(WfProblem), i32, vp, dp, vp, vp]
    L.wf_hvp.argtypes = [vp, C.POINTER(WfProblem), i32, vp, vp, vp]
    L.wf_hvp_noalloc.argtypes = [vp, C.POINTER(WfProblem), i32, vp, vp, vp]
    L.wf_band_E.argtypes = [vp, C.POINTER(WfProblem), i32, vp, dp, vp]
    L.wf_chi2_dtheta.argtypes = [vp, C.POINTER(WfProblem), i32, vp, dp, dp, vp]
    L.wf_set_profiling.argtypes = [vp, i32]
    L.wf_kernel_kinds.argtypes = []
    L.wf_kernel_kind_name.argtypes = [i32]
    L.wf_kernel_kind_name.restype = C.c_char_p
    L.wf_get_kernel_stats.argtypes = [vp, C.POINTER(C.c_int64), dp, dp]
    L.wf_reset_kernel_stats.argtypes = [vp]
    L.wf_set_chain_tiles.argtypes = [vp, i32, i32, i32, i32]
    L.wf_get_chain_tiles.argtypes = [vp, i32, i32, i32, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32),
                                     C.POINTER(i32)]
    for name in EXPORTS:
        fn = getattr(L, name)
        if fn.restype is C.c_int:
            fn.restype = C.c_int
    _lib = L
    return L
