"""Batched Wiener-filter MAP reconstruction and band-power estimation on AMD MI355X.

Python binding of libwf (include/wf.h): every function below marshals torch tensors
(device memory) and numpy arrays (host scalars) into one C-ABI call; all compute runs
in the library's HIP kernels.  There is no CPU fallback: calls raise if the shared
library is missing or the device call fails.

Method: Horowitz, Seljak & Aslanyan, arXiv:1810.00503 (sections 2.2-2.5, appendices
A and C).  Conventions (unitary DFT, half-plane storage [ncomp][n][n/2+1], live and
free modes, S_k = theta[band_k] P_k, spin-2 rotation) are those of include/wf.h.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import Sequence

import numpy as np

from . import _lib as L
from ._lib import (WF_ADJ_GRAD, WF_ADJ_METRIC, WF_F32, WF_F64, WF_MASK, WF_NOT_CONVERGED, WF_OK,  # noqa: F401
                   WF_SOLVE_CONVERGED, WF_SOLVE_MAXITER, WF_SOLVE_NONFINITE, WF_METHOD_LBFGS, WF_METHOD_CG)

__all__ = [
    "load", "Context", "Problem", "LbfgsOpts", "SolveStats", "context", "map_wf_solve", "wf_simulate",
    "sim_fisher", "sim_fisher_rows", "bandpower_qe", "bandpower_qe_batch", "bandpower_iterate", "bmode_leakage_qe", "posterior_error",
    "convergence_by_band",
    "wf_forward",
    "wf_adjoint",
    "wf_chi2_grad", "wf_hvp", "wf_hvp_noalloc", "wf_band_E", "wf_chi2_dtheta",
    "WFError", "kernel_stats", "reset_kernel_stats", "set_profiling", "autograd", "set_chain_tiles", "copy_bandwidth",
    "get_chain_tiles", "GalaxyCatalog", "map_wf_solve_catalog", "catalog_forward", "catalog_adjoint",
]


class WFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libwf error {code}: {msg}")
        self.code = code


def load():
    return L.load()


def _torch():
    import torch
    return torch


class Context:
    """Owns a libwf context (workspace, twiddle tables, captured graphs) on one device."""

    def __init__(self, device: int = 0):
        lib = L.load()
        h = C.c_void_p()
        rc = lib.wf_create(C.byref(h), int(device))
        if rc != 0:
            raise WFError(rc, "wf_create failed")
        self.h = h
        self.device = int(device)
        self.lib = lib

    def close(self):
        if self.h:
            self.lib.wf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc: int, allow_soft: bool = True) -> int:
        if rc < 0:
            raise WFError(rc, self.lib.wf_last_error(self.h).decode(errors="replace"))
        if rc > 0 and not allow_soft:
            raise WFError(rc, "not converged")
        return rc


_contexts: dict[int, Context] = {}


def context(device: int = 0) -> Context:
    if device not in _contexts:
        _contexts[device] = Context(device)
    return _contexts[device]


@dataclasses.dataclass
class LbfgsOpts:
    m: int = 10
    max_iter: int = 20000
    rel_grad_tol: float = 1e-6
    dchi2_tol: float = 0.0
    refresh_every: int = 0
    iters_per_poll: int = 0
    use_graph: int = 1
    precond: int = 0
    method: int = 0   # WF_METHOD_LBFGS or WF_METHOD_CG
    refine: int = 0   # rounds of float64 residual refinement of float32 solves (0 = off)
    refine_tol: float = 1e-10

    def c(self) -> L.WfLbfgsOpts:
        return L.WfLbfgsOpts(self.m, self.max_iter, self.rel_grad_tol, self.dchi2_tol, self.refresh_every,
                             self.iters_per_poll, self.use_graph, self.precond, self.method, self.refine,
                             self.refine_tol)


@dataclasses.dataclass
class SolveStats:
    iters: int
    status: int
    ngrad: int
    chi2: float
    rel_grad: float


class Problem:
    """One map's inputs on the device.

    d [ncomp][n][n] and w [n][n] in the compute dtype (float32 or float64), pshape
    [ncomp][n][n/2+1] float64, band [ncomp][n][n/2+1] int32, theta [nbands] (host)."""

    def __init__(self, w, pshape, band, theta, d=None, ncomp=None, device=None):
        torch = _torch()
        dev = device if device is not None else (w.device if isinstance(w, torch.Tensor) else "cuda:0")
        self.w = torch.as_tensor(w, device=dev).contiguous()
        if self.w.dtype not in (torch.float32, torch.float64):
            raise TypeError("w must be float32 or float64")
        self.rdtype = self.w.dtype
        self.n = int(self.w.shape[-1])
        self.pshape = torch.as_tensor(pshape, dtype=torch.float64, device=dev).contiguous()
        self.ncomp = int(ncomp if ncomp is not None else self.pshape.shape[0])
        self.band = torch.as_tensor(band, dtype=torch.int32, device=dev).contiguous()
        self.theta = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1))
        self.d = None if d is None else torch.as_tensor(d, dtype=self.rdtype, device=dev).contiguous()
        self._check()

    @classmethod
    def for_catalog(cls, n: int, pshape, band, theta, device=None) -> "Problem":
        """A float32 problem whose data is a galaxy catalog (sec. 3.4): prior and grid only,
        no pixel data or weights (map_wf_solve_catalog, catalog_forward / catalog_adjoint)."""
        torch = _torch()
        p = object.__new__(cls)
        dev = device if device is not None else (pshape.device if isinstance(pshape, torch.Tensor) else "cuda:0")
        p.w = None
        p.d = None
        p.rdtype = torch.float32
        p.n = int(n)
        p.pshape = torch.as_tensor(pshape, dtype=torch.float64, device=dev).contiguous()
        p.ncomp = int(p.pshape.shape[0])
        p.band = torch.as_tensor(band, dtype=torch.int32, device=dev).contiguous()
        p.theta = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1))
        p._check()
        return p

    @property
    def device(self):
        return self.pshape.device

    def _check(self):
        n, c = self.n, self.ncomp
        if self.w is not None and tuple(self.w.shape) != (n, n):
            raise ValueError(f"w must be [{n}][{n}]")
        if tuple(self.pshape.shape) != (c, n, n // 2 + 1) or tuple(self.band.shape) != (c, n, n // 2 + 1):
            raise ValueError("pshape and band must be [ncomp][n][n/2+1]")
        if self.d is not None and tuple(self.d.shape) != (c, n, n):
            raise ValueError("d must be [ncomp][n][n]")

    def with_data(self, d) -> "Problem":
        p = object.__new__(Problem)
        p.__dict__.update(self.__dict__)
        p.__dict__.pop("_cstruct", None)
        torch = _torch()
        p.d = torch.as_tensor(d, dtype=self.rdtype, device=self.device).contiguous()
        p._check()
        return p

    def with_theta(self, theta) -> "Problem":
        p = object.__new__(Problem)
        p.__dict__.update(self.__dict__)
        p.__dict__.pop("_cstruct", None)
        p.theta = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1))
        return p

    @property
    def dtype_code(self) -> int:
        return L.WF_F64 if self.rdtype == _torch().float64 else L.WF_F32

    @property
    def cdtype(self):
        torch = _torch()
        return torch.complex128 if self.rdtype == torch.float64 else torch.complex64

    @property
    def nbands(self) -> int:
        return int(self.theta.size)

    def c(self) -> L.WfProblem:
        """The C-ABI struct of this problem: plain pointers to its tensors and to theta.  Built
        once per object and reused while the object still holds the same tensors and theta
        (with_data / with_theta make new objects), so a batch call does not rebuild a struct
        per problem; the cache keeps those objects alive, so their pointers stay valid."""
        objs = (self.d, self.w, self.pshape, self.band, self.theta)
        cached = self.__dict__.get("_cstruct")
        if cached is not None and all(a is b for a, b in zip(cached[0], objs)):
            return cached[1]
        th = self.theta.ctypes.data_as(C.POINTER(C.c_double)) if self.theta.size else None
        cs = L.WfProblem(self.n, self.ncomp, self.dtype_code, self.theta.size,
                         self.d.data_ptr() if self.d is not None else None,
                         self.w.data_ptr() if self.w is not None else None,
                         self.pshape.data_ptr(), self.band.data_ptr(), th)
        self.__dict__["_cstruct"] = (objs, cs)
        return cs

    def device_index(self) -> int:
        return self.device.index or 0


def _stream(dev: int):
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _opts(o):
    return (o or LbfgsOpts()).c()


def _dptr(t):
    return C.cast(C.c_void_p(t.data_ptr()), C.POINTER(C.c_double))


def _out_buffers(torch, given, problems, shape_of, dtype_of, what):
    """Caller-supplied output tensors, checked against the problems, or new ones."""
    if given is None:
        # one allocation per distinct (shape, dtype, device), handed out as views: a batch of
        # many small maps would otherwise spend most of a call in the allocator
        groups = {}
        for i, p in enumerate(problems):
            groups.setdefault((shape_of(p), dtype_of(p), p.device), []).append(i)
        outs = [None] * len(problems)
        for (shape, dt, dev), idx in groups.items():
            big = torch.empty((len(idx),) + tuple(shape), dtype=dt, device=dev)
            for j, t in zip(idx, big.unbind(0)):
                outs[j] = t
        return outs
    given = list(given)
    if len(given) != len(problems):
        raise ValueError(f"{what}: {len(given)} tensors for {len(problems)} problems")
    for i, (t, p) in enumerate(zip(given, problems)):
        if (tuple(t.shape) != shape_of(p) or t.dtype != dtype_of(p) or t.device != p.device
                or not t.is_contiguous()):
            raise ValueError(f"{what}[{i}] must be a contiguous {dtype_of(p)} tensor of shape {shape_of(p)} "
                             f"on {p.device}")
    return given


def map_wf_solve(problems: Sequence[Problem], opts: LbfgsOpts | None = None, want_maps: bool = False,
                 ctx: Context | None = None, out=None, maps_out=None):
    """MAP fields of a batch of problems (uneven sizes allowed).
    Returns (s list of complex [ncomp][n][n/2+1], maps list or None, stats list, rc).
    `out` (and `maps_out`, which implies want_maps) are optional preallocated output tensors,
    one per problem; a loop that passes the same ones every call allocates nothing per call.
    Outputs allocated here are views into one tensor per distinct shape (disjoint rows of it)."""
    torch = _torch()
    problems = list(problems)
    B = len(problems)
    dev = problems[0].device_index() if B else 0
    cx = ctx or context(dev)
    outs = _out_buffers(torch, out, problems, lambda p: (p.ncomp, p.n, p.n // 2 + 1), lambda p: p.cdtype, "out")
    want_maps = want_maps or maps_out is not None
    maps = _out_buffers(torch, maps_out, problems, lambda p: (p.ncomp, p.n, p.n), lambda p: p.rdtype,
                        "maps_out") if want_maps else None
    cps = (L.WfProblem * max(B, 1))(*[p.c() for p in problems])
    s_arr = (C.c_void_p * max(B, 1))(*[o.data_ptr() for o in outs])
    m_arr = (C.c_void_p * max(B, 1))(*[m.data_ptr() for m in maps]) if maps else None
    st = (L.WfSolveStats * max(B, 1))()
    o = _opts(opts)
    rc = cx.lib.map_wf_solve(cx.h, cps, B, C.byref(o), s_arr, m_arr, st, _stream(dev))
    cx.check(rc)
    stats = [SolveStats(st[i].iters, st[i].status, st[i].ngrad, st[i].chi2, st[i].rel_grad) for i in range(B)]
    return outs, maps, stats, rc


class GalaxyCatalog:
    """A galaxy catalog on the device (sec. 3.4): positions pos [ngal][2] (y, x) in pixel units
    (float64, periodic), measured values e [ncomp][ngal] and inverse noise variances
    wgt [ngal] (float32; needed by solves only)."""

    def __init__(self, pos, e=None, wgt=None, device=None):
        torch = _torch()
        dev = device if device is not None else (pos.device if isinstance(pos, torch.Tensor) else "cuda:0")
        self.pos = torch.as_tensor(pos, dtype=torch.float64, device=dev).contiguous()
        if self.pos.dim() != 2 or self.pos.shape[1] != 2:
            raise ValueError("pos must be [ngal][2]")
        self.ngal = int(self.pos.shape[0])
        self.e = None if e is None else torch.as_tensor(e, dtype=torch.float32, device=dev).contiguous()
        self.wgt = None if wgt is None else torch.as_tensor(wgt, dtype=torch.float32, device=dev).contiguous()
        if self.e is not None and (self.e.dim() != 2 or self.e.shape[1] != self.ngal):
            raise ValueError("e must be [ncomp][ngal]")
        if self.wgt is not None and tuple(self.wgt.shape) != (self.ngal,):
            raise ValueError("wgt must be [ngal]")

    def c(self) -> L.WfCatalog:
        return L.WfCatalog(self.ngal, self.pos.data_ptr(), self.e.data_ptr() if self.e is not None else None,
                           self.wgt.data_ptr() if self.wgt is not None else None)


def map_wf_solve_catalog(problems: Sequence[Problem], catalogs: Sequence[GalaxyCatalog],
                         opts: LbfgsOpts | None = None, ctx: Context | None = None, out=None):
    """MAP fields of a batch of catalogs (problems from Problem.for_catalog give the grid and
    prior).  Returns (s list of complex64 [ncomp][n][n/2+1], stats list, rc)."""
    torch = _torch()
    problems, catalogs = list(problems), list(catalogs)
    if len(problems) != len(catalogs):
        raise ValueError("one catalog per problem")
    B = len(problems)
    dev = problems[0].device_index() if B else 0
    cx = ctx or context(dev)
    outs = _out_buffers(torch, out, problems, lambda p: (p.ncomp, p.n, p.n // 2 + 1), lambda p: p.cdtype, "out")
    cps = (L.WfProblem * max(B, 1))(*[p.c() for p in problems])
    cats = (L.WfCatalog * max(B, 1))(*[g.c() for g in catalogs])
    s_arr = (C.c_void_p * max(B, 1))(*[o.data_ptr() for o in outs])
    st = (L.WfSolveStats * max(B, 1))()
    o = _opts(opts)
    rc = cx.lib.map_wf_solve_catalog(cx.h, cps, cats, B, C.byref(o), s_arr, st, _stream(dev))
    cx.check(rc)
    stats = [SolveStats(st[i].iters, st[i].status, st[i].ngrad, st[i].chi2, st[i].rel_grad) for i in range(B)]
    return outs, stats, rc


def catalog_forward(problem: Problem, catalog: GalaxyCatalog, s, ctx: Context | None = None):
    """The field s [ncomp][n][n/2+1] (complex64) at the catalog's positions: [ncomp][ngal]."""
    torch = _torch()
    s = s.contiguous()
    if s.dtype != torch.complex64 or tuple(s.shape) != (problem.ncomp, problem.n, problem.n // 2 + 1):
        raise ValueError("s must be complex64 [ncomp][n][n/2+1]")
    dev = problem.device_index()
    cx = ctx or context(dev)
    g = torch.empty((problem.ncomp, catalog.ngal), dtype=torch.float32, device=s.device)
    cp, cc = problem.c(), catalog.c()
    cx.check(cx.lib.wf_catalog_forward(cx.h, C.byref(cp), C.byref(cc), s.data_ptr(), g.data_ptr(), _stream(dev)))
    return g


def catalog_adjoint(problem: Problem, catalog: GalaxyCatalog, r, flags: int = WF_ADJ_METRIC,
                    ctx: Context | None = None):
    """Adjoint of catalog_forward for r [ncomp][ngal] (float32): complex64 [ncomp][n][n/2+1]."""
    torch = _torch()
    r = r.contiguous()
    if r.dtype != torch.float32 or tuple(r.shape) != (problem.ncomp, catalog.ngal):
        raise ValueError("r must be float32 [ncomp][ngal]")
    dev = problem.device_index()
    cx = ctx or context(dev)
    s = torch.empty((problem.ncomp, problem.n, problem.n // 2 + 1), dtype=torch.complex64, device=r.device)
    cp, cc = problem.c(), catalog.c()
    cx.check(cx.lib.wf_catalog_adjoint(cx.h, C.byref(cp), C.byref(cc), r.data_ptr(), s.data_ptr(), int(flags),
                                       _stream(dev)))
    return s


def wf_simulate(problem: Problem, nsim: int, seed: int, sim0: int = 0, draws=None, theta_true=None,
                boost_band: int = -1, boost_factor: float = 1.0, ctx: Context | None = None):
    """Simulated data maps [nsim][ncomp][n][n] (sec. 2.4)."""
    torch = _torch()
    dev = problem.device_index()
    cx = ctx or context(dev)
    out = torch.empty((nsim, problem.ncomp, problem.n, problem.n), dtype=problem.rdtype, device=problem.device)
    dr = None
    if draws is not None:
        draws = torch.as_tensor(draws, dtype=problem.rdtype, device=problem.device).contiguous()
        if tuple(draws.shape) != (nsim, 2, problem.ncomp, problem.n, problem.n):
            raise ValueError("draws must be [nsim][2][ncomp][n][n]")
        dr = draws.data_ptr()
    tt = None
    if theta_true is not None:
        tt_np = np.ascontiguousarray(np.asarray(theta_true, np.float64))
        tt = tt_np.ctypes.data_as(C.POINTER(C.c_double))
    cp = problem.c()
    rc = cx.lib.wf_simulate(cx.h, C.byref(cp), nsim, C.c_uint64(seed), sim0, dr, tt, boost_band,
                            float(boost_factor), out.data_ptr(), _stream(dev))
    cx.check(rc)
    return out


def _draws_ptr(problem, draws, nsim):
    if draws is None:
        return None, None
    torch = _torch()
    t = torch.as_tensor(draws, dtype=problem.rdtype, device=problem.device).contiguous()
    if tuple(t.shape) != (nsim, 2, problem.ncomp, problem.n, problem.n):
        raise ValueError("draws must be [nsim][2][ncomp][n][n]")
    return t, t.data_ptr()


def sim_fisher(problem: Problem, nsim: int, seed: int, draws=None, opts: LbfgsOpts | None = None,
               ctx: Context | None = None, want_var: bool = False):
    """Simulation noise bias b and Fisher matrix F around problem.theta (eqs. blmv, fisher).
    Returns (F [nb][nb], b [nb], E_sims [nsim][nb], rc) as numpy arrays; with want_var
    (F, b, E_sims, F_var [nb][nb], rc), F_var the Monte Carlo variance of each entry of F."""
    dev = problem.device_index()
    cx = ctx or context(dev)
    nb = problem.nbands
    F = np.zeros((nb, nb))
    b = np.zeros(nb)
    Fv = np.zeros((nb, nb))
    Es = np.zeros((nsim, nb))
    keep, dp = _draws_ptr(problem, draws, nsim)
    cp = problem.c()
    o = _opts(opts)
    rc = cx.lib.sim_fisher(cx.h, C.byref(cp), nsim, C.c_uint64(seed), dp, C.byref(o),
                           F.ctypes.data_as(C.POINTER(C.c_double)), b.ctypes.data_as(C.POINTER(C.c_double)),
                           Fv.ctypes.data_as(C.POINTER(C.c_double)) if want_var else None,
                           Es.ctypes.data_as(C.POINTER(C.c_double)), _stream(dev))
    cx.check(rc)
    del keep
    return (F, b, Es, Fv, rc) if want_var else (F, b, Es, rc)


def bandpower_qe(problem: Problem, nsim: int, seed: int, draws=None, opts: LbfgsOpts | None = None,
                 ctx: Context | None = None):
    """Quadratic band-power estimate.  Returns (theta_hat, E, b, F, rc) as numpy arrays."""
    dev = problem.device_index()
    cx = ctx or context(dev)
    nb = problem.nbands
    th = np.zeros(nb)
    E = np.zeros(nb)
    b = np.zeros(nb)
    F = np.zeros((nb, nb))
    keep, dp = _draws_ptr(problem, draws, nsim)
    cp = problem.c()
    o = _opts(opts)
    ptr = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
    rc = cx.lib.bandpower_qe(cx.h, C.byref(cp), nsim, C.c_uint64(seed), dp, C.byref(o), ptr(th), ptr(E), ptr(b),
                             ptr(F), _stream(dev))
    cx.check(rc)
    del keep
    return th, E, b, F, rc


def bandpower_qe_batch(problems: Sequence[Problem], nsim: int, seed: int, opts: LbfgsOpts | None = None,
                       ctx: Context | None = None):
    """Quadratic band-power estimates of several maps (uneven sizes allowed) with all of their
    solves shared among batched solves; map i draws its simulations from Philox key seed + i.
    Returns (theta_hat list, E list, b list, F list, rc) of numpy arrays."""
    problems = list(problems)
    P = len(problems)
    dev = problems[0].device_index() if P else 0
    cx = ctx or context(dev)
    th = [np.zeros(p.nbands) for p in problems]
    Es = [np.zeros(p.nbands) for p in problems]
    bs = [np.zeros(p.nbands) for p in problems]
    Fs = [np.zeros((p.nbands, p.nbands)) for p in problems]
    dpp = C.POINTER(C.c_double)

    def arr(xs):
        return (dpp * max(P, 1))(*[x.ctypes.data_as(dpp) for x in xs])

    cps = (L.WfProblem * max(P, 1))(*[p.c() for p in problems])
    o = _opts(opts)
    rc = cx.lib.bandpower_qe_batch(cx.h, cps, P, nsim, C.c_uint64(seed), C.byref(o), arr(th), arr(Es), arr(bs),
                                   arr(Fs), _stream(dev))
    cx.check(rc)
    return th, Es, bs, Fs, rc


def _rows_groups(problem, rows, groups):
    """int32 host arrays (or None) for the sampled-row calls."""
    nb = problem.nbands
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int32)
    if r is not None and r.size == 0:
        raise ValueError("rows must name at least one band")
    g = None if groups is None else np.ascontiguousarray(groups, dtype=np.int32)
    if g is not None and g.shape != (nb,):
        raise ValueError("groups must have one id per band")
    ip = lambda a: None if a is None else a.ctypes.data_as(C.POINTER(C.c_int32))  # noqa: E731
    return r, g, ip(r), (0 if r is None else int(r.size)), ip(g)


def sim_fisher_rows(problem: Problem, nsim: int, seed: int, rows=None, groups=None, draws=None,
                    opts: LbfgsOpts | None = None, ctx: Context | None = None):
    """sim_fisher with boosted simulations for the Fisher rows `rows` only, the others
    interpolated along the diagonals within band groups (sec. 3.1).
    Returns (F [nb][nb], b [nb], E_sims [nsim][nb], rc) as numpy arrays."""
    dev = problem.device_index()
    cx = ctx or context(dev)
    nb = problem.nbands
    F = np.zeros((nb, nb))
    b = np.zeros(nb)
    Es = np.zeros((nsim, nb))
    keep, dp = _draws_ptr(problem, draws, nsim)
    r, g, rp, nr, gp = _rows_groups(problem, rows, groups)
    cp = problem.c()
    o = _opts(opts)
    ptr = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
    rc = cx.lib.sim_fisher_rows(cx.h, C.byref(cp), nsim, C.c_uint64(seed), dp, C.byref(o), rp, nr, gp, ptr(F),
                                ptr(b), ptr(Es), _stream(dev))
    cx.check(rc)
    del keep, r, g
    return F, b, Es, rc


def bandpower_iterate(problem: Problem, nsim: int, seed: int, max_iter: int = 3, rel_tol: float = 0.01,
                      floor: float = 0.01, rows=None, groups=None, draws=None, opts: LbfgsOpts | None = None,
                      ctx: Context | None = None):
    """Fiducial iteration of the band-power estimate (sec. 2.3): the fiducial is reset to
    max(theta_hat, floor * previous) and the estimate repeated.  Returns (theta_hat,
    history [n_iter + 1][nb] of fiducials, E, b, F, rc) as numpy arrays."""
    dev = problem.device_index()
    cx = ctx or context(dev)
    nb = problem.nbands
    th = np.zeros(nb)
    hist = np.zeros((max_iter + 1, nb))
    E = np.zeros(nb)
    b = np.zeros(nb)
    F = np.zeros((nb, nb))
    nit = C.c_int32(0)
    keep, dp = _draws_ptr(problem, draws, nsim)
    r, g, rp, nr, gp = _rows_groups(problem, rows, groups)
    cp = problem.c()
    o = _opts(opts)
    ptr = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
    rc = cx.lib.bandpower_iterate(cx.h, C.byref(cp), nsim, C.c_uint64(seed), dp, C.byref(o), rp, nr, gp, max_iter,
                                  rel_tol, floor, ptr(th), ptr(hist), C.byref(nit), ptr(E), ptr(b), ptr(F),
                                  _stream(dev))
    cx.check(rc)
    del keep, r, g
    return th, hist[:nit.value + 1], E, b, F, rc


def bmode_leakage_qe(problem: Problem, nsim: int, seed: int, b_bands, draws=None, opts: LbfgsOpts | None = None,
                     ctx: Context | None = None):
    """B-mode band powers with the E->B leakage as a bias (appendix C).  Returns (theta_B,
    E_B, b_B, F_BB, rc) as numpy arrays over the bands b_bands."""
    dev = problem.device_index()
    cx = ctx or context(dev)
    bb = np.ascontiguousarray(b_bands, dtype=np.int32)
    k = int(bb.size)
    if k == 0:
        raise ValueError("b_bands must name at least one band")
    th, E, b = np.zeros(k), np.zeros(k), np.zeros(k)
    F = np.zeros((k, k))
    keep, dp = _draws_ptr(problem, draws, nsim)
    cp = problem.c()
    o = _opts(opts)
    ptr = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
    rc = cx.lib.bmode_leakage_qe(cx.h, C.byref(cp), nsim, C.c_uint64(seed), dp, C.byref(o),
                                 bb.ctypes.data_as(C.POINTER(C.c_int32)), k, ptr(th), ptr(E), ptr(b), ptr(F),
                                 _stream(dev))
    cx.check(rc)
    del keep
    return th, E, b, F, rc


def posterior_error(problem: Problem, nsim: int, seed: int, draws=None, opts: LbfgsOpts | None = None,
                    want_modes: bool = True, want_pixels: bool = True, ctx: Context | None = None):
    """Posterior error of the Wiener filter from simulations with the problem's prior
    (residual covariance S - S R^T C^-1 R S, appendix A).  Returns (var_modes
    [ncomp][n][n/2+1] or None, var_pix [ncomp][n][n] or None, rc) as device tensors."""
    torch = _torch()
    dev = problem.device_index()
    cx = ctx or context(dev)
    n, c = problem.n, problem.ncomp
    vm = torch.empty((c, n, n // 2 + 1), dtype=problem.rdtype, device=problem.device) if want_modes else None
    vp = torch.empty((c, n, n), dtype=problem.rdtype, device=problem.device) if want_pixels else None
    keep, dp = _draws_ptr(problem, draws, nsim)
    cp = problem.c()
    o = _opts(opts)
    rc = cx.lib.posterior_error(cx.h, C.byref(cp), nsim, C.c_uint64(seed), dp, C.byref(o),
                                None if vm is None else vm.data_ptr(), None if vp is None else vp.data_ptr(),
                                _stream(dev))
    cx.check(rc)
    del keep
    return vm, vp, rc


def convergence_by_band(problem: Problem, tols, opts: LbfgsOpts | None = None, want_fields: bool = False,
                        ctx: Context | None = None):
    """Convergence as a function of scale (appendix B): the MAP of problem.d at the
    reference tolerance (opts.rel_grad_tol) and at each of `tols`, in one batched solve.
    Returns (power [ntol + 1][nb], err_power [ntol][nb], cv [nb], iters [ntol + 1],
    fields (list of ntol + 1 tensors, reference first) or None, rc)."""
    torch = _torch()
    dev = problem.device_index()
    cx = ctx or context(dev)
    t = np.ascontiguousarray(tols, dtype=np.float64)
    nt, nb = int(t.size), problem.nbands
    power = np.zeros((nt + 1, nb))
    err = np.zeros((nt, nb))
    cv = np.zeros(nb)
    its = np.zeros(nt + 1, np.int32)
    fields = None
    outs = None
    if want_fields:
        cdt = torch.complex64 if problem.rdtype == torch.float32 else torch.complex128
        fields = [torch.empty((problem.ncomp, problem.n, problem.n // 2 + 1), dtype=cdt, device=problem.device)
                  for _ in range(nt + 1)]
        outs = (C.c_void_p * (nt + 1))(*[f.data_ptr() for f in fields])
    cp = problem.c()
    o = _opts(opts)
    ptr = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
    rc = cx.lib.convergence_by_band(cx.h, C.byref(cp), nt, ptr(t), C.byref(o), ptr(power), ptr(err), ptr(cv),
                                    its.ctypes.data_as(C.POINTER(C.c_int32)), outs, _stream(dev))
    cx.check(rc)
    return power, err, cv, its, fields, rc


def _batch_shape(problem, t, kind):
    n, c = problem.n, problem.ncomp
    if kind == "s":
        shp = (c, n, n // 2 + 1)
    else:
        shp = (c, n, n)
    if tuple(t.shape) == shp:
        return 1, False
    if t.dim() == 4 and tuple(t.shape[1:]) == shp:
        return int(t.shape[0]), True
    raise ValueError(f"expected [batch]{list(shp)}, got {list(t.shape)}")


def wf_forward(problem: Problem, s, flags: int = 0, ctx: Context | None = None):
    """x = R s (or M R s with WF_MASK) for one field [c][n][n/2+1] or a batch [B][c][n][n/2+1]."""
    torch = _torch()
    s = s.contiguous()
    if s.dtype != problem.cdtype:
        raise TypeError(f"s must be {problem.cdtype}")
    B, batched = _batch_shape(problem, s, "s")
    dev = problem.device_index()
    cx = ctx or context(dev)
    x = torch.empty((B, problem.ncomp, problem.n, problem.n), dtype=problem.rdtype, device=s.device)
    cp = problem.c()
    cx.check(cx.lib.wf_forward(cx.h, C.byref(cp), B, s.data_ptr(), x.data_ptr(), int(flags), _stream(dev)))
    return x if batched else x[0]


def wf_adjoint(problem: Problem, x, flags: int = WF_ADJ_METRIC, ctx: Context | None = None):
    """R^T x (metric adjoint) or the stored-coefficient gradient (WF_ADJ_GRAD)."""
    torch = _torch()
    x = x.contiguous()
    if x.dtype != problem.rdtype:
        raise TypeError(f"x must be {problem.rdtype}")
    B, batched = _batch_shape(problem, x, "x")
    dev = problem.device_index()
    cx = ctx or context(dev)
    s = torch.empty((B, problem.ncomp, problem.n, problem.n // 2 + 1), dtype=problem.cdtype, device=x.device)
    cp = problem.c()
    cx.check(cx.lib.wf_adjoint(cx.h, C.byref(cp), B, x.data_ptr(), s.data_ptr(), int(flags), _stream(dev)))
    return s if batched else s[0]


def wf_chi2_grad(problem: Problem, s, want_grad: bool = True, ctx: Context | None = None):
    """chi^2 of each field (numpy [B]) and d chi^2 / d s (torch, or None)."""
    torch = _torch()
    s = s.contiguous()
    if s.dtype != problem.cdtype:
        raise TypeError(f"s must be {problem.cdtype}")
    B, batched = _batch_shape(problem, s, "s")
    dev = problem.device_index()
    cx = ctx or context(dev)
    chi = np.zeros(B)
    g = torch.empty_like(s) if want_grad else None
    cp = problem.c()
    cx.check(cx.lib.wf_chi2_grad(cx.h, C.byref(cp), B, s.data_ptr(), chi.ctypes.data_as(C.POINTER(C.c_double)),
                                 g.data_ptr() if g is not None else None, _stream(dev)))
    if not batched:
        return chi[0], (g if g is None else g)
    return chi, g


def wf_hvp(problem: Problem, p, ctx: Context | None = None):
    """Curvature product d^2 chi^2 / ds ds . p in the stored-coefficient convention."""
    torch = _torch()
    p = p.contiguous()
    B, batched = _batch_shape(problem, p, "s")
    dev = problem.device_index()
    cx = ctx or context(dev)
    out = torch.empty_like(p)
    cp = problem.c()
    cx.check(cx.lib.wf_hvp(cx.h, C.byref(cp), B, p.data_ptr(), out.data_ptr(), _stream(dev)))
    return out


def wf_hvp_noalloc(problem: Problem, p, out, ctx: Context | None = None):
    """wf_hvp into the caller's `out` (same shape and dtype as p) without any device
    allocation by the library (its buffers live in a fixed per-GPU scratch array).  The call
    is enqueued on the current stream and returns without waiting."""
    p = p.contiguous()
    B, batched = _batch_shape(problem, p, "s")
    if tuple(out.shape) != tuple(p.shape) or out.dtype != p.dtype or not out.is_contiguous():
        raise ValueError("out must be a contiguous tensor shaped and typed like p")
    dev = problem.device_index()
    cx = ctx or context(dev)
    cp = problem.c()
    cx.check(cx.lib.wf_hvp_noalloc(cx.h, C.byref(cp), B, p.data_ptr(), out.data_ptr(), _stream(dev)))
    return out


def wf_band_E(problem: Problem, s, ctx: Context | None = None):
    """E_l of each field with problem's prior: numpy [nbands] or [B][nbands]."""
    s = s.contiguous()
    B, batched = _batch_shape(problem, s, "s")
    dev = problem.device_index()
    cx = ctx or context(dev)
    E = np.zeros((B, problem.nbands))
    cp = problem.c()
    cx.check(cx.lib.wf_band_E(cx.h, C.byref(cp), B, s.data_ptr(), E.ctypes.data_as(C.POINTER(C.c_double)),
                              _stream(dev)))
    return E if batched else E[0]


def wf_chi2_dtheta(problem: Problem, s, gout=None, ctx: Context | None = None):
    """sum_i gout[i] d chi^2(s_i) / d theta_b at fixed fields (numpy [nbands]); gout None =
    ones.  s is one field [c][n][n/2+1] or a batch [B][c][n][n/2+1]."""
    s = s.contiguous()
    B, batched = _batch_shape(problem, s, "s")
    dev = problem.device_index()
    cx = ctx or context(dev)
    out = np.zeros(problem.nbands)
    go = None
    if gout is not None:
        go = np.ascontiguousarray(np.asarray(gout, np.float64).reshape(-1))
        if go.size != B:
            raise ValueError(f"gout must have {B} entries")
    cp = problem.c()
    cx.check(cx.lib.wf_chi2_dtheta(cx.h, C.byref(cp), B, s.data_ptr(),
                                   go.ctypes.data_as(C.POINTER(C.c_double)) if go is not None else None,
                                   out.ctypes.data_as(C.POINTER(C.c_double)), _stream(dev)))
    return out


def copy_bandwidth(nbytes: int = 2 * 1024 ** 3, reps: int = 5, device: int = 0, ctx: Context | None = None) -> float:
    """HBM streaming-copy reference in GB/s (read + write) of the library's copy kernel."""
    torch = _torch()
    cx = ctx or context(device)
    n = nbytes // 16 * 4
    src = torch.empty(n, dtype=torch.float32, device=f"cuda:{device}")
    dst = torch.empty_like(src)
    out = C.c_double()
    torch.cuda.synchronize()
    cx.check(cx.lib.wf_copy_bandwidth(cx.h, src.data_ptr(), dst.data_ptr(), C.c_uint64(n * 4), int(reps),
                                      C.byref(out)))
    return float(out.value)


def set_profiling(on: bool, ctx: Context | None = None):
    cx = ctx or context(0)
    cx.check(cx.lib.wf_set_profiling(cx.h, 1 if on else 0))


def kernel_stats(ctx: Context | None = None) -> dict:
    cx = ctx or context(0)
    k = cx.lib.wf_kernel_kinds()
    la = (C.c_int64 * k)()
    ms = (C.c_double * k)()
    by = (C.c_double * k)()
    cx.check(cx.lib.wf_get_kernel_stats(cx.h, la, ms, by))
    return {cx.lib.wf_kernel_kind_name(i).decode(): dict(launches=la[i], ms=ms[i], bytes=by[i]) for i in range(k)}


def reset_kernel_stats(ctx: Context | None = None):
    cx = ctx or context(0)
    cx.check(cx.lib.wf_reset_kernel_stats(cx.h))


def set_chain_tiles(rbv: int = 0, cpb: int = 1, group: int = 0, reg: int = 0, ctx: Context | None = None):
    """Fix the transform chain's tiles (rbv rows, cpb column blocks, group instances per
    launch, reg = register-staged passes: bit 0 row, bit 1 column inverse, bit 2 column
    forward; or reg = 8: the single-pass kernel of small maps), or return to autotuning
    with rbv = 0."""
    cx = ctx or context(0)
    cx.check(cx.lib.wf_set_chain_tiles(cx.h, int(rbv), int(cpb), int(group), int(reg)))


def get_chain_tiles(n: int, ncomp: int, dtype: int = WF_F32, batch: int = 64, ctx: Context | None = None):
    """(rbv, cpb, group, reg, tuned) in use for this shape and batch size."""
    cx = ctx or context(0)
    a, b, g, r = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    rc = cx.check(cx.lib.wf_get_chain_tiles(cx.h, n, ncomp, dtype, batch, C.byref(a), C.byref(b), C.byref(g),
                                            C.byref(r)))
    return a.value, b.value, g.value, r.value, rc == 0


from . import autograd  # noqa: E402,F401  (torch.autograd.Function wrappers)
