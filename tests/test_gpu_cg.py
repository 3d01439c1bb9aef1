"""Conjugate gradients in the batched engine (an alternative optimiser on the same quadratic):
the MAP is unique, so CG's field is held to the same bars as L-BFGS's against the oracle's
MAP (1e-5 relative L2 in float32, the exact FP64 whitened gradient small, chi^2), plain and
split-preconditioned, batched with uneven shapes, with periodic restarts, and in float64."""
import numpy as np
import pytest

import oracle as O
from paper_1810_00503_amd import workloads as WL
from tests.gpu_util import make_problem, oracle_data, rel_l2

pytestmark = pytest.mark.gpu


def _wl(kind, n):
    return {"density": lambda: WL.density_workload(n, 21, nbands=4, holes=4, target_mask=0.25),
            "shear": lambda: WL.shear_workload(n, 22, nbands_e=3, nbands_b=3),
            "cmb": lambda: WL.cmb_workload(n, 23, nbands=6)}[kind]()


def _solve(lib, probs, **kw):
    s, maps, st, rc = lib.map_wf_solve(probs, lib.LbfgsOpts(**kw), want_maps=True)
    return [x.cpu().numpy() for x in s], [x.cpu().numpy() for x in maps], st, rc


def _check_field(s, d, wl, S, ref, chi2, gbar=3e-6):
    assert rel_l2(s, ref["s"]) < 1e-5
    g = np.sqrt(S) * O.grad_chi2(s, d, wl.W, S)
    g0 = np.sqrt(S) * O.grad_chi2(np.zeros_like(s), d, wl.W, S)
    assert np.linalg.norm(g) <= gbar * np.linalg.norm(g0)
    assert abs(chi2 - ref["chi2"]) <= 1e-5 * ref["chi2"]


@pytest.mark.parametrize("kind,n,precond", [("density", 16, 0), ("shear", 64, 0), ("density", 128, 0),
                                            ("cmb", 64, 1), ("shear", 64, 1)])
def test_cg_map_matches_oracle(lib, kind, n, precond):
    import torch
    print(f"[cg {kind} n={n} precond={precond}]", flush=True)
    wl = _wl(kind, n)
    d = oracle_data(wl, 5)
    S = O.prior_S(wl.pshape, wl.band, wl.theta_fid)
    ref = O.lbfgs_solve(d, wl.W, S, tol=1e-11, max_iter=50000)
    prob = make_problem(lib, torch, wl, "f32", d=d)
    tol = 3e-8 if kind == "cmb" else 1e-7
    s, maps, st, rc = _solve(lib, [prob], rel_grad_tol=tol, method=lib.WF_METHOD_CG, precond=precond)
    sl, _, stl, _ = _solve(lib, [prob], rel_grad_tol=tol, precond=precond)
    print(f"   iters CG {st[0].iters} (exact gradients {st[0].ngrad}), L-BFGS {stl[0].iters}; "
          f"rel_grad {st[0].rel_grad:.2e}", flush=True)
    assert st[0].status == lib.WF_SOLVE_CONVERGED and rc == 0, st[0]
    assert st[0].rel_grad <= tol and st[0].ngrad >= 2
    _check_field(s[0], d, wl, S, ref, st[0].chi2)
    assert rel_l2(O.forward(s[0]), maps[0]) < 3e-6


def test_cg_uneven_batch_and_restarts(lib):
    import torch
    print("[cg uneven batch]", flush=True)
    wls = [_wl("density", 32), _wl("shear", 64), _wl("density", 48), _wl("shear", 16), _wl("density", 128)]
    ds = [oracle_data(wl, 40 + i) for i, wl in enumerate(wls)]
    probs = [make_problem(lib, torch, wl, "f32", d=d) for wl, d in zip(wls, ds)]
    s, _, st, rc = _solve(lib, probs, rel_grad_tol=1e-7, method=lib.WF_METHOD_CG)
    sr, _, str_, rcr = _solve(lib, probs, rel_grad_tol=1e-7, method=lib.WF_METHOD_CG, refresh_every=7)
    assert rc == 0 and rcr == 0
    for i, (wl, d) in enumerate(zip(wls, ds)):
        S = O.prior_S(wl.pshape, wl.band, wl.theta_fid)
        ref = O.lbfgs_solve(d, wl.W, S, tol=1e-11, max_iter=50000)
        _check_field(s[i], d, wl, S, ref, st[i].chi2)
        _check_field(sr[i], d, wl, S, ref, str_[i].chi2)
        # a restart every 7 iterations: at least one exact gradient per 7 iterations
        assert str_[i].ngrad >= 1 + str_[i].iters // 7
        # one instance alone gives the same field as in the batch
        one, _, st1, _ = _solve(lib, [probs[i]], rel_grad_tol=1e-7, method=lib.WF_METHOD_CG)
        assert rel_l2(one[0], s[i]) < 2e-6


def test_cg_float64_and_zero_data(lib):
    import torch
    print("[cg f64, zero data]", flush=True)
    wl = _wl("shear", 32)
    d = oracle_data(wl, 9)
    S = O.prior_S(wl.pshape, wl.band, wl.theta_fid)
    ref = O.lbfgs_solve(d, wl.W, S, tol=1e-12, max_iter=50000)
    prob = make_problem(lib, torch, wl, "f64", d=d)
    s, _, st, rc = _solve(lib, [prob], rel_grad_tol=1e-11, method=lib.WF_METHOD_CG)
    assert rc == 0
    assert rel_l2(s[0], ref["s"]) < 1e-9
    z = make_problem(lib, torch, wl, "f32", d=np.zeros_like(d))
    s0, _, st0, rc0 = _solve(lib, [z], method=lib.WF_METHOD_CG)
    assert rc0 == 0 and st0[0].iters == 0 and np.all(s0[0] == 0)
