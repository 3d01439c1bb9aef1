"""The single-pass transform kernel of small maps (the whole field in one work-group's LDS:
column inverse, row and column forward passes of a solver's curvature product or gradient in
one launch) against the three-pass chain and the oracle: MAP fields, chi^2 and iteration
counts for float32 and float64, spin-0 and spin-2, sides 8 to 128 (radix-3 sides included);
operator calls keep the three passes when it is fixed; the autotuner may choose it.

Bars: the two paths differ only in the order of the partial sums and of the transforms'
rounding; solved to 1e-6 (float32) or 1e-10 (float64), their fields agree within the solve
bar (1e-5 relative L2 in float32, 1e-9 in float64) and each is within it of the oracle's
MAP (1e-5, 1e-9); iteration counts depend on round-off and are not compared."""
import numpy as np
import pytest

import oracle as O
from paper_1810_00503_amd import workloads as WL
from tests.gpu_util import make_problem, oracle_data, rel_l2

pytestmark = pytest.mark.gpu


def _wls(kind, n, k, seed):
    if kind == "shear":
        return [WL.shear_workload(n, seed + i, nbands_e=2, nbands_b=2, b_ratio=0.2) for i in range(k)]
    return [WL.density_workload(n, seed + i, nbands=3, holes=2, target_mask=0.2) for i in range(k)]


@pytest.mark.parametrize("kind,n,dt", [("density", 8, "f32"), ("shear", 16, "f32"), ("density", 24, "f32"),
                                       ("shear", 48, "f32"), ("density", 64, "f32"), ("shear", 96, "f32"),
                                       ("density", 128, "f32"), ("shear", 128, "f32"), ("shear", 64, "f64"),
                                       ("shear", 96, "f64"), ("density", 128, "f64")])
def test_single_pass_matches_three_passes_and_oracle(lib, kind, n, dt):
    import torch
    print(f"[single pass {kind} n={n} {dt}]", flush=True)
    wls = _wls(kind, n, 5, 700 + n)
    ds = [oracle_data(wl, 710 + i) for i, wl in enumerate(wls)]
    probs = [make_problem(lib, torch, wl, dt, d=d) for wl, d in zip(wls, ds)]
    tol = 1e-6 if dt == "f32" else 1e-10
    opts = lib.LbfgsOpts(rel_grad_tol=tol)
    try:
        lib.set_chain_tiles(4, 1, 0, 0)
        s3, _, st3, rc3 = lib.map_wf_solve(probs, opts)
        lib.set_chain_tiles(4, 1, 0, 8)
        assert lib.get_chain_tiles(n, wls[0].ncomp, lib.WF_F32 if dt == "f32" else lib.WF_F64, 5)[3] == 8
        s1, _, st1, rc1 = lib.map_wf_solve(probs, opts)
    finally:
        lib.set_chain_tiles(0)
    print("   single pass:", [(x.status, x.iters, x.ngrad, f"{x.rel_grad:.2e}") for x in st1], flush=True)
    print("   three passes:", [(x.status, x.iters, x.ngrad, f"{x.rel_grad:.2e}") for x in st3], flush=True)
    assert rc1 == lib.WF_OK and rc3 == lib.WF_OK
    bar = 1e-5 if dt == "f32" else 1e-9
    for i in range(len(probs)):
        a, b = s1[i].cpu().numpy(), s3[i].cpu().numpy()
        assert rel_l2(a, b) < bar, (i, rel_l2(a, b))
        assert abs(st1[i].chi2 - st3[i].chi2) <= (1e-6 if dt == "f32" else 1e-12) * abs(st3[i].chi2)
        # iteration counts are not compared: they depend on round-off
    for i in range(2):
        wl, d = wls[i], ds[i]
        ref = O.lbfgs_solve(d, wl.W, O.prior_S(wl.pshape, wl.band, wl.theta_fid), tol=1e-12)
        err = rel_l2(s1[i].cpu().numpy(), ref["s"])
        print(f"   map {i}: iters {st1[i].iters} (three passes {st3[i].iters}), field vs oracle {err:.2e}", flush=True)
        assert err < (1e-5 if dt == "f32" else 1e-9)


def test_single_pass_cg_and_preconditioned(lib):
    import torch
    print("[single pass: CG, preconditioned]", flush=True)
    wls = [WL.cmb_workload(64, 720 + i, nbands=4, target_mask=0.25) for i in range(4)]
    probs = [make_problem(lib, torch, wl, "f32", d=oracle_data(wl, 730 + i)) for i, wl in enumerate(wls)]
    for opts in (lib.LbfgsOpts(rel_grad_tol=1e-6, method=lib.WF_METHOD_CG),
                 lib.LbfgsOpts(rel_grad_tol=1e-6, precond=1)):
        try:
            lib.set_chain_tiles(4, 1, 0, 0)
            s3, _, st3, _ = lib.map_wf_solve(probs, opts)
            lib.set_chain_tiles(4, 1, 0, 8)
            s1, _, st1, _ = lib.map_wf_solve(probs, opts)
        finally:
            lib.set_chain_tiles(0)
        for i in range(len(probs)):
            # both meet the same gradient bar; the badly conditioned CMB maps are compared in
            # the float64 gradient (the energy norm), which is what the tolerance fixes
            wl = wls[i]
            S = O.prior_S(wl.pshape, wl.band, wl.theta_fid)
            d = oracle_data(wl, 730 + i)
            g0 = np.linalg.norm(np.sqrt(S) * O.grad_chi2(np.zeros_like(s1[i].cpu().numpy()), d, wl.W, S))
            for s in (s1[i], s3[i]):
                g = np.linalg.norm(np.sqrt(S) * O.grad_chi2(s.cpu().numpy(), d, wl.W, S))
                assert g <= 3e-6 * g0, g / g0


def test_operators_keep_three_passes_and_tuner_may_choose_it(lib):
    import torch
    print("[single pass: operators, tuner]", flush=True)
    wl = _wls("shear", 32, 1, 740)[0]
    p = make_problem(lib, torch, wl, "f32", d=oracle_data(wl, 741))
    rng = np.random.default_rng(3)
    s = torch.tensor(rng.standard_normal((2, 32, 17)) + 1j * rng.standard_normal((2, 32, 17)),
                     dtype=torch.complex64, device="cuda:0")
    x0 = lib.wf_forward(p, s)
    try:
        lib.set_chain_tiles(4, 1, 0, 8)
        x1 = lib.wf_forward(p, s)
        g1 = lib.wf_adjoint(p, x0)
    finally:
        lib.set_chain_tiles(0)
    assert torch.equal(x0, x1)
    assert torch.equal(g1, lib.wf_adjoint(p, x0))
    # a batch of 64 small maps: the tuner times the single pass beside the three-pass choices
    wls = _wls("density", 64, 64, 750)
    probs = [make_problem(lib, torch, w, "f32", d=oracle_data(w, 760 + i)) for i, w in enumerate(wls)]
    cx = lib.Context(0)
    try:
        _, _, st, rc = lib.map_wf_solve(probs, lib.LbfgsOpts(rel_grad_tol=1e-6), ctx=cx)
        rbv, cpb, grp, reg, tuned = lib.get_chain_tiles(64, 1, lib.WF_F32, 64, ctx=cx)
        print(f"   tuned choice for 64 maps of 64^2: rbv {rbv} cpb {cpb} group {grp} reg {reg}", flush=True)
        assert tuned and rc == lib.WF_OK
        assert reg in range(9)
    finally:
        cx.close()
    with pytest.raises(lib.WFError):
        lib.set_chain_tiles(4, 1, 0, 9)
