"""GPU parity of the posterior-error estimate (residual covariance S - S R^T C^-1 R S of the
Wiener filter, appendix A) against the FP64 oracle with identical simulations: per stored
entry and per pixel.  The residual s - s_hat is small where the data constrain the field,
so its float32 error relative to its own size is larger than that of the MAP: bar 2e-3
relative plus 1e-4 of the map's maximum."""
import numpy as np
import pytest

import oracle as O
from paper_1810_00503_amd import workloads as WL
from tests.gpu_util import make_problem

pytestmark = pytest.mark.gpu


def _check(got, want, what):
    got = got.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(got, want, rtol=2e-3, atol=1e-4 * np.abs(want).max(), err_msg=what)


@pytest.mark.parametrize("ncomp", [1, 2])
def test_posterior_error_matches_oracle_draws(lib, ncomp):
    import torch
    print(f"[posterior_error draws ncomp={ncomp}]", flush=True)
    n = 16
    if ncomp == 1:
        wl = WL.density_workload(n, 90, nbands=3, holes=2, target_mask=0.2)
        wl.pshape = WL.density_pshape(n, kd=n / 3.0)
    else:
        wl = WL.shear_workload(n, 91, nbands_e=2, nbands_b=2, b_ratio=0.2)
    nsim = 4
    draws = WL.white_draws(n, ncomp, nsim, 77)
    prob = make_problem(lib, torch, wl, "f32")
    dt = torch.tensor(draws, dtype=torch.float32, device="cuda:0")
    vm, vp, rc = lib.posterior_error(prob, nsim, 0, draws=dt, opts=lib.LbfgsOpts(rel_grad_tol=1e-7))
    assert rc == 0
    om, op = O.posterior_error(wl.W, wl.pshape, wl.band, wl.theta_fid, draws, tol=1e-11)
    _check(vm, om, "var_modes")
    _check(vp, op, "var_pix")


def test_posterior_error_philox_and_single_output(lib):
    import torch
    print("[posterior_error philox]", flush=True)
    n, nsim, seed = 16, 3, 4242
    wl = WL.density_workload(n, 92, nbands=2, holes=2, target_mask=0.2)
    wl.pshape = WL.density_pshape(n, kd=n / 3.0)
    prob = make_problem(lib, torch, wl, "f32")
    opts = lib.LbfgsOpts(rel_grad_tol=1e-7)
    vm, vp, rc = lib.posterior_error(prob, nsim, seed, opts=opts)
    assert rc == 0
    draws = O.philox.draws_for_sims(seed, range(nsim), n, 1)
    om, op = O.posterior_error(wl.W, wl.pshape, wl.band, wl.theta_fid, draws, tol=1e-11)
    _check(vm, om, "var_modes")
    _check(vp, op, "var_pix")
    vm2, vp2, _ = lib.posterior_error(prob, nsim, seed, opts=opts, want_pixels=False)
    assert vp2 is None
    assert torch.equal(vm, vm2)
    with pytest.raises(lib.WFError):
        lib.posterior_error(prob, nsim, seed, want_modes=False, want_pixels=False)
    with pytest.raises(lib.WFError):
        lib.posterior_error(prob, 0, seed)


def test_posterior_error_shear512_full_size(lib):
    """The 512^2 E/B shear workload (two simulations, Philox path) against the oracle."""
    import torch
    print("[posterior_error 512^2 shear]", flush=True)
    wl = WL.shear_eb()
    prob = make_problem(lib, torch, wl, "f32")
    nsim, seed = 2, 99
    vm, vp, rc = lib.posterior_error(prob, nsim, seed, opts=lib.LbfgsOpts(rel_grad_tol=1e-6))   # the workload's tolerance
    assert rc == 0
    draws = O.philox.draws_for_sims(seed, range(nsim), wl.n, wl.ncomp)
    om, op = O.posterior_error(wl.W, wl.pshape, wl.band, wl.theta_fid, draws, tol=1e-9)
    gm, gp = vm.cpu().numpy().astype(np.float64), vp.cpu().numpy().astype(np.float64)
    em = np.linalg.norm(gm - om) / np.linalg.norm(om)
    ep = np.linalg.norm(gp - op) / np.linalg.norm(op)
    print(f"  relative L2: var_modes {em:.2e}, var_pix {ep:.2e}", flush=True)
    assert em < 2e-4 and ep < 2e-4
