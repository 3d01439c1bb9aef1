"""GPU parity of the sampled-Fisher-row estimate and of the fiducial iteration (the
Fisher matrix's smoothness, sec. 3.1; the iterated fiducial, sec. 2.3) against the FP64
oracle, with identical draws on both sides.  Bars as for the full estimate: E, b, F and
Theta_hat to 1e-4 (F and Theta_hat also absolutely, relative to their largest entry)."""
import numpy as np
import pytest

import oracle as O
from paper_1810_00503_amd import workloads as WL
from tests.gpu_util import make_problem, oracle_data

pytestmark = pytest.mark.gpu


def _workload(ncomp):
    n = 16
    if ncomp == 1:
        wl = WL.density_workload(n, 90, nbands=5, holes=2, target_mask=0.2)
        wl.pshape = WL.density_pshape(n, kd=n / 3.0)
        return wl, None, [0, 2, 4]
    wl = WL.shear_workload(n, 91, nbands_e=3, nbands_b=3, b_ratio=0.2)
    return wl, [0, 0, 0, 1, 1, 1], [0, 2, 3, 5]


def test_all_rows_equal_the_full_estimate(lib):
    import torch
    print("[sim_fisher_rows all rows]", flush=True)
    wl, _, _ = _workload(1)
    prob = make_problem(lib, torch, wl, "f32")
    opts = lib.LbfgsOpts(rel_grad_tol=1e-8)
    F, b, Es, _ = lib.sim_fisher(prob, 2, 5, opts=opts)
    F2, b2, Es2, _ = lib.sim_fisher_rows(prob, 2, 5, rows=list(range(wl.nbands)), opts=opts)
    np.testing.assert_array_equal(F, F2)
    np.testing.assert_array_equal(b, b2)
    np.testing.assert_array_equal(Es, Es2)


@pytest.mark.parametrize("ncomp", [1, 2])
def test_sampled_rows_match_oracle(lib, ncomp):
    import torch
    print(f"[sim_fisher_rows ncomp={ncomp}]", flush=True)
    wl, groups, rows = _workload(ncomp)
    nsim = 3
    draws = WL.white_draws(wl.n, ncomp, nsim, 123)
    prob = make_problem(lib, torch, wl, "f32")
    dt = torch.tensor(draws, dtype=torch.float32, device="cuda:0")
    opts = lib.LbfgsOpts(rel_grad_tol=1e-8)
    F, b, Es, _ = lib.sim_fisher_rows(prob, nsim, 0, rows=rows, groups=groups, draws=dt, opts=opts)
    bo, Fo, Eso = O.sim_fisher_rows(wl.W, wl.pshape, wl.band, wl.theta_fid, wl.nbands, draws, rows, groups, tol=1e-11)
    np.testing.assert_allclose(Es, Eso, rtol=1e-4)
    np.testing.assert_allclose(b, bo, rtol=1e-4)
    np.testing.assert_allclose(F, Fo, rtol=1e-4, atol=1e-4 * np.abs(Fo).max())
    np.testing.assert_array_equal(F, F.T)


@pytest.mark.parametrize("ncomp", [1, 2])
def test_fiducial_iteration_matches_oracle(lib, ncomp):
    import torch
    print(f"[bandpower_iterate ncomp={ncomp}]", flush=True)
    wl, groups, rows = _workload(ncomp)
    nsim = 3
    draws = WL.white_draws(wl.n, ncomp, nsim, 321)
    d = oracle_data(wl, 17)
    prob = make_problem(lib, torch, wl, "f32", d=d)
    dt = torch.tensor(draws, dtype=torch.float32, device="cuda:0")
    opts = lib.LbfgsOpts(rel_grad_tol=1e-8)
    th, hist, E, b, F, _ = lib.bandpower_iterate(prob, nsim, 0, max_iter=2, rel_tol=0.0, floor=0.05, rows=rows,
                                                 groups=groups, draws=dt, opts=opts)
    tho, histo = O.bandpower_iterate(d, wl.W, wl.pshape, wl.band, wl.theta_fid, wl.nbands, draws, 2, 0.0, 0.05,
                                     rows, groups, tol=1e-11)
    assert hist.shape == (3, wl.nbands)
    for t in range(3):
        np.testing.assert_allclose(hist[t], histo[t], rtol=2e-4, atol=1e-4 * np.abs(histo[t]).max(), err_msg=f"t={t}")
    np.testing.assert_allclose(th, tho, rtol=2e-4, atol=1e-4 * np.abs(tho).max())


def test_fiducial_iteration_one_step_is_the_estimate(lib):
    import torch
    print("[bandpower_iterate one step]", flush=True)
    wl, _, _ = _workload(1)
    prob = make_problem(lib, torch, wl, "f32", d=oracle_data(wl, 3))
    opts = lib.LbfgsOpts(rel_grad_tol=1e-8)
    th, E, b, F, _ = lib.bandpower_qe(prob, 2, 11, opts=opts)
    th1, hist, E1, b1, F1, _ = lib.bandpower_iterate(prob, 2, 11, max_iter=1, opts=opts)
    np.testing.assert_array_equal(th, th1)
    np.testing.assert_array_equal(E, E1)
    np.testing.assert_array_equal(F, F1)
    np.testing.assert_array_equal(hist[1], np.maximum(th, 0.01 * wl.theta_fid))


def test_bad_rows_and_groups_are_rejected(lib):
    import torch
    wl, groups, _ = _workload(2)
    prob = make_problem(lib, torch, wl, "f32")
    for rows, grp in (([2, 1], None), ([0, 0, 3], None), ([0, 6], None), ([0, 1, 2], groups)):
        with pytest.raises(lib.WFError):
            lib.sim_fisher_rows(prob, 1, 0, rows=rows, groups=grp)
    with pytest.raises(ValueError):
        lib.sim_fisher_rows(prob, 1, 0, rows=[])
    with pytest.raises(lib.WFError):
        lib.bandpower_iterate(prob, 1, 0, max_iter=0)
    with pytest.raises(lib.WFError):
        lib.bandpower_iterate(prob, 1, 0, floor=0.0)


def test_bmode_leakage_matches_oracle(lib):
    """B-mode leakage bias (appendix C), identical draws: theta_B, E_B, b_B, F_BB to 1e-4."""
    import torch
    print("[bmode_leakage_qe]", flush=True)
    wl = WL.shear_workload(16, 93, nbands_e=2, nbands_b=2, b_ratio=0.3)
    nsim = 3
    draws = WL.white_draws(wl.n, 2, nsim, 444)
    d = oracle_data(wl, 45)
    prob = make_problem(lib, torch, wl, "f32", d=d)
    dt = torch.tensor(draws, dtype=torch.float32, device="cuda:0")
    B = [2, 3]
    th, E, b, F, rc = lib.bmode_leakage_qe(prob, nsim, 0, B, draws=dt, opts=lib.LbfgsOpts(rel_grad_tol=1e-7))
    assert rc == 0
    tho, Eo, bo, Fo = O.bmode_leakage_qe(d, wl.W, wl.pshape, wl.band, wl.theta_fid, wl.nbands, draws, B, tol=1e-11)
    np.testing.assert_allclose(E, Eo, rtol=1e-4)
    np.testing.assert_allclose(b, bo, rtol=1e-4)
    np.testing.assert_allclose(F, Fo, rtol=1e-4, atol=1e-4 * np.abs(Fo).max())
    np.testing.assert_allclose(th, tho, rtol=2e-4, atol=1e-4 * np.abs(tho).max())
    for bad in ([3, 2], [0, 4]):
        with pytest.raises(lib.WFError):
            lib.bmode_leakage_qe(prob, 1, 0, bad)
