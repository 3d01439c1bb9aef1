"""GPU parity of the convergence-by-scale diagnostic (appendix B).  Loose solutions depend
on rounding (where an iteration stops), so the returned fields themselves are checked:
the reference against the oracle's MAP, every looser field against its own stop criterion
(the oracle's exact FP64 gradient), and the band sums against the oracle's band power of
the same fields."""
import numpy as np
import pytest

import oracle as O
from paper_1810_00503_amd import workloads as WL
from tests.gpu_util import make_problem, oracle_data, rel_l2

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["density", "shear"])
def test_convergence_by_band(lib, kind):
    import torch
    print(f"[convergence_by_band {kind}]", flush=True)
    n = 64
    if kind == "density":
        wl = WL.density_workload(n, 44, nbands=6, holes=4, target_mask=0.25)
    else:
        wl = WL.shear_workload(n, 45, nbands_e=3, nbands_b=3, b_ratio=0.2)
    d = oracle_data(wl, 8)
    prob = make_problem(lib, torch, wl, "f32", d=d)
    tols = [1e-2, 1e-3, 1e-4]
    power, err, cv, its, fields, rc = lib.convergence_by_band(prob, tols, lib.LbfgsOpts(rel_grad_tol=1e-7),
                                                              want_fields=True)
    assert rc == 0
    S = O.prior_S(wl.pshape, wl.band, wl.theta_fid)
    ref = O.lbfgs_solve(d, wl.W, S, tol=1e-10)["s"]
    f = [x.cpu().numpy().astype(np.complex128) for x in fields]
    assert rel_l2(f[0], ref) < 1e-5
    fr = O.free_mask(n)[None] & (S > 0)
    g0 = np.linalg.norm(O.whitened_grad(np.zeros_like(ref), d, wl.W, S))
    for t, tol in enumerate(tols):
        w = np.where(fr, f[t + 1] / np.sqrt(np.where(S > 0, S, 1.0)), 0)
        rg = np.linalg.norm(O.whitened_grad(w, d, wl.W, S)) / g0
        print(f"  tol {tol:.0e}: iterations {its[t + 1]}, exact relative gradient {rg:.2e}", flush=True)
        assert rg <= 1.5 * tol
    assert its[1] <= its[2] <= its[3] <= its[0]
    for i in range(len(tols) + 1):
        np.testing.assert_allclose(power[i], O.band_power(f[i], S, wl.band, wl.nbands), rtol=1e-5)
    for t in range(len(tols)):
        want = O.band_power(f[t + 1] - f[0], S, wl.band, wl.nbands)
        np.testing.assert_allclose(err[t], want, rtol=1e-3, atol=1e-6 * power[0].max())
    np.testing.assert_allclose(cv, O.cosmic_variance(S, wl.band, wl.nbands), rtol=1e-15)
    # a looser tolerance leaves more error in the map
    tot = err.sum(1)
    assert tot[0] > tot[1] > tot[2]


def test_convergence_by_band_rejects_bad_tolerances(lib):
    import torch
    wl = WL.density_workload(16, 46, nbands=2, holes=1, target_mask=0.1)
    prob = make_problem(lib, torch, wl, "f32", d=oracle_data(wl, 1))
    with pytest.raises(lib.WFError):
        lib.convergence_by_band(prob, [1e-3, 0.0])
    with pytest.raises(lib.WFError):
        lib.convergence_by_band(prob, [])
