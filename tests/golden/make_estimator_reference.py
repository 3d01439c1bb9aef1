"""Writes the oracle's sampled-row Fisher estimate of the 256^2 density workload and its
B-mode leakage estimate of the 512^2 E/B shear workload, at full size with a reduced number of
simulations (tests/golden/estimators_full.json).

Calls only the oracle and the seeded input generators.  The data maps are those of
make_bandpower_reference.py (the oracle's simulation of each workload from its truth, white
normals of seed DATA_SEED); the simulations use the Philox4x32-10 stream of seed SIM_SEED
(simulations 0 .. NSIM - 1), which the library's own simulation reproduces; every solve runs to
a relative gradient of TOL.  Stored: for the density workload b and F from simulations of the
Fisher rows ROWS (the other rows interpolated), for the shear workload Theta_hat_B, E_B, b_B
and F_BB over its B bands.

    python tests/golden/make_estimator_reference.py        # about three minutes on one core
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_1810_00503_amd import workloads as WL  # noqa: E402

TOL = 1e-9
ROWS = [0, 3, 6, 9, 11]


def data_of(wl, seed):
    return O.simulate(WL.white_draws(wl.n, wl.ncomp, 1, seed)[0], O.prior_S(wl.pshape, wl.band, wl.theta_true), wl.W)


def main():
    out = {}
    t = time.time()
    wl = WL.density_bands(256)
    nsim, sim_seed = 3, 2102
    draws = O.philox.draws_for_sims(sim_seed, range(nsim), wl.n, wl.ncomp)
    b, F, _ = O.sim_fisher_rows(wl.W, wl.pshape, wl.band, wl.theta_fid, wl.nbands, draws, ROWS, tol=TOL)
    out["density256_rows"] = dict(workload=wl.name, n=wl.n, ncomp=wl.ncomp, nbands=wl.nbands, rows=ROWS,
                                  sim_seed=sim_seed, nsim=nsim,
                                  sims="Philox4x32-10 key sim_seed, simulations 0 .. nsim-1", rel_grad_tol=TOL,
                                  b=b.tolist(), F=F.tolist(), seconds=round(time.time() - t, 1))
    print("density256_rows", out["density256_rows"]["seconds"], "s", flush=True)
    t = time.time()
    wl = WL.shear_eb(512)
    nsim, data_seed, sim_seed = 2, 3101, 3102
    bb = [l for l in range(wl.nbands) if l >= wl.nbands // 2]   # the B bands follow the E bands
    d = data_of(wl, data_seed)
    draws = O.philox.draws_for_sims(sim_seed, range(nsim), wl.n, wl.ncomp)
    th, E, b, F = O.bmode_leakage_qe(d, wl.W, wl.pshape, wl.band, wl.theta_fid, wl.nbands, draws, bb, tol=TOL)
    out["shear512_leakage"] = dict(workload=wl.name, n=wl.n, ncomp=wl.ncomp, nbands=wl.nbands, b_bands=bb,
                                   data_seed=data_seed,
                                   data="oracle simulate of white_draws(n, ncomp, 1, data_seed) at theta_true",
                                   sim_seed=sim_seed, nsim=nsim,
                                   sims="Philox4x32-10 key sim_seed, simulations 0 .. nsim-1", rel_grad_tol=TOL,
                                   theta_hat_B=th.tolist(), E_B=E.tolist(), b_B=b.tolist(), F_BB=F.tolist(),
                                   seconds=round(time.time() - t, 1))
    print("shear512_leakage", out["shear512_leakage"]["seconds"], "s", flush=True)
    with open(os.path.join(HERE, "estimators_full.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
