"""Writes the oracle's band-power estimates of the 256^2 density and 512^2 E/B shear workloads
at full size with a reduced number of simulations (tests/golden/bandpowers_full.json).

Calls only the oracle and the seeded input generators.  Per workload: the data map is the
oracle's simulation of the workload from its truth (white normals of seed DATA_SEED); the
simulations use the Philox4x32-10 stream of seed SIM_SEED (simulations 0 .. NSIM - 1), which
the library's own simulation reproduces; every solve runs to a relative gradient of TOL.
Stored: E of the data map, b, F and Theta_hat.

    python tests/golden/make_bandpower_reference.py        # a few minutes on one core
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_1810_00503_amd import workloads as WL  # noqa: E402

TOL = 1e-9
CASES = [("density256", lambda: WL.density_bands(256), 2101, 2102, 3),
         ("shear512", lambda: WL.shear_eb(512), 3101, 3102, 2)]


def main():
    out = {}
    for name, make, data_seed, sim_seed, nsim in CASES:
        wl = make()
        t = time.time()
        d = O.simulate(WL.white_draws(wl.n, wl.ncomp, 1, data_seed)[0], O.prior_S(wl.pshape, wl.band, wl.theta_true),
                       wl.W)
        draws = O.philox.draws_for_sims(sim_seed, range(nsim), wl.n, wl.ncomp)
        th, E, b, F = O.bandpower_qe(d, wl.W, wl.pshape, wl.band, wl.theta_fid, wl.nbands, draws, tol=TOL)
        out[name] = dict(workload=wl.name, n=wl.n, ncomp=wl.ncomp, nbands=wl.nbands, data_seed=data_seed,
                         data="oracle simulate of white_draws(n, ncomp, 1, data_seed) at theta_true",
                         sim_seed=sim_seed, nsim=nsim, sims="Philox4x32-10 key sim_seed, simulations 0 .. nsim-1",
                         rel_grad_tol=TOL, theta_hat=th.tolist(), E=E.tolist(), b=b.tolist(), F=F.tolist(),
                         seconds=round(time.time() - t, 1))
        print(name, out[name]["seconds"], "s", flush=True)
    with open(os.path.join(HERE, "bandpowers_full.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
