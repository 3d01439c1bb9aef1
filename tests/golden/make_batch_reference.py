"""Writes the oracle's band-power estimates of three maps of the 96-map uneven batch at full size
(a 128^2 CMB map, a 256^2 density map and a 512^2 shear map, its maps MAPS), which the library
estimates together in shared batched solves (tests/golden/batch_full.json).

Calls only the oracle and the seeded input generators.  Map j's data is the oracle's simulation
of its workload from its truth (white normals of seed DATA_SEED0 + j); its simulations are the
Philox4x32-10 stream of key SIM_SEED + j (simulations 0 .. NSIM - 1), as the library's batched
estimate draws them; every solve (preconditioned) runs to a relative gradient of TOL.  Stored:
E, b, F and Theta_hat of each map.

    python tests/golden/make_batch_reference.py        # about three minutes on one core
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_1810_00503_amd import workloads as WL  # noqa: E402

TOL = 1e-10
MAPS = [17, 23, 13]
NSIM = 2
DATA_SEED0 = 6100
SIM_SEED = 6000


def main():
    wls = WL.uneven_batch(96)
    out = dict(maps=MAPS, nsim=NSIM, data_seed0=DATA_SEED0, sim_seed=SIM_SEED, rel_grad_tol=TOL,
               data="oracle simulate of white_draws(n, ncomp, 1, data_seed0 + j) at theta_true",
               sims="Philox4x32-10 key sim_seed + j, simulations 0 .. nsim-1", estimates=[])
    for j, i in enumerate(MAPS):
        wl = wls[i]
        t = time.time()
        d = O.simulate(WL.white_draws(wl.n, wl.ncomp, 1, DATA_SEED0 + j)[0],
                       O.prior_S(wl.pshape, wl.band, wl.theta_true), wl.W)
        draws = O.philox.draws_for_sims(SIM_SEED + j, range(NSIM), wl.n, wl.ncomp)
        th, E, b, F = O.bandpower_qe(d, wl.W, wl.pshape, wl.band, wl.theta_fid, wl.nbands, draws, tol=TOL,
                                     precond=True)
        out["estimates"].append(dict(map=i, workload=wl.name, n=wl.n, ncomp=wl.ncomp, nbands=wl.nbands,
                                     theta_hat=th.tolist(), E=E.tolist(), b=b.tolist(), F=F.tolist(),
                                     seconds=round(time.time() - t, 1)))
        print(wl.name, out["estimates"][-1]["seconds"], "s", flush=True)
    with open(os.path.join(HERE, "batch_full.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
