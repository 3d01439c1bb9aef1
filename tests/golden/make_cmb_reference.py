"""Writes the oracle's MAP of the 1024^2 flat-sky CMB workload (tests/golden/cmb1024_map.npy,
complex64 [1][1024][513], and cmb1024_map.json with how it was made).

Calls only the oracle and the seeded input generators: the data map is the oracle's
simulation of the CMB patch workload from its truth (white normals of seed DATA_SEED), solved
with the oracle's preconditioned L-BFGS to a relative whitened gradient of TOL.  The GPU
tests regenerate the same data map and compare their fields with this one.

    python tests/golden/make_cmb_reference.py        # about 15 minutes on one core
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

N = 1024
DATA_SEED = 4101
TOL = 1e-11


def main():
    wl = WL.cmb_patch(N)
    draws = WL.white_draws(N, 1, 1, DATA_SEED)
    d = O.simulate(draws[0], O.prior_S(wl.pshape, wl.band, wl.theta_true), wl.W)
    S = O.prior_S(wl.pshape, wl.band, wl.theta_fid)
    t = time.time()
    r = O.lbfgs_solve(d, wl.W, S, tol=TOL, precond=True, max_iter=20000)
    el = time.time() - t
    assert r["status"] == 0, r["status"]
    np.save(os.path.join(HERE, "cmb1024_map.npy"), r["s"].astype(np.complex64))
    meta = dict(workload="cmb_patch(1024)", data="oracle simulate of white_draws(1024, 1, 1, %d) at theta_true"
                % DATA_SEED, prior="theta_fid", solver="oracle lbfgs_solve, precond=True, m=10",
                rel_grad_tol=TOL, rel_grad=r["rel_grad"], iters=r["iters"], chi2=r["chi2"], seconds=round(el, 1),
                stored="complex64 field [1][1024][513] (partners filled)")
    with open(os.path.join(HERE, "cmb1024_map.json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps(meta))


if __name__ == "__main__":
    main()
