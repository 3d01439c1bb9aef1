"""Writes the oracle's MAP of one CMB map of the 96-map uneven batch
(tests/golden/uneven_cmb<index>_map.npy, complex64 [1][n][n/2+1], and a .json with how it was made).

Calls only the oracle and the seeded input generators: map <index> of uneven_batch(96) (its mask and
noise), with data the oracle's simulation from the truth of Philox stream (key 5100 + index,
simulation 0), solved with the oracle's preconditioned L-BFGS to a relative whitened gradient of TOL.
The GPU test solves the same data inside the uneven batch and compares its fields with this one.

    python tests/golden/make_uneven_cmb_reference.py 75    # the last 768^2 CMB map, ~15 minutes on one core
    python tests/golden/make_uneven_cmb_reference.py 88    # the last 1024^2 CMB map, ~20 minutes on one core
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

TOL = 1e-11
SEED0 = 5100


def data_of(wl, index):
    """The map's data: the oracle's simulation at the truth from Philox key SEED0 + index, simulation 0."""
    draws = O.philox.draws_for_sims(SEED0 + index, [0], wl.n, wl.ncomp)[0]
    return O.simulate(draws, O.prior_S(wl.pshape, wl.band, wl.theta_true), wl.W)


def main(index):
    wl = WL.uneven_batch(96)[index]
    assert wl.name.startswith("uneven-cmb"), wl.name
    d = data_of(wl, index)
    S = O.prior_S(wl.pshape, wl.band, wl.theta_fid)
    t = time.time()
    r = O.lbfgs_solve(d, wl.W, S, tol=TOL, precond=True, max_iter=40000)
    el = time.time() - t
    assert r["status"] == 0, r["status"]
    np.save(os.path.join(HERE, f"uneven_cmb{index}_map.npy"), r["s"].astype(np.complex64))
    meta = dict(workload=f"uneven_batch(96)[{index}] ({wl.name})",
                data=f"oracle simulate of philox draws_for_sims({SEED0 + index}, [0]) at theta_true",
                prior="theta_fid", solver="oracle lbfgs_solve, precond=True, m=10", rel_grad_tol=TOL,
                rel_grad=r["rel_grad"], iters=r["iters"], chi2=r["chi2"], seconds=round(el, 1),
                stored=f"complex64 field [1][{wl.n}][{wl.n // 2 + 1}] (partners filled)")
    with open(os.path.join(HERE, f"uneven_cmb{index}_map.json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps(meta))


if __name__ == "__main__":
    main(int(sys.argv[1]))
