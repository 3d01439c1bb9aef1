"""Shared helpers of the GPU parity tests: problems built from the seeded workloads,
host copies, error measures.  Inputs come from paper_1810_00503_amd.workloads and, where
a data map is needed, from the oracle's simulation; nothing here comes from the HIP path."""
import numpy as np

import oracle as O
from paper_1810_00503_amd import workloads as WL


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def make_problem(wf, torch, wl, dtype="f32", theta=None, d=None):
    td = torch.float32 if dtype == "f32" else torch.float64
    dev = "cuda:0"
    th = wl.theta_fid if theta is None else theta
    return wf.Problem(torch.tensor(wl.W, dtype=td, device=dev), wl.pshape, wl.band, th,
                      d=None if d is None else torch.tensor(d, dtype=td, device=dev))


def oracle_data(wl, seed, theta=None):
    """A data map simulated by the oracle from the workload's truth (or `theta`)."""
    draws = WL.white_draws(wl.n, wl.ncomp, 1, seed)
    S_true = O.prior_S(wl.pshape, wl.band, wl.theta_true if theta is None else theta)
    return O.simulate(draws[0], S_true, wl.W)


def random_half(rng, ncomp, n, free_only=True):
    h = n // 2
    s = rng.standard_normal((ncomp, n, h + 1)) + 1j * rng.standard_normal((ncomp, n, h + 1))
    if free_only:
        s = np.where(O.free_mask(n)[None], s, 0)
    return s


def fill_partners(s):
    n = s.shape[1]
    out = s.copy()
    out[:, n // 2 + 1:, 0] = np.conj(s[:, 1:n // 2, 0][:, ::-1])
    return out
