"""Pins of the oracle's B-mode leakage-bias estimate (appendix C): without a mask and with
homogeneous noise E and B decouple, so the bias is the closed-form noise bias of the B bands
and F_BB the closed-form Fisher block; with a mask E power leaks into B and the bias exceeds
the noise-only one; the estimate is unbiased over data realisations (fixed seeds)."""
import math

import numpy as np

import oracle as O
from paper_1810_00503_amd import workloads as WL


def _shear(n, seed, masked, sigma2=0.3):
    rng = np.random.default_rng(seed)
    pshape = WL.shear_pshape(n, b_ratio=0.2)
    band = np.stack([WL.log_band_map(n, 2)] * 2).astype(np.int32)
    band[1] = np.where(band[1] >= 0, band[1] + 2, -1)
    W = np.full((n, n), 1.0 / sigma2)
    if masked:
        W = np.where(WL.circle_holes(n, rng, 3, n / 6, n / 4), W, 0.0)
    return pshape, band, 4, W, np.ones(4)


def test_unmasked_leakage_bias_is_the_noise_only_mean():
    n, sigma2 = 16, 0.3
    pshape, band, nb, W, theta = _shear(n, 1, False, sigma2)
    draws = WL.white_draws(n, 2, 40, 11)
    d = O.simulate(WL.white_draws(n, 2, 1, 12)[0], O.prior_S(pshape, band, theta), W)
    th, EB, bB, FBB = O.bmode_leakage_qe(d, W, pshape, band, theta, nb, draws, [2, 3], tol=1e-10)
    # the simulations carry no B power: <E_B> is the closed-form mean at Theta_B = 0
    th0 = theta.copy()
    th0[[2, 3]] = 0.0
    bc, _, Fc = O.homogeneous_band_moments(pshape, band, theta, th0, nb, sigma2)
    # the statistic of one band sums ~N_l squared normals: relative spread sqrt(2 / N_l) per sim
    S = O.prior_S(pshape, band, theta)
    fr = O.free_mask(n)[None] & (S > 0)
    for j, l in enumerate([2, 3]):
        N = 2 * int(np.sum(fr & (band == l)))
        assert abs(bB[j] - bc[l]) < 5.0 * bc[l] * math.sqrt(2.0 / N / len(draws)), (l, bB[j], bc[l])
        assert abs(FBB[j, j] - Fc[l, l]) < 0.3 * Fc[l, l]


def test_masked_leakage_exceeds_noise_only_bias():
    """Same draws with and without E power (paired): with a mask the E power raises E_B."""
    n = 16
    pshape, band, nb, W, theta = _shear(n, 2, True, sigma2=0.05)
    draws = WL.white_draws(n, 2, 30, 21)
    d = O.simulate(WL.white_draws(n, 2, 1, 22)[0], O.prior_S(pshape, band, theta), W)
    _, _, bB, _ = O.bmode_leakage_qe(d, W, pshape, band, theta, nb, draws, [2, 3], tol=1e-10)
    S = O.prior_S(pshape, band, theta)
    th_leak = theta.copy()
    th_leak[[2, 3]] = 0.0
    S_leak = O.prior_S(pshape, band, th_leak)
    S0 = O.prior_S(pshape, band, np.zeros(nb))

    def EB(Ssim, dr):
        return O.band_E(O.lbfgs_solve(O.simulate(dr, Ssim, W), W, S, tol=1e-10)["s"], S, band, theta, nb)[[2, 3]]

    El = np.array([EB(S_leak, dr) for dr in draws])
    En = np.array([EB(S0, dr) for dr in draws])
    np.testing.assert_allclose(bB, El.mean(0), rtol=1e-10)   # the bias is the mean of these simulations
    diff = El - En
    z = diff.mean(0) / (diff.std(0) / math.sqrt(len(draws)))
    assert z[0] > 4.0, (diff.mean(0), z)


def test_leakage_estimate_is_unbiased():
    """b_B and F_BB from one set of simulations; Theta_hat_B = F_BB^-1 (E_B(d) - b_B) over
    data realisations drawn at the fiducial amplitudes averages to Theta_B."""
    n = 16
    pshape, band, nb, W, theta = _shear(n, 3, True)
    S = O.prior_S(pshape, band, theta)
    draws = WL.white_draws(n, 2, 60, 31)
    d0 = O.simulate(WL.white_draws(n, 2, 1, 32)[0], S, W)
    _, _, bB, FBB = O.bmode_leakage_qe(d0, W, pshape, band, theta, nb, draws, [2, 3], tol=1e-10)
    est = []
    for dr in WL.white_draws(n, 2, 120, 33):
        d = O.simulate(dr, S, W)
        E = O.band_E(O.lbfgs_solve(d, W, S, tol=1e-10)["s"], S, band, theta, nb)
        est.append(np.linalg.solve(FBB, E[[2, 3]] - bB))
    est = np.array(est)
    sd = est.std(0) / math.sqrt(len(est))
    # b_B and F_BB carry their own simulation noise: allow it beside the realisations' spread
    assert np.all(np.abs(est.mean(0) - theta[[2, 3]]) < 4.0 * sd + 0.15), (est.mean(0), sd)
