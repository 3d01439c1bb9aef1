"""Pins of the oracle's posterior-error estimate (the residual covariance S - S R^dag C^-1 R S
of the Wiener filter, appendix A after eq. eq:wiener): the dense diagonal against the
closed form of unmasked homogeneous noise, and the simulation estimate against the dense
diagonal within Monte Carlo error (fixed seeds, so deterministic)."""
import math

import numpy as np

import oracle as O
from paper_1810_00503_amd import workloads as WL


def _setup(n, seed, masked):
    rng = np.random.default_rng(seed)
    pshape = WL.density_pshape(n, kd=n / 3.0)
    band = WL.log_band_map(n, 2)[None].astype(np.int32)
    theta = np.array([0.7, 1.2])
    W = rng.uniform(1.0, 4.0, (n, n))
    if masked:
        W = np.where(WL.circle_holes(n, rng, 2, n / 8, n / 5), W, 0.0)
    return pshape, band, theta, W


def test_dense_posterior_variance_homogeneous_closed_form():
    """Unmasked white noise sigma^2: each free coefficient has posterior variance
    S sigma^2 / (S + sigma^2), and every pixel (2 / n^2) times their sum (each free entry
    stands for the modes k and -k)."""
    n, sigma2 = 12, 0.4
    pshape, band, theta, _ = _setup(n, 1, False)
    W = np.full((n, n), 1.0 / sigma2)
    S = O.prior_S(pshape, band, theta)
    vm, vp = O.dense_posterior_variance(W, S)
    fr = O.free_mask(n)[None] & (S > 0)
    want = np.where(fr, S * sigma2 / (S + sigma2), 0.0)
    for ky in range(n // 2 + 1, n):   # the kx = 0 conjugate partners mirror their free entries
        want[:, ky, 0] = want[:, n - ky, 0]
    np.testing.assert_allclose(vm, want, rtol=1e-10, atol=1e-14)
    pix = 2.0 * np.sum(np.where(fr, S * sigma2 / (S + sigma2), 0.0)) / n ** 2
    np.testing.assert_allclose(vp, np.full((1, n, n), pix), rtol=1e-10)


def test_sim_signal_has_the_prior_variance():
    n = 8
    pshape, band, theta, _ = _setup(n, 2, False)
    S = O.prior_S(pshape, band, theta)
    draws = WL.white_draws(n, 1, 4000, 3)
    acc = np.zeros(S.shape)
    for dr in draws:
        acc += np.abs(O.sim_signal(dr, S)) ** 2
    acc /= len(draws)
    live = S > 0
    live[:, n // 2, :] = False
    z = np.abs(acc[live] - S[live]) / (S[live] / math.sqrt(len(draws)))
    assert z.max() < 5.0, z.max()
    assert np.all(acc[~live] == 0)


def test_posterior_error_simulations_match_dense_diagonal():
    n, nsim = 12, 150
    pshape, band, theta, W = _setup(n, 4, True)
    S = O.prior_S(pshape, band, theta)
    draws = WL.white_draws(n, 1, nsim, 5)
    vm, vp = O.posterior_error(W, pshape, band, theta, draws)
    dm, dp = O.dense_posterior_variance(W, S)
    on = dm > 0
    zm = np.abs(vm[on] - dm[on]) / (dm[on] * math.sqrt(2.0 / nsim))
    zp = np.abs(vp - dp) / (dp * math.sqrt(2.0 / nsim))
    assert zm.max() < 5.5 and zp.max() < 5.5, (zm.max(), zp.max())
    assert np.all(vm[~on] == 0)
    # band-summed and map-summed: Monte Carlo errors average down
    assert abs(vm.sum() / dm.sum() - 1.0) < 3.0 / math.sqrt(nsim)
    assert abs(vp.sum() / dp.sum() - 1.0) < 3.0 / math.sqrt(nsim)


def test_band_power_single_entries():
    """Brute force on fields with one nonzero stored entry: a free entry with S > 0 adds
    |v|^2 to its band only; a partner, a dead entry or an entry with S = 0 adds nothing."""
    n = 8
    pshape, band, theta, _ = _setup(n, 6, False)
    S = O.prior_S(pshape, band, theta)
    cases = [((0, 1, 2), True), ((0, 3, 0), True), ((0, 6, 0), False), ((0, 4, 1), False), ((0, 0, 0), False),
             ((0, 2, 4), False)]
    for (c, ky, kx), counts in cases:
        s = np.zeros(S.shape, np.complex128)
        s[c, ky, kx] = 3.0 - 4.0j
        got = O.band_power(s, S, band, 2)
        want = np.zeros(2)
        if counts and S[c, ky, kx] > 0 and band[c, ky, kx] >= 0:
            want[band[c, ky, kx]] = 25.0
        np.testing.assert_array_equal(got, want, err_msg=str((ky, kx)))


def test_cosmic_variance_counts_modes():
    n = 12
    pshape, band, theta, _ = _setup(n, 7, False)
    S = O.prior_S(pshape, band, theta)
    cv = O.cosmic_variance(S, band, 2)
    for l in range(2):
        N = 0
        for ky in range(n):
            for kx in range(n // 2 + 1):
                free = (kx > 0 and kx < n // 2 and ky != n // 2) or (kx == 0 and 0 < ky < n // 2)
                N += 2 * int(free and S[0, ky, kx] > 0 and band[0, ky, kx] == l)
        assert cv[l] == math.sqrt(2.0 / N)
