"""Pins of the oracle's MAP solve, band powers and simulation estimates.

The MAP solution is pinned to the dense Wiener filter (appendix A), to the diagonal
closed form of the unmasked homogeneous case, to the noiseless limit and to the
optimality conditions; the band-power pieces to their closed forms, to finite
differences in Theta, to the dense traces and (statistically, with fixed seeds) to
their expectations."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1810_00503_amd import workloads as WL


def _small(n, ncomp, seed, masked=True, nb=3):
    rng = np.random.default_rng(seed)
    if ncomp == 1:
        pshape = WL.density_pshape(n, kd=n / 3.0)
    else:
        pshape = WL.shear_pshape(n, b_ratio=0.2)
    band = np.stack([WL.log_band_map(n, nb)] * ncomp).astype(np.int32)
    if ncomp == 2:
        band[1] = np.where(band[1] >= 0, band[1] + nb, -1)
    nbt = nb * ncomp
    W = rng.uniform(2.0, 8.0, (n, n))
    if masked:
        W = np.where(WL.circle_holes(n, rng, 2, n / 8, n / 5), W, 0.0)
    theta = rng.uniform(0.3, 1.0, nbt)
    return pshape, band, nbt, W, theta


@pytest.mark.parametrize("ncomp,n", [(1, 12), (1, 16), (2, 12)])
def test_map_equals_dense_wiener_filter(ncomp, n):
    pshape, band, nb, W, theta = _small(n, ncomp, 5 + n + ncomp)
    S = O.prior_S(pshape, band, theta)
    rng = np.random.default_rng(99)
    d = np.where(W[None] > 0, rng.standard_normal((ncomp, n, n)), 0.0)
    sol = O.lbfgs_solve(d, W, S, m=10, tol=1e-12)
    wf = O.wiener_dense(d, W, S)
    err = np.linalg.norm(sol["s"] - wf["s"]) / np.linalg.norm(wf["s"])
    assert err < 1e-9, err
    # chi^2 at the optimum equals d^T C^-1 d
    assert abs(sol["chi2"] - wf["chi2_min"]) <= 1e-9 * wf["chi2_min"]
    # the gradient vanishes at the dense solution
    g = O.grad_chi2(wf["s"], d, W, S)
    g0 = O.grad_chi2(np.zeros_like(wf["s"]), d, W, S)
    assert np.linalg.norm(g) <= 1e-9 * np.linalg.norm(g0)


def test_density64_map_vs_dense_wiener_filter():
    """64^2 density case (m = 10, tol 1e-8) against the 4096 x 4096 direct inversion."""
    wl = WL.density64()
    S = O.prior_S(wl.pshape, wl.band, wl.theta_fid)
    draws = WL.white_draws(wl.n, 1, 1, wl.seed)
    d = O.simulate(draws[0], O.prior_S(wl.pshape, wl.band, wl.theta_true), wl.W)
    sol = O.lbfgs_solve(d, wl.W, S, m=10, tol=1e-8)
    wf = O.wiener_dense(d, wl.W, S)
    xs, xw = O.forward(sol["s"]), O.forward(wf["s"])
    err = np.linalg.norm(xs - xw) / np.linalg.norm(xw)
    assert err < 1e-6, err
    obs = wl.W > 0
    assert np.max(np.abs(xs - xw)[0][obs]) < 1e-4 * np.max(np.abs(xw))


@pytest.mark.parametrize("n", [16, 24])
def test_homogeneous_unmasked_closed_form(n):
    pshape, band, nb, _, theta = _small(n, 1, 3 + n, masked=False)
    S = O.prior_S(pshape, band, theta)
    sigma2 = 0.3
    W = np.full((n, n), 1.0 / sigma2)
    d = np.random.default_rng(n).standard_normal((1, n, n))
    sol = O.lbfgs_solve(d, W, S, tol=1e-12)
    # closed form written out per mode from the unitary DFT of d (numpy's FFT)
    t = np.fft.rfft2(d[0], norm="ortho")
    expect = np.where(S[0] > 0, S[0] / (S[0] + sigma2) * t, 0)
    live = O.live_mask(n)
    np.testing.assert_allclose(sol["s"][0][live], expect[live], atol=1e-10)


def test_noiseless_unmasked_returns_data():
    n = 16
    pshape, band, nb, _, theta = _small(n, 1, 44, masked=False)
    S = O.prior_S(pshape, band, theta)
    d = np.random.default_rng(4).standard_normal((1, n, n))
    W = np.full((n, n), 1e10)
    sol = O.lbfgs_solve(d, W, S, tol=1e-13, max_iter=5000)
    # the reconstruction is d with its dead modes (DC, Nyquist lines) removed
    dl = d[0] - np.mean(d[0])
    t = np.fft.fft2(dl)
    t[n // 2, :] = 0
    t[:, n // 2] = 0
    proj = np.fft.ifft2(t).real
    np.testing.assert_allclose(O.forward(sol["s"])[0], proj, atol=1e-6)


def test_linearity_of_map():
    n = 12
    pshape, band, nb, W, theta = _small(n, 2, 8)
    S = O.prior_S(pshape, band, theta)
    rng = np.random.default_rng(2)
    d1 = rng.standard_normal((2, n, n))
    d2 = rng.standard_normal((2, n, n))
    s1 = O.lbfgs_solve(d1, W, S, tol=1e-12)["s"]
    s2 = O.lbfgs_solve(d2, W, S, tol=1e-12)["s"]
    s12 = O.lbfgs_solve(d1 + 2.5 * d2, W, S, tol=1e-12)["s"]
    np.testing.assert_allclose(s12, s1 + 2.5 * s2, atol=1e-9 * np.abs(s12).max())


@pytest.mark.parametrize("ncomp", [1, 2])
def test_band_E_is_minus_half_theta_derivative(ncomp):
    """d chi^2 / d Theta_b = -2 E_b: central differences in Theta (O(h^2))."""
    n = 12
    pshape, band, nb, W, theta = _small(n, ncomp, 31)
    S = O.prior_S(pshape, band, theta)
    rng = np.random.default_rng(5)
    fr = O.free_mask(n)[None] & (S > 0)
    s = np.where(fr, rng.standard_normal(S.shape) + 1j * rng.standard_normal(S.shape), 0)
    d = rng.standard_normal((ncomp, n, n))
    E = O.band_E(s, S, band, theta, nb)
    for b in range(nb):
        hh = 1e-4 * theta[b]
        tp, tm = theta.copy(), theta.copy()
        tp[b] += hh
        tm[b] -= hh
        fd = (O.chi2(s, d, W, O.prior_S(pshape, band, tp)) - O.chi2(s, d, W, O.prior_S(pshape, band, tm))) / (2 * hh)
        assert abs(fd + 2 * E[b]) <= 1e-6 * abs(2 * E[b]) + 1e-9


def test_dense_traces_match_homogeneous_closed_forms():
    n = 12
    pshape, band, nb, _, theta = _small(n, 1, 17, masked=False)
    sigma2 = 0.4
    W = np.full((n, n), 1.0 / sigma2)
    b, F = O.dense_bias_fisher(W, pshape, band, theta, nb)
    _, bc, Fc = O.homogeneous_band_moments(pshape, band, theta, theta, nb, sigma2)
    np.testing.assert_allclose(b, bc, rtol=1e-10)
    np.testing.assert_allclose(F, Fc, rtol=1e-10, atol=1e-12 * np.abs(Fc).max())


def test_philox_known_answers():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    for r in rows:
        v = [int(x, 16) for x in r]
        ctr = np.array([v[0:4]], np.uint32)
        key = np.array(v[4:6], np.uint32)
        out = O.philox4x32_10(ctr, key)[0]
        assert [int(x) for x in out] == v[6:10]


def test_philox_normals_moments():
    z = O.normals_for_sim(12345, 3, 400000)
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * math.sqrt(2 / z.size)
    assert abs(np.mean(z ** 4) - 3) < 0.05


def test_simulation_matches_prior_and_noise_statistics():
    """Pixel variance of an unmasked simulation = n^-2 sum_full S_k + sigma^2."""
    n = 32
    pshape, band, nb, _, theta = _small(n, 1, 3, masked=False)
    S = O.prior_S(pshape, band, theta)
    sigma2 = 0.25
    W = np.full((n, n), 1.0 / sigma2)
    draws = WL.white_draws(n, 1, 200, 77)
    var = np.mean([O.simulate(dr, S, W).var() for dr in draws])
    fr = O.free_mask(n) & (S[0] > 0)
    expect = 2.0 * S[0][fr].sum() / n ** 2 + sigma2
    assert abs(var - expect) < 0.03 * expect


def test_sim_bias_and_fisher_converge_to_closed_forms():
    """Unmasked homogeneous noise: the simulation b and F (eqs. blmv, fisher) approach
    the closed forms at the 1/sqrt(N_sim) rate (fixed seed: deterministic)."""
    n = 16
    pshape, band, nb, _, theta = _small(n, 1, 91, masked=False, nb=2)
    sigma2 = 0.5
    W = np.full((n, n), 1.0 / sigma2)
    draws = WL.white_draws(n, 1, 48, 5)
    b, F, Es = O.sim_fisher(W, pshape, band, theta, nb, draws, tol=1e-10)
    _, bc, Fc = O.homogeneous_band_moments(pshape, band, theta, theta, nb, sigma2)
    sd = Es.std(0) / math.sqrt(len(draws))
    assert np.all(np.abs(b - bc) < 4 * sd + 1e-12)
    assert np.all(np.abs(np.diag(F) - np.diag(Fc)) < 0.25 * np.diag(Fc))


def test_sim_bias_matches_dense_trace_masked():
    n = 12
    pshape, band, nb, W, theta = _small(n, 1, 66, nb=2)
    draws = WL.white_draws(n, 1, 64, 9)
    b, F, Es = O.sim_fisher(W, pshape, band, theta, nb, draws, tol=1e-10)
    bd, Fd = O.dense_bias_fisher(W, pshape, band, theta, nb)
    sd = Es.std(0) / math.sqrt(len(draws))
    assert np.all(np.abs(b - bd) < 4 * sd)
    assert np.all(np.abs(np.diag(F) - np.diag(Fd)) < 0.3 * np.diag(Fd))


def test_bandpower_estimate_unbiased():
    """Theta_hat with the exact (dense) b and F is unbiased over data realisations:
    its mean equals Theta_true within Monte Carlo error (fixed seeds)."""
    n = 12
    pshape, band, nb, W, theta_fid = _small(n, 1, 12, nb=2)
    theta_true = np.ones(nb)
    S_true = O.prior_S(pshape, band, theta_true)
    S_fid = O.prior_S(pshape, band, theta_fid)
    bd, Fd = O.dense_bias_fisher(W, pshape, band, theta_fid, nb)
    draws = WL.white_draws(n, 1, 160, 31)
    est = []
    for dr in draws:
        d = O.simulate(dr, S_true, W)
        E = O.band_E(O.lbfgs_solve(d, W, S_fid, tol=1e-10)["s"], S_fid, band, theta_fid, nb)
        est.append(O.newton_update(theta_fid, Fd, E, bd))
    est = np.array(est)
    sd = est.std(0) / math.sqrt(len(est))
    assert np.all(np.abs(est.mean(0) - theta_true) < 4 * sd), (est.mean(0), sd)


def _pcg_iterates(d, W, S, P, k):
    """The first k iterates of textbook (preconditioned) conjugate gradients (Hestenes and
    Stiefel; Nocedal & Wright, Numerical Optimization, algorithm 5.3) on the whitened normal
    equations D w = S^1/2 R^T W d, from w = 0; P is the diagonal preconditioner or None."""
    fr = O.free_mask(S.shape[1])[None] & (S > 0)
    w = np.zeros(S.shape, np.complex128)
    r = -O.whitened_grad(w, d, W, S)          # b - D w at w = 0
    z = r if P is None else np.where(fr, P, 0) * r
    p = z.copy()
    rz = np.vdot(r, z).real
    out = []
    for _ in range(k):
        Dp = O.whitened_hvp(p, W, S)
        a = rz / np.vdot(p, Dp).real
        w = w + a * p
        r = r - a * Dp
        z = r if P is None else np.where(fr, P, 0) * r
        rz_new = np.vdot(r, z).real
        p = z + (rz_new / rz) * p
        rz = rz_new
        out.append(w.copy())
    return out


@pytest.mark.parametrize("ncomp,m,precond", [(1, 1, False), (1, 10, False), (2, 3, False), (1, 10, True),
                                             (2, 1, True)])
def test_lbfgs_iterates_equal_conjugate_gradients(ncomp, m, precond):
    """On a quadratic with exact line searches, L-BFGS with any history length m >= 1 and
    initial matrix gamma I (or gamma P) takes the same steps as conjugate gradients (with
    preconditioner P): each direction is a multiple of the (preconditioned) CG direction and
    the exact step removes the multiple (Nocedal & Wright, secs. 5.1 and 7.2).  Pins the
    oracle's two-loop recursion, its curvature pairs, its scaling and its preconditioner use,
    none of which change the converged MAP.  Iterate k of the oracle (max_iter = k) is
    compared with iterate k of CG, for k up to 12."""
    n = 12
    pshape, band, nb, W, theta = _small(n, ncomp, 70 + 3 * m + ncomp)
    S = O.prior_S(pshape, band, theta)
    rng = np.random.default_rng(71)
    d = np.where(W[None] > 0, rng.standard_normal((ncomp, n, n)), 0.0)
    P = O.precond_diag(W, S) if precond else None
    cg = _pcg_iterates(d, W, S, P, 12)
    for k in range(1, 13):
        w = O.lbfgs_solve(d, W, S, m=m, tol=0.0, max_iter=k, precond=precond)["w"]
        err = np.linalg.norm(w - cg[k - 1]) / np.linalg.norm(cg[k - 1])
        assert err < 1e-9, (k, err)
