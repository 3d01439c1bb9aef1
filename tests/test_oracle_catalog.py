"""Pins of the oracle's catalog-level response (sec. 3.4: the field evaluated at each galaxy's
own position instead of binned maps): it reduces to R at pixel positions, is periodic, has a
closed form for a single Fourier mode (spin-0 and spin-2), its adjoint passes the dot-product
test, the objective's gradient is exact by central differences, the MAP equals the dense
Wiener filter of the catalog, and one galaxy per pixel centre reproduces the map solve."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1810_00503_amd import workloads as WL
from tests.gpu_util import fill_partners


def _rand_field(rng, S):
    fr = O.free_mask(S.shape[1])[None] & (S > 0)
    z = rng.standard_normal(S.shape) + 1j * rng.standard_normal(S.shape)
    return fill_partners(np.where(fr, np.sqrt(S) * z, 0))


@pytest.mark.parametrize("ncomp", [1, 2])
def test_integer_positions_reduce_to_the_map_response(ncomp):
    n = 12
    rng = np.random.default_rng(1)
    s = fill_partners(np.where(O.free_mask(n)[None], rng.standard_normal((ncomp, n, n // 2 + 1))
                                  + 1j * rng.standard_normal((ncomp, n, n // 2 + 1)), 0))
    yy, xx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    pos = np.stack([yy.ravel(), xx.ravel()], 1).astype(np.float64)
    g = O.catalog_forward(s, pos)
    np.testing.assert_allclose(g, O.forward(s).reshape(ncomp, -1), atol=1e-12 * np.abs(g).max())
    # periodic in both coordinates
    rp = rng.uniform(0, n, (50, 2))
    np.testing.assert_allclose(O.catalog_forward(s, rp + np.array([n, -2 * n])), O.catalog_forward(s, rp),
                               atol=1e-10 * np.abs(g).max())


def test_single_mode_closed_form():
    """One free mode k0 with coefficient c: gamma(r) = (2/n) Re(c exp(2 pi i k0.r / n)) for
    spin-0; for spin-2 E alone, (gamma1, gamma2) = (cos 2a, sin 2a) times that, a = atan2(ky, kx)."""
    n = 16
    rng = np.random.default_rng(2)
    pos = rng.uniform(0, n, (40, 2))
    ky, kx = 3, 2
    c = 0.7 - 0.4j
    s = np.zeros((1, n, n // 2 + 1), np.complex128)
    s[0, ky, kx] = c
    ph = 2 * math.pi * (ky * pos[:, 0] + kx * pos[:, 1]) / n
    expect = 2.0 / n * (c * np.exp(1j * ph)).real
    np.testing.assert_allclose(O.catalog_forward(s, pos)[0], expect, atol=1e-13)
    s2 = np.zeros((2, n, n // 2 + 1), np.complex128)
    s2[0, ky, kx] = c
    a = math.atan2(ky, kx)
    g = O.catalog_forward(s2, pos)
    np.testing.assert_allclose(g[0], math.cos(2 * a) * expect, atol=1e-13)
    np.testing.assert_allclose(g[1], math.sin(2 * a) * expect, atol=1e-13)


@pytest.mark.parametrize("ncomp", [1, 2])
def test_catalog_adjoint_dot_product(ncomp):
    n = 12
    rng = np.random.default_rng(3)
    pos = rng.uniform(0, n, (300, 2))
    s = fill_partners(np.where(O.free_mask(n)[None], rng.standard_normal((ncomp, n, n // 2 + 1))
                                  + 1j * rng.standard_normal((ncomp, n, n // 2 + 1)), 0))
    r = rng.standard_normal((ncomp, 300))
    lhs = float(np.sum(O.catalog_forward(s, pos) * r))
    rhs = O.inner_half(s, O.catalog_adjoint(r, pos, n))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def _catalog_problem(n, seed, nbpc=2, per_pixel=2.0):
    cat = WL.shear_catalog(n, seed, ngal_mean=per_pixel, target_mask=0.2, nbands_e=nbpc, nbands_b=nbpc, b_ratio=0.2)
    S = O.prior_S(cat.pshape, cat.band, cat.theta_fid)
    zs, zn = WL.catalog_draws(n, 2, cat.ngal, seed + 1)
    e = O.catalog_simulate(zs, zn, O.prior_S(cat.pshape, cat.band, cat.theta_true), cat.wgt, cat.pos)
    return cat, S, e


def test_catalog_gradient_central_differences():
    n = 12
    cat, S, e = _catalog_problem(n, 11)
    rng = np.random.default_rng(4)
    fr = O.free_mask(n)[None] & (S > 0)
    w = np.where(fr, rng.standard_normal(S.shape) + 1j * rng.standard_normal(S.shape), 0)
    g = O.catalog_whitened_grad(w, e, cat.wgt, cat.pos, S)
    sq = np.sqrt(S)
    for _ in range(3):
        v = np.where(fr, rng.standard_normal(S.shape) + 1j * rng.standard_normal(S.shape), 0)
        h = 0.3
        cp = O.catalog_chi2(fill_partners(np.where(fr, sq * (w + h * v), 0)), e, cat.wgt, cat.pos, S)
        cm = O.catalog_chi2(fill_partners(np.where(fr, sq * (w - h * v), 0)), e, cat.wgt, cat.pos, S)
        # chi^2 = 2 |w|^2_free + data term in the whitened variable, whose gradient (per real
        # coordinate) is 4 Re(conj(g) v): exact for a quadratic
        fd = (cp - cm) / (2 * h)
        an = 4.0 * float(np.sum((np.conj(g) * v).real))
        assert abs(fd - an) <= 1e-9 * abs(an)
    # the curvature is the gradient difference
    v = np.where(fr, rng.standard_normal(S.shape) + 1j * rng.standard_normal(S.shape), 0)
    Dv = O.catalog_whitened_hvp(v, cat.wgt, cat.pos, S)
    np.testing.assert_allclose(Dv, O.catalog_whitened_grad(w + v, e, cat.wgt, cat.pos, S) - g, atol=1e-10)


def test_catalog_map_equals_dense_wiener_filter():
    n = 8
    cat, S, e = _catalog_problem(n, 21)
    sol = O.catalog_lbfgs_solve(e, cat.wgt, cat.pos, S, tol=1e-12)
    wf = O.catalog_wiener_dense(e, cat.wgt, cat.pos, S)
    assert sol["status"] == 0
    assert np.linalg.norm(sol["s"] - wf["s"]) <= 1e-9 * np.linalg.norm(wf["s"])
    assert abs(sol["chi2"] - wf["chi2_min"]) <= 1e-9 * wf["chi2_min"]


def test_one_galaxy_per_pixel_centre_is_the_map_solve():
    n = 12
    rng = np.random.default_rng(5)
    wl = WL.shear_workload(n, 33, nbands_e=2, nbands_b=2, b_ratio=0.2)
    S = O.prior_S(wl.pshape, wl.band, wl.theta_fid)
    d = O.simulate(WL.white_draws(n, 2, 1, 34)[0], O.prior_S(wl.pshape, wl.band, wl.theta_true), wl.W)
    iy, ix = np.nonzero(wl.W > 0)
    pos = np.stack([iy, ix], 1).astype(np.float64)
    e = d[:, iy, ix]
    grid = O.lbfgs_solve(d, wl.W, S, tol=1e-12)
    cat = O.catalog_lbfgs_solve(e, wl.W[iy, ix], pos, S, tol=1e-12)
    assert np.linalg.norm(cat["s"] - grid["s"]) <= 1e-9 * np.linalg.norm(grid["s"])
    assert abs(cat["chi2"] - grid["chi2"]) <= 1e-9 * grid["chi2"]
    del rng
