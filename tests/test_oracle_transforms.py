"""Pins of the oracle's response operator R, its adjoint, chi^2, gradient and curvature.

Each check compares against something other than the oracle itself: a brute-force
DFT written out term by term, analytic derivatives of a plane wave (appendix C's
differential operator), the exactness of central differences on a quadratic, and
the identities an isometry must satisfy."""
import cmath
import math

import numpy as np
import pytest

import oracle as O


def _rand_half(rng, ncomp, n):
    h = n // 2
    s = rng.standard_normal((ncomp, n, h + 1)) + 1j * rng.standard_normal((ncomp, n, h + 1))
    return np.where(O.free_mask(n)[None], s, 0)


def _fill(s):
    n = s.shape[1]
    out = s.copy()
    for iy in range(n // 2 + 1, n):
        out[:, iy, 0] = np.conj(s[:, n - iy, 0])
    return out


@pytest.mark.parametrize("n", [4, 6, 8])
def test_forward_is_bruteforce_inverse_dft(n):
    """x_j = n^-1 sum over the full plane of s_k e^{+2 pi i k.j/n}; each free entry and its
    conjugate mirror contribute 2 Re(s_k e^{i theta})."""
    rng = np.random.default_rng(n)
    s = _rand_half(rng, 1, n)
    fr = O.free_mask(n)
    x = O.forward(s)[0]
    ref = np.zeros((n, n))
    for iy in range(n):
        ky = iy if iy < n // 2 else iy - n
        for kx in range(n // 2 + 1):
            if not fr[iy, kx]:
                continue
            for y in range(n):
                for xx in range(n):
                    th = 2 * math.pi * (kx * xx + ky * y) / n
                    ref[y, xx] += 2.0 * (s[0, iy, kx] * cmath.exp(1j * th)).real / n
    np.testing.assert_allclose(x, ref, atol=1e-12)


@pytest.mark.parametrize("n", [4, 6, 8])
def test_adjoint_is_bruteforce_forward_dft(n):
    rng = np.random.default_rng(10 + n)
    x = rng.standard_normal((1, n, n))
    t = O.adjoint(x)[0]
    live = O.live_mask(n)
    for iy in range(n):
        ky = iy if iy < n // 2 else iy - n
        for kx in range(n // 2 + 1):
            v = 0j
            for y in range(n):
                for xx in range(n):
                    v += x[0, y, xx] * cmath.exp(-2j * math.pi * (kx * xx + ky * y) / n)
            v /= n
            assert abs(t[iy, kx] - (v if live[iy, kx] else 0)) < 1e-12


@pytest.mark.parametrize("ncomp", [1, 2])
@pytest.mark.parametrize("n", [8, 12, 32])
def test_adjoint_dot_product_and_parseval(n, ncomp):
    """<R s, x> = <s, R^T x> in the full-plane metric; |R s| = |s| (R is an isometry)."""
    rng = np.random.default_rng(100 * n + ncomp)
    s = _fill(_rand_half(rng, ncomp, n))
    x = rng.standard_normal((ncomp, n, n))
    lhs = float(np.sum(O.forward(s) * x))
    rhs = O.inner_half(s, O.adjoint(x))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)
    Rs = O.forward(s)
    assert abs(np.sum(Rs * Rs) - O.inner_half(s, s)) <= 1e-12 * np.sum(Rs * Rs)


@pytest.mark.parametrize("n", [16, 24])
def test_spin2_matches_plane_wave_derivatives(n):
    """Appendix C: g1 = (dx^2 - dy^2) phi_E - 2 dx dy phi_B, g2 = 2 dx dy phi_E + (dx^2 - dy^2) phi_B.
    For phi = cos(2 pi (a x + b y)/n) the derivatives are analytic; the convergence
    kappa = lap(phi) = -|k|^2 phi has unitary coefficient -|k|^2 n/2 at (b, a)."""
    h = n // 2
    for (a, b) in [(1, 2), (3, -1), (0, 2), (2, 0), (h - 1, -(h - 1))]:
        kp = 2 * math.pi / n
        kx, ky = a * kp, b * kp
        yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
        c = np.cos(kx * xx + ky * yy)
        for comp in (0, 1):
            s = np.zeros((2, n, h + 1), np.complex128)
            iy = b % n
            coef = -(kx * kx + ky * ky) * n / 2.0
            if a == 0 and iy > h:
                s[comp, n - iy, 0] = coef      # store the free entry of the pair
            else:
                s[comp, iy, a] = coef
            g = O.forward(s)
            dxx, dyy, dxy = -kx * kx * c, -ky * ky * c, -kx * ky * c
            if comp == 0:
                exp1, exp2 = dxx - dyy, 2 * dxy
            else:
                exp1, exp2 = -2 * dxy, dxx - dyy
            np.testing.assert_allclose(g[0], exp1, atol=1e-10)
            np.testing.assert_allclose(g[1], exp2, atol=1e-10)


def _problem(rng, n, ncomp, masked=True):
    pshape = np.stack([1.0 / (1.0 + O.signed_k(n)[0] ** 2 + O.signed_k(n)[1] ** 2)] * ncomp)
    pshape = pshape * (1.0 if ncomp == 1 else np.array([1.0, 0.3])[:, None, None])
    band = np.zeros(pshape.shape, np.int32)
    S = O.prior_S(pshape, band, [0.7])
    W = rng.uniform(0.5, 3.0, (n, n))
    if masked:
        W[rng.uniform(size=(n, n)) < 0.25] = 0.0
    d = rng.standard_normal((ncomp, n, n))
    return S, W, d


@pytest.mark.parametrize("ncomp", [1, 2])
def test_gradient_equals_central_differences(ncomp):
    """chi^2 is quadratic, so the central difference is exact for any step; the
    gradient convention is d/dRe + i d/dIm per stored coefficient."""
    n = 8
    rng = np.random.default_rng(7 + ncomp)
    S, W, d = _problem(rng, n, ncomp)
    fr = O.free_mask(n)[None] & (S > 0)
    s = np.where(fr, rng.standard_normal(S.shape) + 1j * rng.standard_normal(S.shape), 0)
    g = O.grad_chi2(s, d, W, S)
    for _ in range(6):
        e = np.where(fr, rng.standard_normal(S.shape) + 1j * rng.standard_normal(S.shape), 0)
        hstep = 0.37
        fd = (O.chi2(s + hstep * e, d, W, S) - O.chi2(s - hstep * e, d, W, S)) / (2 * hstep)
        an = float(np.sum((np.conj(g) * e).real))
        assert abs(fd - an) <= 1e-9 * (abs(fd) + 1)
    # every single coordinate as well (exhaustive at 8^2)
    iy, kx = np.nonzero(fr[0])
    for j in range(0, iy.size, 5):
        for part in (1.0, 1j):
            e = np.zeros(S.shape, np.complex128)
            e[0, iy[j], kx[j]] = part
            fd = (O.chi2(s + e, d, W, S) - O.chi2(s - e, d, W, S)) / 2.0
            an = float((np.conj(g[0, iy[j], kx[j]]) * part).real)
            assert abs(fd - an) <= 1e-9 * (abs(fd) + 1)


@pytest.mark.parametrize("ncomp", [1, 2])
def test_whitened_curvature_is_gradient_difference(ncomp):
    n = 12
    rng = np.random.default_rng(21 + ncomp)
    S, W, d = _problem(rng, n, ncomp)
    fr = O.free_mask(n)[None] & (S > 0)
    w = np.where(fr, rng.standard_normal(S.shape) + 1j * rng.standard_normal(S.shape), 0)
    p = np.where(fr, rng.standard_normal(S.shape) + 1j * rng.standard_normal(S.shape), 0)
    lhs = O.whitened_hvp(p, W, S)
    rhs = O.whitened_grad(w + p, d, W, S) - O.whitened_grad(w, d, W, S)
    np.testing.assert_allclose(lhs, rhs, atol=1e-11)
    # the whitened gradient is the raw gradient / 4 times S^1/2 (chain rule)
    s = np.sqrt(S) * w
    g_raw = O.grad_chi2(s, d, W, S)
    np.testing.assert_allclose(O.whitened_grad(w, d, W, S), np.where(fr, np.sqrt(S) * g_raw / 4.0, 0), atol=1e-11)
