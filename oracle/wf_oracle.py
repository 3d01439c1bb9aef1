"""FP64 CPU oracle of the Wiener-filter-as-MAP hot path (test infrastructure only).

Written from the paper's equations; each function cites the passage it follows.
numpy's FFT is the one library primitive used per transform; numpy.linalg provides
the Cholesky factorisation and small dense solves.  Nothing here is blocked, fused
or reordered beyond what the equations state, so it can be checked by eye.

Conventions the paper leaves open (fixed identically for the HIP library):

* grid n x n (n even), pixel (y, x); signed wavenumbers k = (kx, ky) in [-n/2, n/2);
* unitary DFT: (F x)_k = n^-1 sum_j x_j exp(-2 pi i k.j/n); the response R is
  F^-1 restricted to Hermitian spectra (sec. 2, eq. ddecomp; R is an isometry);
* live modes: k != 0, |kx| < n/2, |ky| < n/2 and prior S_k > 0; everything else is
  dead (not a variable).  Half-plane storage [ncomp][n][n/2+1]; the independent
  ("free") entries are kx in [1, n/2) (every row but ky = -n/2) and kx = 0 with
  ky in [1, n/2); the rows kx = 0, ky in (n/2, n) hold their conjugate partners;
* S_k = Theta_{band(k)} P_k is the variance of the unitary coefficient
  (band -1: amplitude fixed at 1);
* spin-2 (appendix C): with kappa = -k^2 phi absorbed into S, the shear spectra are
  g1 = cos2a E - sin2a B, g2 = sin2a E + cos2a B, a = atan2(ky, kx) (per-mode
  rotation, orthogonal, so R stays an isometry);
* the L-BFGS variable is the whitened field w = S^-1/2 s on the free entries, with
  the Euclidean inner product of their real and imaginary parts; f = chi^2 / 4.

Parity status: every function below is pinned by the not-gpu tests in
tests/test_oracle_*.py: brute-force DFT, plane-wave derivatives, finite
differences of chi^2 in s and in Theta, the dense Wiener filter (also for the
preconditioned solve), closed forms of the homogeneous unmasked case, Philox known
answers; the dense noise bias and Fisher matrix by derivatives of ln det C of an
independently built pixel covariance (masked, off-diagonals included); the
simulation b and F, every entry, within their own Monte Carlo error of the dense
ones; the full estimate with simulation b and F unbiased over data realisations;
the sampled-row Fisher matrix and the fiducial iteration by reduction to the full
estimate and closed-form histories; the catalog response by the map response at
pixel positions, periodicity, single-mode closed forms (spin-0 and spin-2), the
dot-product test with its adjoint, exact central differences of its objective, and
its MAP against the dense Wiener filter of the catalog and, for one galaxy per pixel
centre, against the map solve.  Iteration counts of the solver are not pinned (the
paper prints none).
This module is test infrastructure: only the tests, the smoke check and the
benchmark's CPU-baseline leg use it; the library never does.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "signed_k", "live_mask", "free_mask", "partner_mask", "prior_S", "full_plane",
    "forward", "adjoint", "inner_half", "chi2", "grad_chi2", "whitened_grad", "whitened_hvp",
    "lbfgs_solve", "wiener_dense", "band_E", "dchi2_dtheta", "simulate", "sim_fisher",
    "bandpower_qe", "dense_bias_fisher", "newton_update", "precond_diag",
    "homogeneous_band_moments", "band_groups", "fisher_from_columns", "sim_fisher_rows",
    "fiducial_iteration", "bandpower_iterate", "fisher_scale", "sim_signal", "posterior_error",
    "dense_posterior_variance", "band_power", "cosmic_variance", "bmode_leakage_qe",
    "catalog_forward", "catalog_adjoint", "catalog_chi2", "catalog_whitened_grad", "catalog_whitened_hvp",
    "catalog_lbfgs_solve", "catalog_wiener_dense", "catalog_simulate",
]


# ----------------------------------------------------------------------------- conventions

def signed_k(n: int):
    """(ky, kx) float64 broadcastable to the half plane [n][n/2+1]."""
    iy = np.arange(n)
    ky = np.where(iy < n // 2, iy, iy - n).astype(np.float64)[:, None]
    kx = np.arange(n // 2 + 1, dtype=np.float64)[None, :]
    return ky, kx


def live_mask(n: int) -> np.ndarray:
    """Live modes of the half plane: not DC, not on either Nyquist line."""
    iy = np.arange(n)[:, None]
    kx = np.arange(n // 2 + 1)[None, :]
    return ~(((iy == 0) & (kx == 0)) | (iy == n // 2) | (kx == n // 2))


def free_mask(n: int) -> np.ndarray:
    """Independent live entries of the half plane (conjugate partners excluded)."""
    iy = np.arange(n)[:, None]
    kx = np.arange(n // 2 + 1)[None, :]
    return live_mask(n) & ((kx > 0) | ((iy >= 1) & (iy < n // 2)))


def partner_mask(n: int) -> np.ndarray:
    iy = np.arange(n)[:, None]
    kx = np.arange(n // 2 + 1)[None, :]
    return live_mask(n) & (kx == 0) & (iy > n // 2)


def prior_S(pshape: np.ndarray, band: np.ndarray, theta) -> np.ndarray:
    """S_k = Theta_{b(k)} P_k (sec. 2.3, eqs. pi / pilin); 0 on dead modes."""
    theta = np.asarray(theta, np.float64)
    amp = np.where(band >= 0, theta[np.clip(band, 0, None)] if theta.size else 1.0, 1.0)
    n = pshape.shape[1]
    S = amp * pshape
    S = np.where(live_mask(n)[None] & (S > 0), S, 0.0)
    return S


def _rotation_full(n: int):
    """cos 2a, sin 2a on the full plane (appendix C rotation); (1, 0) at k = 0."""
    k = np.fft.fftfreq(n, 1.0 / n)
    ky = k[:, None]
    kx = k[None, :]
    k2 = kx * kx + ky * ky
    with np.errstate(invalid="ignore", divide="ignore"):
        c2 = np.where(k2 > 0, (kx * kx - ky * ky) / k2, 1.0)
        s2 = np.where(k2 > 0, 2.0 * kx * ky / k2, 0.0)
    return c2, s2


def full_plane(half: np.ndarray, free: np.ndarray) -> np.ndarray:
    """Full-plane [n][n] spectrum from the free half-plane entries by Hermitian symmetry."""
    n = half.shape[0]
    F = np.zeros((n, n), np.complex128)
    iy, kx = np.nonzero(free)
    v = half[iy, kx]
    F[iy, kx] = v
    F[(-iy) % n, (-kx) % n] = np.conj(v)
    return F


# ----------------------------------------------------------------------------- response R

def forward(s: np.ndarray, free: np.ndarray | None = None) -> np.ndarray:
    """x = R s (eq. ddecomp without noise): [ncomp][n][n/2+1] complex -> [ncomp][n][n] real.

    Only the free entries of s are read.  Spin-0: x = F^-1 s.  Spin-2: rotate (E, B)
    to (g1, g2) per mode (appendix C) and invert each component."""
    ncomp, n = s.shape[0], s.shape[1]
    fr = free_mask(n) if free is None else free
    full = [full_plane(s[c], fr if fr.ndim == 2 else fr[c]) for c in range(ncomp)]
    if ncomp == 2:
        c2, s2 = _rotation_full(n)
        full = [c2 * full[0] - s2 * full[1], s2 * full[0] + c2 * full[1]]
    out = np.empty((ncomp, n, n))
    for c in range(ncomp):
        z = np.fft.ifft2(full[c]) * n
        assert np.max(np.abs(z.imag)) <= 1e-9 * (np.max(np.abs(z.real)) + 1e-300)
        out[c] = z.real
    return out


def adjoint(x: np.ndarray) -> np.ndarray:
    """R^T x in the full-plane metric: unitary forward DFT, inverse rotation, dead modes
    zeroed; conjugate partners are filled (they are part of the half plane)."""
    ncomp, n = x.shape[0], x.shape[1]
    t = [np.fft.fft2(x[c]) / n for c in range(ncomp)]
    if ncomp == 2:
        c2, s2 = _rotation_full(n)
        t = [c2 * t[0] + s2 * t[1], -s2 * t[0] + c2 * t[1]]
    live = live_mask(n)
    return np.stack([np.where(live, tc[:, : n // 2 + 1], 0.0) for tc in t])


def inner_half(a: np.ndarray, b: np.ndarray) -> float:
    """Full-plane inner product Re sum_k conj(a_k) b_k for half-plane arrays that carry
    every entry of the half plane (columns 0 and n/2 count once, the others twice)."""
    n = a.shape[1]
    wgt = np.full(n // 2 + 1, 2.0)
    wgt[0] = 1.0
    wgt[-1] = 1.0
    return float(np.sum(wgt[None, None, :] * (np.conj(a) * b).real))


# ----------------------------------------------------------------------------- objective

def _free_with_prior(S):
    n = S.shape[1]
    return free_mask(n)[None] & (S > 0)


def chi2(s, d, W, S) -> float:
    """chi^2 = s^dag S^-1 s + (d - R s)^T N^-1 (d - R s) (sec. 2.2, eq. eq_chi), with
    the mask folded into W = M N^-1 and the prior sum taken over the full plane."""
    fr = _free_with_prior(S)
    prior = 0.0
    for c in range(S.shape[0]):
        Fs = full_plane(s[c], fr[c])
        Sf = full_plane(S[c].astype(np.complex128), fr[c]).real
        nz = Sf > 0
        prior += float(np.sum(np.abs(Fs[nz]) ** 2 / Sf[nz]))
    x = forward(np.where(fr, s, 0), fr)
    r = d - x
    return prior + float(np.sum(W[None] * r * r))


def grad_chi2(s, d, W, S) -> np.ndarray:
    """d chi^2 / d s per stored coefficient (d/dRe + i d/dIm): 4 g on the free entries,
    g = S^-1 s - R^dag N^-1 (d - R s) (eq. eq_cost); 0 elsewhere."""
    fr = _free_with_prior(S)
    sf = np.where(fr, s, 0)
    x = forward(sf, fr)
    Fr = adjoint(W[None] * (d - x))
    with np.errstate(divide="ignore", invalid="ignore"):
        g = np.where(fr, sf / np.where(fr, S, 1.0) - Fr, 0)
    return 4.0 * g


def whitened_grad(w, d, W, S) -> np.ndarray:
    """Gradient of f = chi^2/4 in w = S^-1/2 s: w - S^1/2 R^T W (d - R S^1/2 w)."""
    fr = _free_with_prior(S)
    sq = np.sqrt(S)
    x = forward(np.where(fr, sq * w, 0), fr)
    return np.where(fr, w - sq * adjoint(W[None] * (d - x)), 0)


def whitened_hvp(p, W, S) -> np.ndarray:
    """Curvature of f applied to p: p + S^1/2 R^T W R S^1/2 p (eq. eq_curv, whitened)."""
    fr = _free_with_prior(S)
    sq = np.sqrt(S)
    x = forward(np.where(fr, sq * p, 0), fr)
    return np.where(fr, p + sq * adjoint(W[None] * x), 0)


def _dot(a, b) -> float:
    return float(np.vdot(a, b).real)


def precond_diag(W, S) -> np.ndarray:
    """Diagonal of the optional noise-aware initial inverse Hessian in the whitened
    variable: P_k = 1 / (1 + S_k <W>), <W> the pixel mean of W (masked pixels count as 0).
    It approximates the inverse of D = I + S^1/2 R^T W R S^1/2 when W is replaced by its
    mean (R is an isometry), which makes very red spectra tractable; the paper itself
    solves without a preconditioner (sec. 3)."""
    return 1.0 / (1.0 + S * float(np.mean(W)))


def lbfgs_solve(d, W, S, m: int = 10, tol: float = 1e-10, max_iter: int = 20000,
                dchi2_tol: float = 0.0, x0=None, precond: bool = False):
    """MAP field by L-BFGS (sec. 2.2): textbook two-loop recursion (Nocedal & Wright,
    Numerical Optimization, 2nd ed., algorithms 7.4/7.5) in the whitened variable,
    H0 = gamma I with gamma = s.y / y.y of the newest pair, and the exact line search of
    a quadratic, alpha = -g.p / p.D p (eq. eq_chib).  Starts from w = 0 unless given
    (the start does not matter for a convex problem).  Stops when
    |g| <= tol |g(0)|, or |delta chi^2| < dchi2_tol (sec. 3), or after max_iter.
    precond: H0 = gamma diag(P) with P = precond_diag(W, S) and gamma = s.y / y.P y (same
    stop test, same minimum).

    Returns dict(s, w, iters, rel_grad, chi2, status) with s on the free entries and
    its conjugate partners filled."""
    return _lbfgs(lambda w: whitened_grad(w, d, W, S), lambda p: whitened_hvp(p, W, S),
                  lambda s_: chi2(s_, d, W, S), S, precond_diag(W, S) if precond else None, m, tol, max_iter,
                  dchi2_tol, x0)


def _lbfgs(grad, hvp, chi2_of, S, Pdiag, m, tol, max_iter, dchi2_tol, x0):
    """The L-BFGS iteration of lbfgs_solve for a whitened gradient grad(w) and curvature
    product hvp(p) of any linear response."""
    fr = _free_with_prior(S)
    sq = np.sqrt(S)
    P = np.where(fr, Pdiag, 0.0) if Pdiag is not None else None
    w = np.zeros_like(S, dtype=np.complex128) if x0 is None else np.where(fr, x0, 0).astype(np.complex128)
    g = grad(np.zeros_like(w))
    g0 = math.sqrt(_dot(g, g))
    if w.any():
        g = grad(w)
    pairs: list[tuple[np.ndarray, np.ndarray, float]] = []
    it = 0
    status = 0
    rel = math.sqrt(_dot(g, g)) / g0 if g0 > 0 else 0.0
    while True:
        rel = math.sqrt(_dot(g, g)) / g0 if g0 > 0 else 0.0
        if rel <= tol:
            break
        if it >= max_iter:
            status = 1
            break
        q = g.copy()
        alph = []
        for sv, yv, rho in reversed(pairs):
            a = rho * _dot(sv, q)
            q = q - a * yv
            alph.append(a)
        if pairs:
            sv, yv, _ = pairs[-1]
            if P is None:
                q = (_dot(sv, yv) / _dot(yv, yv)) * q
            else:
                q = (_dot(sv, yv) / _dot(yv, P * yv)) * (P * q)
        elif P is not None:
            q = P * q
        for (sv, yv, rho), a in zip(pairs, reversed(alph)):
            b = rho * _dot(yv, q)
            q = q + sv * (a - b)
        p = -q
        Dp = hvp(p)
        pDp = _dot(p, Dp)
        if not (pDp > 0):
            status = 2
            break
        alpha = -_dot(g, p) / pDp
        w_new = w + alpha * p
        g_new = grad(w_new)
        sv, yv = w_new - w, g_new - g
        sy = _dot(sv, yv)
        if sy > 1e-12 * math.sqrt(_dot(sv, sv) * _dot(yv, yv)):
            pairs.append((sv, yv, 1.0 / sy))
            if len(pairs) > m:
                pairs.pop(0)
        dchi = 4.0 * (alpha * _dot(g, p) + 0.5 * alpha * alpha * pDp)
        w, g = w_new, g_new
        it += 1
        if dchi2_tol > 0 and abs(dchi) < dchi2_tol:
            break
    s_ = np.where(fr, sq * w, 0)
    s_ = _fill_partners(s_)
    return dict(s=s_, w=w, iters=it, rel_grad=rel, chi2=chi2_of(s_), status=status)


def _fill_partners(s):
    n = s.shape[1]
    out = s.copy()
    iy = np.arange(n // 2 + 1, n)
    out[:, iy, 0] = np.conj(s[:, n - iy, 0])
    out[:, n // 2, :] = 0
    return out


# ----------------------------------------------------------------------------- dense Wiener filter

def _coords(S):
    """Real coordinates of the field: (comp, iy, kx, part) of each free entry with S > 0."""
    fr = _free_with_prior(S)
    cc, iy, kx = np.nonzero(fr)
    comp = np.concatenate([cc, cc])
    yy = np.concatenate([iy, iy])
    xx = np.concatenate([kx, kx])
    part = np.concatenate([np.zeros_like(cc), np.ones_like(cc)])
    return comp, yy, xx, part


def _response_matrix(S):
    """A with x = A theta for the real coordinates theta (Re, Im of each free entry):
    column j is R applied to the j-th unit coordinate."""
    ncomp, n = S.shape[0], S.shape[1]
    fr = _free_with_prior(S)
    comp, yy, xx, part = _coords(S)
    A = np.empty((ncomp * n * n, comp.size))
    for j in range(comp.size):
        e = np.zeros(S.shape, np.complex128)
        e[comp[j], yy[j], xx[j]] = 1.0 if part[j] == 0 else 1.0j
        A[:, j] = forward(e, fr).reshape(-1)
    return A, (comp, yy, xx, part)


def wiener_dense(d, W, S):
    """Exact Wiener filter s = S R^dag C^-1 d, C = R S R^dag + N (appendix A, eq. eq:wiener),
    in the real coordinates of the field (each of Re, Im carries variance S_k / 2);
    masked pixels (W = 0) are dropped from d and C.  Also returns
    chi^2_min = d^T C^-1 d.  Dense: O(n^6); for n <= 64 only."""
    A, (comp, yy, xx, part) = _response_matrix(S)
    var = 0.5 * S[comp, yy, xx]
    obs = np.broadcast_to(W[None] > 0, d.shape).reshape(-1)
    Ao = A[obs]
    C = (Ao * var[None, :]) @ Ao.T
    C[np.diag_indices_from(C)] += 1.0 / np.broadcast_to(W[None], d.shape).reshape(-1)[obs]
    L = np.linalg.cholesky(C)
    do = d.reshape(-1)[obs]
    u = np.linalg.solve(L.T, np.linalg.solve(L, do))
    theta = var * (Ao.T @ u)
    s = np.zeros(S.shape, np.complex128)
    np.add.at(s, (comp[part == 0], yy[part == 0], xx[part == 0]), theta[part == 0])
    np.add.at(s, (comp[part == 1], yy[part == 1], xx[part == 1]), 1j * theta[part == 1])
    return dict(s=_fill_partners(s), chi2_min=float(do @ u))


def dense_bias_fisher(W, pshape, band, theta, nbands):
    """Exact noise bias and Fisher matrix of the band powers (appendix A, eqs. bl and
    eq:wf_exact_f read as the Gaussian-likelihood derivatives):
    b_l = 1/2 tr(C^-1 Q_l), F_ll' = 1/2 tr(C^-1 Q_l C^-1 Q_l'), Q_l = R Pi_l R^dag,
    evaluated as b_l = 1/2 sum_{j in l} pi_j G_jj, F_ll' = 1/2 sum pi_j pi_j' G_jj'^2 with
    G = A^T C^-1 A over the real field coordinates (pi_j = P_k / 2).  n <= 32."""
    S = prior_S(pshape, band, theta)
    A, (comp, yy, xx, part) = _response_matrix(S)
    var = 0.5 * S[comp, yy, xx]
    ncomp = S.shape[0]
    n = S.shape[1]
    obs = np.broadcast_to(W[None] > 0, (ncomp, n, n)).reshape(-1)
    Ao = A[obs]
    C = (Ao * var[None, :]) @ Ao.T
    C[np.diag_indices_from(C)] += 1.0 / np.broadcast_to(W[None], (ncomp, n, n)).reshape(-1)[obs]
    G = Ao.T @ np.linalg.solve(C, Ao)
    pi = 0.5 * pshape[comp, yy, xx]
    bj = band[comp, yy, xx]
    b = np.zeros(nbands)
    F = np.zeros((nbands, nbands))
    for l in range(nbands):
        il = np.nonzero(bj == l)[0]
        b[l] = 0.5 * np.sum(pi[il] * np.diag(G)[il])
        for l2 in range(nbands):
            i2 = np.nonzero(bj == l2)[0]
            F[l, l2] = 0.5 * np.sum((pi[il][:, None] * pi[i2][None, :]) * G[np.ix_(il, i2)] ** 2)
    return b, F


# ----------------------------------------------------------------------------- band powers

def band_E(s, S_fid, band, theta_fid, nbands) -> np.ndarray:
    """E_l = 1/2 sum_{k in band l} |s_k|^2 / (Theta_fid,l S_fid,k) over the full plane
    (sec. 2.3, eq. el)."""
    ncomp, n = S_fid.shape[0], S_fid.shape[1]
    fr = _free_with_prior(S_fid)
    E = np.zeros(nbands)
    for c in range(ncomp):
        Fs = full_plane(s[c], fr[c])
        Sf = full_plane(S_fid[c].astype(np.complex128), fr[c]).real
        Bf = full_plane((band[c] + 1).astype(np.complex128), fr[c]).real.round().astype(int) - 1
        for l in range(nbands):
            sel = (Bf == l) & (Sf > 0)
            E[l] += 0.5 * np.sum(np.abs(Fs[sel]) ** 2 / (theta_fid[l] * Sf[sel]))
    return E


def dchi2_dtheta(s, pshape, band, theta, nbands) -> np.ndarray:
    """d chi^2 / d Theta_b at fixed s: the prior term's derivative,
    -sum_{k in b, full plane} |s_k|^2 / (Theta_b^2 P_k)."""
    S = prior_S(pshape, band, theta)
    return -2.0 * band_E(s, S, band, np.asarray(theta, np.float64), nbands)


def sim_signal(draw, S_true):
    """The signal of a simulation (sec. 2.4): s_k = (S_true,k / 2)^1/2 (z_re + i z_im) on
    the free entries from part 0 of draw, partners their conjugates, dead entries 0."""
    n = S_true.shape[1]
    h = n // 2
    fr = _free_with_prior(S_true)
    zr = draw[0][:, :, 0:2 * h:2][:, :, :h]
    zi = draw[0][:, :, 1:2 * h:2][:, :, :h]
    z = np.zeros(S_true.shape, np.complex128)
    z[:, :, :h] = zr + 1j * zi
    return _fill_partners(np.where(fr, np.sqrt(0.5 * S_true) * z, 0))


def simulate(draw, S_true, W):
    """One simulated data map (sec. 2.4 and the procedure summary): a Gaussian random
    field with spectrum S_true (sim_signal), x = R s, plus pixel noise of variance 1/W,
    zero on masked pixels.
    draw: [2][ncomp][n][n] standard normals (part 0 signal, part 1 noise)."""
    fr = _free_with_prior(S_true)
    x = forward(sim_signal(draw, S_true), fr)
    with np.errstate(divide="ignore"):
        sig = np.where(W > 0, 1.0 / np.sqrt(np.where(W > 0, W, 1.0)), 0.0)
    return np.where(W[None] > 0, x + sig[None] * draw[1], 0.0)


def _boosted_S(pshape, band, theta_fid, lb, factor):
    th = np.asarray(theta_fid, np.float64).copy()
    if lb >= 0:
        th[lb] *= factor
    return prior_S(pshape, band, th)


def sim_fisher(W, pshape, band, theta_fid, nbands, draws, m=10, tol=1e-8, max_iter=20000, return_var=False,
               precond=False):
    """Simulation noise bias and Fisher matrix (sec. 2.4):
    b_l = < E_l(Theta_fid, s_hat[d_sim]) > over sims drawn at Theta_fid (eq. blmv);
    F_ll' Delta_l' = < E_l(s_hat[d_sim at Theta_fid + Delta_l' e_l']) - E_l(s_hat[d_sim]) >
    (eq. fisher) with common random numbers, Delta_l' = Theta_fid,l' and every solve
    using the fiducial prior; F is symmetrised.  Returns (b, F, E_sims[nsim][nbands]),
    and with return_var also F_var: per entry the variance of the mean, i.e. the sample
    variance over the simulations of each one's symmetrised estimate divided by nsim
    (zero with a single simulation).  precond: the solves use the diagonal preconditioner
    (same minima)."""
    theta_fid = np.asarray(theta_fid, np.float64)
    S_fid = prior_S(pshape, band, theta_fid)
    nsim = draws.shape[0]
    Es = np.zeros((nsim, nbands))
    Fs = np.zeros((nsim, nbands, nbands))
    for i in range(nsim):
        d0 = simulate(draws[i], S_fid, W)
        E0 = band_E(lbfgs_solve(d0, W, S_fid, m, tol, max_iter, precond=precond)["s"], S_fid, band, theta_fid,
                    nbands)
        Es[i] = E0
        for l2 in range(nbands):
            S2 = _boosted_S(pshape, band, theta_fid, l2, 2.0)
            d2 = simulate(draws[i], S2, W)
            E2 = band_E(lbfgs_solve(d2, W, S_fid, m, tol, max_iter, precond=precond)["s"], S_fid, band, theta_fid,
                        nbands)
            Fs[i, :, l2] = (E2 - E0) / theta_fid[l2]
    b = Es.mean(0)
    F = Fs.mean(0)
    if not return_var:
        return b, 0.5 * (F + F.T), Es
    Fsym = 0.5 * (Fs + Fs.transpose(0, 2, 1))
    Fvar = Fsym.var(0, ddof=1) / nsim if nsim > 1 else np.zeros((nbands, nbands))
    return b, 0.5 * (F + F.T), Es, Fvar


FISHER_FLOOR = 1e-9


def newton_update(theta_fid, F, E, b):
    """Theta_hat = Theta_fid + F^-1 (E - b) (sec. 2.3, eq. eq:wfmv), on the bands that carry
    information: a band whose Fisher diagonal is not positive or is below FISHER_FLOOR of the
    largest (its E does not respond to its amplitude, e.g. beyond a spectrum's cut-off) keeps
    its fiducial amplitude and the step is solved on the other bands."""
    theta_fid = np.asarray(theta_fid, np.float64)
    d = np.diag(F)
    use = np.nonzero(d > FISHER_FLOOR * max(d.max(), 0.0))[0]
    out = theta_fid.copy()
    if use.size:
        out[use] = theta_fid[use] + np.linalg.solve(F[np.ix_(use, use)], (E - b)[use])
    return out


def bandpower_qe(d, W, pshape, band, theta_fid, nbands, draws, m=10, tol=1e-8, max_iter=20000, precond=False):
    """Quadratic band-power estimate (procedure summary, sec. 2.5): MAP of the data,
    E_l of it, simulation b and F, Newton step.  Returns (theta_hat, E, b, F)."""
    theta_fid = np.asarray(theta_fid, np.float64)
    S_fid = prior_S(pshape, band, theta_fid)
    sh = lbfgs_solve(d, W, S_fid, m, tol, max_iter, precond=precond)["s"]
    E = band_E(sh, S_fid, band, theta_fid, nbands)
    b, F, _ = sim_fisher(W, pshape, band, theta_fid, nbands, draws, m, tol, max_iter, precond=precond)
    return newton_update(theta_fid, F, E, b), E, b, F


# ----------------------------------------------------------------------------- sampled Fisher rows
# The Fisher matrix is smooth and close to translation invariant along its diagonals, so
# only a few of its rows need their own simulations and the rest can be interpolated
# (sec. 3.1, discussion of the iteration count against box size).  The paper gives no
# interpolation rule; the one used here: bands form groups of consecutive indices (one
# group per spectrum, e.g. E and B).  The response is interpolated in units of a per-band
# scale D (the variance of E_l over the fiducial simulations, which estimates F_ll for
# the optimal quadratic estimator, so the interpolated quantity is close to a correlation
# and varies slowly even where F_ll spans orders of magnitude):
# r[l, l2] = Fr[l, l2] / sqrt(D_l D_l2).  A column l2 of r that has no simulations of its
# own is taken from the nearest simulated columns a < l2 < b of its group at the same
# diagonal offset (row l + (a - l2) of column a, row l + (b - l2) of column b, each row
# shift kept inside the row's own group), linearly in the band index; with one of the
# two rows outside its group the other is used; beyond the first or last simulated
# column of a group the one neighbour is used with the row clamped into its group.
# Fr = sqrt(D_l D_l2) r, and F is symmetrised afterwards, as in the full estimate.

def band_groups(nbands, groups=None):
    """[(start, stop)] of the band groups (consecutive indices with equal group id)."""
    g = np.zeros(nbands, np.int64) if groups is None else np.asarray(groups, np.int64)
    out = []
    start = 0
    for l in range(1, nbands + 1):
        if l == nbands or g[l] != g[start]:
            out.append((start, l))
            start = l
    return out


def fisher_scale(Es):
    """Per-band scale D_l: the sample variance of E_l over the simulations (1 where it is
    not positive or there is a single simulation)."""
    Es = np.asarray(Es, np.float64)
    if Es.shape[0] < 2:
        return np.ones(Es.shape[1])
    v = Es.var(0, ddof=1)
    return np.where(v > 0, v, 1.0)


def fisher_from_columns(Fcols, rows, nbands, groups=None, scale=None):
    """Symmetrised F from the simulated columns Fcols[:, j] = Fr[:, rows[j]] (see above);
    scale = D (None: all ones)."""
    rows = [int(r) for r in rows]
    D = np.ones(nbands) if scale is None else np.asarray(scale, np.float64)
    sq = np.sqrt(D)
    Fr = np.zeros((nbands, nbands))
    for j, r in enumerate(rows):
        Fr[:, r] = Fcols[:, j]
    rn = Fr / np.outer(sq, sq)
    grp = band_groups(nbands, groups)
    gof = {}
    for gi, (g0, g1) in enumerate(grp):
        for l in range(g0, g1):
            gof[l] = (g0, g1)
    for l2 in range(nbands):
        if l2 in rows:
            continue
        g0, g1 = gof[l2]
        below = [r for r in rows if g0 <= r < l2]
        above = [r for r in rows if l2 < r < g1]
        if not below and not above:
            raise ValueError(f"band group [{g0}, {g1}) has no simulated column")
        a = max(below) if below else None
        b = min(above) if above else None
        for l in range(nbands):
            h0, h1 = gof[l]
            va = vb = None
            if a is not None and h0 <= l + (a - l2) < h1:
                va = rn[l + (a - l2), a]
            if b is not None and h0 <= l + (b - l2) < h1:
                vb = rn[l + (b - l2), b]
            if va is not None and vb is not None:
                v = va + (vb - va) * (l2 - a) / (b - a)
            elif va is not None:
                v = va
            elif vb is not None:
                v = vb
            else:
                s_ = a if a is not None else b
                v = rn[min(max(l + (s_ - l2), h0), h1 - 1), s_]
            Fr[l, l2] = sq[l] * sq[l2] * v
    return 0.5 * (Fr + Fr.T)


def sim_fisher_rows(W, pshape, band, theta_fid, nbands, draws, rows, groups=None, m=10, tol=1e-8,
                    max_iter=20000):
    """sim_fisher with simulations for the boosted bands in `rows` only, the other columns
    interpolated (fisher_from_columns).  Returns (b, F, E_sims)."""
    theta_fid = np.asarray(theta_fid, np.float64)
    S_fid = prior_S(pshape, band, theta_fid)
    nsim = draws.shape[0]
    Es = np.zeros((nsim, nbands))
    Fc = np.zeros((nsim, nbands, len(rows)))
    for i in range(nsim):
        d0 = simulate(draws[i], S_fid, W)
        E0 = band_E(lbfgs_solve(d0, W, S_fid, m, tol, max_iter)["s"], S_fid, band, theta_fid, nbands)
        Es[i] = E0
        for j, l2 in enumerate(rows):
            S2 = _boosted_S(pshape, band, theta_fid, int(l2), 2.0)
            d2 = simulate(draws[i], S2, W)
            E2 = band_E(lbfgs_solve(d2, W, S_fid, m, tol, max_iter)["s"], S_fid, band, theta_fid, nbands)
            Fc[i, :, j] = (E2 - E0) / theta_fid[int(l2)]
    return Es.mean(0), fisher_from_columns(Fc.mean(0), rows, nbands, groups, fisher_scale(Es)), Es


# ----------------------------------------------------------------------------- fiducial iteration
# The fiducial spectrum is itself updated from the estimate and the estimate repeated
# (sec. 2.3, after eq. pilin): a band power must not reach zero, which would remove its
# projection; the update keeps each band at or above `floor` times its previous value.

def fiducial_iteration(estimate, theta0, max_iter, rel_tol, floor):
    """Theta_fid,0 = theta0; theta_hat_t = estimate(Theta_fid,t-1); Theta_fid,t =
    max(theta_hat_t, floor * Theta_fid,t-1); stop after max_iter estimates or once
    max_l |Theta_fid,t - Theta_fid,t-1| / Theta_fid,t-1 <= rel_tol.  Returns
    (theta_hat of the last estimate, [Theta_fid,0 .. Theta_fid,T])."""
    hist = [np.asarray(theta0, np.float64).copy()]
    th = None
    for _ in range(max_iter):
        prev = hist[-1]
        th = np.asarray(estimate(prev), np.float64)
        nxt = np.maximum(th, floor * prev)
        hist.append(nxt)
        if np.max(np.abs(nxt - prev) / prev) <= rel_tol:
            break
    return th, hist


def bandpower_iterate(d, W, pshape, band, theta0, nbands, draws, max_iter, rel_tol, floor, rows=None, groups=None,
                      m=10, tol=1e-8, solve_max_iter=20000):
    """fiducial_iteration of the quadratic estimate (bandpower_qe, with the Fisher matrix
    from all rows or from the sampled `rows`).  Returns (theta_hat, history)."""
    def est(th_fid):
        S_fid = prior_S(pshape, band, th_fid)
        sh = lbfgs_solve(d, W, S_fid, m, tol, solve_max_iter)["s"]
        E = band_E(sh, S_fid, band, th_fid, nbands)
        if rows is None:
            b, F, _ = sim_fisher(W, pshape, band, th_fid, nbands, draws, m, tol, solve_max_iter)
        else:
            b, F, _ = sim_fisher_rows(W, pshape, band, th_fid, nbands, draws, rows, groups, m, tol, solve_max_iter)
        return newton_update(th_fid, F, E, b)
    return fiducial_iteration(est, theta0, max_iter, rel_tol, floor)


# ----------------------------------------------------------------------------- B-mode leakage bias
# Appendix C: instead of the full Fisher analysis for the B bands, realisations of the E->B
# leakage are averaged into a bias, like the noise bias.  Reading used here: simulations
# drawn with the fiducial E power and no B power, solved with the fiducial prior, give
# b_B = <E_B> = noise bias + leakage; the B block of the Fisher matrix comes from boosted B
# bands only (eq. fisher); with <E> linear in the true amplitudes,
# Theta_hat_B = F_BB^-1 (E_B(d) - b_B).

def bmode_leakage_qe(d, W, pshape, band, theta_fid, nbands, draws, b_bands, m=10, tol=1e-8, max_iter=20000):
    """Returns (theta_hat_B, E_B of the data, b_B, F_BB) over the bands b_bands."""
    theta_fid = np.asarray(theta_fid, np.float64)
    B = [int(l) for l in b_bands]
    th_leak = theta_fid.copy()
    th_leak[B] = 0.0
    S_fid = prior_S(pshape, band, theta_fid)
    S_leak = prior_S(pshape, band, th_leak)
    E = band_E(lbfgs_solve(d, W, S_fid, m, tol, max_iter)["s"], S_fid, band, theta_fid, nbands)
    Eleak = np.zeros((len(draws), nbands))
    Fr = np.zeros((nbands, len(B)))
    for i, dr in enumerate(draws):
        Eleak[i] = band_E(lbfgs_solve(simulate(dr, S_leak, W), W, S_fid, m, tol, max_iter)["s"], S_fid, band,
                          theta_fid, nbands)
        E0 = band_E(lbfgs_solve(simulate(dr, S_fid, W), W, S_fid, m, tol, max_iter)["s"], S_fid, band, theta_fid,
                    nbands)
        for j, l2 in enumerate(B):
            S2 = _boosted_S(pshape, band, theta_fid, l2, 2.0)
            E2 = band_E(lbfgs_solve(simulate(dr, S2, W), W, S_fid, m, tol, max_iter)["s"], S_fid, band, theta_fid,
                        nbands)
            Fr[:, j] += (E2 - E0) / theta_fid[l2]
    Fr /= len(draws)
    FBB = Fr[B, :]
    FBB = 0.5 * (FBB + FBB.T)
    bB = Eleak.mean(0)[B]
    return np.linalg.solve(FBB, E[B] - bB), E[B], bB, FBB


# ----------------------------------------------------------------------------- posterior errors
# The Wiener filter's residual s - s_hat has covariance S - S R^dag C^-1 R S (appendix A,
# after eq. eq:wiener).  Its diagonal, per harmonic entry and per pixel (x = R (s - s_hat)),
# is estimated from simulations drawn with the solve's own prior: signal and data of each
# simulation, the MAP of the data, the residual.

def posterior_error(W, pshape, band, theta, draws, m=10, tol=1e-10, max_iter=20000):
    """Simulation estimate of the posterior variance: var_modes [ncomp][n][n/2+1] =
    mean |s - s_hat|^2 per stored entry (partners mirror their free entries, dead 0),
    var_pix [ncomp][n][n] = mean (R (s - s_hat))^2."""
    S = prior_S(pshape, band, theta)
    vm = np.zeros(S.shape)
    vp = None
    for dr in draws:
        s = sim_signal(dr, S)
        sh = lbfgs_solve(simulate(dr, S, W), W, S, m, tol, max_iter)["s"]
        r = s - sh
        x = forward(r, _free_with_prior(S))
        vm += np.abs(r) ** 2
        vp = x ** 2 if vp is None else vp + x ** 2
    return vm / len(draws), vp / len(draws)


def dense_posterior_variance(W, S):
    """Exact diagonal of S - S R^dag C^-1 R S (dense, n <= 16): per stored entry the sum of
    the posterior variances of its real and imaginary coordinates (var - var^2 G_jj with
    G = A^T C^-1 A over the observed pixels), and per pixel the diagonal of
    A (V - V G V) A^T."""
    A, (comp, yy, xx, part) = _response_matrix(S)
    var = 0.5 * S[comp, yy, xx]
    ncomp, n = S.shape[0], S.shape[1]
    obs = np.broadcast_to(W[None] > 0, (ncomp, n, n)).reshape(-1)
    Ao = A[obs]
    C = (Ao * var[None, :]) @ Ao.T
    C[np.diag_indices_from(C)] += 1.0 / np.broadcast_to(W[None], (ncomp, n, n)).reshape(-1)[obs]
    G = Ao.T @ np.linalg.solve(C, Ao)
    P = np.diag(var) - (var[:, None] * G) * var[None, :]
    vm = np.zeros(S.shape)
    np.add.at(vm, (comp, yy, xx), np.diag(P))
    vm = _fill_partners(vm.astype(np.complex128)).real
    vp = np.einsum("pj,jk,pk->p", A, P, A).reshape(ncomp, n, n)
    return vm, vp


# ----------------------------------------------------------------------------- convergence by scale
# Appendix B compares a map solved to a loose tolerance with a tightly converged one scale by
# scale, against the cosmic-variance limit: here per band, by the band power of the map and
# of its difference from the reference.

def band_power(s, S, band, nbands) -> np.ndarray:
    """sum over the free entries k of band l with S_k > 0 of |s_k|^2."""
    fr = _free_with_prior(S)
    out = np.zeros(nbands)
    for l in range(nbands):
        sel = fr & (band == l)
        out[l] = np.sum(np.abs(s[sel]) ** 2)
    return out


def cosmic_variance(S, band, nbands) -> np.ndarray:
    """sqrt(2 / N_l), N_l the full-plane modes of band l (two per free entry with S > 0)."""
    fr = _free_with_prior(S)
    out = np.zeros(nbands)
    for l in range(nbands):
        N = 2 * int(np.sum(fr & (band == l)))
        out[l] = math.sqrt(2.0 / N) if N > 0 else 0.0
    return out


# ----------------------------------------------------------------------------- catalog response
# Sec. 3.4: instead of binned shear maps, the likelihood of the measured ellipticities of a
# catalog of galaxies at their own positions.  The field is the band-limited Fourier series of
# the harmonic coefficients (the same modes, rotation and unitary normalisation as R),
# evaluated exactly at each galaxy position r_g in pixel units (a non-uniform DFT):
# gamma_a(r_g) = n^-1 sum_{k live, full plane} gamma~_a,k exp(2 pi i k.r_g / n); at integer
# positions this is R s.  chi^2 = s^dag S^-1 s + sum_{a,g} wgt_g (e_a,g - gamma_a(r_g))^2.

def _catalog_phases(pos, n):
    """exp(2 pi i k.r_g / n) for every galaxy (rows) and full-plane mode (columns, [ky][kx])."""
    k = np.fft.fftfreq(n, 1.0 / n)
    ky = np.repeat(k, n)
    kx = np.tile(k, n)
    ph = 2.0 * math.pi * (np.outer(pos[:, 0], ky) + np.outer(pos[:, 1], kx)) / n
    return np.exp(1j * ph)


def catalog_forward(s, pos, free=None) -> np.ndarray:
    """gamma [ncomp][ngal] at the positions pos [ngal][2] (y, x) of the field s
    [ncomp][n][n/2+1] (free entries read; spin-2 rotated as in forward)."""
    ncomp, n = s.shape[0], s.shape[1]
    fr = free_mask(n) if free is None else free
    full = [full_plane(s[c], fr if fr.ndim == 2 else fr[c]) for c in range(ncomp)]
    if ncomp == 2:
        c2, s2 = _rotation_full(n)
        full = [c2 * full[0] - s2 * full[1], s2 * full[0] + c2 * full[1]]
    E = _catalog_phases(np.asarray(pos, np.float64), n)
    out = np.empty((ncomp, len(pos)))
    for c in range(ncomp):
        z = E @ full[c].reshape(-1) / n
        assert np.max(np.abs(z.imag)) <= 1e-9 * (np.max(np.abs(z.real)) + 1e-300)
        out[c] = z.real
    return out


def catalog_adjoint(r, pos, n) -> np.ndarray:
    """R_cat^T r in the full-plane metric for r [ncomp][ngal]: per full-plane mode
    n^-1 sum_g r_g exp(-2 pi i k.r_g / n), inverse rotation, dead entries zeroed."""
    ncomp = r.shape[0]
    E = _catalog_phases(np.asarray(pos, np.float64), n)
    t = [(np.conj(E).T @ r[c]).reshape(n, n) / n for c in range(ncomp)]
    if ncomp == 2:
        c2, s2 = _rotation_full(n)
        t = [c2 * t[0] + s2 * t[1], -s2 * t[0] + c2 * t[1]]
    live = live_mask(n)
    return np.stack([np.where(live, tc[:, : n // 2 + 1], 0.0) for tc in t])


def catalog_chi2(s, e, wgt, pos, S) -> float:
    """chi^2 of a catalog (eq. eq_chi with the catalog response)."""
    fr = _free_with_prior(S)
    prior = 0.0
    for c in range(S.shape[0]):
        Fs = full_plane(s[c], fr[c])
        Sf = full_plane(S[c].astype(np.complex128), fr[c]).real
        nz = Sf > 0
        prior += float(np.sum(np.abs(Fs[nz]) ** 2 / Sf[nz]))
    r = e - catalog_forward(np.where(fr, s, 0), pos, fr)
    return prior + float(np.sum(wgt[None] * r * r))


def catalog_whitened_grad(w, e, wgt, pos, S) -> np.ndarray:
    fr = _free_with_prior(S)
    sq = np.sqrt(S)
    g = catalog_forward(np.where(fr, sq * w, 0), pos, fr)
    return np.where(fr, w - sq * catalog_adjoint(wgt[None] * (e - g), pos, S.shape[1]), 0)


def catalog_whitened_hvp(p, wgt, pos, S) -> np.ndarray:
    fr = _free_with_prior(S)
    sq = np.sqrt(S)
    g = catalog_forward(np.where(fr, sq * p, 0), pos, fr)
    return np.where(fr, p + sq * catalog_adjoint(wgt[None] * g, pos, S.shape[1]), 0)


def catalog_lbfgs_solve(e, wgt, pos, S, m: int = 10, tol: float = 1e-10, max_iter: int = 20000):
    """MAP field of a catalog by the L-BFGS of lbfgs_solve (same recursion and line search)."""
    return _lbfgs(lambda w: catalog_whitened_grad(w, e, wgt, pos, S),
                  lambda p: catalog_whitened_hvp(p, wgt, pos, S),
                  lambda s_: catalog_chi2(s_, e, wgt, pos, S), S, None, m, tol, max_iter, 0.0, None)


def catalog_wiener_dense(e, wgt, pos, S):
    """Exact Wiener filter of a catalog (appendix A, eq. eq:wiener, with the catalog response):
    s = S R^dag C^-1 e, C = R S R^dag + diag(1 / wgt) per component.  Small cases only."""
    comp, yy, xx, part = _coords(S)
    fr = _free_with_prior(S)
    ng = len(pos)
    A = np.empty((S.shape[0] * ng, comp.size))
    for j in range(comp.size):
        u = np.zeros(S.shape, np.complex128)
        u[comp[j], yy[j], xx[j]] = 1.0 if part[j] == 0 else 1.0j
        A[:, j] = catalog_forward(u, pos, fr).reshape(-1)
    var = 0.5 * S[comp, yy, xx]
    C = (A * var[None, :]) @ A.T
    C[np.diag_indices_from(C)] += 1.0 / np.tile(wgt, S.shape[0])
    L = np.linalg.cholesky(C)
    u_ = np.linalg.solve(L.T, np.linalg.solve(L, e.reshape(-1)))
    theta = var * (A.T @ u_)
    s_ = np.zeros(S.shape, np.complex128)
    np.add.at(s_, (comp[part == 0], yy[part == 0], xx[part == 0]), theta[part == 0])
    np.add.at(s_, (comp[part == 1], yy[part == 1], xx[part == 1]), 1j * theta[part == 1])
    return dict(s=_fill_partners(s_), chi2_min=float(e.reshape(-1) @ u_))


def catalog_simulate(draw_signal, draw_noise, S_true, wgt, pos):
    """A simulated catalog: the signal of sim_signal (normals draw_signal [ncomp][n][n], as part
    0 of a grid draw) at the galaxy positions plus noise of variance 1 / wgt_g
    (normals draw_noise [ncomp][ngal])."""
    s_ = sim_signal(np.stack([draw_signal, np.zeros_like(draw_signal)]), S_true)
    return catalog_forward(s_, pos, _free_with_prior(S_true)) + draw_noise / np.sqrt(wgt)[None]


# ----------------------------------------------------------------------------- closed forms

def homogeneous_band_moments(pshape, band, theta_fid, theta_true, nbands, sigma2):
    """Unmasked homogeneous noise, full-plane sums per band (diagonal C in Fourier space):
    <E_l> = 1/2 sum P_k (S_true + s2) / (S_fid + s2)^2, b_l = 1/2 sum P_k / (S_fid + s2),
    F_ll' = delta_ll' 1/2 sum P_k^2 / (S_fid + s2)^2."""
    S_fid = prior_S(pshape, band, theta_fid)
    S_tr = prior_S(pshape, band, theta_true)
    n = pshape.shape[1]
    fr = free_mask(n)[None] & (S_fid > 0)
    mean = np.zeros(nbands)
    b = np.zeros(nbands)
    F = np.zeros((nbands, nbands))
    for l in range(nbands):
        sel = fr & (band == l)
        # each free entry stands for two full-plane modes
        P, Sf, St = pshape[sel], S_fid[sel], S_tr[sel]
        mean[l] = np.sum(P * (St + sigma2) / (Sf + sigma2) ** 2)
        b[l] = np.sum(P / (Sf + sigma2))
        F[l, l] = np.sum(P * P / (Sf + sigma2) ** 2)
    return mean, b, F
