"""Seeded synthetic workloads: masks, noise maps, prior shapes, band maps, white draws.

This module is the one place that both the HIP path's callers and the CPU oracle's
callers take their inputs from.  It holds none of the method's arithmetic: no
transform, no objective, no solver.  It only tabulates the input functions the
workloads are defined by (P(k) shapes, band edges, mask geometry, noise levels)
and draws white Gaussian numbers from a seeded numpy generator.

Array conventions (shared with the library's C-ABI):

* pixel maps are ``[n][n]`` (row y, column x), float64;
* harmonic tables are ``[ncomp][n][n//2+1]`` over the half plane: row index
  ``iy`` holds the signed wavenumber ``ky = iy`` for ``iy < n/2`` and
  ``iy - n`` otherwise, column ``kx = 0 .. n/2``;
* ``pshape`` is the prior shape P_k (variance of the unitary Fourier coefficient),
  ``band`` the band index of each mode (-1 = not in any band, fixed at amplitude 1);
* ``draws`` for ``nsim`` simulations is ``[nsim][2][ncomp][n][n]`` standard normals:
  part 0 feeds the signal (entries ``[c][ky][2kx]`` / ``[c][ky][2kx+1]`` are the
  real / imaginary normal of mode (ky, kx), kx < n/2), part 1 the pixel noise.

The five workloads follow the method's test cases (projected density, cosmic shear
with E and B modes, flat-sky CMB temperature, a batch of uneven sizes); the
paper's own masks, CLASS spectra and HEALPix maps are not available, so seeded
synthetic stand-ins with the stated shapes, sizes and value ranges are used.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Workload", "kmag_half", "log_band_map", "linear_band_map",
    "density_pshape", "shear_pshape", "cmb_pshape", "circle_holes",
    "white_draws", "density64", "density_bands", "shear_eb", "cmb_patch", "uneven_batch",
    "density_workload", "shear_workload", "cmb_workload",
]


@dataclasses.dataclass
class Workload:
    """One map's inputs.  ``theta_fid`` multiplies ``pshape`` band by band."""
    name: str
    n: int
    ncomp: int
    pshape: np.ndarray          # [ncomp][n][n/2+1] float64
    band: np.ndarray            # [ncomp][n][n/2+1] int32
    nbands: int
    theta_true: np.ndarray      # [nbands] float64 (all ones: the truth)
    theta_fid: np.ndarray       # [nbands] float64
    noise_var: np.ndarray       # [n][n] float64 (per-pixel noise variance)
    mask: np.ndarray            # [n][n] bool (True = observed)
    seed: int

    @property
    def W(self) -> np.ndarray:
        """Inverse-noise weight with the mask folded in: M N^-1 (0 on masked pixels)."""
        return np.where(self.mask, 1.0 / self.noise_var, 0.0)

    @property
    def masked_fraction(self) -> float:
        return float(1.0 - self.mask.mean())


# ----------------------------------------------------------------------------- grids

def signed_ky(n: int) -> np.ndarray:
    iy = np.arange(n)
    return np.where(iy < n // 2, iy, iy - n).astype(np.float64)


def kmag_half(n: int) -> np.ndarray:
    """|k| in grid units on the half plane [n][n/2+1], float64."""
    ky = signed_ky(n)[:, None]
    kx = np.arange(n // 2 + 1, dtype=np.float64)[None, :]
    return np.sqrt(kx * kx + ky * ky)


def _bands_from_edges(kmag: np.ndarray, edges: np.ndarray) -> np.ndarray:
    """Half-open bins [e_l, e_{l+1}); a value exactly on an edge goes to the upper bin."""
    idx = np.searchsorted(edges, kmag, side="right") - 1
    nb = len(edges) - 1
    idx = np.where((kmag >= edges[0]) & (kmag < edges[-1]), idx, -1)
    return np.clip(idx, -1, nb - 1).astype(np.int32)


def log_band_map(n: int, nbands: int) -> np.ndarray:
    """nbands log-spaced |k| bins spanning [1, n/2); [n][n/2+1] int32."""
    edges = np.geomspace(1.0, n / 2.0, nbands + 1)
    return _bands_from_edges(kmag_half(n), edges)


def linear_band_map(n: int, nbands: int) -> np.ndarray:
    """nbands linearly spaced |k| bins spanning [1, n/2); [n][n/2+1] int32."""
    edges = np.linspace(1.0, n / 2.0, nbands + 1)
    return _bands_from_edges(kmag_half(n), edges)


# ----------------------------------------------------------------------------- spectra

def density_pshape(n: int, A: float = 1.0, k0: float = 1.0, kd: float = 20.0) -> np.ndarray:
    """P(k) = A (k/k0)^-2 exp(-(k/kd)^2) in grid units; P(0) := 0."""
    k = kmag_half(n)
    with np.errstate(divide="ignore"):
        p = A * (k / k0) ** -2.0 * np.exp(-(k / kd) ** 2)
    p[k == 0] = 0.0
    return p[None]


def shear_pshape(n: int, A: float = 1.0, ld: float = 300.0, b_ratio: float = 0.01) -> np.ndarray:
    """E: P(l) = A l^-1.5 exp(-(l/ld)^2) in grid units; B = b_ratio * E.  [2][n][n/2+1]."""
    k = kmag_half(n)
    with np.errstate(divide="ignore"):
        pe = A * k ** -1.5 * np.exp(-(k / ld) ** 2)
    pe[k == 0] = 0.0
    return np.stack([pe, b_ratio * pe])


def cmb_pshape(n: int, theta_pix_arcmin: float = 1.7, A: float = 2.0 * math.pi * 1e3) -> np.ndarray:
    """C_l = A/(l(l+1)) exp(-(l/1500)^2)(1 + 0.1 sin(l/40)), l = 2 pi |k| / (n theta_pix);
    the per-coefficient variance is C_l / Omega_pix (Omega_pix = theta_pix^2, uK^2)."""
    th = theta_pix_arcmin * math.pi / (180.0 * 60.0)
    ell = 2.0 * math.pi * kmag_half(n) / (n * th)
    with np.errstate(divide="ignore", invalid="ignore"):
        cl = A / (ell * (ell + 1.0)) * np.exp(-(ell / 1500.0) ** 2) * (1.0 + 0.1 * np.sin(ell / 40.0))
    cl[ell == 0] = 0.0
    return (cl / (th * th))[None]


# ----------------------------------------------------------------------------- masks

def _cut_disc(m: np.ndarray, cy: float, cx: float, r: float) -> None:
    """m &= (pixel outside the disc), evaluated only inside the disc's bounding box (every
    pixel outside the box is farther than r from the centre)."""
    n = m.shape[0]
    y0, y1 = max(0, int(np.ceil(cy - r))), min(n - 1, int(np.floor(cy + r)))
    x0, x1 = max(0, int(np.ceil(cx - r))), min(n - 1, int(np.floor(cx + r)))
    if y0 > y1 or x0 > x1:
        return
    yy, xx = np.mgrid[y0:y1 + 1, x0:x1 + 1]
    m[y0:y1 + 1, x0:x1 + 1] &= (yy - cy) ** 2 + (xx - cx) ** 2 > r * r


def circle_holes(n: int, rng: np.random.Generator, count: int, rmin: float, rmax: float,
                 mask: np.ndarray | None = None) -> np.ndarray:
    """Cut `count` discs of radius U(rmin, rmax) at uniform centres (True = observed)."""
    m = np.ones((n, n), bool) if mask is None else mask.copy()
    for _ in range(count):
        cy, cx = rng.uniform(0, n, 2)
        r = rng.uniform(rmin, rmax)
        _cut_disc(m, cy, cx, r)
    return m


def _holes_until(n, rng, mask, target, rmin, rmax):
    """Add discs one at a time until the masked fraction reaches `target`."""
    while 1.0 - mask.mean() < target:
        cy, cx = rng.uniform(0, n, 2)
        r = rng.uniform(rmin, rmax)
        _cut_disc(mask, cy, cx, r)
    return mask


# ----------------------------------------------------------------------------- draws

def white_draws(n: int, ncomp: int, nsim: int, seed: int, dtype=np.float64) -> np.ndarray:
    """[nsim][2][ncomp][n][n] standard normals (part 0 signal, part 1 noise)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((nsim, 2, ncomp, n, n)).astype(dtype)


def _theta_fid(rng, nbands, randomize):
    if not randomize:
        return np.ones(nbands)
    # the fiducial model: truth rescaled band by band by U(0.01, 1)
    return rng.uniform(0.01, 1.0, nbands)


# ----------------------------------------------------------------------------- workloads

def density_workload(n: int, seed: int, nbands: int = 12, holes: int = 40, rmin=4.0, rmax=12.0,
                     stripe_frac: float = 0.10, noise0: float = 0.05, target_mask: float | None = 0.30,
                     randomize_fid: bool = True, name="density") -> Workload:
    """Projected density: red P(k), holes plus one stripe, log-normal per-pixel noise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = circle_holes(n, rng, holes, rmin * n / 256.0 if n < 256 else rmin,
                     rmax * n / 256.0 if n < 256 else rmax)
    if stripe_frac > 0:
        w = max(1, int(round(stripe_frac * n)))
        y0 = int(rng.integers(0, n - w + 1))
        m[y0:y0 + w, :] = False
    if target_mask is not None:
        m = _holes_until(n, rng, m, target_mask - 0.02, max(1.0, rmin * n / 256.0 if n < 256 else rmin),
                         max(1.5, rmax * n / 256.0 if n < 256 else rmax))
    var = noise0 * rng.lognormal(0.0, 0.5, (n, n))
    band = log_band_map(n, nbands)[None]
    return Workload(name, n, 1, density_pshape(n), band, nbands, np.ones(nbands),
                    _theta_fid(rng, nbands, randomize_fid), var, m, seed)


def shear_workload(n: int, seed: int, nbands_e: int = 10, nbands_b: int = 10, sigma_e: float = 0.3,
                   ngal_mean: float = 10.0, target_mask: float = 0.15, randomize_fid: bool = True,
                   b_ratio: float = 0.01, name="shear") -> Workload:
    """Joint E/B shear: per-pixel noise sigma_e^2 / n_gal with n_gal ~ Poisson(ngal_mean);
    empty pixels are masked and discs (radius 4-12 px, scaled below 512) are added
    until the masked fraction is target_mask +- 1 %."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ngal = rng.poisson(ngal_mean, (n, n))
    m = ngal > 0
    sc = min(1.0, n / 512.0)
    m = _holes_until(n, rng, m, target_mask - 0.01, max(1.0, 4.0 * sc), max(1.5, 12.0 * sc))
    var = np.where(ngal > 0, sigma_e ** 2 / np.maximum(ngal, 1), 1.0)
    be = log_band_map(n, nbands_e)
    bb = np.where(log_band_map(n, nbands_b) >= 0, log_band_map(n, nbands_b) + nbands_e, -1)
    band = np.stack([be, bb]).astype(np.int32)
    nb = nbands_e + nbands_b
    return Workload(name, n, 2, shear_pshape(n, b_ratio=b_ratio), band, nb, np.ones(nb),
                    _theta_fid(rng, nb, randomize_fid), var, m, seed)


def cmb_workload(n: int, seed: int, nbands: int = 40, holes: int = 300, gal_frac: float = 0.10,
                 depth_uk_arcmin: float = 6.0, theta_pix_arcmin: float = 1.7,
                 randomize_fid: bool = True, name="cmb", target_mask: float | None = None) -> Workload:
    """Flat-sky CMB temperature: point-source holes (r 3-10 px, scaled below 1024),
    a galactic-cut band of gal_frac of the rows, scan-striped noise
    sigma^2 = (depth/theta_pix)^2 <hits>/hits with hits = 1 + |sin(x/50)| Poisson(20).
    target_mask: further holes until that masked fraction (- 2 %) is reached."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sc = min(1.0, n / 1024.0)
    nh = max(1, int(round(holes * (n / 1024.0) ** 2)))
    m = circle_holes(n, rng, nh, max(1.0, 3.0 * sc), max(1.5, 10.0 * sc))
    w = max(1, int(round(gal_frac * n)))
    y0 = int(rng.integers(0, n - w + 1))
    m[y0:y0 + w, :] = False
    if target_mask is not None:
        m = _holes_until(n, rng, m, target_mask - 0.02, max(1.0, 3.0 * sc), max(1.5, 10.0 * sc))
    xx = np.arange(n, dtype=np.float64)[None, :]
    hits = 1.0 + np.abs(np.sin(xx / 50.0)) * rng.poisson(20.0, (n, n))
    var = (depth_uk_arcmin / theta_pix_arcmin) ** 2 * hits.mean() / hits
    band = linear_band_map(n, nbands)[None]
    return Workload(name, n, 1, cmb_pshape(n, theta_pix_arcmin), band, nbands, np.ones(nbands),
                    _theta_fid(rng, nbands, randomize_fid), var, m, seed)


@dataclasses.dataclass
class Catalog:
    """A galaxy catalog over an n x n patch: positions (y, x) in pixel units, per-galaxy
    inverse noise variance, and the E/B shear prior of the shear workload."""
    name: str
    n: int
    pos: np.ndarray        # [ngal][2] float64 in [0, n)
    wgt: np.ndarray        # [ngal] 1 / sigma_e^2
    mask: np.ndarray       # [n][n] observed pixels (galaxies only there)
    pshape: np.ndarray
    band: np.ndarray
    nbands: int
    theta_true: np.ndarray
    theta_fid: np.ndarray
    seed: int
    ncomp: int = 2

    @property
    def ngal(self) -> int:
        return int(self.pos.shape[0])


def shear_catalog(n: int, seed: int, ngal_mean: float = 10.0, sigma_e: float = 0.3, target_mask: float = 0.15,
                  nbands_e: int = 10, nbands_b: int = 10, b_ratio: float = 0.01, name="shear-catalog") -> Catalog:
    """Galaxy catalog for the E/B shear workload: Poisson(ngal_mean) galaxies per observed
    pixel, each at a uniform random position inside its pixel; discs (radius 4-12 px, scaled
    below 512) masked until target_mask; per-component shape noise sigma_e per galaxy."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sc = min(1.0, n / 512.0)
    m = _holes_until(n, rng, np.ones((n, n), bool), target_mask, max(1.0, 4.0 * sc), max(1.5, 12.0 * sc))
    counts = np.where(m, rng.poisson(ngal_mean, (n, n)), 0)
    iy, ix = np.nonzero(counts)
    reps = counts[iy, ix]
    py = np.repeat(iy, reps).astype(np.float64) + rng.uniform(0.0, 1.0, reps.sum())
    px = np.repeat(ix, reps).astype(np.float64) + rng.uniform(0.0, 1.0, reps.sum())
    pos = np.stack([py, px], 1)
    wgt = np.full(pos.shape[0], 1.0 / sigma_e ** 2)
    be = log_band_map(n, nbands_e)
    bb = np.where(log_band_map(n, nbands_b) >= 0, log_band_map(n, nbands_b) + nbands_e, -1)
    band = np.stack([be, bb]).astype(np.int32)
    nb = nbands_e + nbands_b
    return Catalog(name, n, pos, wgt, m, shear_pshape(n, b_ratio=b_ratio), band, nb, np.ones(nb),
                   _theta_fid(rng, nb, True), seed)


def catalog_draws(n: int, ncomp: int, ngal: int, seed: int, dtype=np.float64):
    """(signal normals [ncomp][n][n], noise normals [ncomp][ngal]) of one simulated catalog."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.standard_normal((ncomp, n, n)).astype(dtype), rng.standard_normal((ncomp, ngal)).astype(dtype))


def density64(n: int = 64) -> Workload:
    """64^2 density, P = (k/k0)^-2 exp(-(k/20)^2), 8 discs r 4-8 px + 4-px border,
    sigma^2 = 0.1 U(0.5, 2); compared against the dense Wiener filter."""
    seed = 1000
    rng = np.random.Generator(np.random.PCG64(seed))
    sc = n / 64.0
    m = circle_holes(n, rng, 8, 4.0 * sc, 8.0 * sc)
    b = max(1, int(round(4 * sc)))
    m[:b, :] = False
    m[-b:, :] = False
    m[:, :b] = False
    m[:, -b:] = False
    var = 0.1 * rng.uniform(0.5, 2.0, (n, n))
    nb = 8
    band = log_band_map(n, nb)[None]
    return Workload("density64", n, 1, density_pshape(n), band, nb, np.ones(nb),
                    np.ones(nb), var, m, seed)


def density_bands(n: int = 256) -> Workload:
    """The density band-power workload: 12 log bands, 40 holes plus a stripe (~30 % masked),
    log-normal per-pixel noise 0.05 lognormal(0, 0.5); 256^2 by default."""
    return density_workload(n, 2000, nbands=12, name=f"density{n}-bands")


def shear_eb(n: int = 512) -> Workload:
    """The joint E/B shear workload: 10 E and 10 B bands, P_B = 0.01 P_E, sigma_e = 0.3 with
    n_gal ~ Poisson(10), ~15 % masked; 512^2 by default."""
    return shear_workload(n, 3000, name=f"shear{n}-eb")


def cmb_patch(n: int = 1024) -> Workload:
    """The flat-sky CMB temperature patch: 40 linear bands, 300 point-source holes plus a 10 %
    galactic cut, scan-striped noise at 6 uK-arcmin mean depth; 1024^2 by default."""
    return cmb_workload(n, 4000, name=f"cmb{n}-patch")


def uneven_batch(count: int = 96, sizes=(128, 192, 256, 384, 512, 768, 1024)) -> list[Workload]:
    """Uneven-size batch: maps of the three kinds with sides drawn from `sizes`."""
    rng = np.random.Generator(np.random.PCG64(5000))
    out = []
    for i in range(count):
        n = int(rng.choice(sizes))
        kind = int(rng.integers(0, 3))
        frac = float(rng.uniform(0.10, 0.40))
        s = 5000 + 1 + i
        if kind == 0:
            out.append(density_workload(n, s, target_mask=frac, name=f"uneven-density{n}"))
        elif kind == 1:
            out.append(shear_workload(n, s, target_mask=frac, name=f"uneven-shear{n}"))
        else:
            out.append(cmb_workload(n, s, target_mask=frac, name=f"uneven-cmb{n}"))
    return out
