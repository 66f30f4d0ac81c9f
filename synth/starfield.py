"""Seeded synthetic star fields and coefficient draws.

Recipe (the paper's NEAT and Pan-STARRS images are not available, so these
stand in for them with the shapes of its workloads, 256x256 up to chip and
tile sizes):

* sky: Poisson(1000) counts per pixel;
* stars: positions uniform over the pixel area, flux 10**U(3, 5), circular
  Gaussian profile F/(2 pi s^2) exp(-r^2 / 2 s^2) with s = FWHM / 2.35482,
  sampled at pixel centres and truncated at ceil(5 s) pixels, added without
  noise;
* R = float32(sky + stars).

Coefficients a[n][m] are drawn U(-0.05, 0.05) with the constant spatial term
of one chosen basis set to 1, and are returned as float32 so that the CPU
oracle (which promotes them to float64) and the GPU library see identical
values.

Every draw goes through ``numpy.random.SeedSequence(seed).spawn(4)``, whose
children feed the sky, the stars, the coefficients and extra noise.
"""

import math
import numpy as np

SKY_LEVEL = 1000.0
FWHM_TO_SIGMA = 1.0 / 2.35482


def sky_sigma() -> float:
    """Nominal sky noise in ADU: sqrt of the Poisson sky level."""
    return math.sqrt(SKY_LEVEL)


def _streams(seed: int):
    ss = np.random.SeedSequence(seed)
    return [np.random.default_rng(s) for s in ss.spawn(4)]


def render_stars(height, width, xs, ys, flux, fwhm):
    """Sum of truncated, pixel-centre-sampled Gaussian stars (float64)."""
    img = np.zeros(height * width, dtype=np.float64)
    s = np.asarray(fwhm, dtype=np.float64) * FWHM_TO_SIGMA
    rad = np.ceil(5.0 * s).astype(np.int64)
    cx = np.rint(xs).astype(np.int64)
    cy = np.rint(ys).astype(np.int64)
    for r in np.unique(rad):
        sel = np.nonzero(rad == r)[0]
        d = np.arange(-r, r + 1)
        dy, dx = np.meshgrid(d, d, indexing="ij")
        px = cx[sel, None, None] + dx[None]
        py = cy[sel, None, None] + dy[None]
        ss = s[sel, None, None]
        val = (flux[sel, None, None] / (2.0 * math.pi * ss * ss)
               * np.exp(-((px - xs[sel, None, None]) ** 2 + (py - ys[sel, None, None]) ** 2)
                        / (2.0 * ss * ss)))
        ok = (px >= 0) & (px < width) & (py >= 0) & (py < height)
        img += np.bincount((py * width + px)[ok], weights=val[ok], minlength=height * width)
    return img.reshape(height, width)


def star_field(height, width, n_stars, fwhm_fn=None, seed=0, with_sky=True):
    """Reference-like image: Poisson sky plus Gaussian stars, float32.

    ``fwhm_fn(x, y, W, H)`` gives the star FWHM in pixels at a position
    (default 2.5 everywhere).
    """
    sky_rng, star_rng, _, _ = _streams(seed)
    if with_sky:
        sky = sky_rng.poisson(SKY_LEVEL, size=(height, width)).astype(np.float64)
    else:
        sky = np.zeros((height, width))
    xs = star_rng.uniform(-0.5, width - 0.5, n_stars)
    ys = star_rng.uniform(-0.5, height - 0.5, n_stars)
    flux = 10.0 ** star_rng.uniform(3.0, 5.0, n_stars)
    if fwhm_fn is None:
        fwhm = np.full(n_stars, 2.5)
    else:
        fwhm = np.asarray(fwhm_fn(xs, ys, width, height), dtype=np.float64) * np.ones(n_stars)
    img = sky + render_stars(height, width, xs, ys, flux, fwhm)
    return img.astype(np.float32)


def coefficients(n_basis, n_spatial, const_index=None, seed=0, scale=0.05):
    """a[n][m] ~ U(-scale, scale) as float32, a[const_index][0] = 1."""
    _, _, coef_rng, _ = _streams(seed)
    a = coef_rng.uniform(-scale, scale, size=(n_basis, n_spatial))
    if const_index is not None:
        a[const_index, 0] = 1.0
    return a.astype(np.float32)


def poisson_noise(image, seed=0):
    """float32(Poisson(max(image, 0))) from the noise stream of ``seed``."""
    _, _, _, noise_rng = _streams(seed)
    lam = np.maximum(np.asarray(image, dtype=np.float64), 0.0)
    return noise_rng.poisson(lam).astype(np.float32)


def uniform_image(height, width, seed=0, lo=-1.0, hi=1.0):
    """float32 image of independent U(lo, hi) values (noise stream)."""
    _, _, _, noise_rng = _streams(seed)
    return noise_rng.uniform(lo, hi, size=(height, width)).astype(np.float32)


def workload_inputs(wl, seed=None):
    """(R, a) of a workload from the recipe above."""
    seed = wl.seed if seed is None else seed
    R = star_field(wl.height, wl.width, wl.n_stars, wl.fwhm, seed)
    a = coefficients(wl.n_basis, wl.n_spatial, wl.const_basis, seed)
    return R, a


def second_image(wl, seed=None):
    """A second star field of the workload's shape (independent of R).

    Used where I only has to be a realistic image (timing, sampled parity),
    not a function of R.
    """
    seed = (wl.seed if seed is None else seed) + 1000
    return star_field(wl.height, wl.width, wl.n_stars, wl.fwhm, seed)
