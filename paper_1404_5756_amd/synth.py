"""Seeded synthetic workloads (grids, masks, sigma fields, input fields, observations).

This module only draws inputs; it holds none of the filter's arithmetic.  It is
the one module both the oracle-based tests and the GPU path take inputs from.
The paper's grids, bathymetry, length-scale climatology and observations are
not available, so every workload is synthetic with the shapes and value ranges
of the paper's two configurations (Sec. 4: Mediterranean 1/16 deg grid,
72 levels, half resolution here; Sec. 5: global 1/4 deg, 50 levels,
length scales varying with latitude).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.ndimage import gaussian_filter

SEEDS = {"c1": 14045756, "c2": 1, "c3": 2, "c4": 3, "c5": 4}


def _rng(seed, *sub):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, *sub])))


def smooth_noise(rng, ny, nx, width):
    """White noise smoothed with a Gaussian of `width` grid points, rescaled to [0, 1]."""
    z = gaussian_filter(rng.standard_normal((ny, nx)), width, mode="wrap")
    z -= z.min()
    return z / max(z.max(), 1e-300)


def blob_mask(rng, ny, nx, land_fraction, width=8.0):
    """Smoothed random blobs; the land_fraction quantile is land (0), the rest sea (1)."""
    z = gaussian_filter(rng.standard_normal((ny, nx)), width, mode="wrap")
    thr = np.quantile(z, land_fraction)
    return (z > thr).astype(np.uint8)


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nlev: int
    nfields: int
    mask: np.ndarray            # [1][ny][nx] uint8
    sigma_x: np.ndarray         # [1][ny][nx] float64
    sigma_y: np.ndarray
    n_img: int = 4
    qmode: str = "fit"
    seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def points(self):
        return self.nx * self.ny * self.nlev * self.nfields

    def field(self, dtype=np.float32, nfields=None, nlev=None, sub=0):
        """N(0,1) input [nfields][nlev][ny][nx], one sub-stream per field."""
        nf = self.nfields if nfields is None else nfields
        nl = self.nlev if nlev is None else nlev
        out = np.empty((nf, nl, self.ny, self.nx), dtype=dtype)
        for f in range(nf):
            out[f] = _rng(self.seed, 100 + sub, f).standard_normal((nl, self.ny, self.nx), dtype=np.float64
                                                                    ).astype(dtype)
        return out


def c1_impulse_box():
    """64x64, one level, all sea, sigma = 4: impulse at (32, 32) and an N(0,1) field."""
    n = 64
    w = Workload("c1_64x64_allsea_sigma4", n, n, 1, 1, np.ones((1, n, n), np.uint8),
                 np.full((1, n, n), 4.0), np.full((1, n, n), 4.0), n_img=0, qmode="literal", seed=SEEDS["c1"])
    imp = np.zeros((1, 1, n, n))
    imp[0, 0, 32, 32] = 1.0
    w.extra["impulse"] = imp
    return w


def c2_regional(nlev=72):
    """871x253, 72 levels, T and S; ~40% land in smoothed blobs; sigma in [2, 10] varying smoothly."""
    seed = SEEDS["c2"]
    rng = _rng(seed, 0)
    nx, ny = 871, 253
    mask = blob_mask(rng, ny, nx, 0.40, 8.0)[None]
    s = 2.0 + 8.0 * smooth_noise(_rng(seed, 1), ny, nx, 20.0)
    return Workload("c2_871x253x72_T+S", nx, ny, nlev, 2, mask, s[None], s[None].copy(), seed=seed)


def c3_global(nlev=50):
    """1440x720 (1/4 deg), 50 levels; ~30% land; sigma = 1.5 + 10.5 cos^2(latitude)."""
    seed = SEEDS["c3"]
    nx, ny = 1440, 720
    mask = blob_mask(_rng(seed, 0), ny, nx, 0.30, 10.0)[None]
    lat = np.deg2rad(-90.0 + (np.arange(ny) + 0.5) * 0.25)
    s = np.repeat((1.5 + 10.5 * np.cos(lat) ** 2)[:, None], nx, axis=1)
    return Workload("c3_1440x720x50", nx, ny, nlev, 1, mask, s[None], s[None].copy(), seed=seed)


def c3_anisotropic(nlev=50):
    """The C3 grid with anisotropic, spatially inhomogeneous length scales (Sec. 5: tropical
    scales up to ~350 km, i.e. ~12 grid points at 1/4 deg, with zonal correlations longer than
    meridional ones there): zonal sigma_x = 1.5 + 10.5 cos^2(latitude) as in C3, meridional
    sigma_y = sigma_x / (1 + exp(-(lat/15 deg)^2)) (half the zonal scale at the equator, equal
    at high latitude), and a patch of short scales (x 0.4) standing for a western boundary
    current such as the Kuroshio Extension."""
    w = c3_global(nlev)
    nx, ny = w.nx, w.ny
    lat = -90.0 + (np.arange(ny) + 0.5) * 0.25
    sx = w.sigma_x[0].copy()
    sy = sx / (1.0 + np.exp(-(lat / 15.0) ** 2))[:, None]
    jj, ii = np.mgrid[0:ny, 0:nx]
    patch = np.exp(-(((ii - 0.38 * nx) / (0.05 * nx)) ** 2 + ((jj - 0.65 * ny) / (0.04 * ny)) ** 2))
    scale = 1.0 - 0.6 * patch
    return Workload("c3_aniso_1440x720x50", nx, ny, nlev, 1, w.mask, (sx * scale)[None], (sy * scale)[None],
                    seed=w.seed)


def c3_depth(nlev=50):
    """The C3 grid with a depth-dependent mask and length scales (Sec. 5: the global
    configuration's land grows with depth and its length scales depend on depth): level k
    thresholds C3's smoothed blob field at the land fraction 0.30 + 0.25 k/(nlev-1), so land
    only grows downwards, and sigma shrinks with depth, times (1 - 0.3 k/(nlev-1))."""
    seed = SEEDS["c3"]
    nx, ny = 1440, 720
    z = gaussian_filter(_rng(seed, 0).standard_normal((ny, nx)), 10.0, mode="wrap")
    fr = 0.30 + 0.25 * np.arange(nlev) / max(nlev - 1, 1)
    mask = np.stack([(z > np.quantile(z, f)).astype(np.uint8) for f in fr])
    lat = np.deg2rad(-90.0 + (np.arange(ny) + 0.5) * 0.25)
    s2 = np.repeat((1.5 + 10.5 * np.cos(lat) ** 2)[:, None], nx, axis=1)
    sig = np.stack([s2 * (1.0 - 0.3 * k / max(nlev - 1, 1)) for k in range(nlev)])
    return Workload("c3_depth_1440x720x50", nx, ny, nlev, 1, mask, sig, sig.copy(), seed=seed)


def c2_depth(nlev=72):
    """The C2 grid (T and S) with a depth-dependent mask and length scales (Sec. 4: the
    regional model's bathymetry): level k thresholds C2's smoothed blob field at the land
    fraction 0.40 + 0.25 k/(nlev-1), so land only grows downwards, and sigma is C2's field
    times (1 - 0.3 k/(nlev-1))."""
    seed = SEEDS["c2"]
    nx, ny = 871, 253
    z = gaussian_filter(_rng(seed, 0).standard_normal((ny, nx)), 8.0, mode="wrap")
    fr = 0.40 + 0.25 * np.arange(nlev) / max(nlev - 1, 1)
    mask = np.stack([(z > np.quantile(z, f)).astype(np.uint8) for f in fr])
    s2 = 2.0 + 8.0 * smooth_noise(_rng(seed, 1), ny, nx, 20.0)
    sig = np.stack([s2 * (1.0 - 0.3 * k / max(nlev - 1, 1)) for k in range(nlev)])
    return Workload("c2_depth_871x253x72_T+S", nx, ny, nlev, 2, mask, sig, sig.copy(), seed=seed)


def c4_batch(nitems=64):
    """64 grids with nx~U[128,1024], ny~U[128,768], nlev~U[1,75], land~U[0.1,0.5], sigma in [2, 8]."""
    seed = SEEDS["c4"]
    rng = _rng(seed, 0)
    items = []
    for k in range(nitems):
        nx = int(rng.integers(128, 1025))
        ny = int(rng.integers(128, 769))
        nlev = int(rng.integers(1, 76))
        land = float(rng.uniform(0.1, 0.5))
        r = _rng(seed, 1, k)
        mask = blob_mask(r, ny, nx, land, 6.0)[None]
        s = 2.0 + 6.0 * smooth_noise(_rng(seed, 2, k), ny, nx, 12.0)
        items.append(Workload(f"c4_item{k}_{nx}x{ny}x{nlev}", nx, ny, nlev, 1, mask, s[None], s[None].copy(),
                              seed=seed * 1000 + k))
    return items


def c5_observations(w: Workload, nobs=200_000, seed=None):
    """Observation positions (level, x, y) with all four bilinear corners at sea."""
    rng = _rng(SEEDS["c5"] if seed is None else seed, 0)
    m = w.mask[0]
    lev, xs, ys = [], [], []
    while len(lev) < nobs:
        n = 2 * (nobs - len(lev)) + 1000
        k = rng.integers(0, w.nlev, n)
        x = rng.uniform(0, w.nx - 1, n)
        y = rng.uniform(0, w.ny - 1, n)
        i, j = np.floor(x).astype(int), np.floor(y).astype(int)
        i1, j1 = np.minimum(i + 1, w.nx - 1), np.minimum(j + 1, w.ny - 1)
        ok = (m[j, i] & m[j, i1] & m[j1, i] & m[j1, i1]).astype(bool)
        lev += k[ok].tolist()
        xs += x[ok].tolist()
        ys += y[ok].tolist()
    return (np.array(lev[:nobs], np.int32), np.array(xs[:nobs]), np.array(ys[:nobs]))


def random_case(seed, ny, nx, nlev=1, land=0.3, n_img=2, sigma=(1.0, 8.0), width=3.0, qmode="literal",
                mask_3d=False, sigma_3d=False):
    """Small randomised grid for parity tests: blob mask, smooth sigma, given n_img."""
    rng = _rng(seed, 0)
    ml = nlev if mask_3d else 1
    sl = nlev if sigma_3d else 1
    mask = np.stack([blob_mask(_rng(seed, 1, l), ny, nx, land, width) for l in range(ml)]) if land > 0 \
        else np.ones((ml, ny, nx), np.uint8)
    lo, hi = sigma
    sx = np.stack([lo + (hi - lo) * smooth_noise(_rng(seed, 2, l), ny, nx, width * 2) for l in range(sl)])
    sy = np.stack([lo + (hi - lo) * smooth_noise(_rng(seed, 3, l), ny, nx, width * 2) for l in range(sl)])
    w = Workload(f"rand{seed}_{nx}x{ny}x{nlev}", nx, ny, nlev, 1, mask, sx, sy, n_img=n_img, qmode=qmode,
                 seed=seed)
    del rng
    return w
