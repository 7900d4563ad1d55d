"""Seeded synthetic shear catalogues with the shape of the paper's
aperture-mass workload (Sec. 3: 10^6 galaxies at 35 per square arcmin, about
7.9 square degrees, reconstruction grids of 512^2 to 2048^2 points).

The paper's ray-traced catalogue is not available, so this stands in for it:
  * positions area-uniform on a square field [0, L) x [0, L) arcmin with
    L = sqrt(n / density) (flat sky);
  * intrinsic ellipticity: both components Gaussian with sigma_e = 0.3,
    redrawn until |e| < 1;
  * lensing signal: singular isothermal halos, centres uniform on the field,
    Einstein radii log-uniform in [0.05, 0.5] arcmin, one halo per 100
    square arcmin; a galaxy at distance r from a halo gets the tangential
    shear gamma_t = theta_E / (2 r), capped at 0.5 and cut beyond
    r = 60 theta_E, added to its intrinsic ellipticity as
    (e1, e2) += -gamma_t (cos 2phi, sin 2phi);
  * the catalogue is shuffled (input order carries no spatial structure).
numpy PCG64 with seed = 1000 * config + stream (0 positions, 1 intrinsic
shapes, 2 halos, 3 shuffle).  Nothing here is aperture-mass arithmetic: the
GPU library and the CPU oracle both take these arrays as their inputs.
"""

from __future__ import annotations

import math

import numpy as np

APERTURE_CONFIG = 6        # seed family of the aperture-mass workload
PAPER_DENSITY = 35.0       # galaxies per square arcmin (Sec. 3)


def _rng(config: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(1000 * config + stream))


def shear_catalog(n: int, density: float = PAPER_DENSITY, config: int = APERTURE_CONFIG,
                  sigma_e: float = 0.3, halos: bool = True):
    """Returns ((x, y, e1, e2), side): float64 arrays in arcmin and the field side."""
    side = math.sqrt(n / density) if n > 0 else 1.0
    pos = _rng(config, 0).random((2, n)) * side
    x, y = pos[0].copy(), pos[1].copy()
    r_int = _rng(config, 1)
    e = r_int.normal(0.0, sigma_e, (2, n))
    bad = np.hypot(e[0], e[1]) >= 1.0
    while bad.any():
        e[:, bad] = r_int.normal(0.0, sigma_e, (2, int(bad.sum())))
        bad = np.hypot(e[0], e[1]) >= 1.0
    e1, e2 = e[0].copy(), e[1].copy()
    if halos and n > 0:
        rh = _rng(config, 2)
        n_halo = max(1, int(round(side * side / 100.0)))
        hc = rh.random((2, n_halo)) * side
        th_e = np.exp(rh.uniform(math.log(0.05), math.log(0.5), n_halo))
        order = np.argsort(x, kind="stable")
        xs = x[order]
        for h in range(n_halo):
            reach = 60.0 * th_e[h]                      # gamma_t below 1/120 further out
            lo, hi = np.searchsorted(xs, [hc[0, h] - reach, hc[0, h] + reach])
            cand = order[lo:hi]
            dx, dy = x[cand] - hc[0, h], y[cand] - hc[1, h]
            r2 = dx * dx + dy * dy
            near = r2 < reach * reach
            idx, dxn, dyn, r2n = cand[near], dx[near], dy[near], np.maximum(r2[near], 1e-12)
            g = np.minimum(th_e[h] / (2.0 * np.sqrt(r2n)), 0.5)
            e1[idx] -= g * (dxn * dxn - dyn * dyn) / r2n
            e2[idx] -= g * (2.0 * dxn * dyn) / r2n
    perm = _rng(config, 3).permutation(n)
    return (x[perm], y[perm], e1[perm], e2[perm]), side


def field_grid(side: float, n: int):
    """n x n reconstruction points centred in the cells of the field:
    (x0, y0, dx, dy, nx, ny) with point (i, j) at ((i + 0.5) side/n, ...)."""
    d = side / n
    return (0.5 * d, 0.5 * d, d, d, n, n)


def config_aperture(n: int = 1_000_000):
    """The paper's workload: 10^6 galaxies at 35 per square arcmin."""
    return shear_catalog(n)
