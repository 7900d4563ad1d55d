"""Seeded synthetic catalogues with the shapes of the paper's workloads.

The paper's own catalogue (galaxies from an N-body simulation, RA and Dec in
0..90 deg, with a flat random catalogue over the same region; Sec. 2.2) is not
available, so clustered Neyman-Scott catalogues stand in for the data and
area-uniform points stand in for the randoms.

Recipe (all in float64 degrees, numpy PCG64, seed = 1000*config + stream):
  * area-uniform on a patch [ra0, ra0+W) x [dec0, dec0+H): RA uniform, sin(Dec)
    uniform between sin(dec0) and sin(dec0+H);
  * Neyman-Scott: parents area-uniform, each with `children` points displaced
    by a Gaussian of width sigma (deg) in the local tangent plane
    (dDec = sigma*g2, dRA = sigma*g1/cos(Dec_parent)); on a patch a child that
    falls outside is drawn again, on the full sky Dec is reflected at the poles
    and RA wrapped;
  * the finished catalogue is shuffled, so the input order carries no spatial
    structure;
  * bin edges are log-spaced in theta (equal steps in ln theta, which equal
    steps in log10 theta also give), endpoints exact.

Nothing in this module is pair-counting arithmetic: the GPU library and the CPU
oracle both take the arrays returned here as their inputs.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Patch:
    ra0: float
    width: float
    dec0: float
    height: float

    @property
    def full_sky(self) -> bool:
        return self.width >= 360.0 and self.height >= 180.0


FULL_SKY = Patch(0.0, 360.0, -90.0, 180.0)


def centred_patch(width: float, height: float | None = None, ra0: float = 0.0) -> Patch:
    """Patch of `width` x `height` degrees centred on the equator."""
    h = width if height is None else height
    return Patch(ra0, width, -0.5 * h, h)


def _rng(config: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(1000 * config + stream))


def uniform_patch(n: int, patch: Patch, rng: np.random.Generator):
    """n points uniform in solid angle on `patch`; returns (ra, dec) in degrees."""
    ra = patch.ra0 + patch.width * rng.random(n)
    s0 = math.sin(math.radians(patch.dec0))
    s1 = math.sin(math.radians(patch.dec0 + patch.height))
    dec = np.degrees(np.arcsin(np.clip(s0 + (s1 - s0) * rng.random(n), -1.0, 1.0)))
    if patch.full_sky:
        ra = np.mod(ra, 360.0)
    return ra.astype(np.float64), dec.astype(np.float64)


def _inside(ra, dec, patch: Patch):
    return (ra >= patch.ra0) & (ra < patch.ra0 + patch.width) & \
           (dec >= patch.dec0) & (dec < patch.dec0 + patch.height)


def neyman_scott(n_parents: int, children: int, sigma_deg, patch: Patch,
                 rng: np.random.Generator, shuffle: bool = True):
    """Clustered catalogue: n_parents area-uniform parents, `children` points
    around each (sigma_deg: scalar, or one value per parent)."""
    pra, pdec = uniform_patch(n_parents, patch, rng)
    sig = np.broadcast_to(np.asarray(sigma_deg, dtype=np.float64), (n_parents,))
    pra = np.repeat(pra, children)
    pdec = np.repeat(pdec, children)
    sig = np.repeat(sig, children)
    n = pra.size
    ra = np.empty(n)
    dec = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        g = rng.standard_normal((2, todo.size))
        d = pdec[todo] + sig[todo] * g[1]
        cosd = np.maximum(np.cos(np.radians(pdec[todo])), 1e-12)
        r = pra[todo] + sig[todo] * g[0] / cosd
        if patch.full_sky:
            over = d > 90.0
            under = d < -90.0
            d = np.where(over, 180.0 - d, np.where(under, -180.0 - d, d))
            r = np.where(over | under, r + 180.0, r)
            r = np.mod(r, 360.0)
            ra[todo] = r
            dec[todo] = d
            todo = todo[:0]
        else:
            ok = _inside(r, d, patch)
            ra[todo[ok]] = r[ok]
            dec[todo[ok]] = d[ok]
            todo = todo[~ok]
    if shuffle:
        p = rng.permutation(n)
        ra, dec = ra[p], dec[p]
    return ra, dec


def log_edges(theta_min: float, theta_max: float, n_bins: int) -> np.ndarray:
    """n_bins+1 edges with equal steps in ln(theta); endpoints exact."""
    k = np.arange(n_bins + 1, dtype=np.float64)
    lo, hi = math.log(theta_min), math.log(theta_max)
    e = np.exp(lo + k * ((hi - lo) / n_bins))
    e[0], e[-1] = theta_min, theta_max
    return e


def linear_edges(theta_min: float, theta_max: float, n_bins: int) -> np.ndarray:
    """n_bins+1 evenly spaced edges; endpoints exact."""
    e = theta_min + np.arange(n_bins + 1, dtype=np.float64) * ((theta_max - theta_min) / n_bins)
    e[0], e[-1] = theta_min, theta_max
    return e


def _job(name, D, R, edges, **extra):
    d = {"name": name, "D": D, "R": R, "edges": edges}
    d.update(extra)
    return d


def config_small(scale: float = 1.0):
    """10,000 clustered points (500 parents x 20, sigma 0.05 deg) and 10,000
    randoms on a 10 x 10 deg patch; 30 log bins 0.01-10 deg.  `scale` shrinks
    the parent and random counts for quick tests."""
    patch = centred_patch(10.0)
    npar = max(1, int(round(500 * scale)))
    D = neyman_scott(npar, 20, 0.05, patch, _rng(1, 1))
    R = uniform_patch(max(2, int(round(10_000 * scale))), patch, _rng(1, 2))
    return _job("small", D, R, log_edges(0.01, 10.0, 30), patch=patch)


def config_1m(n_parents: int = 50_000, n_random: int = 1_000_000):
    """1,000,000 clustered points (50,000 parents x 20, sigma 0.05 deg) and
    1,000,000 randoms on a 100 x 100 deg patch; 40 log bins 0.01-20 deg."""
    patch = centred_patch(100.0)
    D = neyman_scott(n_parents, 20, 0.05, patch, _rng(2, 1))
    R = uniform_patch(n_random, patch, _rng(2, 2))
    return _job("clustered_1M_vs_random_1M_100deg_40logbins", D, R,
                log_edges(0.01, 20.0, 40), patch=patch)


def config_batched(n_mocks: int = 256, n_random: int = 1_000_000,
                   parents_lo: int = 2_500, parents_hi: int = 20_000):
    """256 clustered mocks (parents uniform in 2,500..20,000, 20 children,
    sigma 0.05 deg; 50k..400k points) and one shared 1,000,000-point random
    catalogue on a 50 x 50 deg patch; 25 log bins 0.02-5 deg.  The mocks are
    returned as a list of (ra, dec)."""
    patch = centred_patch(50.0)
    sizes = _rng(3, 3).integers(parents_lo, parents_hi + 1, size=n_mocks)
    mocks = [neyman_scott(int(p), 20, 0.05, patch, _rng(3, 100 + m))
             for m, p in enumerate(sizes)]
    R = uniform_patch(n_random, patch, _rng(3, 2))
    return {"name": "batched_mocks", "mocks": mocks, "R": R,
            "edges": log_edges(0.02, 5.0, 25), "patch": patch}


def config_large(n_parents: int = 200_000, n_random: int = 8_000_000):
    """4,000,000 clustered points on the full sky (200,000 parents x 20, sigma
    log-uniform in 0.01-0.2 deg per parent) and 8,000,000 full-sky randoms;
    50 log bins 0.005-30 deg."""
    rng = _rng(4, 0)
    sig = np.exp(rng.uniform(math.log(0.01), math.log(0.2), size=n_parents))
    D = neyman_scott(n_parents, 20, sig, FULL_SKY, _rng(4, 1))
    R = uniform_patch(n_random, FULL_SKY, _rng(4, 2))
    return _job("large_fullsky", D, R, log_edges(0.005, 30.0, 50), patch=FULL_SKY)


def paper_shape(n: int):
    """Unclustered stand-in for the paper's timing runs: n data and n random
    points area-uniform on RA, Dec in [0, 90) deg; 254 log bins 0.001-90 deg."""
    patch = Patch(0.0, 90.0, 0.0, 90.0)
    D = uniform_patch(n, patch, _rng(6, 1))
    R = uniform_patch(n, patch, _rng(6, 2))
    return _job(f"paper_shape_{n}", D, R, log_edges(0.001, 90.0, 254), patch=patch)


def serve_stream(n_requests: int, rate_hz: float, n_patches: int = 32,
                 n_min: int = 1_000, n_max: int = 2_000_000,
                 n_random: int = 1_000_000, seed_config: int = 5):
    """Poisson request stream.  Each request: a clustered catalogue of N points
    (N log-uniform in [n_min, n_max], 20 children per parent, sigma 0.05 deg)
    on one of `n_patches` pool patches (side 5-50 deg), with 10-50 log bins
    over [0.01 deg, min(side/2, 20 deg)].  Returns (patches, requests) where
    patches[p] = {"patch", "R"} holds the pool's random catalogue (generated
    lazily by the caller through `pool_random`) and each request is a dict with
    arrival time (s), patch index and generator parameters; `request_catalog`
    materialises its points."""
    rng = _rng(seed_config, 3)
    sides = rng.uniform(5.0, 50.0, size=n_patches)
    patches = [{"patch": centred_patch(float(s), ra0=float(40.0 * p)), "side": float(s),
                "n_random": n_random} for p, s in enumerate(sides)]
    t = np.cumsum(rng.exponential(1.0 / rate_hz, size=n_requests))
    reqs = []
    for q in range(n_requests):
        n = int(math.floor(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        p = int(rng.integers(0, n_patches))
        b = int(rng.integers(10, 51))
        tmax = min(patches[p]["side"] / 2.0, 20.0)
        reqs.append({"id": q, "t": float(t[q]), "patch": p, "n": max(n, 2),
                     "edges": log_edges(0.01, tmax, b)})
    return patches, reqs


def pool_random(patches, p: int, seed_config: int = 5):
    pp = patches[p]
    return uniform_patch(pp["n_random"], pp["patch"], _rng(seed_config, 1000 + p))


def request_catalog(patches, req, seed_config: int = 5):
    pp = patches[req["patch"]]
    npar = max(1, (req["n"] + 19) // 20)
    ra, dec = neyman_scott(npar, 20, 0.05, pp["patch"], _rng(seed_config, 10_000 + req["id"]))
    return ra[: req["n"]], dec[: req["n"]]
