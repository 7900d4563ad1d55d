"""Pins of the aperture-mass oracle (Sec. 3, Eq. 3-5) against facts that do
not come from the oracle itself: closed-form limits and special points of the
filter, exact sums on symmetric galaxy rings, the spin-2 symmetries of the
tangential ellipticity, linearity, and the aperture cut at its boundary."""
import math

import numpy as np
import pytest

import oracle

G = 0.2  # ellipticity amplitude used by the ring pins


def _ring(k: int, r: float, pattern: str, centre=(0.0, 0.0)):
    phi = 2.0 * np.pi * np.arange(k) / k
    x = centre[0] + r * np.cos(phi)
    y = centre[1] + r * np.sin(phi)
    c2, s2 = np.cos(2 * phi), np.sin(2 * phi)
    if pattern == "tangential":   # stretched along the circle around the centre
        e1, e2 = -G * c2, -G * s2
    elif pattern == "radial":     # stretched towards the centre
        e1, e2 = G * c2, G * s2
    else:                         # tangential rotated by 45 degrees: no E mode
        e1, e2 = G * s2, -G * c2
    return x, y, e1, e2


def _field(seed: int, n: int, radius: float):
    rng = np.random.default_rng(seed)
    r = radius * np.sqrt(rng.uniform(0.0, 1.0, n))
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    e = rng.normal(0.0, 0.3, (2, n))
    return r * np.cos(phi), r * np.sin(phi), e[0], e[1]


def test_filter_limit_at_zero():
    # tanh(u)/u -> 1, so Q(0) keeps only the logistic factor
    q0 = 1.0 / (1.0 + math.exp(6.0) + math.exp(-47.0))
    assert oracle.q_nfw(0.0) == pytest.approx(q0, rel=1e-15)
    # continuity: the logistic factor moves by ~150 x relative, tanh(u)/u by u^2/3
    assert oracle.q_nfw(1e-9) == pytest.approx(q0, rel=2e-7)


@pytest.mark.parametrize("x,other", [(0.04, -45.0), (0.94, -135.0)])
def test_filter_where_one_exponent_vanishes(x, other):
    # at x = 6/150 the first exponent is 0, at x = 47/50 the second one is
    q = oracle.q_nfw(x)
    u = x / 0.15
    expect = 1.0 / (2.0 + math.exp(other)) * math.tanh(u) / u
    assert q == pytest.approx(expect, rel=1e-12)


def test_filter_plateau_is_the_tanh_profile():
    # for 0.1 < x < 0.6 both exponentials are below e^-9; check the
    # logistic factor is ~1 there, so a wrong sign in either exponent fails
    for x in (0.1, 0.3, 0.6):
        u = x / 0.15
        assert oracle.q_nfw(x) == pytest.approx(math.tanh(u) / u, rel=2e-4)
    assert oracle.q_nfw(1.5) < 1e-10   # beyond the radius the filter dies


def test_tangential_ring_snr_and_sign():
    k, r, theta = 12, 1.3, 2.0
    out = oracle.aperture_points(_ring(k, r, "tangential"), [0.0], [0.0], theta, 7.0)
    assert out["n_in"][0] == k
    # every galaxy has eps_t = +G and the same Q, so SNR = sqrt(2K) exactly
    assert out["snr"][0] == pytest.approx(math.sqrt(2 * k), rel=1e-13)
    assert out["map"][0] == pytest.approx(k * G * oracle.q_nfw(r / theta) / 7.0, rel=1e-13)
    assert out["map"][0] > 0.0


def test_radial_ring_is_negative_and_cross_ring_is_zero():
    k, r, theta = 16, 0.7, 1.0
    rad = oracle.aperture_points(_ring(k, r, "radial"), [0.0], [0.0], theta, 1.0)
    assert rad["snr"][0] == pytest.approx(-math.sqrt(2 * k), rel=1e-13)
    cross = oracle.aperture_points(_ring(k, r, "cross"), [0.0], [0.0], theta, 1.0)
    assert abs(cross["s1"][0]) < 1e-15 * k
    assert cross["s2"][0] == pytest.approx(rad["s2"][0], rel=1e-13)


def _rotate(cat, alpha):
    x, y, e1, e2 = cat
    ca, sa = math.cos(alpha), math.sin(alpha)
    c2, s2 = math.cos(2 * alpha), math.sin(2 * alpha)
    return x * ca - y * sa, x * sa + y * ca, e1 * c2 - e2 * s2, e1 * s2 + e2 * c2


@pytest.mark.parametrize("alpha", [math.pi / 4, 0.37, 2.0])
def test_spin_two_rotation_invariance(alpha):
    # rotating positions by alpha about the point and ellipticities by 2 alpha
    # leaves eps_t, hence M_ap and SNR, unchanged; a wrong sign of either
    # 2phi term or phi in place of 2phi changes them
    theta = 3.0
    cat = _field(1, 400, 0.95 * theta)
    a = oracle.aperture_points(cat, [0.0], [0.0], theta, 2.5)
    b = oracle.aperture_points(_rotate(cat, alpha), [0.0], [0.0], theta, 2.5)
    assert a["n_in"][0] == b["n_in"][0] == 400
    assert b["s1"][0] == pytest.approx(a["s1"][0], rel=1e-10, abs=1e-12 * a["qe_abs"][0])
    assert b["s2"][0] == pytest.approx(a["s2"][0], rel=1e-12)


def test_mirror_symmetry():
    theta = 2.0
    x, y, e1, e2 = _field(2, 300, 0.9 * theta)
    a = oracle.aperture_points((x, y, e1, e2), [0.0], [0.0], theta, 1.0)
    b = oracle.aperture_points((x, -y, e1, -e2), [0.0], [0.0], theta, 1.0)
    assert b["s1"][0] == pytest.approx(a["s1"][0], rel=1e-12, abs=1e-13 * a["qe_abs"][0])


def test_linear_in_ellipticity_and_inverse_in_density():
    theta = 2.0
    x, y, e1, e2 = _field(3, 200, 2.5)
    _, _, f1, f2 = _field(4, 200, 2.5)
    pts = ([0.0, 0.3], [0.0, -0.4])
    a = oracle.aperture_points((x, y, e1, e2), *pts, theta, 1.0)
    b = oracle.aperture_points((x, y, f1, f2), *pts, theta, 1.0)
    c = oracle.aperture_points((x, y, e1 + f1, e2 + f2), *pts, theta, 1.0)
    scale = a["qe_abs"] + b["qe_abs"]
    assert np.all(np.abs(c["map"] - a["map"] - b["map"]) <= 1e-13 * scale)
    d = oracle.aperture_points((x, y, e1, e2), *pts, theta, 4.0)
    np.testing.assert_allclose(d["map"] * 4.0, a["map"], rtol=1e-15)
    np.testing.assert_array_equal(d["snr"], a["snr"])


def test_cut_at_the_filter_radius():
    theta = 2.0
    below = np.nextafter(theta, 0.0)
    x = np.array([theta, 0.0, below, 0.0, 0.0])
    y = np.array([0.0, -theta, 0.0, 0.0, 1.0])
    e = np.full(5, 0.1)
    out = oracle.aperture_points((x, y, e, e), [0.0], [0.0], theta, 1.0)
    # at exactly theta_max (two galaxies) out, just inside in, on the point out
    assert out["n_in"][0] == 2
    empty = oracle.aperture_points((x[:2], y[:2], e[:2], e[:2]), [0.0], [0.0], theta, 1.0)
    assert empty["n_in"][0] == 0 and empty["map"][0] == 0.0 and math.isnan(empty["snr"][0])


def test_grid_is_the_points_it_names():
    theta = 1.5
    cat = _field(5, 500, 4.0)
    grid = (-1.0, -0.75, 0.25, 0.3, 7, 5)
    g = oracle.aperture_grid(cat, grid, theta, 3.0)
    ix, iy = np.meshgrid(np.arange(7), np.arange(5))
    px = -1.0 + ix.ravel() * 0.25
    py = -0.75 + iy.ravel() * 0.3
    p = oracle.aperture_points(cat, px, py, theta, 3.0)
    for k in ("map", "snr", "n_in"):
        np.testing.assert_array_equal(g[k], p[k])


def test_translation_invariance():
    theta = 2.0
    x, y, e1, e2 = _field(6, 300, 2.2)
    a = oracle.aperture_points((x, y, e1, e2), [0.1], [-0.2], theta, 1.0)
    b = oracle.aperture_points((x + 64.0, y - 32.0, e1, e2), [64.1], [-32.2], theta, 1.0)
    assert a["n_in"][0] == b["n_in"][0]
    assert b["s1"][0] == pytest.approx(a["s1"][0], rel=1e-9, abs=1e-11 * a["qe_abs"][0])
