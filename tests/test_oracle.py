"""Pins for the CPU oracle: each check ties it to something other than itself
(hand-worked geometry, high-precision mathematics, exact identities, the
closed form for isotropic points).  CPU only."""
import json
import math
import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


# ------------------------------------------------------------------ sincosd

def _true_sincos_deg(x: float):
    with mpmath.workdps(60):
        t = mpmath.mpf(x) * mpmath.pi / 180
        return mpmath.sin(t), mpmath.cos(t)


def _ulps(got: float, true) -> float:
    tf = float(true)
    if tf == 0.0:
        return abs(got) / math.ulp(0.0) if got else 0.0
    return float(abs(mpmath.mpf(got) - true)) / math.ulp(tf)


def test_sincosd_exact_at_quarter_turns():
    # sin/cos of multiples of 90 deg are exactly 0 or +-1 (degree-domain reduction)
    for k in list(range(-12, 13)) + [4 * 10**6 + 1, -(4 * 10**7) - 3]:
        s, c = oracle.sincosd(90.0 * k)
        m = k % 4
        es, ec = [(0.0, 1.0), (1.0, 0.0), (0.0, -1.0), (-1.0, 0.0)][m]
        assert s == es and c == ec, (k, s, c)


def test_sincosd_within_two_ulps_of_true_value():
    rng = np.random.default_rng(7)
    xs = list(rng.uniform(-1000.0, 1000.0, 1500))
    xs += list(rng.uniform(-1e-3, 1e-3, 200)) + [30.0, 60.0, 45.0, 135.0, 1e-300, 89.999999, 1e15 + 17.5]
    worst = 0.0
    for x in xs:
        s, c = oracle.sincosd(x)
        ts, tc = _true_sincos_deg(x)
        worst = max(worst, _ulps(s, ts), _ulps(c, tc))
    assert worst <= 2.0, worst


def test_unit_vectors_known_points_and_norm():
    v = oracle.unit_vectors([0.0, 90.0, 17.0, 0.0], [0.0, 0.0, 90.0, -90.0])
    assert tuple(v[0]) == (1.0, 0.0, 0.0)
    assert abs(v[1][0]) == 0.0 and v[1][1] == 1.0 and v[1][2] == 0.0
    assert v[2][2] == 1.0 and abs(v[2][0]) == 0.0 and abs(v[2][1]) == 0.0
    assert v[3][2] == -1.0
    rng = np.random.default_rng(3)
    ra = rng.uniform(0, 360, 5000)
    dec = rng.uniform(-90, 90, 5000)
    u = oracle.unit_vectors(ra, dec)
    assert np.max(np.abs(np.sum(u * u, axis=1) - 1.0)) < 1e-15
    # against an independent evaluation (numpy, radians) -- a sign or axis slip would show
    r, d = np.radians(ra), np.radians(dec)
    ref = np.stack([np.cos(d) * np.cos(r), np.cos(d) * np.sin(r), np.sin(d)], axis=1)
    assert np.max(np.abs(u - ref)) < 1e-15


def test_chord2_edges_match_high_precision():
    th = synth.log_edges(0.005, 30.0, 50)
    e = oracle.chord2_edges(th)
    for t, ek in zip(th, e):
        with mpmath.workdps(50):
            true = 4 * mpmath.sin(mpmath.mpf(float(t)) * mpmath.pi / 360) ** 2
        assert abs(mpmath.mpf(float(ek)) - true) <= 4 * math.ulp(float(true))


# ----------------------------------------------------------- hand-built cases

def _load_golden():
    with open(os.path.join(HERE, "golden", "handbuilt_pairs.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _load_golden(), ids=lambda c: c["name"])
def test_handbuilt_counts(case):
    A = np.array(case["A"], dtype=np.float64)
    if case["auto"]:
        got = oracle.count((A[:, 0], A[:, 1]), case["edges"], auto=True)
    else:
        B = np.array(case["B"], dtype=np.float64)
        got = oracle.count((A[:, 0], A[:, 1]), case["edges"], B=(B[:, 0], B[:, 1]), auto=False)
    assert got.tolist() == case["expected"]


# ------------------------------------------- brute force against Appendix A

def _sep_appendix_a(ra1, dec1, ra2, dec2):
    """Appendix A separation, arctan read as atan2 (numpy, radians)."""
    d1, d2 = np.radians(dec1), np.radians(dec2)
    da = np.radians(ra2 - ra1)
    A = np.cos(d2) ** 2 * np.sin(da) ** 2
    B = np.cos(d1) * np.sin(d2) - np.sin(d1) * np.cos(d2) * np.cos(da)
    C = np.sin(d1) * np.sin(d2) + np.cos(d1) * np.cos(d2) * np.cos(da)
    return np.degrees(np.arctan2(np.sqrt(A + B * B), C))


def _sep_mp(ra1, dec1, ra2, dec2):
    with mpmath.workdps(40):
        k = mpmath.pi / 180
        d1, d2, da = mpmath.mpf(dec1) * k, mpmath.mpf(dec2) * k, (mpmath.mpf(ra2) - mpmath.mpf(ra1)) * k
        A = mpmath.cos(d2) ** 2 * mpmath.sin(da) ** 2
        B = mpmath.cos(d1) * mpmath.sin(d2) - mpmath.sin(d1) * mpmath.cos(d2) * mpmath.cos(da)
        C = mpmath.sin(d1) * mpmath.sin(d2) + mpmath.cos(d1) * mpmath.cos(d2) * mpmath.cos(da)
        return mpmath.atan2(mpmath.sqrt(A + B * B), C) / k


def _exact_bins(raA, decA, raB, decB, edges, auto):
    """Counts from the Appendix A angle.  Pairs whose double precision angle
    is within 1e-9 relative of an edge are settled in 40-digit arithmetic;
    pairs within 1e-12 of an edge in that arithmetic are edge-ambiguous (the
    pinned binary64 chord decides them) and are put in the lower bin, with
    amb[k] counting those at edge k."""
    edges = np.asarray(edges)
    counts = np.zeros(edges.size + 1, dtype=np.int64)
    amb = np.zeros(edges.size, dtype=np.int64)
    for i in range(raA.size):
        if auto:
            rb, db = raA[i + 1:], decA[i + 1:]
        else:
            rb, db = raB, decB
        th = _sep_appendix_a(raA[i], decA[i], rb, db)
        idx = np.searchsorted(edges, th, side="right")
        if th.size:
            scale = np.maximum(edges, 1e-300)[None, :]
            rel = np.min(np.abs(th[:, None] - edges[None, :]) / scale, axis=1)
        else:
            rel = np.zeros(0)
        for j in np.nonzero(rel < 1e-9)[0]:
            t = _sep_mp(raA[i], decA[i], rb[j], db[j])
            near = [k for k, e in enumerate(edges)
                    if abs(t - mpmath.mpf(float(e))) <= mpmath.mpf(1e-12) * max(abs(float(e)), 1e-300)]
            if near:
                amb[near[0]] += 1
                idx[j] = near[0]
            else:
                idx[j] = sum(1 for e in edges if mpmath.mpf(float(e)) <= t)
        counts += np.bincount(idx, minlength=edges.size + 1)
    return counts, amb


def _assert_counts_valid(got, want, amb):
    """got must equal want after moving m_k <= amb[k] pairs across edge k
    from the lower bin (index k) to the upper bin (index k+1)."""
    d = np.asarray(got, dtype=np.int64) - want
    assert d.sum() == 0
    carry = 0
    for k in range(amb.size):
        carry = carry - d[k]          # pairs moved up across edge k
        assert 0 <= carry <= amb[k], (k, carry, amb[k], d.tolist())
    assert carry == d[-1]


def test_brute_force_against_appendix_a_auto_and_cross():
    c = synth.config_small(scale=0.04)          # 20 parents x 20 = 400 pts, 400 randoms
    (ra, dec), (rr, dr) = c["D"], c["R"]
    edges = c["edges"]
    want, amb = _exact_bins(ra, dec, None, None, edges, True)
    assert amb.sum() == 0
    got = oracle.count((ra, dec), edges, auto=True)
    assert got.tolist() == want.tolist()
    want, amb = _exact_bins(ra, dec, rr, dr, edges, False)
    assert amb.sum() == 0
    got = oracle.count((ra, dec), edges, B=(rr, dr), auto=False)
    assert got.tolist() == want.tolist()


def test_brute_force_wide_angles_and_poles():
    # full sky, including pairs beyond 90 deg (where the printed arctan breaks)
    # and pole-to-equator pairs lying exactly on the 90 deg edge
    rng = np.random.default_rng(11)
    ra, dec = synth.uniform_patch(300, synth.FULL_SKY, rng)
    ra = np.concatenate([ra, [0.0, 200.0, 10.0]])
    dec = np.concatenate([dec, [90.0, -90.0, 0.0]])
    edges = synth.linear_edges(0.0, 180.0, 18)
    want, amb = _exact_bins(ra, dec, None, None, edges, True)
    assert amb.sum() >= 2
    got = oracle.count((ra, dec), edges, auto=True)
    _assert_counts_valid(got, want, amb)


# -------------------------------------------------------------- invariants

def test_pair_totals_union_symmetry_permutation_rows():
    c = synth.config_small(scale=0.1)           # 1,000 + 1,000 points
    A, R, edges = c["D"], c["R"], c["edges"]
    nA, nR = A[0].size, R[0].size
    dd = oracle.count(A, edges)
    rr = oracle.count(R, edges)
    dr = oracle.count(A, edges, B=R, auto=False)
    rd = oracle.count(R, edges, B=A, auto=False)
    assert int(dd.sum()) == nA * (nA - 1) // 2
    assert int(dr.sum()) == nA * nR
    assert dr.tolist() == rd.tolist()                       # cross symmetry
    U = (np.concatenate([A[0], R[0]]), np.concatenate([A[1], R[1]]))
    uu = oracle.count(U, edges)
    assert uu.tolist() == (dd + rr + dr).tolist()           # auto(A u B) = auto A + auto B + cross
    p = np.random.default_rng(5).permutation(nA)
    assert oracle.count((A[0][p], A[1][p]), edges).tolist() == dd.tolist()
    parts = [oracle.count(A, edges, rows=(a, b)) for a, b in [(0, 1), (1, 333), (333, 999), (999, nA)]]
    assert np.sum(parts, axis=0).tolist() == dd.tolist()
    parts = [oracle.count(A, edges, B=R, auto=False, rows=(a, b)) for a, b in [(0, 400), (400, nA)]]
    assert np.sum(parts, axis=0).tolist() == dr.tolist()


def test_degenerate_sizes():
    e = [1.0, 2.0]
    assert oracle.count((np.zeros(0), np.zeros(0)), e).tolist() == [0, 0, 0]
    assert oracle.count((np.zeros(1), np.zeros(1)), e).tolist() == [0, 0, 0]
    assert oracle.count((np.zeros(0), np.zeros(0)), e, B=(np.zeros(3), np.zeros(3)), auto=False).tolist() == [0, 0, 0]


def test_isotropic_sphere_closed_form():
    """Uniform points on the sphere: a pair falls in [t1, t2) with probability
    (cos t1 - cos t2)/2; pair indicators are pairwise independent (for a fixed
    point the other is still uniform), so Var = M p (1-p) exactly."""
    n = 3000
    ra, dec = synth.uniform_patch(n, synth.FULL_SKY, np.random.default_rng(2024))
    edges = np.array([0.5, 1, 2, 4, 8, 16, 32, 64, 90, 120, 150, 179], dtype=np.float64)
    got = oracle.count((ra, dec), edges).astype(np.float64)
    M = n * (n - 1) / 2
    full = np.concatenate([[0.0], edges, [180.0]])
    for k in range(full.size - 1):
        t1, t2 = math.radians(full[k]), math.radians(full[k + 1])
        p = math.sin(0.5 * (t1 + t2)) * math.sin(0.5 * (t2 - t1))   # = (cos t1 - cos t2)/2
        z = (got[k] - M * p) / math.sqrt(M * p * (1 - p))
        assert abs(z) < 5.0, (k, got[k], M * p, z)


# ----------------------------------------------------------- Landy-Szalay

def _ls_exact(DD, DR, RR, nD, nR):
    nDD = Fraction(nD * (nD - 1), 2)
    nDR = Fraction(nD * nR)
    nRR = Fraction(nR * (nR - 1), 2)
    out = []
    for a, b, c in zip(DD, DR, RR):
        dd, dr, rr = Fraction(int(a)) / nDD, Fraction(int(b)) / nDR, Fraction(int(c)) / nRR
        out.append((dd - 2 * dr + rr) / rr)
    return out


def test_wtheta_exact_rational_and_identities():
    rng = np.random.default_rng(9)
    nD, nR = 123_457, 998_001
    RR = rng.integers(1, 10**11, 40).astype(np.uint64)
    DD = rng.integers(0, 10**10, 40).astype(np.uint64)
    DR = rng.integers(0, 10**11, 40).astype(np.uint64)
    w = oracle.wtheta(DD, DR, RR, nD, nR)
    for got, want in zip(w, _ls_exact(DD, DR, RR, nD, nR)):
        assert abs(got - float(want)) <= 1e-13 * max(1.0, abs(float(want)))
    # equal normalised counts -> w = 0 exactly: with nD = nR = n, DD = RR = c and
    # DR = 2cn/(n-1) all three normalise to the same number; RR = 0 -> NaN
    nD = nR = 1001
    c = np.array([500, 0], dtype=np.uint64)
    w = oracle.wtheta(c, np.array([1001, 0], dtype=np.uint64), c, nD, nR)
    assert w[0] == 0.0 and math.isnan(w[1])


def _estimators_exact(DD, DR, RR, nD, nR):
    """The four estimators in exact rational arithmetic (textbook forms)."""
    nDD = Fraction(nD * (nD - 1), 2)
    nDR = Fraction(nD * nR)
    nRR = Fraction(nR * (nR - 1), 2)
    out = {0: [], 1: [], 2: [], 3: []}
    for a, b, c in zip(DD, DR, RR):
        dd, dr, rr = Fraction(int(a)) / nDD, Fraction(int(b)) / nDR, Fraction(int(c)) / nRR
        out[0].append((dd - 2 * dr + rr) / rr)
        out[1].append(dd / rr - 1)
        out[2].append(dd / dr - 1)
        out[3].append(dd * rr / (dr * dr) - 1)
    return out


def test_estimators_exact_rational_and_zero_for_proportional_counts():
    rng = np.random.default_rng(19)
    nD, nR = 54_321, 700_001
    DD = rng.integers(1, 10**10, 30).astype(np.uint64)
    DR = rng.integers(1, 10**11, 30).astype(np.uint64)
    RR = rng.integers(1, 10**11, 30).astype(np.uint64)
    want = _estimators_exact(DD, DR, RR, nD, nR)
    for kind in range(4):
        got = oracle.estimator(kind, DD, DR, RR, nD, nR)
        for g, wv in zip(got, want[kind]):
            assert abs(g - float(wv)) <= 1e-13 * max(1.0, abs(float(wv))), kind
    assert np.array_equal(oracle.estimator(0, DD, DR, RR, nD, nR), oracle.wtheta(DD, DR, RR, nD, nR))
    # counts proportional to the pair totals (an unclustered sky) give 0 for
    # every estimator: nD = nR = n, DD = RR = c, DR = 2cn/(n-1)
    n = 1001
    c = np.array([500, 1500], dtype=np.uint64)
    dr = np.array([1001, 3003], dtype=np.uint64)
    for kind in range(4):
        assert np.all(oracle.estimator(kind, c, dr, c, n, n) == 0.0), kind
    # natural ignores DR, Davis-Peebles ignores RR
    assert np.array_equal(oracle.estimator(1, DD, None, RR, nD, nR), oracle.estimator(1, DD, DR, RR, nD, nR))
    assert np.array_equal(oracle.estimator(2, DD, DR, None, nD, nR), oracle.estimator(2, DD, DR, RR, nD, nR))

