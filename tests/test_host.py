"""Host-side checks of libpc.so that need no GPU: the exported ABI, the host
tables (edges, guard band, cell table) and argument validation."""
import glob
import os
import re

import numpy as np
import pytest

import oracle
import synth
import paper_1208_3658_amd as pc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        names |= set(re.findall(r"\b(pc_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_library_loads_and_exports_every_declared_function():
    L = pc.lib()
    names = _declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert pc.pc_version().startswith("pc ")


EDGE_SETS = {
    "log_30": synth.log_edges(0.01, 10.0, 30),
    "log_40": synth.log_edges(0.01, 20.0, 40),
    "log_50": synth.log_edges(0.005, 30.0, 50),
    "paper_254": synth.log_edges(0.001, 90.0, 254),
    "linear_zero_180": synth.linear_edges(0.0, 180.0, 36),
    "linear_fine": synth.linear_edges(0.0, 10.0, 50),
    "tiny": np.array([1e-5, 2e-5, 1e-3, 0.5]),
}


@pytest.mark.parametrize("name", sorted(EDGE_SETS))
def test_chord2_edges_match_oracle_bitwise(name):
    e = EDGE_SETS[name]
    got = pc.pc_chord2_edges(e)
    want = oracle.chord2_edges(e)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


def _c32_variants(a64, b64):
    """binary32 squared chords as the kernel may form them: plain products and
    sums, and fused multiply-adds (exact product + sum, rounded once)."""
    a32 = a64.astype(np.float32)
    b32 = b64.astype(np.float32)
    d = (a32 - b32).astype(np.float32)
    plain = (d[:, 0] * d[:, 0]).astype(np.float32)
    plain = (plain + (d[:, 1] * d[:, 1]).astype(np.float32)).astype(np.float32)
    plain = (plain + (d[:, 2] * d[:, 2]).astype(np.float32)).astype(np.float32)
    dd = d.astype(np.float64)
    f = (dd[:, 0] * dd[:, 0]).astype(np.float32).astype(np.float64)
    f = (dd[:, 1] * dd[:, 1] + f).astype(np.float32).astype(np.float64)
    f = (dd[:, 2] * dd[:, 2] + f).astype(np.float32)
    return plain, f


def _c64(a, b):
    d = a - b
    c = d[:, 0] * d[:, 0]
    c = c + d[:, 1] * d[:, 1]
    c = c + d[:, 2] * d[:, 2]
    return c


def _pairs_near_edges(theta, per_edge=400, seed=1):
    """Point pairs whose separation is theta_k (1 + eps) for tiny eps, in
    random places and orientations on the sphere."""
    rng = np.random.default_rng(seed)
    ra1, dec1, ra2, dec2 = [], [], [], []
    for t in theta:
        if t <= 0 or t >= 179:
            continue
        eps = np.concatenate([rng.uniform(-1e-3, 1e-3, per_edge // 2),
                              rng.uniform(-1e-6, 1e-6, per_edge // 4),
                              rng.uniform(-1e-9, 1e-9, per_edge // 4)])
        r0 = rng.uniform(0, 360, eps.size)
        d0 = rng.uniform(-60, 60, eps.size)
        sep = t * (1.0 + eps)
        horiz = rng.random(eps.size) < 0.5
        ra1.append(r0)
        dec1.append(d0)
        # meridian offsets: exact separation; equatorial offsets: approximately
        ra2.append(np.where(horiz, r0 + sep, r0))
        dec2.append(np.where(horiz, 0.0 * d0, np.clip(d0 + sep, -90, 90)))
        dec1[-1] = np.where(horiz, 0.0 * d0, d0)
    return (np.concatenate(ra1), np.concatenate(dec1), np.concatenate(ra2), np.concatenate(dec2))


@pytest.mark.parametrize("name", sorted(EDGE_SETS))
def test_guard_band_separates_binary32_from_binary64_decisions(name):
    theta = EDGE_SETS[name]
    e = oracle.chord2_edges(theta)
    lo, hi = pc.pc_guard_band(theta)
    ra1, dec1, ra2, dec2 = _pairs_near_edges(theta)
    a = oracle.unit_vectors(ra1, dec1)
    b = oracle.unit_vectors(ra2, dec2)
    c64 = _c64(a, b)
    for c32 in _c32_variants(a, b):
        for k in range(e.size):
            above = c32 > hi[k]
            below = c32 < lo[k]
            assert np.all(c64[above] >= e[k]), (name, k)
            assert np.all(c64[below] < e[k]), (name, k)
    # the band is narrow: relative width at most ~0.6% for edges >= 0.001 deg
    pos = e > 1e-12
    assert np.all((hi[pos].astype(np.float64) - lo[pos]) / e[pos] < 0.2)
    assert np.all(hi >= lo)


def _emulate_kernel(theta, A, B=None):
    """Bin all pairs as the mixed kernel does (cell table + guard band +
    binary64 re-check), with emulated binary32 chords; returns counts."""
    info, ent = pc.pc_debug_lut32(theta)
    e64 = oracle.chord2_edges(theta)
    xa = oracle.unit_vectors(*A)
    if B is None:
        i, j = np.triu_indices(xa.shape[0], 1)
        a, b = xa[i], xa[j]
    else:
        xb = oracle.unit_vectors(*B)
        i, j = np.meshgrid(np.arange(xa.shape[0]), np.arange(xb.shape[0]), indexing="ij")
        a, b = xa[i.ravel()], xb[j.ravel()]
    c64 = _c64(a, b)
    counts = []
    for c32 in _c32_variants(a, b):
        key = np.clip(c32.view(np.uint32), info["clamp_lo"], info["clamp_hi"])
        cell = (key >> info["shift"]) - (info["clamp_lo"] >> info["shift"])
        E = ent[cell]
        lo = E[:, 1].view(np.float32)
        hi = E[:, 2].view(np.float32)
        # as the kernel does it: d = RN32(hi - c); off_lo, plus one row when
        # the sign bit of d is set; a chord is flagged for the re-check when
        # max(bits(d) - wbits, 0) = 0, and the re-check moves the flagged
        # chords that lie in the band (lo <= c <= hi) to their binary64 row
        with np.errstate(invalid="ignore", over="ignore"):
            d = (hi - c32).astype(np.float32)
        bd = d.view(np.uint32)
        row = (E[:, 0] + (bd >> 31) * info["row_bytes"]) // info["row_bytes"]
        flagged = bd <= E[:, 3]
        band = (c32 >= lo) & ~(c32 > hi)
        assert np.all(flagged[band]), "an in-band chord was not flagged"
        assert np.array_equal(row[~band], np.where(c32 > hi, E[:, 0] + info["row_bytes"], E[:, 0])[~band]
                              // info["row_bytes"])
        row = row.astype(np.int64)
        fix = flagged & band
        row[fix] = np.searchsorted(e64, c64[fix], side="right")
        counts.append(np.bincount(row, minlength=theta.size + 1).astype(np.uint64))
    return counts


@pytest.mark.parametrize("name", ["log_30", "paper_254", "linear_zero_180", "linear_fine", "tiny"])
def test_cell_table_logic_reproduces_oracle(name):
    theta = EDGE_SETS[name]
    c = synth.config_small(scale=0.06)                  # 600 clustered + 600 random
    A = c["D"]
    if name in ("linear_zero_180",):
        A = synth.uniform_patch(700, synth.FULL_SKY, np.random.default_rng(4))
    want = oracle.count(A, theta)
    for got in _emulate_kernel(theta, A):
        assert got.tolist() == want.tolist()
    want = oracle.count(A, theta, B=c["R"], auto=False)
    for got in _emulate_kernel(theta, A, c["R"]):
        assert got.tolist() == want.tolist()


def _gram_c32_variants(a64, b64, rng):
    """binary32 squared chords in Gram form as the matrix cores and the vector
    path form them: both points centred on o (within half the pair's chord of
    a, or of b), rounded to binary32, c = |b'|^2 + |a'|^2 + sum_k a'_k (-2 b'_k)
    summed in several orders (one rounding at the end; a rounding after every
    product and addition, forward and backward; the vector path's fused
    multiply-add chain with |a'|^2 added exactly)."""
    s = np.sqrt(_c64(a64, b64))
    w = rng.normal(size=a64.shape)
    w /= np.linalg.norm(w, axis=1)[:, None]
    r = (0.5 * s * rng.uniform(0.0, 0.999, s.size))[:, None]
    out = []
    for near in (a64, b64):
        o = near + r * w
        A = (a64 - o).astype(np.float32)
        B = (b64 - o).astype(np.float32)
        f = lambda x: x.astype(np.float32)
        na = f(f(f(A[:, 0] * A[:, 0]) + f(A[:, 1] * A[:, 1])) + f(A[:, 2] * A[:, 2]))
        nb = f(f(f(B[:, 0] * B[:, 0]) + f(B[:, 1] * B[:, 1])) + f(B[:, 2] * B[:, 2]))
        terms = [nb.astype(np.float64)] + [A[:, k].astype(np.float64) * (-2.0 * B[:, k].astype(np.float64))
                                           for k in range(3)] + [na.astype(np.float64)]
        out.append(f(sum(terms)))                          # exact sum, one rounding
        acc = f(terms[0])
        for t in terms[1:]:
            acc = f(acc + f(t))                            # rounded products and sums
        out.append(acc)
        acc = f(terms[-1])
        for t in terms[-2::-1]:
            acc = f(acc + f(t))
        out.append(acc)
        # the vector path's order: fused multiply-adds of z, y, x from
        # |b'|^2 (each product exact, one rounding each), then |a'|^2 added
        # exactly (the kernel compares the partial sum with thresholds
        # shifted by |a'|^2)
        acc = nb
        for k in (2, 1, 0):
            acc = f(A[:, k].astype(np.float64) * (-2.0 * B[:, k].astype(np.float64)) + acc.astype(np.float64))
        out.append(na.astype(np.float64) + acc.astype(np.float64))
    return out


@pytest.mark.parametrize("name", sorted(EDGE_SETS))
def test_gram_guard_band_separates_matrix_core_chords(name):
    """The matrix-core path's band holds for chords formed from coordinates
    centred within half the chord of either point."""
    theta = EDGE_SETS[name]
    e = oracle.chord2_edges(theta)
    lo, hi = pc.pc_guard_band(theta, gram=True)
    ra1, dec1, ra2, dec2 = _pairs_near_edges(theta, seed=7)
    a = oracle.unit_vectors(ra1, dec1)
    b = oracle.unit_vectors(ra2, dec2)
    c64 = _c64(a, b)
    rng = np.random.default_rng(11)
    for c32 in _gram_c32_variants(a, b, rng):
        for k in range(e.size):
            assert np.all(c64[c32 > hi[k]] >= e[k]), (name, k)
            assert np.all(c64[c32 < lo[k]] < e[k]), (name, k)
    # relative error bound: the band is narrow at every scale
    pos = e > 1e-30
    assert np.all((hi[pos].astype(np.float64) - lo[pos]) / e[pos] < 1e-4)
    assert np.all(hi >= lo)


def _few_edge_rows(c32, c64, e64, lo, hi, k0, m):
    """Rows as the few-edge binning forms them: k0 + #{k < m : c32 > hi[k0+k]},
    and the binary64 row for chords inside one of those m bands."""
    row = np.full(c32.size, k0, dtype=np.int64)
    band = np.zeros(c32.size, dtype=bool)
    for k in range(k0, k0 + m):
        gt = c32 > hi[k]
        row += gt
        band |= ~gt & (c32 >= lo[k])
    row[band] = np.searchsorted(e64, c64[band], side="right")
    return row


@pytest.mark.parametrize("gram", [False, True])
@pytest.mark.parametrize("name", ["log_40", "paper_254", "linear_zero_180", "tiny"])
def test_few_edge_binning_reproduces_the_oracle(name, gram):
    """Few-edge binning (compare with the m <= 3 edges inside a pair's proven
    chord interval, re-check in-band chords) on emulated binary32 chords --
    plain differences, or tile-centred Gram chords with the matrix-core band --
    gives the binary64 bins, for every interval of 1-3 consecutive edges that
    holds the exact chord."""
    theta = EDGE_SETS[name]
    e64 = oracle.chord2_edges(theta)
    lo, hi = pc.pc_guard_band(theta, gram=gram)
    ra1, dec1, ra2, dec2 = _pairs_near_edges(theta, per_edge=200, seed=3)
    a = oracle.unit_vectors(ra1, dec1)
    b = oracle.unit_vectors(ra2, dec2)
    c64 = _c64(a, b)
    want = np.searchsorted(e64, c64, side="right")
    rng = np.random.default_rng(5)
    variants = _gram_c32_variants(a, b, rng) if gram else list(_c32_variants(a, b))
    checked = 0
    for c32 in variants:
        for m in (1, 2, 3):
            for shift in range(m + 1):
                # intervals [k0, k0 + m] that contain each pair's exact row
                k0 = want - shift
                ok = (k0 >= 0) & (k0 + m <= e64.size)
                for k in np.unique(k0[ok]):
                    sel = ok & (k0 == k)
                    got = _few_edge_rows(c32[sel], c64[sel], e64, lo, hi, int(k), m)
                    assert np.array_equal(got, want[sel]), (name, gram, m, int(k))
                    checked += int(sel.sum())
    assert checked > 0


def _f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def _fma32(a, b, c):
    """binary32 fused multiply-add, emulated: the product of two binary32
    values is exact in binary64; the sum is rounded to binary64, then to
    binary32 (a double rounding, far below the thresholds' margins)."""
    return _f32(np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64))


def _fused_d_variants(a64, b64, h_ref, gram, rng):
    """d = h_ref - c as the vector few-edge paths form it, in one chain of
    binary32 roundings: differences of the binary32 unit vectors and three
    fused multiply-adds (x, y, z and z, y, x), or tile-centred Gram chords
    (centre within half the chord of either point): na, bw by fused
    multiply-adds, S = h - na, T = S - bw, then the products 2 a'_k b'_k."""
    out = []
    if not gram:
        s = _f32(a64.astype(np.float32) - b64.astype(np.float32))
        for order in ((0, 1, 2), (2, 1, 0)):
            d = _f32(h_ref)
            for k in order:
                d = _fma32(-s[:, k], s[:, k], d)
            out.append(d)
        return out
    sc = np.sqrt(_c64(a64, b64))
    w = rng.normal(size=a64.shape)
    w /= np.linalg.norm(w, axis=1)[:, None]
    r = (0.5 * sc * rng.uniform(0.0, 0.999, sc.size))[:, None]
    for near in (a64, b64):
        o = near + r * w
        A = (a64 - o).astype(np.float32)
        B = (b64 - o).astype(np.float32)
        na = _fma32(A[:, 2], A[:, 2], _fma32(A[:, 1], A[:, 1], _f32(A[:, 0].astype(np.float64) ** 2)))
        bw = _fma32(B[:, 2], B[:, 2], _fma32(B[:, 1], B[:, 1], _f32(B[:, 0].astype(np.float64) ** 2)))
        T = _f32(_f32(np.float64(h_ref) - na) - bw.astype(np.float64))
        d = T
        for k in (2, 1, 0):
            d = _fma32(-A[:, k], -2.0 * B[:, k], d)
        out.append(d)
    return out


def _fused_d_edge(d_ref, h, k, ref):
    """d of edge k from the reference edge's d: RN32(d_ref + RN32(h_k - h_ref))."""
    if k == ref:
        return d_ref
    delta = _f32(np.float64(h[k]) - np.float64(h[ref]))
    return _f32(d_ref.astype(np.float64) + np.float64(delta))


@pytest.mark.parametrize("gram", [False, True])
@pytest.mark.parametrize("name", sorted(EDGE_SETS))
def test_fused_thresholds_separate_binary32_from_binary64_decisions(name, gram):
    """The vector few-edge paths' fused differences d = h - c (for the
    reference edge, and for an edge one or two above it through RN32(h_k -
    h_ref)): d < 0 only for chords at or above the edge in binary64, d > w
    only for chords below it."""
    theta = EDGE_SETS[name]
    e = oracle.chord2_edges(theta)
    h, w = pc.pc_debug_fused_band(theta, gram=gram)
    ra1, dec1, ra2, dec2 = _pairs_near_edges(theta, per_edge=200, seed=13)
    a = oracle.unit_vectors(ra1, dec1)
    b = oracle.unit_vectors(ra2, dec2)
    c64 = _c64(a, b)
    rng = np.random.default_rng(17)
    near = np.searchsorted(e, c64)  # pairs are generated around each edge
    checked = 0
    for k in range(e.size):
        if e[k] <= 0:
            assert h[k] == -np.finfo(np.float32).max and w[k] == 0.0
            continue
        sel = (near == k) | (near == k + 1)
        if not np.any(sel):
            continue
        for ref in range(max(k - 2, 0), k + 1):
            if e[ref] <= 0:
                continue  # an edge at 0 is never in a few-edge item
            for d_ref in _fused_d_variants(a[sel], b[sel], h[ref], gram, rng):
                d = _fused_d_edge(d_ref, h, k, ref)
                assert np.all(c64[sel][d < 0] >= e[k]), (name, gram, k, ref)
                assert np.all(c64[sel][d > w[k]] < e[k]), (name, gram, k, ref)
                checked += int(sel.sum())
    assert checked > 0
    # the flag window is as narrow as the guard band of the same chords
    lo, hi = pc.pc_guard_band(theta, gram=gram)
    fin = np.isfinite(lo) & (e > 0)
    assert np.all(w[fin] <= 2.0 * (hi[fin].astype(np.float64) - lo[fin]))


@pytest.mark.parametrize("gram", [False, True])
@pytest.mark.parametrize("name", ["log_40", "paper_254", "linear_zero_180", "tiny"])
def test_fused_few_edge_binning_reproduces_the_oracle(name, gram):
    """Few-edge binning as the vector paths do it: for an interval of m <= 3
    consecutive edges holding the exact chord, the row is k0 + #{t : d_t < 0}
    with d_t from the smallest edge's fused difference, and a chord with 0 <=
    d_t <= w_t for some t takes its binary64 row.  (An edge at 0 is never in
    such an interval: every chord lies above it.)"""
    theta = EDGE_SETS[name]
    e64 = oracle.chord2_edges(theta)
    h, w = pc.pc_debug_fused_band(theta, gram=gram)
    wb = w.view(np.uint32)
    ra1, dec1, ra2, dec2 = _pairs_near_edges(theta, per_edge=160, seed=23)
    a = oracle.unit_vectors(ra1, dec1)
    b = oracle.unit_vectors(ra2, dec2)
    c64 = _c64(a, b)
    want = np.searchsorted(e64, c64, side="right")
    rng = np.random.default_rng(29)
    checked = 0
    for m in (1, 2, 3):
        for shift in range(m + 1):
            k0 = want - shift
            ok = (k0 >= 0) & (k0 + m <= e64.size)
            ok &= e64[np.clip(k0, 0, e64.size - 1)] > 0
            for k in np.unique(k0[ok]):
                sel = ok & (k0 == k)
                ref = int(k)
                for d_ref in _fused_d_variants(a[sel], b[sel], h[ref], gram, rng):
                    row = np.full(d_ref.size, int(k), dtype=np.int64)
                    flag = np.zeros(d_ref.size, dtype=bool)
                    for t in range(int(k), int(k) + m):
                        d = _fused_d_edge(d_ref, h, t, ref)
                        bits = d.view(np.uint32)
                        row += bits >> 31
                        flag |= bits <= wb[t]
                    row[flag] = np.searchsorted(e64, c64[sel][flag], side="right")
                    assert np.array_equal(row, want[sel]), (name, gram, m, int(k))
                    checked += int(sel.sum())
    assert checked > 0


@pytest.mark.parametrize("name", sorted(EDGE_SETS))
def test_cell_entries_hold_band_width_bits(name):
    """A cell entry is (off_lo, lo, hi, wbits): a finite hi only in one-band
    cells, with wbits the bits of RN32(hi - lo); no band: lo = hi = +inf,
    wbits 0; several bands: lo = -inf, hi = +inf, wbits all ones."""
    info, ent = pc.pc_debug_lut32(EDGE_SETS[name])
    lo = ent[:, 1].view(np.float32)
    hi = ent[:, 2].view(np.float32)
    fin = np.isfinite(hi)
    assert np.array_equal(ent[fin, 3], (hi[fin] - lo[fin]).astype(np.float32).view(np.uint32))
    assert np.all(hi[~fin] == np.inf)
    none = ~fin & (lo == np.inf)
    multi = ~fin & (lo == -np.inf)
    assert np.all(none | multi | fin)
    assert np.all(ent[none, 3] == 0) and np.all(ent[multi, 3] == 0xFFFFFFFF)
    assert int(np.sum(multi)) == info["multi"]


def test_wtheta_matches_oracle_bitwise():
    rng = np.random.default_rng(2)
    DD = rng.integers(0, 10**12, 50).astype(np.uint64)
    DR = rng.integers(0, 10**12, 50).astype(np.uint64)
    RR = rng.integers(1, 10**12, 50).astype(np.uint64)
    RR[3] = 0
    got = pc.pc_wtheta(DD, DR, RR, 1_000_003, 2_000_001)
    want = oracle.wtheta(DD, DR, RR, 1_000_003, 2_000_001)
    assert np.array_equal(np.isnan(got), np.isnan(want))
    f = ~np.isnan(want)
    assert np.array_equal(got[f].view(np.uint64), want[f].view(np.uint64))


def test_estimators_match_oracle_bitwise():
    rng = np.random.default_rng(23)
    DD = rng.integers(0, 10**12, 60).astype(np.uint64)
    DR = rng.integers(0, 10**12, 60).astype(np.uint64)
    RR = rng.integers(0, 10**12, 60).astype(np.uint64)
    DR[5] = 0
    RR[7] = 0
    for kind in range(4):
        got = pc.pc_estimator(kind, DD, DR, RR, 777_777, 3_000_001)
        want = oracle.estimator(kind, DD, DR, RR, 777_777, 3_000_001)
        assert np.array_equal(np.isnan(got), np.isnan(want)), kind
        f = ~np.isnan(want)
        assert np.array_equal(got[f].view(np.uint64), want[f].view(np.uint64)), kind
    assert np.array_equal(pc.pc_estimator(1, DD, None, RR, 10, 20), oracle.estimator(1, DD, None, RR, 10, 20))
    with pytest.raises(pc.PcError):
        pc.pc_estimator(4, DD, DR, RR, 10, 20)
    with pytest.raises(pc.PcError):
        pc.pc_estimator(3, DD, None, RR, 10, 20)


@pytest.mark.parametrize("args,fragment", [
    (((np.zeros(3), np.array([0.0, 91.0, 0.0])), [1.0, 2.0]), "Dec"),
    (((np.array([0.0, np.nan]), np.zeros(2)), [1.0, 2.0]), "finite"),
    (((np.zeros(3), np.zeros(3)), [2.0, 1.0]), "increasing"),
    (((np.zeros(3), np.zeros(3)), [1.0]), ">= 2"),
    (((np.zeros(3), np.zeros(3)), [1.0, 181.0]), "[0, 180]"),
    (((np.zeros(3), np.zeros(3)), [-1.0, 1.0]), "[0, 180]"),
    (((np.zeros(3), np.zeros(3)), list(np.linspace(0.0, 90.0, 1025))), "<= 1024"),
])
def test_invalid_arguments_rejected_before_any_device_work(args, fragment):
    with pytest.raises(pc.PcError) as ex:
        pc.pc_count(*args)
    assert ex.value.code == pc.PC_ERR_INVALID
    assert fragment in str(ex.value)


def test_invalid_row_range_and_wtheta_arguments():
    A = (np.zeros(5), np.zeros(5))
    with pytest.raises(pc.PcError) as ex:
        pc.pc_count_ex(A, [1.0, 2.0], rows=(3, 9))
    assert ex.value.code == pc.PC_ERR_INVALID
    with pytest.raises(pc.PcError):
        pc.pc_wtheta([1], [1], [1], 1, 5)


def test_server_config_is_validated_before_the_device():
    with pytest.raises(pc.PcError) as ex:
        pc.Server({"no_such_key": 1})
    assert ex.value.code == pc.PC_ERR_INVALID
    with pytest.raises(pc.PcError) as ex:
        pc.Server({"mode": 5})
    assert ex.value.code == pc.PC_ERR_INVALID


def test_tuning_cache_file_is_validated(tmp_path):
    good = tmp_path / "tune.jsonl"
    good.write_text('{"device": "gfx950:256", "edges_class": 6, "pairs_class": 40, "cols": 16, "chunk": 4, '
                    '"matrix_cores": 0, "kernel_ms": 70.1}\n\n'
                    '{"device": "gfx950:256", "edges_class": 5, "pairs_class": 45, "cols": 32, "chunk": 8, '
                    '"matrix_cores": 1, "kernel_ms": 500.0}\n')
    pc.pc_autotune_load(good)
    for bad in ['{"device": "x", "edges_class": 6, "pairs_class": 40, "cols": 12, "chunk": 4, "matrix_cores": 0}',
                '{"device": "x", "edges_class": 6, "pairs_class": 40, "cols": 16, "chunk": 0, "matrix_cores": 0}',
                '{"device": "x", "edges_class": 6, "cols": 16, "chunk": 4, "matrix_cores": 0}',
                '{"device": "x", "edges_class": 6, "pairs_class": 40, "cols": 16, "chunk": 4, "matrix_cores": 2}']:
        f = tmp_path / "bad.jsonl"
        f.write_text(bad + "\n")
        with pytest.raises(pc.PcError) as ex:
            pc.pc_autotune_load(f)
        assert ex.value.code == pc.PC_ERR_INVALID
    with pytest.raises(pc.PcError):
        pc.pc_autotune_load(tmp_path / "missing.jsonl")



@pytest.mark.parametrize("change,fragment", [
    ({"theta": 0.0}, "theta_max"),
    ({"theta": float("nan")}, "theta_max"),
    ({"n_gal": -1.0}, "n_gal"),
    ({"grid": (0.0, 0.0, 0.0, 1.0, 4, 4)}, "spacings"),
    ({"grid": (0.0, float("inf"), 1.0, 1.0, 4, 4)}, "grid origin"),
    ({"grid": (0.0, 0.0, 1.0, 1.0, -1, 4)}, "grid size"),
    ({"grid": (0.0, 0.0, 1.0, 1.0, 65536, 65536)}, "grid size"),
    ({"nan_at": 3}, "non-finite"),
])
def test_aperture_arguments_rejected_before_any_device_work(change, fragment):
    x = np.linspace(0.0, 5.0, 10)
    cat = [x, x[::-1].copy(), np.full(10, 0.1), np.full(10, -0.1)]
    if "nan_at" in change:
        cat[1][change["nan_at"]] = np.nan
    grid = change.get("grid", (0.0, 0.0, 1.0, 1.0, 4, 4))
    with pytest.raises(pc.PcError) as ei:
        pc.pc_aperture_mass(tuple(cat), grid, change.get("theta", 2.0), change.get("n_gal", 35.0))
    assert ei.value.code == pc.PC_ERR_INVALID
    assert fragment in str(ei.value)


def test_shear_catalogue_recipe():
    (x, y, e1, e2), side = synth.shear_catalog(20000, density=35.0, config=9)
    assert side == pytest.approx((20000 / 35.0) ** 0.5)
    assert x.min() >= 0.0 and x.max() < side and y.min() >= 0.0 and y.max() < side
    assert np.all(np.isfinite(e1)) and np.all(np.isfinite(e2))
    again = synth.shear_catalog(20000, density=35.0, config=9)[0]
    assert all(np.array_equal(a, b) for a, b in zip((x, y, e1, e2), again))
    g = synth.field_grid(side, 64)
    assert g[4] == g[5] == 64 and g[0] == pytest.approx(0.5 * side / 64)


def test_aperture_filter_table_matches_the_definition():
    """The map kernel reads Eq. 4's Q(x) from a table (1024 cubic cells over
    [0, 1]); evaluated with the kernel's binary32 steps it stays within
    2.5e-7 of the oracle's binary64 Q on 2e6 + seeded points -- far inside the
    map tolerance (1e-4 of sum Q|eps|), and of the size of Q' times the
    binary32 rounding of x itself (the steep logistic near x = 0.04)."""
    rng = np.random.default_rng(404)
    x = np.concatenate([np.linspace(0.0, 1.0, 400_001), rng.random(100_000), [0.0, 1e-12, 0.5, 1.0]])
    q = pc.pc_debug_ap_filter(x)
    ref = np.array([oracle.q_nfw(v) for v in x])
    err = np.abs(q - ref)
    assert err.max() <= 2.5e-7, (err.max(), x[err.argmax()])
    # away from the steep part the error is a few binary32 ulps of Q
    flat = (x > 0.1) & (x < 0.85)
    assert np.all(err[flat] <= 8 * 2.0 ** -24 * np.maximum(ref[flat], 1e-3))


def test_bin_presets():
    """The paper's presets (Sec. 2.1): limits and evenly spaced, natural-log or
    log10 bins, by count or by width in the preset's scale."""
    e = pc.pc_bin_edges(pc.PC_BINS_LN, 0.01, 20.0, n_bins=40)
    assert e.size == 41 and e[0] == 0.01 and e[-1] == 20.0
    assert np.allclose(e, synth.log_edges(0.01, 20.0, 40), rtol=1e-14, atol=0)
    assert np.all(np.diff(np.log(e)) > 0) and np.allclose(np.diff(np.log(e)), np.log(2000.0) / 40, rtol=1e-9)
    # equal steps in log10 theta give the same edges as in ln theta
    assert np.allclose(pc.pc_bin_edges(pc.PC_BINS_LOG10, 0.01, 20.0, n_bins=40), e, rtol=1e-14, atol=0)
    # by width: a decade split in 0.1-decade bins; ln widths; even widths, last bin narrower
    d = pc.pc_bin_edges(pc.PC_BINS_LOG10, 0.1, 10.0, width=0.1)
    assert d.size == 21 and np.allclose(np.log10(d), np.linspace(-1, 1, 21), atol=1e-14)
    assert pc.pc_bin_edges(pc.PC_BINS_LN, 0.1, 10.0, width=np.log(10.0) / 10).size == 21
    lin = pc.pc_bin_edges(pc.PC_BINS_EVEN, 0.0, 30.0, width=0.6)
    assert lin.size == 51 and np.allclose(lin, synth.linear_edges(0.0, 30.0, 50), rtol=0, atol=1e-12)
    odd = pc.pc_bin_edges(pc.PC_BINS_EVEN, 0.0, 1.0, width=0.3)
    assert odd.tolist() == [0.0, 0.3, 0.6, 0.8999999999999999, 1.0] or odd.tolist() == [0.0, 0.3, 0.6, 0.9, 1.0]
    # the edges are usable as they are
    assert pc.pc_chord2_edges(e).size == 41
    for bad in [dict(preset=pc.PC_BINS_LN, lo_deg=0.0, hi_deg=1.0, n_bins=4),
                dict(preset=pc.PC_BINS_EVEN, lo_deg=2.0, hi_deg=1.0, n_bins=4),
                dict(preset=pc.PC_BINS_EVEN, lo_deg=0.0, hi_deg=181.0, n_bins=4),
                dict(preset=pc.PC_BINS_EVEN, lo_deg=0.0, hi_deg=10.0, n_bins=2000),
                dict(preset=pc.PC_BINS_EVEN, lo_deg=0.0, hi_deg=10.0),
                dict(preset=7, lo_deg=0.0, hi_deg=10.0, n_bins=4)]:
        with pytest.raises(pc.PcError) as ex:
            pc.pc_bin_edges(**bad)
        assert ex.value.code == pc.PC_ERR_INVALID
