"""GPU parity: libpc.so on gfx950 against the CPU oracle, through the C ABI.

Counts must be bit-exact (integers); unit vectors bit-exact; w(theta) within
1e-12 relative.  Every kernel is checked: mixed binary32 + binary64 re-check
(with and without the matrix-core path) and plain binary64."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
import paper_1208_3658_amd as pc  # noqa: E402

pytestmark = pytest.mark.gpu
MODES = [pc.PC_MIXED, pc.PC_MIXED | pc.PC_MATRIX_CORES, pc.PC_FP64_PLAIN]


def dev(cat):
    return tuple(torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in cat)


def test_unit_vectors_bitwise():
    rng = np.random.default_rng(8)
    ra = np.concatenate([[0, 90, 180, 270, 360, -90, -720.5, 1e6 + 0.25, 45, 12.3456789, 359.999999999],
                         rng.uniform(-1000, 1000, 3000)])
    dec = np.concatenate([[0, 90, -90, 45, -45, 0, 89.9999999, -89.9999999, 30, 0.001, -0.001],
                          rng.uniform(-90, 90, 3000)])
    want = oracle.unit_vectors(ra, dec)
    for cat in [(ra, dec), dev((ra, dec))]:
        x64, x32 = pc.pc_unit_vectors(cat)
        assert np.array_equal(x64.view(np.uint64), want.view(np.uint64))
        assert np.array_equal(x32.view(np.uint32), want.astype(np.float32).view(np.uint32))


@pytest.mark.parametrize("mode", MODES)
def test_small_config_dd_dr_rr_and_wtheta(mode):
    c = synth.config_small(scale=0.3)                  # 3,000 clustered + 3,000 random
    D, R, e = c["D"], c["R"], c["edges"]
    dd, dr, rr = pc.pc_count_batch([{"A": dev(D), "edges": e}, {"A": dev(D), "B": dev(R), "edges": e, "auto": False},
                                    {"A": dev(R), "edges": e}], mode=mode)
    odd, odr, orr = oracle.count(D, e), oracle.count(D, e, B=R, auto=False), oracle.count(R, e)
    assert dd.tolist() == odd.tolist()
    assert dr.tolist() == odr.tolist()
    assert rr.tolist() == orr.tolist()
    nD, nR = D[0].size, R[0].size
    w = pc.pc_wtheta(dd[1:-1], dr[1:-1], rr[1:-1], nD, nR)
    ow = oracle.wtheta(odd[1:-1], odr[1:-1], orr[1:-1], nD, nR)
    f = ~np.isnan(ow)
    assert np.array_equal(np.isnan(w), np.isnan(ow))
    assert np.all(np.abs(w[f] - ow[f]) <= 1e-12 * np.maximum(1.0, np.abs(ow[f])))


SIZES = [0, 1, 2, 3, 63, 64, 65, 255, 256, 257, 511, 513, 1000, 2049]


@pytest.mark.parametrize("mode", MODES)
def test_ragged_sizes_auto_and_cross(mode):
    rng = np.random.default_rng(5)
    e = synth.log_edges(0.05, 8.0, 12)
    patch = synth.centred_patch(12.0)
    for n in SIZES:
        A = synth.uniform_patch(n, patch, rng) if n else (np.zeros(0), np.zeros(0))
        got = pc.pc_count_ex(dev(A) if n else A, e, mode=mode)
        assert got.tolist() == oracle.count(A, e).tolist(), n
        assert int(got.sum()) == n * (n - 1) // 2
        nb = (n * 7) % 300 + 1
        B = synth.uniform_patch(nb, patch, rng)
        got = pc.pc_count_ex(A, e, B=dev(B), auto=False, mode=mode)
        assert got.tolist() == oracle.count(A, e, B=B, auto=False).tolist(), (n, nb)
        assert int(got.sum()) == n * nb


@pytest.mark.parametrize("mode", MODES)
def test_row_ranges(mode):
    c = synth.config_small(scale=0.2)
    D, R, e = c["D"], c["R"], c["edges"]
    n = D[0].size
    Dd, Rd = dev(D), dev(R)
    cuts = [0, 1, 300, 301, 1777, n]
    tot_a = np.zeros(e.size + 1, dtype=np.uint64)
    tot_c = np.zeros(e.size + 1, dtype=np.uint64)
    for a, b in zip(cuts[:-1], cuts[1:]):
        ga = pc.pc_count_ex(Dd, e, rows=(a, b), mode=mode)
        assert ga.tolist() == oracle.count(D, e, rows=(a, b)).tolist(), (a, b)
        gc = pc.pc_count_ex(Dd, e, B=Rd, auto=False, rows=(a, b), mode=mode)
        assert gc.tolist() == oracle.count(D, e, B=R, auto=False, rows=(a, b)).tolist(), (a, b)
        tot_a += ga
        tot_c += gc
    assert tot_a.tolist() == pc.pc_count_ex(Dd, e, mode=mode).tolist()
    assert tot_c.tolist() == pc.pc_count_ex(Dd, e, B=Rd, auto=False, mode=mode).tolist()


@pytest.mark.parametrize("mode", MODES)
def test_batch_with_mixed_edge_sets_equals_single_jobs(mode):
    rng = np.random.default_rng(12)
    A = synth.neyman_scott(150, 20, 0.2, synth.Patch(0, 90, 0, 90), rng)
    B = synth.uniform_patch(2500, synth.Patch(0, 90, 0, 90), rng)
    S = synth.uniform_patch(1200, synth.FULL_SKY, rng)
    sets = [synth.log_edges(0.001, 90.0, 254), synth.linear_edges(0.0, 30.0, 50), synth.log_edges(0.01, 10, 30),
            synth.linear_edges(0.0, 180.0, 36)]
    jobs = [{"A": dev(A), "edges": sets[0]},
            {"A": dev(A), "B": dev(B), "edges": sets[1], "auto": False},
            {"A": dev(B), "edges": sets[2], "rows": (100, 2000)},
            {"A": dev(S), "edges": sets[3]},
            {"A": dev(A), "edges": sets[1]}]
    got = pc.pc_count_batch(jobs, mode=mode)
    want = [oracle.count(A, sets[0]), oracle.count(A, sets[1], B=B, auto=False),
            oracle.count(B, sets[2], rows=(100, 2000)), oracle.count(S, sets[3]), oracle.count(A, sets[1])]
    for g, w in zip(got, want):
        assert g.tolist() == w.tolist()
    single = pc.pc_count_ex(dev(A), sets[0], mode=mode)
    assert single.tolist() == got[0].tolist()


def _near_edge_catalogue(theta, per_edge=24, seed=3):
    """Points placed so that many pairs sit within a few binary32 ulps of
    the edges: pairs on a meridian separated by theta_k (1 + eps)."""
    rng = np.random.default_rng(seed)
    ra, dec = [], []
    for t in theta:
        if not (0 < t < 150):
            continue
        for s in range(per_edge):
            r0 = rng.uniform(0, 360)
            d0 = rng.uniform(-60, 60 - t)
            eps = rng.choice([0.0, 1e-12, -1e-12, 1e-9, -1e-9, 3e-8, -3e-8, 1e-7, -1e-7, 1e-6, -1e-6, 1e-4])
            ra += [r0, r0]
            dec += [d0, d0 + t * (1 + eps)]
    return np.array(ra), np.array(dec)


@pytest.mark.parametrize("mode", MODES)
def test_adversarial_near_edge_pairs_exact(mode):
    for theta in [synth.log_edges(0.01, 20.0, 40), synth.linear_edges(0.0, 60.0, 30)]:
        A = _near_edge_catalogue(theta)
        got = pc.pc_count_ex(dev(A), theta, mode=mode)
        assert got.tolist() == oracle.count(A, theta).tolist()
        # pairs placed at the edges land in the guard bands: the mixed kernel
        # re-checks them in binary64; the binary64 kernel has nothing to re-check
        rk = pc.pc_debug_last_rechecks()
        n = A[0].size
        if mode == pc.PC_FP64_PLAIN:
            assert rk == 0
        else:
            assert 0 < rk <= n * (n - 1) // 2


def test_antipodes_poles_duplicates_full_sky():
    e = synth.linear_edges(0.0, 180.0, 18)
    ra = np.array([0, 180, 0, 0, 33, 33, 90, 270, 10, 10] * 20, dtype=np.float64)
    dec = np.array([0, 0, 90, -90, 45, 45, 0, 0, -30, 30] * 20, dtype=np.float64)
    for mode in MODES:
        got = pc.pc_count_ex(dev((ra, dec)), e, mode=mode)
        assert got.tolist() == oracle.count((ra, dec), e).tolist()


def test_resident_handles_and_host_inputs():
    c = synth.config_small(scale=0.1)
    D, R, e = c["D"], c["R"], c["edges"]
    hD = pc.pc_catalog_upload(dev(D))
    hR = pc.pc_catalog_upload(R)                      # host arrays
    try:
        assert pc.pc_count_h(hD, e).tolist() == oracle.count(D, e).tolist()
        assert pc.pc_count_h(hD, e, hB=hR, auto=False).tolist() == oracle.count(D, e, B=R, auto=False).tolist()
        assert pc.pc_count_h(hR, e, mode=pc.PC_FP64_PLAIN).tolist() == oracle.count(R, e).tolist()
    finally:
        pc.pc_catalog_release(hD)
        pc.pc_catalog_release(hR)
    with pytest.raises(pc.PcError):
        pc.pc_count_h(hD, e)


def test_invalid_device_input_reported():
    ra = torch.zeros(100, dtype=torch.float64, device="cuda")
    dec = torch.zeros(100, dtype=torch.float64, device="cuda")
    dec[17] = 95.0
    with pytest.raises(pc.PcError) as ex:
        pc.pc_count((ra, dec), [1.0, 2.0])
    assert ex.value.code == pc.PC_ERR_INVALID
    dec[17] = float("nan")
    with pytest.raises(pc.PcError):
        pc.pc_count((ra, dec), [1.0, 2.0])


def test_repeatable_counts():
    # 20 runs cycling through the kernels and work distributions (mixed,
    # matrix cores, every pair visited, binary64; the tuner's 18 launch
    # shapes are compared inside pc_autotune): integer counts, so any race
    # between waves would show as a difference
    c = synth.config_small(scale=0.5)
    D, e = dev(c["D"]), c["edges"]
    first = pc.pc_count(D, e)
    modes = [pc.PC_MIXED, pc.PC_MIXED | pc.PC_MATRIX_CORES, pc.PC_MIXED | pc.PC_NO_PRUNE, pc.PC_FP64_PLAIN]
    for k in range(20):
        assert pc.pc_count_ex(D, e, mode=modes[k % 4]).tolist() == first.tolist(), k


def test_1m_config_sampled_rows_and_decompositions():
    """The 1M-point configuration at full size, in the launch bench.py times:
    exact totals, both kernels identical, sampled rows against the oracle,
    and a row decomposition that must add up to the full count."""
    c = synth.config_1m()
    D, R, e = c["D"], c["R"], c["edges"]
    n = D[0].size
    Dd, Rd = dev(D), dev(R)
    jobs = [{"A": Dd, "edges": e}, {"A": Dd, "B": Rd, "edges": e, "auto": False}, {"A": Rd, "edges": e}]
    mixed = pc.pc_count_batch(jobs, mode=pc.PC_MIXED)
    st = pc.pc_debug_last_pruning()
    assert st["few_items"] > 0 and st["gram_items"] > 0
    plain = pc.pc_count_batch(jobs, mode=pc.PC_FP64_PLAIN)
    matrix = pc.pc_count_batch(jobs, mode=pc.PC_MIXED | pc.PC_MATRIX_CORES)
    assert pc.pc_debug_last_pruning()["mfma_items"] > 0
    for m, p, x in zip(mixed, plain, matrix):
        assert m.tolist() == p.tolist()
        assert m.tolist() == x.tolist()
    assert int(mixed[0].sum()) == n * (n - 1) // 2
    assert int(mixed[1].sum()) == n * R[0].size
    assert int(mixed[2].sum()) == R[0].size * (R[0].size - 1) // 2
    rows = [(0, 64), (437_000, 437_100), (n - 80, n)]
    for r in rows:
        assert pc.pc_count_ex(Dd, e, rows=r).tolist() == oracle.count(D, e, rows=r).tolist(), r
        assert pc.pc_count_ex(Dd, e, B=Rd, auto=False, rows=r).tolist() == \
            oracle.count(D, e, B=R, auto=False, rows=r).tolist(), r
    parts = [pc.pc_count_ex(Dd, e, rows=r) for r in [(0, 333_333), (333_333, 777_777), (777_777, n)]]
    assert np.sum(parts, axis=0).tolist() == mixed[0].tolist()


@pytest.mark.parametrize("mode", MODES)
def test_whole_tile_pair_binning_matches_every_pair(mode):
    """Compact clusters far apart: whole tile pairs fall inside one bin (an
    interior bin, the overflow, and -- for piled-up duplicates -- the
    underflow), so they are binned without visiting their pairs; counts must
    equal the oracle and the run that visits every pair."""
    rng = np.random.default_rng(21)
    parts = []
    for ra0, dec0, s, n in [(10, 0, 0.02, 700), (40, 5, 0.02, 900), (11, 1, 0.03, 600), (200, -40, 0.02, 800)]:
        parts.append((ra0 + s * rng.standard_normal(n), np.clip(dec0 + s * rng.standard_normal(n), -90, 90)))
    parts.append((np.full(600, 123.0), np.full(600, -7.0)))          # 600 identical points
    A = (np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts]))
    B = synth.uniform_patch(1500, synth.FULL_SKY, rng)
    e = np.array([0.001, 0.5, 2.0, 25.0, 35.0, 120.0])
    want_a = oracle.count(A, e)
    want_c = oracle.count(A, e, B=B, auto=False)
    got = pc.pc_count_ex(dev(A), e, mode=mode)
    stats = pc.pc_debug_last_pruning()
    assert got.tolist() == want_a.tolist()
    assert stats["survivors"] < stats["pairs_total"]
    assert stats["pairs_computed"] < stats["pairs_total"]
    assert pc.pc_count_ex(dev(A), e, mode=mode | pc.PC_NO_PRUNE).tolist() == want_a.tolist()
    assert pc.pc_count_ex(dev(A), e, B=dev(B), auto=False, mode=mode).tolist() == want_c.tolist()
    assert pc.pc_count_ex(dev(A), e, B=dev(B), auto=False, mode=mode | pc.PC_NO_PRUNE).tolist() == want_c.tolist()
    # rows and the pruned path together
    assert pc.pc_count_ex(dev(A), e, rows=(650, 2900), mode=mode).tolist() == \
        oracle.count(A, e, rows=(650, 2900)).tolist()


@pytest.mark.parametrize("mode", MODES)
def test_tile_pairs_around_the_last_edge(mode):
    """Clusters whose separations sit just below, at and just above the last
    edge (20 deg): the prune pass bins a tile pair past the last edge from
    its squared centre distance, without the square root; tile pairs on
    either side of that bound must give the oracle's counts, pruned or not."""
    rng = np.random.default_rng(33)
    parts = [(0.3 * rng.standard_normal(2000), 0.3 * rng.standard_normal(2000))]
    for k, d in enumerate([19.0, 19.8, 19.95, 20.0, 20.05, 20.2, 21.0, 23.0]):
        # clusters on a small circle around (0, 0), each at distance ~d
        pa = 2 * np.pi * k / 8
        ra0, dec0 = d * np.cos(pa), d * np.sin(pa)
        parts.append((ra0 + 0.3 * rng.standard_normal(700), dec0 + 0.3 * rng.standard_normal(700)))
    A = (np.concatenate([p[0] for p in parts[:1]]), np.concatenate([p[1] for p in parts[:1]]))
    B = (np.concatenate([p[0] for p in parts[1:]]) % 360.0, np.concatenate([p[1] for p in parts[1:]]))
    A = (A[0] % 360.0, A[1])
    AB = (np.concatenate([A[0], B[0]]), np.concatenate([A[1], B[1]]))
    e = synth.log_edges(0.1, 20.0, 12)
    want_cross = oracle.count(A, e, B=B, auto=False)
    want_auto = oracle.count(AB, e)
    assert want_cross[-1] > 0 and want_cross[-2] > 0  # pairs on both sides of the last edge
    for extra in (0, pc.PC_NO_PRUNE):
        assert pc.pc_count_ex(dev(A), e, B=dev(B), auto=False, mode=mode | extra).tolist() == want_cross.tolist()
        assert pc.pc_count_ex(dev(AB), e, mode=mode | extra).tolist() == want_auto.tolist()


def test_pruning_skips_most_pairs_on_the_1m_shape():
    c = synth.config_1m(n_parents=5_000, n_random=100_000)
    D, R, e = dev(c["D"]), dev(c["R"]), c["edges"]
    got = pc.pc_count_ex(D, e, B=R, auto=False)
    st = pc.pc_debug_last_pruning()
    rk = pc.pc_debug_last_rechecks()
    assert st["pairs_total"] == 100_000 * 100_000
    assert st["pairs_computed"] < 0.35 * st["pairs_total"]
    # guard-band re-checks: a small fraction of the computed pairs, but some
    assert 0 < rk < 1e-3 * st["pairs_computed"]
    # few-edge work units: survivors, or open sub-blocks of split survivors
    assert 0 < st["few_items"] <= 4 * st["survivors"]
    assert 0 < st["split_items"] <= st["survivors"]
    assert got.tolist() == pc.pc_count_ex(D, e, B=R, auto=False, mode=pc.PC_NO_PRUNE).tolist()


@pytest.mark.parametrize("mode", MODES)
def test_matrix_core_path_far_clusters_and_edge_pairs(mode):
    """Two compact clusters 15 deg apart, each 10 full tiles, and a copy of the
    first shifted by exactly 12 deg along the meridian (2560 pairs on the 12
    deg edge).  With the matrix-core flag, full tile pairs whose chords are all
    at least twice the smaller tile radius and whose chord interval holds at
    most 3 edges get their chords from the matrix cores with their own guard
    band (sparse edges); dense edges around 12 deg leave them to the vector
    path.  Counts must equal the oracle either way."""
    rng = np.random.default_rng(33)
    n = 2560
    ra1, dec1 = 100 + 0.5 * rng.standard_normal(n), 0.5 * rng.standard_normal(n)
    ra2, dec2 = 100 + 0.5 * rng.standard_normal(n), 15 + 0.5 * rng.standard_normal(n)
    A = (np.concatenate([ra1, ra2]), np.concatenate([dec1, dec2]))
    B = (ra1.copy(), dec1 + 12.0)
    for e, sparse in [(np.array([0.01, 1.0, 5.0, 12.0, 15.0, 30.0]), True),
                      (np.array([0.01, 1.0, 5.0, 9.0, 11.0, 11.9, 12.0, 12.1, 13.0, 14.0, 15.0, 16.0, 18.0, 30.0]),
                       False)]:
        got = pc.pc_count_ex(dev(A), e, mode=mode)
        st = pc.pc_debug_last_pruning()
        assert got.tolist() == oracle.count(A, e).tolist()
        gotc = pc.pc_count_ex(dev(A), e, B=dev(B), auto=False, mode=mode)
        stc = pc.pc_debug_last_pruning()
        assert gotc.tolist() == oracle.count(A, e, B=B, auto=False).tolist()
        if mode & pc.PC_MATRIX_CORES and sparse:
            assert st["mfma_items"] > 0 and stc["mfma_items"] > 0
        if mode == pc.PC_MIXED and sparse:
            assert st["gram_items"] > 0 and stc["gram_items"] > 0
        elif not mode & pc.PC_MATRIX_CORES:
            assert st["mfma_items"] == 0 and stc["mfma_items"] == 0


@pytest.mark.parametrize("mode", MODES)
def test_edge_at_zero_with_ragged_gram_items(mode):
    """An edge at 0 (its band is (-inf, -inf): every chord lies above it) in
    few-edge items whose i-tile is ragged: the i slots past the end count
    nowhere (marked -infinity in the Gram form) and must never be taken for
    in-band chords or counted above the zero edge."""
    rng = np.random.default_rng(41)
    for n_a, n_b in [(300, 700), (45, 513), (257, 256)]:
        A = (100 + 0.4 * rng.standard_normal(n_a), 0.4 * rng.standard_normal(n_a))
        B = (100 + 0.4 * rng.standard_normal(n_b), 15 + 0.4 * rng.standard_normal(n_b))
        for e in (np.array([0.0, 14.0, 16.0]), np.array([0.0, 1e-9, 13.0, 15.0, 17.0]),
                  synth.linear_edges(0.0, 90.0, 9)):
            got = pc.pc_count_ex(dev(A), e, B=dev(B), auto=False, mode=mode)
            assert got.tolist() == oracle.count(A, e, B=B, auto=False).tolist(), (n_a, n_b, e.size)
            if mode == pc.PC_MIXED and e.size == 3:
                assert pc.pc_debug_last_pruning()["gram_items"] > 0
            AB = (np.concatenate([A[0], B[0]]), np.concatenate([A[1], B[1]]))
            assert pc.pc_count_ex(dev(AB), e, mode=mode).tolist() == oracle.count(AB, e).tolist(), (n_a, n_b)


@pytest.mark.parametrize("mode", [pc.PC_MIXED, pc.PC_MIXED | pc.PC_MATRIX_CORES])
def test_split_items_match_oracle(mode):
    """Clustered points on a 10-degree patch with 30 log bins: most surviving
    tile pairs are split into 64-point j sub-blocks (some binned whole by the
    prune pass, the rest counted with their own edges); DD and DR must equal
    the oracle, and the run that visits every pair, exactly."""
    c = synth.config_small(scale=0.5)
    D, R, e = c["D"], c["R"], c["edges"]
    dd = pc.pc_count_ex(dev(D), e, mode=mode)
    st = pc.pc_debug_last_pruning()
    assert st["split_items"] > 0
    assert dd.tolist() == oracle.count(D, e).tolist()
    assert dd.tolist() == pc.pc_count_ex(dev(D), e, mode=pc.PC_MIXED | pc.PC_NO_PRUNE).tolist()
    dr = pc.pc_count_ex(dev(D), e, B=dev(R), auto=False, mode=mode)
    assert pc.pc_debug_last_pruning()["split_items"] > 0
    assert dr.tolist() == oracle.count(D, e, B=R, auto=False).tolist()


def test_many_edge_sets_cycle_the_table_cache():
    # more distinct edge sets than the library keeps device tables for: old
    # tables are dropped and rebuilt when they come back; counts stay exact
    rng = np.random.default_rng(47)
    A = synth.uniform_patch(400, synth.centred_patch(20.0), rng)
    Ad = dev(A)
    sets = [synth.log_edges(0.05 + 0.001 * k, 10.0 + 0.01 * k, 10 + k % 20) for k in range(300)]
    for k, e in enumerate(sets + sets[:5]):
        got = pc.pc_count_ex(Ad, e)
        if k % 37 == 0 or k >= 300:
            assert got.tolist() == oracle.count(A, e).tolist(), k
        else:
            assert int(got.sum()) == 400 * 399 // 2


def test_concurrent_calls_on_distinct_streams():
    # the C ABI is thread-safe on distinct streams: four host threads count
    # different catalogues and edge sets at once; each result equals the
    # same call made alone
    import threading
    rng = np.random.default_rng(48)
    cases = []
    for k in range(4):
        A = synth.neyman_scott(60 + 20 * k, 20, 0.3, synth.centred_patch(30.0), rng)
        B = synth.uniform_patch(3000 + 500 * k, synth.centred_patch(30.0), rng)
        e = synth.log_edges(0.02 * (k + 1), 15.0, 12 + 6 * k)
        cases.append((dev(A), dev(B), e, A, B))
    torch.cuda.synchronize()
    alone = [(pc.pc_count_ex(a, e), pc.pc_count_ex(a, e, B=b, auto=False)) for a, b, e, _, _ in cases]
    streams = [torch.cuda.Stream() for _ in cases]
    got = [None] * len(cases)
    errors = []

    def work(k):
        try:
            a, b, e, _, _ = cases[k]
            out = []
            for _ in range(5):
                out.append((pc.pc_count_ex(a, e, stream=streams[k]),
                            pc.pc_count_ex(a, e, B=b, auto=False, stream=streams[k])))
            got[k] = out
        except Exception as ex:  # reported below
            errors.append(repr(ex))

    threads = [threading.Thread(target=work, args=(k,)) for k in range(len(cases))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(120)
    assert not errors, errors
    for k, (dd, dr) in enumerate(alone):
        for gdd, gdr in got[k]:
            assert gdd.tolist() == dd.tolist() and gdr.tolist() == dr.tolist(), k
    a, b, e, A, B = cases[0]
    assert alone[0][1].tolist() == oracle.count(A, e, B=B, auto=False).tolist()


@pytest.mark.parametrize("mode", MODES)
def test_largest_edge_set(mode):
    # 1024 edges, the most a call takes: the widest histograms and cell
    # tables in LDS, pairs spread over every bin
    rng = np.random.default_rng(49)
    A = synth.uniform_patch(1500, synth.centred_patch(60.0), rng)
    B = synth.uniform_patch(900, synth.centred_patch(60.0), rng)
    e = synth.log_edges(0.05, 80.0, 1023)
    assert e.size == 1024
    got = pc.pc_count_ex(dev(A), e, mode=mode)
    assert got.tolist() == oracle.count(A, e).tolist()
    got = pc.pc_count_ex(dev(A), e, B=dev(B), auto=False, mode=mode)
    assert got.tolist() == oracle.count(A, e, B=B, auto=False).tolist()
    lin = synth.linear_edges(0.0, 180.0, 1023)
    got = pc.pc_count_ex(dev(A), lin, mode=mode)
    assert got.tolist() == oracle.count(A, lin).tolist()


@pytest.mark.parametrize("seed", range(12))
def test_seeded_random_configurations(seed):
    # random shapes drawn from a seed: patch size, clustering, sizes (ragged),
    # edge sets (log or linear, 1..300 bins, zero edge or not), kernel, auto
    # or cross, row range; every result against the oracle
    rng = np.random.default_rng(1000 + seed)
    side = float(rng.choice([2.0, 10.0, 45.0, 120.0]))
    patch = synth.centred_patch(side) if side < 120 else synth.FULL_SKY
    nA, nB = int(rng.integers(0, 2600)), int(rng.integers(1, 1800))
    if rng.random() < 0.5 and nA >= 20:
        A = synth.neyman_scott(max(1, nA // 20), 20, float(rng.uniform(0.01, 0.5)), patch, rng)
    else:
        A = synth.uniform_patch(nA, patch, rng) if nA else (np.zeros(0), np.zeros(0))
    B = synth.uniform_patch(nB, patch, rng)
    nbins = int(rng.integers(1, 300))
    if rng.random() < 0.5:
        lo = float(10 ** rng.uniform(-3, 0))
        e = synth.log_edges(lo, float(min(180.0, lo * 10 ** rng.uniform(0.5, 4))), nbins)
    else:
        e = synth.linear_edges(0.0 if rng.random() < 0.5 else float(rng.uniform(0, 5)), float(rng.uniform(5, 180)), nbins)
    mode = MODES[int(rng.integers(0, len(MODES)))]
    n = A[0].size
    r0 = int(rng.integers(0, n + 1))
    r1 = int(rng.integers(r0, n + 1))
    Ad = dev(A) if n else A
    got = pc.pc_count_ex(Ad, e, mode=mode, rows=(r0, r1))
    assert got.tolist() == oracle.count(A, e, rows=(r0, r1)).tolist(), (seed, n, nbins, mode, r0, r1)
    got = pc.pc_count_ex(Ad, e, B=dev(B), auto=False, mode=mode)
    assert got.tolist() == oracle.count(A, e, B=B, auto=False).tolist(), (seed, n, nB, nbins, mode)


@pytest.mark.parametrize("seed", range(4))
def test_seeded_random_batches(seed):
    # 3..12 jobs in one launch: shared and distinct catalogues, auto and
    # cross, row ranges, several edge sets; each job against the oracle
    rng = np.random.default_rng(3000 + seed)
    patch = synth.centred_patch(float(rng.choice([5.0, 30.0, 90.0])))
    cats = [synth.uniform_patch(int(rng.integers(1, 1500)), patch, rng) for _ in range(4)]
    devs = [dev(c) for c in cats]
    sets = [synth.log_edges(0.01, 20.0, int(rng.integers(2, 60))), synth.linear_edges(0.0, 90.0, int(rng.integers(1, 40)))]
    jobs, want = [], []
    for _ in range(int(rng.integers(3, 13))):
        a, b = int(rng.integers(0, 4)), int(rng.integers(0, 4))
        e = sets[int(rng.integers(0, 2))]
        if rng.random() < 0.5:
            n = cats[a][0].size
            r0 = int(rng.integers(0, n + 1))
            r1 = int(rng.integers(r0, n + 1))
            jobs.append({"A": devs[a], "edges": e, "rows": (r0, r1)})
            want.append(oracle.count(cats[a], e, rows=(r0, r1)))
        else:
            jobs.append({"A": devs[a], "B": devs[b], "edges": e, "auto": False})
            want.append(oracle.count(cats[a], e, B=cats[b], auto=False))
    mode = MODES[seed % len(MODES)]
    got = pc.pc_count_batch(jobs, mode=mode)
    for k, (g, w) in enumerate(zip(got, want)):
        assert g.tolist() == w.tolist(), (seed, k)


@pytest.mark.parametrize("mode", MODES + [pc.PC_MIXED | pc.PC_NO_PRUNE])
def test_histogram_flushed_every_few_items(mode):
    """The wrap guard's flush (LDS uint32 histogram -> uint64 counts before a
    word could wrap, Sec. 2.1 per-block histograms) normally fires every ~10^6
    items; lowered to 1, 2 and 3 items through the debug hook, each wave
    flushes between most of its ~tens of items.  Counts equal the oracle."""
    c = synth.config_small(scale=6.0)   # 60,000 + 60,000 on the 10 x 10 deg patch: most tile pairs survive
    D, R, e = c["D"], c["R"], c["edges"]
    Dd, Rd = dev(D), dev(R)
    jobs = [{"A": Dd, "edges": e}, {"A": Dd, "B": Rd, "edges": e, "auto": False}, {"A": Rd, "edges": e}]
    want = [oracle.count(D, e), oracle.count(D, e, B=R, auto=False), oracle.count(R, e)]
    try:
        for every in (1, 2, 3):
            pc.pc_debug_set_flush_every(every)
            got = pc.pc_count_batch(jobs, mode=mode)
            launch = pc.pc_debug_last_launch()
            work = pc.pc_debug_last_pruning()["survivors"] if not mode & pc.PC_NO_PRUNE else launch["items"]
            assert work >= 4 * launch["grid"], (work, launch)     # several items per wave
            for g, w in zip(got, want):
                assert g.tolist() == w.tolist(), every
    finally:
        pc.pc_debug_set_flush_every(0)
    for g, w in zip(pc.pc_count_batch(jobs, mode=mode), want):
        assert g.tolist() == w.tolist()


def test_allocation_failures_report_nomem_leave_outputs_untouched_and_recover():
    """Device allocations made to fail from the host (workspace, edge-set
    table, resident catalogue, aperture work space): each call reports
    PC_ERR_NOMEM, writes nothing, and the next call works; a hundred failed
    calls leave device memory where it was."""
    c = synth.config_small(scale=0.1)
    D, e = dev(c["D"]), c["edges"]
    want = pc.pc_count(D, e)                       # the edge set's table is cached from here on
    assert want.tolist() == oracle.count(c["D"], e).tolist()
    a = pc.as_catalog(D)
    sentinel = np.uint64(0xDEADBEEFCAFE)
    counts = np.full(e.size + 1, sentinel, dtype=np.uint64)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    try:
        for _ in range(100):
            pc.pc_debug_fail_allocations(1)
            rc = pc.lib().pc_count(a.ref(), None, e.ctypes.data, e.size, 1, counts.ctypes.data, None)
            assert rc == pc.PC_ERR_NOMEM, rc
            assert "out of memory" in pc.pc_last_error()
            assert np.all(counts == sentinel)
        torch.cuda.synchronize()
        assert abs(torch.cuda.mem_get_info()[0] - free0) < (64 << 20)
        assert pc.pc_count(D, e).tolist() == want.tolist()
        # a new edge set: its table's allocation fails, then the call works
        e2 = synth.linear_edges(0.0, 7.5, 17)
        pc.pc_debug_fail_allocations(1)
        with pytest.raises(pc.PcError) as ex:
            pc.pc_count(D, e2)
        assert ex.value.code == pc.PC_ERR_NOMEM
        assert pc.pc_count(D, e2).tolist() == oracle.count(c["D"], e2).tolist()
        # a resident catalogue
        pc.pc_debug_fail_allocations(1)
        with pytest.raises(pc.PcError) as ex:
            pc.pc_catalog_upload(D)
        assert ex.value.code == pc.PC_ERR_NOMEM
        h = pc.pc_catalog_upload(D)
        assert pc.pc_count_h(h, e).tolist() == want.tolist()
        pc.pc_catalog_release(h)
        # the aperture-mass map's work space
        cat, side = synth.shear_catalog(2000, config=23)
        pc.pc_debug_fail_allocations(1)
        with pytest.raises(pc.PcError) as ex:
            pc.pc_aperture_mass(cat, (0.0, 0.0, side / 8, side / 8, 8, 8), 2.0, 35.0)
        assert ex.value.code == pc.PC_ERR_NOMEM
        assert pc.pc_aperture_mass(cat, (0.0, 0.0, side / 8, side / 8, 8, 8), 2.0, 35.0)["n_in"].size == 64
    finally:
        pc.pc_debug_fail_allocations(0)



@pytest.mark.parametrize("mode", MODES)
def test_128_point_tiles_match_the_oracle(mode):
    """The counting path compiled for 128-point tiles (the tuner's other
    submatrix size, Sec. 2.1): the small configuration's DD, DR and RR, ragged
    sizes, row ranges and a resident catalogue (re-ordered for the smaller
    tiles) equal the oracle; its pruning and sub-block paths are exercised."""
    try:
        pc.pc_debug_set_tile(128)
        c = synth.config_small(scale=0.3)
        D, R, e = c["D"], c["R"], c["edges"]
        got = pc.pc_count_batch([{"A": dev(D), "edges": e}, {"A": dev(D), "B": dev(R), "edges": e, "auto": False},
                                 {"A": dev(R), "edges": e}], mode=mode)
        want = [oracle.count(D, e), oracle.count(D, e, B=R, auto=False), oracle.count(R, e)]
        for g, w in zip(got, want):
            assert g.tolist() == w.tolist()
        if mode == pc.PC_MIXED:
            assert pc.pc_debug_last_pruning()["split_items"] > 0
        # two compact clusters 15 deg apart with sparse edges: tile pairs
        # across them meet one or two edges (few-edge and Gram-form units)
        rng = np.random.default_rng(34)
        n = 1280
        F = (np.concatenate([100 + 0.5 * rng.standard_normal(n), 100 + 0.5 * rng.standard_normal(n)]),
             np.concatenate([0.5 * rng.standard_normal(n), 15 + 0.5 * rng.standard_normal(n)]))
        ef = np.array([0.01, 1.0, 5.0, 12.0, 15.0, 30.0])
        assert pc.pc_count_ex(dev(F), ef, mode=mode).tolist() == oracle.count(F, ef).tolist()
        if mode == pc.PC_MIXED:
            st = pc.pc_debug_last_pruning()
            assert st["few_items"] > 0 and st["gram_items"] > 0
        rng = np.random.default_rng(55)
        patch = synth.centred_patch(12.0)
        e2 = synth.log_edges(0.05, 8.0, 12)
        for n in (1, 2, 127, 128, 129, 255, 257, 1000):
            A = synth.uniform_patch(n, patch, rng)
            assert pc.pc_count_ex(dev(A), e2, mode=mode).tolist() == oracle.count(A, e2).tolist(), n
            B = synth.uniform_patch(n * 3 % 200 + 1, patch, rng)
            assert pc.pc_count_ex(dev(A), e2, B=dev(B), auto=False, mode=mode).tolist() == \
                oracle.count(A, e2, B=B, auto=False).tolist(), n
        for rows in [(0, 1), (129, 1000), (1777, D[0].size)]:
            assert pc.pc_count_ex(dev(D), e, rows=rows, mode=mode).tolist() == oracle.count(D, e, rows=rows).tolist()
        h = pc.pc_catalog_upload(dev(D))
        try:
            assert pc.pc_count_h(h, e, mode=mode).tolist() == want[0].tolist()
        finally:
            pc.pc_catalog_release(h)
    finally:
        pc.pc_debug_set_tile(0)


@pytest.mark.parametrize("tile", [256, 128])
def test_compact_cell_table_matches_oracle(tile):
    """The 8-byte cell table (bits(hi) and the width bits rounded up, with the
    row offset in their low bits; every flagged chord re-checked in binary64)
    forced on: the small configuration's DD, DR and RR, pairs within a few
    ulps of the edges, the paper's 254 log bins, and ragged sizes equal the
    oracle, with less LDS per wave than the 16-byte table.  With 254 bins the
    default launch takes it by itself (more waves per CU)."""
    try:
        pc.pc_debug_set_tile(tile)
        c = synth.config_small(scale=0.3)
        D, R, e = c["D"], c["R"], c["edges"]
        jobs = [{"A": dev(D), "edges": e}, {"A": dev(D), "B": dev(R), "edges": e, "auto": False},
                {"A": dev(R), "edges": e}]
        want = [oracle.count(D, e), oracle.count(D, e, B=R, auto=False), oracle.count(R, e)]
        pc.pc_debug_set_compact_table(-1)
        pc.pc_count_batch(jobs)
        full = pc.pc_debug_last_launch()["lds_bytes"]
        pc.pc_debug_set_compact_table(1)
        got = pc.pc_count_batch(jobs)
        for g, w in zip(got, want):
            assert g.tolist() == w.tolist()
        assert pc.pc_debug_last_launch()["lds_bytes"] < full
        for theta in [synth.log_edges(0.01, 20.0, 40), synth.linear_edges(0.0, 60.0, 30)]:
            A = _near_edge_catalogue(theta)
            assert pc.pc_count_ex(dev(A), theta).tolist() == oracle.count(A, theta).tolist()
            assert pc.pc_debug_last_rechecks() > 0
        rng = np.random.default_rng(71)
        ep = synth.log_edges(0.001, 90.0, 254)
        A = synth.uniform_patch(2500, synth.centred_patch(30.0), rng)
        B = synth.uniform_patch(1700, synth.centred_patch(30.0), rng)
        assert pc.pc_count_ex(dev(A), ep).tolist() == oracle.count(A, ep).tolist()
        assert pc.pc_count_ex(dev(A), ep, B=dev(B), auto=False).tolist() == oracle.count(A, ep, B=B, auto=False).tolist()
        compact = pc.pc_debug_last_launch()["lds_bytes"]
        pc.pc_debug_set_compact_table(0)
        assert pc.pc_count_ex(dev(A), ep, B=dev(B), auto=False).tolist() == oracle.count(A, ep, B=B, auto=False).tolist()
        assert pc.pc_debug_last_launch()["lds_bytes"] == compact
        pc.pc_debug_set_compact_table(1)
        e2 = synth.log_edges(0.05, 8.0, 12)
        for n in (1, 2, 127, 129, 255, 257, 1000):
            A = synth.uniform_patch(n, synth.centred_patch(12.0), rng)
            assert pc.pc_count_ex(dev(A), e2).tolist() == oracle.count(A, e2).tolist(), n
    finally:
        pc.pc_debug_set_compact_table(0)
        pc.pc_debug_set_tile(0)
