"""GPU parity of every configuration at its stated size, in the launch the
benchmark times (one pc_count_batch of all jobs, launch parameters from the
tuner), through the C ABI.

* small (10k + 10k) and 1M (1M + 1M): DD, DR and RR of the whole launch
  against the oracle's full counts stored in tests/golden/ (written by
  tests/golden/make_config_goldens.py from oracle/ and synth/ alone), bit for
  bit, in the mixed, mixed + matrix-core and binary64 kernels and with tuned
  launch parameters.  The paper's own check is this comparison for DR
  (Sec. 2.2, CPU-GPU consistency).
* batched (256 mocks of 50k-400k points x one shared 1M random catalogue, 513
  jobs in one launch) and large (4M clustered + 8M random, full sky): the
  whole launch is compared job by job with the oracle where the oracle
  finishes in seconds (every pair of the smallest mocks' DD and DR), with
  seeded row windows of every job type (DD, DR and RR) otherwise, and the
  whole-launch counts must equal the sum of row-range launches that split
  each sampled job around its window.  The large RR is checked against the
  isotropic closed form p_k = (cos t_k - cos t_k+1)/2 on all 8M points.
"""
import hashlib
import json
import math
import os
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
import paper_1208_3658_amd as pc  # noqa: E402

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
MODES = {"mixed": pc.PC_MIXED, "matrix_cores": pc.PC_MIXED | pc.PC_MATRIX_CORES, "fp64": pc.PC_FP64_PLAIN}


def dev(cat):
    return tuple(torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in cat)


def sha256(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<f8").tobytes()).hexdigest()


def note(msg):
    print(msg, file=sys.stderr, flush=True)


def load_golden(fname, c):
    path = os.path.join(GOLDEN, fname)
    assert os.path.exists(path), f"{path} missing: run tests/golden/make_config_goldens.py"
    with open(path) as f:
        g = json.load(f)
    have = {"D_ra": sha256(c["D"][0]), "D_dec": sha256(c["D"][1]), "R_ra": sha256(c["R"][0]),
            "R_dec": sha256(c["R"][1]), "edges": sha256(c["edges"])}
    assert have == g["input_sha256"], (
        "the generator draws different catalogues on this machine than the ones the golden counts were "
        f"computed on ({fname}); re-run tests/golden/make_config_goldens.py")
    return {k: np.array(v, dtype=np.uint64) for k, v in g["counts"].items()}


def ddrrr_jobs(D, R, e):
    return [{"A": D, "edges": e}, {"A": D, "B": R, "edges": e, "auto": False}, {"A": R, "edges": e}]


def check_wtheta(counts, want, nD, nR):
    w = pc.pc_wtheta(counts[0][1:-1], counts[1][1:-1], counts[2][1:-1], nD, nR)
    ow = oracle.wtheta(want["DD"][1:-1], want["DR"][1:-1], want["RR"][1:-1], nD, nR)
    f = ~np.isnan(ow)
    assert np.array_equal(np.isnan(w), np.isnan(ow))
    assert np.all(np.abs(w[f] - ow[f]) <= 1e-12 * np.maximum(1.0, np.abs(ow[f])))


def check_against(counts, want, label):
    for got, key in zip(counts, ("DD", "DR", "RR")):
        assert got.tolist() == want[key].tolist(), (label, key)


# ---------------------------------------------------------------- small, 1M

@pytest.fixture(scope="module")
def small():
    c = synth.config_small()
    return c, load_golden("config_small_10k.json", c)


@pytest.fixture(scope="module")
def onem():
    c = synth.config_1m()
    return c, load_golden("config_1m.json", c)


@pytest.mark.parametrize("mode", list(MODES))
def test_small_config_full_size_all_kernels(small, mode):
    """10,000 clustered + 10,000 random points (the small configuration in
    full): DD, DR, RR of one launch equal the oracle's full counts."""
    c, want = small
    D, R, e = dev(c["D"]), dev(c["R"]), c["edges"]
    got = pc.pc_count_batch(ddrrr_jobs(D, R, e), mode=MODES[mode])
    check_against(got, want, mode)
    check_wtheta(got, want, c["D"][0].size, c["R"][0].size)
    # host-memory inputs and every pair visited give the same counts
    got_h = pc.pc_count_batch(ddrrr_jobs(c["D"], c["R"], e), mode=MODES[mode] | pc.PC_NO_PRUNE)
    check_against(got_h, want, mode + "+no_prune")


def test_small_config_tuned_launch(small):
    """pc_autotune runs every launch candidate on the batch (they must agree);
    the tuned launch and the tuner's own counts equal the oracle."""
    c, want = small
    D, R, e = dev(c["D"]), dev(c["R"]), c["edges"]
    jobs = ddrrr_jobs(D, R, e)
    counts, cfg = pc.pc_autotune(jobs)
    check_against(counts, want, "autotune")
    check_against(pc.pc_count_batch(jobs, mode=pc.PC_MIXED | pc.PC_TUNED), want, f"tuned {cfg}")


@pytest.mark.parametrize("mode", list(MODES))
def test_1m_config_full_size_all_kernels(onem, mode):
    """The benchmark's workload in full (1,999,999,000,000 pairs in one
    launch): DD, DR and RR equal the oracle's full counts bit for bit."""
    c, want = onem
    D, R, e = dev(c["D"]), dev(c["R"]), c["edges"]
    note(f"1M workload, mode {mode}")
    got = pc.pc_count_batch(ddrrr_jobs(D, R, e), mode=MODES[mode])
    check_against(got, want, mode)
    check_wtheta(got, want, c["D"][0].size, c["R"][0].size)
    if mode == "mixed":
        st = pc.pc_debug_last_pruning()
        assert st["few_items"] > 0 and st["gram_items"] > 0 and st["split_items"] > 0
    if mode == "matrix_cores":
        assert pc.pc_debug_last_pruning()["mfma_items"] > 0


def test_1m_config_full_size_128_point_tiles(onem):
    """The same launch cut into 128-point tiles (the tuner's other size)."""
    c, want = onem
    D, R, e = dev(c["D"]), dev(c["R"]), c["edges"]
    try:
        pc.pc_debug_set_tile(128)
        check_against(pc.pc_count_batch(ddrrr_jobs(D, R, e)), want, "tile 128")
    finally:
        pc.pc_debug_set_tile(0)


def test_1m_config_tuned_launch_as_benchmarked(onem):
    """Exactly what bench.py times: tune on the batch, then PC_TUNED steps."""
    c, want = onem
    D, R, e = dev(c["D"]), dev(c["R"]), c["edges"]
    jobs = ddrrr_jobs(D, R, e)
    note("1M workload: tuning")
    counts, cfg = pc.pc_autotune(jobs)
    check_against(counts, want, "autotune")
    for k in range(2):
        check_against(pc.pc_count_batch(jobs, mode=pc.PC_MIXED | pc.PC_TUNED), want, f"tuned {cfg} step {k}")


# ------------------------------------------------- row windows, decomposition

def window_check(Adev, A, e, n, rows, full, Bdev=None, B=None, auto=True, mode=pc.PC_MIXED):
    """The window rows = (a, b) against the oracle; the whole-launch counts
    `full` against the sum of the row-range launches [0, a), [a, b), [b, n)."""
    kw = {} if auto else {"B": Bdev, "auto": False}
    okw = {} if auto else {"B": B, "auto": False}
    a, b = rows
    mid = pc.pc_count_ex(Adev, e, rows=(a, b), mode=mode, **kw)
    assert mid.tolist() == oracle.count(A, e, rows=(a, b), **okw).tolist(), rows
    parts = [mid]
    if a > 0:
        parts.append(pc.pc_count_ex(Adev, e, rows=(0, a), mode=mode, **kw))
    if b < n:
        parts.append(pc.pc_count_ex(Adev, e, rows=(b, n), mode=mode, **kw))
    assert np.sum(parts, axis=0).tolist() == full.tolist(), rows


def seeded_windows(n, k, width, seed):
    rng = np.random.default_rng(seed)
    starts = sorted({0, n - width, *(int(x) for x in rng.integers(0, n - width, k - 2))})
    return [(s, s + width) for s in starts]


# ---------------------------------------------------------------- batched

@pytest.fixture(scope="module")
def batched():
    note("generating the batched configuration (256 mocks, 1M randoms)")
    c = synth.config_batched()
    R = dev(c["R"])
    mocks = [dev(m) for m in c["mocks"]]
    jobs = []
    for m in mocks:
        jobs += [{"A": m, "edges": c["edges"]}, {"A": m, "B": R, "edges": c["edges"], "auto": False}]
    jobs.append({"A": R, "edges": c["edges"]})
    note("batched: tuning and the tuned launch")
    tuned_counts, cfg = pc.pc_autotune(jobs)
    got = pc.pc_count_batch(jobs, mode=pc.PC_MIXED | pc.PC_TUNED)
    return {"c": c, "R": R, "mocks": mocks, "jobs": jobs, "got": got, "tuned_counts": tuned_counts, "cfg": cfg}


def test_batched_config_full_launch_totals_and_kernels(batched):
    """513 jobs in one launch: exact pair totals per job; the tuner's
    candidates, the tuned launch, the binary64 kernel and the matrix-core
    path give the same counts."""
    c, got = batched["c"], batched["got"]
    nR = c["R"][0].size
    for q, m in enumerate(c["mocks"]):
        n = m[0].size
        assert int(got[2 * q].sum()) == n * (n - 1) // 2
        assert int(got[2 * q + 1].sum()) == n * nR
    assert int(got[-1].sum()) == nR * (nR - 1) // 2
    for a, b in zip(got, batched["tuned_counts"]):
        assert a.tolist() == b.tolist()
    for mode in (pc.PC_FP64_PLAIN, pc.PC_MIXED | pc.PC_MATRIX_CORES):
        note(f"batched: mode {mode:#x}")
        other = pc.pc_count_batch(batched["jobs"], mode=mode)
        for q, (a, b) in enumerate(zip(got, other)):
            assert a.tolist() == b.tolist(), (mode, q)


def test_batched_config_smallest_mocks_whole_jobs_vs_oracle(batched):
    """Every pair of the two smallest mocks' DD and DR jobs (2 x ~5e10 pairs
    for the oracle) as counted inside the 513-job launch."""
    c, got = batched["c"], batched["got"]
    sizes = np.array([m[0].size for m in c["mocks"]])
    for q in np.argsort(sizes, kind="stable")[:2]:
        m = c["mocks"][q]
        note(f"batched: oracle on mock {q} ({m[0].size} points)")
        assert got[2 * q].tolist() == oracle.count(m, c["edges"]).tolist(), q
        assert got[2 * q + 1].tolist() == oracle.count(m, c["edges"], B=c["R"], auto=False).tolist(), q


def test_batched_config_seeded_row_windows_every_job_type(batched):
    """Seeded mocks and windows: DD and DR rows of the mock and RR rows of the
    shared random catalogue against the oracle, each job of the launch equal
    to the sum of launches split around its window."""
    c, got, e = batched["c"], batched["got"], batched["c"]["edges"]
    rng = np.random.default_rng(3003)
    for q in sorted(int(x) for x in rng.choice(len(c["mocks"]), 4, replace=False)):
        m, md = c["mocks"][q], batched["mocks"][q]
        n = m[0].size
        for rows in seeded_windows(n, 3, 48, 100 + q):
            window_check(md, m, e, n, rows, got[2 * q])
            window_check(md, m, e, n, rows, got[2 * q + 1], Bdev=batched["R"], B=c["R"], auto=False)
    nR = c["R"][0].size
    for rows in seeded_windows(nR, 4, 48, 3004):
        window_check(batched["R"], c["R"], e, nR, rows, got[-1])


# ---------------------------------------------------------------- large

@pytest.fixture(scope="module")
def large():
    note("generating the large configuration (4M clustered + 8M random, full sky)")
    c = synth.config_large()
    D, R = dev(c["D"]), dev(c["R"])
    jobs = ddrrr_jobs(D, R, c["edges"])
    note("large: tuning and the tuned launch")
    tuned_counts, cfg = pc.pc_autotune(jobs)
    got = pc.pc_count_batch(jobs, mode=pc.PC_MIXED | pc.PC_TUNED)
    return {"c": c, "D": D, "R": R, "jobs": jobs, "got": got, "tuned_counts": tuned_counts}


def test_large_config_full_launch_totals_kernels_and_closed_form(large):
    c, got = large["c"], large["got"]
    n, nr = c["D"][0].size, c["R"][0].size
    assert int(got[0].sum()) == n * (n - 1) // 2
    assert int(got[1].sum()) == n * nr
    assert int(got[2].sum()) == nr * (nr - 1) // 2
    for a, b in zip(got, large["tuned_counts"]):
        assert a.tolist() == b.tolist()
    for mode in (pc.PC_FP64_PLAIN, pc.PC_MIXED | pc.PC_MATRIX_CORES):
        note(f"large: mode {mode:#x}")
        other = pc.pc_count_batch(large["jobs"], mode=mode)
        for a, b in zip(got, other):
            assert a.tolist() == b.tolist(), mode
    # RR of the 8M full-sky randoms: for points uniform on the sphere the
    # bin of a pair is independent of where its first point lies, so the
    # pair indicators are pairwise independent and RR_k has mean M p_k and
    # variance M p_k (1 - p_k) exactly, p_k = (cos t_k - cos t_k+1)/2
    rr = got[2]
    M = nr * (nr - 1) / 2
    full = np.concatenate([[0.0], c["edges"], [180.0]])
    zs = []
    for k in range(full.size - 1):
        t1, t2 = math.radians(full[k]), math.radians(full[k + 1])
        p = math.sin(0.5 * (t1 + t2)) * math.sin(0.5 * (t2 - t1))
        zs.append((float(rr[k]) - M * p) / math.sqrt(M * p * (1 - p)))
    assert max(abs(z) for z in zs) < 5.0, zs
    # 52 independent-ish z-scores: their mean square near 1
    assert 0.3 < float(np.mean(np.square(zs))) < 3.0, zs


def test_large_config_seeded_row_windows_every_job_type(large):
    c, got, e = large["c"], large["got"], large["c"]["edges"]
    n, nr = c["D"][0].size, c["R"][0].size
    for rows in seeded_windows(n, 4, 40, 4004):
        window_check(large["D"], c["D"], e, n, rows, got[0])
        window_check(large["D"], c["D"], e, n, rows, got[1], Bdev=large["R"], B=c["R"], auto=False)
    for rows in seeded_windows(nr, 4, 40, 4005):
        window_check(large["R"], c["R"], e, nr, rows, got[2])
