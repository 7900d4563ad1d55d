"""The w(theta) server's admission policy, on the CPU: the library's own
policy function (the one the server applies to its queue) fed with chosen
memory figures, and a discrete-event run of it against a fake executor and a
fake free-memory figure: first-come-first-served order, no oversubscription,
in-flight and pairs-per-launch limits, requests that can never fit, queueing
deadlines and cancellation."""
import heapq

import numpy as np
import pytest

pc = pytest.importorskip("paper_1208_3658_amd")

GB = 1 << 30
A, NF, EX, W = pc.ADMIT, pc.NEVER_FITS, pc.EXPIRED, pc.WAIT


def plan(need_gb, free_gb, total_gb=288, pairs=None, age=None, reserved_gb=0, inflight=0, **cfg):
    n = len(need_gb)
    need = [int(x * GB) for x in need_gb]
    pairs = [1e9] * n if pairs is None else pairs
    age = [0.0] * n if age is None else age
    cfg.setdefault("hbm_budget_bytes", 4 * GB)
    return pc.pc_debug_admission_plan(need, pairs, age, int(free_gb * GB), int(total_gb * GB),
                                      int(reserved_gb * GB), inflight, cfg).tolist()


def test_first_come_first_served_within_free_memory():
    # 10 GB free - 4 GB budget = 6 GB: the first two fit, the third does not and
    # holds back the fourth although the fourth alone would fit
    assert plan([2, 2, 3, 1], free_gb=10) == [A, A, W, W]
    # bytes held by running batches count against the free memory
    assert plan([2, 2, 3, 1], free_gb=10, reserved_gb=3) == [A, W, W, W]
    assert plan([2], free_gb=5) == [W]
    assert plan([], free_gb=10) == []


def test_requests_that_can_never_fit_fail_wherever_they_stand():
    # 8 GB device, 4 GB budget: a 5 GB request can never run
    assert plan([1, 5, 1], free_gb=8, total_gb=8) == [A, NF, A]
    assert plan([3, 5, 1], free_gb=6, total_gb=8) == [W, NF, W]
    assert plan([4], free_gb=8, total_gb=8) == [A]          # exactly the budget's complement fits
    # a budget beyond the device (and a huge configured one, clamped) rejects everything
    assert plan([1, 1], free_gb=8, total_gb=8, hbm_budget_bytes=1 << 62) == [NF, NF]
    assert plan([1], free_gb=8, total_gb=8, hbm_budget_bytes=1e30) == [NF]


def test_inflight_and_pairs_per_launch_limits():
    assert plan([1] * 5, free_gb=100, inflight=61, max_inflight=64) == [A, A, A, W, W]
    assert plan([1] * 2, free_gb=100, inflight=64, max_inflight=64) == [W, W]
    # the first request of a launch is exempt from the pairs limit
    assert plan([1, 1, 1], free_gb=100, pairs=[3e12, 1e9, 1e9], max_batch_pairs=2e12) == [A, W, W]
    assert plan([1, 1, 1], free_gb=100, pairs=[1e12, 9e11, 2e11], max_batch_pairs=2e12) == [A, A, W]


def test_queueing_deadline():
    assert plan([1, 1, 1], free_gb=100, age=[0.5, 2.0, 0.1], deadline_s=1.0) == [A, EX, A]
    # expiry applies behind a waiting request too; no deadline by default
    assert plan([50, 1, 1], free_gb=20, age=[0.1, 3.0, 0.2], deadline_s=1.0) == [W, EX, W]
    assert plan([1], free_gb=100, age=[1e6]) == [A]


def test_invalid_policy_arguments():
    with pytest.raises(pc.PcError) as e:
        plan([1], free_gb=10, bogus_key=1)
    assert e.value.code == pc.PC_ERR_INVALID
    with pytest.raises(pc.PcError):
        plan([1], free_gb=10, inflight=-1)
    with pytest.raises(ValueError):
        pc.pc_debug_admission_plan([1, 2], [1.0], [0.0, 0.0], 10, 10)


def _simulate(reqs, free0, total, cfg, cancel_at=()):
    """Discrete-event run: `reqs` = (arrival_s, need_bytes, pairs); a batch
    runs for 1 ms + pairs / 3e13 s on one of `streams` fake streams; the fake
    free memory drops by what running batches hold.  Cancellations at given
    times remove waiting requests.  Returns per-request (admit time, end
    time, status) and the launch log."""
    budget = cfg.get("hbm_budget_bytes", 4 * GB)
    streams = cfg.get("streams", 2)
    queue, running, log = [], [], []
    result = {}
    events = [(t, 0, i) for i, (t, _, _) in enumerate(reqs)]
    events += [(t, 1, i) for t, i in cancel_at]
    heapq.heapify(events)
    busy = 0
    now = 0.0
    while events or queue:
        if events:
            now, kind, x = heapq.heappop(events)
            if kind == 0:
                queue.append(x)
            elif kind == 1 and x in queue:
                queue.remove(x)
                result[x] = (None, now, "cancelled")
            elif kind == 2:                      # a batch ends
                busy -= 1
                for i in x:
                    result[i] = (result[i][0], now, "ok")
                running = [b for b in running if b is not x]
        elif not running:
            break
        while busy < streams and queue:
            held = sum(reqs[i][1] for b in running for i in b)
            free = free0 - held
            outcome = pc.pc_debug_admission_plan(
                [reqs[i][1] for i in queue], [reqs[i][2] for i in queue], [now - reqs[i][0] for i in queue],
                free, total, held, sum(len(b) for b in running), cfg)
            batch = [i for i, o in zip(queue, outcome) if o == A]
            for i, o in zip(queue, outcome):
                if o == NF:
                    result[i] = (None, now, "nomem")
                elif o == EX:
                    result[i] = (None, now, "expired")
            queue = [i for i, o in zip(queue, outcome) if o == W]
            if not batch:
                break
            assert held + sum(reqs[i][1] for i in batch) <= free0 - budget, "memory oversubscribed"
            for i in batch:
                result[i] = (now, None, "running")
            b = tuple(batch)
            running.append(b)
            busy += 1
            log.append((now, b))
            heapq.heappush(events, (now + 1e-3 + sum(reqs[i][2] for i in batch) / 3e13, 2, b))
        if not events and queue and not running:
            break
    return result, log


def test_fake_executor_run_keeps_order_memory_and_limits():
    rng = np.random.default_rng(31)
    n = 400
    t = np.cumsum(rng.exponential(0.004, n))
    need = (128 * np.exp(rng.uniform(np.log(1e3), np.log(2e6), n)) + (1 << 20)).astype(np.int64)
    need[::97] = 300 * GB                       # never fit on a 288 GB device
    pairs = (need / 128.0) ** 2 / 2
    cfg = {"hbm_budget_bytes": 4 * GB, "max_inflight": 16, "streams": 2, "max_batch_pairs": 2e12,
           "deadline_s": 0.5}
    free0 = 12 * GB                              # a busy device: little memory free
    res, log = _simulate(list(zip(t, need, pairs)), free0, 288 * GB, cfg, cancel_at=[(t[10] + 1e-6, 10)])
    assert len(res) == n
    assert all(res[i][2] == "nomem" for i in range(0, n, 97))
    assert res[10][2] in ("cancelled", "ok")
    admitted = [i for _, b in log for i in b]
    assert admitted == sorted(admitted), "admission out of submission order"
    assert all(len(b) <= 16 for _, b in log)
    assert all(len(b) == 1 or sum(pairs[i] for i in b) <= 2e12 for _, b in log)
    for i, (ta, te, st) in res.items():
        if st == "ok":
            assert ta - t[i] <= 0.5 + 1e-12, "admitted after its deadline"
        if st == "expired":
            assert te - t[i] > 0.5
    assert sum(1 for r in res.values() if r[2] == "ok") > n // 2


def test_fake_executor_burst_expires_late_requests():
    # 60 requests of 2e6 points at once: one launch each (pairs limit), two
    # streams, ~70 ms per launch; those still queued after 0.2 s expire
    n = 60
    need = np.full(n, 128 * 2_000_000 + (1 << 20), dtype=np.int64)
    pairs = np.full(n, 2e12)
    cfg = {"hbm_budget_bytes": 4 * GB, "streams": 2, "max_batch_pairs": 2e12, "deadline_s": 0.2}
    res, log = _simulate(list(zip(np.zeros(n), need, pairs)), 64 * GB, 288 * GB, cfg)
    status = [res[i][2] for i in range(n)]
    assert status.count("expired") > n // 2 and status.count("ok") >= 4
    first_expired = status.index("expired")
    assert all(s == "ok" for s in status[:first_expired]) and all(s == "expired" for s in status[first_expired:])
    assert all(len(b) == 1 for _, b in log)


def test_budget_from_environment_and_string_keys(monkeypatch):
    need, pairs, age = [int(3 * GB)], [1e9], [0.0]
    # default budget 4 GiB: 3 GiB fits in 8 GiB free
    assert pc.pc_debug_admission_plan(need, pairs, age, 8 * GB, 288 * GB).tolist() == [A]
    monkeypatch.setenv("PC_HBM_BUDGET_BYTES", str(6 * GB))
    assert pc.pc_debug_admission_plan(need, pairs, age, 8 * GB, 288 * GB).tolist() == [W]
    # an explicit key wins over the environment
    assert pc.pc_debug_admission_plan(need, pairs, age, 8 * GB, 288 * GB, config={"hbm_budget_bytes": 0}).tolist() == [A]
    monkeypatch.setenv("PC_HBM_BUDGET_BYTES", "lots")
    with pytest.raises(pc.PcError):
        pc.pc_debug_admission_plan(need, pairs, age, 8 * GB, 288 * GB)
    monkeypatch.delenv("PC_HBM_BUDGET_BYTES")
    assert pc.pc_debug_admission_plan(need, pairs, age, 8 * GB, 288 * GB, config={"log_path": "/tmp/x.jsonl"}).tolist() == [A]
    with pytest.raises(pc.PcError):
        pc.pc_debug_admission_plan(need, pairs, age, 8 * GB, 288 * GB, config={"log_path": 3})


def test_smallest_first_policy_with_ageing():
    pairs = [3e12, 1e9, 5e11]
    # fewest pairs first: the two small requests share a launch, the big one waits
    assert plan([3, 1, 2], free_gb=100, pairs=pairs, policy=1, max_batch_pairs=2e12) == [W, A, A]
    # a request past the ageing limit goes first whatever its size
    assert plan([3, 1, 2], free_gb=100, pairs=pairs, age=[2.0, 0.0, 0.0], policy=1, aging_s=1.0,
                max_batch_pairs=2e12) == [A, W, W]
    # first come, first served by default
    assert plan([3, 1, 2], free_gb=100, pairs=pairs, max_batch_pairs=2e12) == [A, W, W]
    with pytest.raises(pc.PcError):
        plan([1], free_gb=100, policy=2)


def test_fake_executor_smallest_first_serves_everyone():
    rng = np.random.default_rng(33)
    n = 300
    t = np.cumsum(rng.exponential(0.004, n))
    npts = np.exp(rng.uniform(np.log(1e3), np.log(2e6), n))
    need = (128 * npts + (1 << 20)).astype(np.int64)
    pairs = npts ** 2 / 2
    cfg = {"hbm_budget_bytes": 4 * GB, "max_inflight": 16, "streams": 2, "max_batch_pairs": 2e12,
           "policy": 1, "aging_s": 0.5}
    res, log = _simulate(list(zip(t, need, pairs)), 64 * GB, 288 * GB, cfg)
    assert all(res[i][2] == "ok" for i in range(n))               # nobody starves
    waits = np.array([res[i][0] - t[i] for i in range(n)])
    fifo, _ = _simulate(list(zip(t, need, pairs)), 64 * GB, 288 * GB, {**cfg, "policy": 0})
    fifo_waits = np.array([fifo[i][0] - t[i] for i in range(n)])
    assert np.median(waits) <= np.median(fifo_waits) + 1e-12


# ------------------------------------------------------ parts and their sizes

def _pairs(n, a, b):
    """DD pairs of rows [a, b) of an n-point catalogue (i < j, i in range)."""
    k = b - a
    return k * (n - 1 - a) - k * (k - 1) // 2


def test_large_requests_run_as_row_range_parts_that_cover_every_pair():
    """A 2M-point request on a 1M-random patch, with RR to count, cut into
    parts of about 5e11 pairs: data rows then random rows, contiguous and
    disjoint (so the parts' counts add up to the whole, Sec. 2.1), each part
    at most one row past the slice."""
    n, nr, slice_pairs = 2_000_000, 1_000_000, 5e11
    parts = pc.pc_debug_request_parts(n, nr, 41, True, slice_pairs)
    data = [p["rows"] for p in parts if p["rows"][0] < p["rows"][1]]
    rr = [p["rr_rows"] for p in parts if p["rr_rows"][0] < p["rr_rows"][1]]
    assert data[0][0] == 0 and data[-1][1] == n
    assert all(x[1] == y[0] for x, y in zip(data, data[1:]))
    assert rr[0][0] == 0 and rr[-1][1] == nr
    assert all(x[1] == y[0] for x, y in zip(rr, rr[1:]))
    total = n * (n - 1) // 2 + n * nr + nr * (nr - 1) // 2
    got = sum(_pairs(n, a, b) + (b - a) * nr for a, b in data) + sum(_pairs(nr, c, d) for c, d in rr)
    assert got == total
    for a, b in data:
        row = (n - 1 - a) + nr          # the first row is the largest
        assert _pairs(n, a, b) + (b - a) * nr < slice_pairs + row
    assert len(parts) >= total / (slice_pairs + n + nr)
    # RR already cached: no random rows; slicing off: one part with everything
    assert all(p["rr_rows"][0] == p["rr_rows"][1] for p in pc.pc_debug_request_parts(n, nr, 41, False))
    one = pc.pc_debug_request_parts(n, nr, 41, True, 0)
    assert len(one) == 1 and one[0]["rows"] == (0, n) and one[0]["rr_rows"] == (0, nr)


def test_admission_need_counts_the_launch_workspace():
    """The bytes admission reserves for a request come from the batch
    runner's own plan: converted and ordered copies (~100 B per point), plus
    16 bytes per pair of 256-point tiles for the survivor lists -- for a
    2M-point request against 1M randoms with RR, over 1.2 GB in one part, so
    a 1 GB budget window holds it back while its 5e11-pair parts fit."""
    n, nr = 2_000_000, 1_000_000
    T, TR = -(-n // 256), -(-nr // 256)
    items = T * (T + 1) // 2 + T * TR + TR * (TR + 1) // 2
    whole = pc.pc_debug_request_parts(n, nr, 41, True, 0)[0]["need_bytes"]
    assert whole >= 16 * items + 100 * n
    assert whole > 1.2e9
    parts = pc.pc_debug_request_parts(n, nr, 41, True, 5e11)
    worst = max(p["need_bytes"] for p in parts)
    assert worst < whole
    avail_gb = 4 + 1.0                       # budget 4 GB + a 1 GB window
    assert plan([whole / GB], free_gb=avail_gb) == [W]
    assert plan([worst / GB], free_gb=avail_gb) == [A] or worst > GB
    # a small request's need is small
    small = pc.pc_debug_request_parts(5_000, nr, 20, False)[0]["need_bytes"]
    assert small < 40e6

