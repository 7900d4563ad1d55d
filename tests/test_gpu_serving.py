"""GPU tests of the w(theta) server: results in the continuously batched mix
equal the same request alone and the oracle; admission by device memory;
RR cache; latency statistics."""
import time

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
import paper_1208_3658_amd as pc  # noqa: E402

pytestmark = pytest.mark.gpu


def _patches_and_requests(n_req, n_min=200, n_max=20_000, n_random=20_000):
    patches, reqs = synth.serve_stream(n_req, rate_hz=50.0, n_patches=3, n_min=n_min, n_max=n_max,
                                       n_random=n_random, seed_config=7)
    rands = [synth.pool_random(patches, p, 7) for p in range(len(patches))]
    cats = [synth.request_catalog(patches, r, 7) for r in reqs]
    return patches, reqs, rands, cats


def test_served_results_equal_alone_and_oracle():
    patches, reqs, rands, cats = _patches_and_requests(24)
    srv = pc.Server({"streams": 2, "max_inflight": 16})
    try:
        for p, R in enumerate(rands):
            srv.set_random(p, R)
        ids = []
        t0 = time.perf_counter()
        for r, cat in zip(reqs, cats):                 # arrivals spread over the running batches
            while time.perf_counter() - t0 < r["t"]:
                time.sleep(0.001)
            src = tuple(torch.from_numpy(x).cuda() for x in cat) if r["id"] % 2 else cat
            ids.append(srv.submit(src, r["patch"], r["edges"]))
        srv.drain()
        st = srv.stats()
        assert st["completed"] == len(reqs) and st["failed"] == 0
        assert st["batches"] >= 2
        for jid, r, cat in zip(ids, reqs, cats):
            res = srv.poll(jid)
            R = rands[r["patch"]]
            e = r["edges"]
            # the same request alone
            dd, dr, rr = pc.pc_count_batch([{"A": cat, "edges": e}, {"A": cat, "B": R, "edges": e, "auto": False},
                                            {"A": R, "edges": e}])
            assert res["DD"].tolist() == dd.tolist()
            assert res["DR"].tolist() == dr.tolist()
            assert res["RR"].tolist() == rr.tolist()
            w_alone = pc.pc_wtheta(dd[1:-1], dr[1:-1], rr[1:-1], cat[0].size, R[0].size)
            assert np.array_equal(np.isnan(res["w"]), np.isnan(w_alone))
            f = ~np.isnan(w_alone)
            assert np.array_equal(res["w"][f], w_alone[f])
            assert res["latency_s"] > 0
            if cat[0].size <= 3000:                     # oracle on the small requests
                assert res["DD"].tolist() == oracle.count(cat, e).tolist()
                assert res["DR"].tolist() == oracle.count(cat, e, B=R, auto=False).tolist()
        assert st["p99_s"] >= st["p50_s"] > 0
        assert st["rr_cached"] >= 1
    finally:
        srv.close()


def test_admission_rejects_requests_that_can_never_fit():
    srv = pc.Server({"hbm_budget_bytes": 1 << 62})
    try:
        R = synth.uniform_patch(1000, synth.centred_patch(10.0), np.random.default_rng(1))
        srv.set_random(0, R)
        jid = srv.submit(R, 0, synth.log_edges(0.1, 5.0, 10))
        srv.drain()
        with pytest.raises(pc.PcError) as ex:
            srv.poll(jid)
        assert ex.value.code == pc.PC_ERR_NOMEM
        assert srv.stats()["failed"] == 1
    finally:
        srv.close()


def test_submit_validation_and_unknown_patch():
    srv = pc.Server()
    try:
        R = synth.uniform_patch(500, synth.centred_patch(10.0), np.random.default_rng(2))
        with pytest.raises(pc.PcError) as ex:
            srv.submit(R, 3, [1.0, 2.0])
        assert ex.value.code == pc.PC_ERR_INVALID
        srv.set_random(3, R)
        with pytest.raises(pc.PcError):
            srv.submit(R, 3, [2.0, 1.0])
        with pytest.raises(pc.PcError):
            srv.submit((R[0], np.full(R[0].size, 100.0)), 3, [1.0, 2.0])
    finally:
        srv.close()


def test_server_config_errors():
    with pytest.raises(pc.PcError):
        pc.Server({"no_such_key": 1})
    with pytest.raises(pc.PcError):
        pc.Server({"mode": 7})


def _big_and_small(seed):
    rng = np.random.default_rng(seed)
    patch = synth.centred_patch(50.0)
    R = synth.uniform_patch(1_000_000, patch, rng)
    big = synth.uniform_patch(1_000_000, patch, rng)           # tens of ms on the device
    small = [synth.uniform_patch(n, patch, rng) for n in (1500, 2500)]
    return R, big, small, synth.log_edges(0.01, 10.0, 20)


def _alone(cat, R, e):
    return pc.pc_count_batch([{"A": cat, "edges": e}, {"A": cat, "B": R, "edges": e, "auto": False},
                              {"A": R, "edges": e}])


def test_cancel_queued_running_and_finished_requests():
    R, big, (s1, s2), e = _big_and_small(41)
    srv = pc.Server({"streams": 1, "max_inflight": 1})
    try:
        srv.set_random(0, R)
        a = srv.submit(big, 0, e)
        b = srv.submit(s1, 0, e)        # queued behind a (one request on the device at a time)
        c = srv.submit(s2, 0, e)
        assert srv.cancel(b) is True
        with pytest.raises(pc.PcError) as ex:
            srv.poll(b)
        assert ex.value.code == pc.PC_ERR_CANCELLED
        with pytest.raises(pc.PcError) as ex:
            srv.cancel(b)               # already polled: unknown now
        assert ex.value.code == pc.PC_ERR_INVALID
        srv.drain()
        assert srv.cancel(a) is False   # finished first: the answer stays
        for jid, cat in ((a, big), (c, s2)):
            res = srv.poll(jid)
            dd, dr, rr = _alone(cat, R, e)
            assert res["DD"].tolist() == dd.tolist() and res["DR"].tolist() == dr.tolist()
            assert res["RR"].tolist() == rr.tolist()
        # cancelling a running request discards its answer
        d = srv.submit(big, 0, e)
        while srv.stats()["inflight"] == 0 and srv.stats()["completed"] < 3:
            time.sleep(0.0005)
        was_running = srv.cancel(d)
        srv.drain()
        st = srv.stats()
        if was_running:
            with pytest.raises(pc.PcError) as ex:
                srv.poll(d)
            assert ex.value.code == pc.PC_ERR_CANCELLED and st["cancelled"] == 2
        else:                               # it finished before the cancel arrived
            assert srv.poll(d)["DD"].tolist() == _alone(big, R, e)[0].tolist() and st["cancelled"] == 1
    finally:
        srv.close()


def test_queueing_deadline_fails_requests_that_wait_too_long():
    # request a is admitted and held from the host before its launch (a debug
    # gate), so b waits behind it for as long as the test says, whatever the
    # kernel's duration on this device
    R, big, (s1, _), e = _big_and_small(42)
    srv = pc.Server({"streams": 1, "max_inflight": 1, "deadline_s": 0.5})
    try:
        srv.set_random(0, R)
        srv.hold(True)
        a = srv.submit(big, 0, e)
        t0 = time.time()
        while srv.stats()["inflight"] == 0:
            assert time.time() - t0 < 0.4, "request a was not admitted"
            time.sleep(0.001)
        b = srv.submit(s1, 0, e)        # no slot while a holds it
        time.sleep(0.8)
        assert srv.stats()["queued"] == 1
        srv.hold(False)
        srv.drain()
        assert srv.poll(a)["DD"].sum() == big[0].size * (big[0].size - 1) // 2
        with pytest.raises(pc.PcError) as ex:
            srv.poll(b)
        assert ex.value.code == pc.PC_ERR_CANCELLED
        st = srv.stats()
        assert st["expired"] == 1 and st["completed"] == 1
    finally:
        srv.close()


def test_two_streams_run_two_batches_at_once():
    # one request per launch; the second arrives while the first runs and is
    # taken by the other stream's worker: two batches on the device together
    R, big, (s1, _), e = _big_and_small(43)
    srv = pc.Server({"streams": 2, "max_batch_pairs": 1})
    try:
        srv.set_random(0, R)
        srv.submit(R, 0, e)             # RR of the patch counted (and cached) first
        srv.drain()
        a = srv.submit(big, 0, e)
        b = srv.submit(big, 0, e)
        srv.drain()
        st = srv.stats()
        assert st["max_concurrent_batches"] == 2
        ra, rb = srv.poll(a), srv.poll(b)
        dd, dr, rr = _alone(big, R, e)
        for res in (ra, rb):
            assert res["DD"].tolist() == dd.tolist() and res["DR"].tolist() == dr.tolist()
            assert res["RR"].tolist() == rr.tolist()
    finally:
        srv.close()


def test_request_log_has_one_line_per_finished_request(tmp_path):
    import json
    log = tmp_path / "requests.jsonl"
    patches, reqs, rands, cats = _patches_and_requests(6, n_max=5_000, n_random=5_000)
    srv = pc.Server({"streams": 2, "log_path": str(log)})
    try:
        for p, R in enumerate(rands):
            srv.set_random(p, R)
        ids = [srv.submit(cat, r["patch"], r["edges"]) for r, cat in zip(reqs, cats)]
        srv.drain()
        lines = [json.loads(l) for l in log.read_text().splitlines()]
        assert sorted(l["id"] for l in lines) == sorted(ids)
        for l, r, cat in zip(sorted(lines, key=lambda l: l["id"]), reqs, cats):
            assert l["status"] == 0 and l["error"] == "" and l["batch"] >= 0
            assert l["n"] == cat[0].size and l["n_edges"] == len(r["edges"]) and l["latency_s"] > 0
        for jid in ids:
            srv.poll(jid)
    finally:
        srv.close()


def test_replacing_a_patch_random_catalogue_mid_stream():
    R1, big, (s1, s2), e = _big_and_small(44)
    R2 = synth.uniform_patch(300_000, synth.centred_patch(50.0), np.random.default_rng(45))
    srv = pc.Server({"streams": 2, "max_batch_pairs": 1})
    try:
        srv.set_random(0, R1)
        a = srv.submit(big, 0, e)           # long: still running when the patch is replaced
        b = srv.submit(s1, 0, e)
        srv.set_random(0, R2)
        c = srv.submit(s2, 0, e)            # submitted after the replacement: uses R2
        srv.drain()
        res = {j: srv.poll(j) for j in (a, b, c)}
        dd, dr, rr = _alone(s2, R2, e)
        assert res[c]["DR"].tolist() == dr.tolist() and res[c]["RR"].tolist() == rr.tolist()
        # the earlier requests: DR, RR and w all from one and the same random catalogue
        for j, cat in ((a, big), (b, s1)):
            matches = []
            for R in (R1, R2):
                dd, dr, rr = _alone(cat, R, e)
                w = pc.pc_wtheta(dd[1:-1], dr[1:-1], rr[1:-1], cat[0].size, R[0].size)
                matches.append(res[j]["DR"].tolist() == dr.tolist() and res[j]["RR"].tolist() == rr.tolist()
                               and np.array_equal(res[j]["w"], w, equal_nan=True))
            assert any(matches)
    finally:
        srv.close()


def test_destroy_drops_waiting_requests_and_returns():
    R, big, (s1, _), e = _big_and_small(46)
    srv = pc.Server({"streams": 1, "max_inflight": 1})
    srv.set_random(0, R)
    for _ in range(3):
        srv.submit(big, 0, e)               # one runs, the others wait
    t0 = time.perf_counter()
    srv.close()
    assert time.perf_counter() - t0 < 30.0


def test_large_request_runs_in_parts_small_ones_finish_first():
    """A request of ~2e12 pairs with a slice of 2e11 runs as ~10 row-range
    parts in successive launches (counts over disjoint rows add up exactly,
    Sec. 2.1); a small request submitted after it joins an early launch and
    finishes first.  Both answers equal the same requests counted alone."""
    R, big, (s1, _), e = _big_and_small(44)
    srv = pc.Server({"streams": 1, "slice_pairs": 2e11})
    try:
        srv.set_random(0, R)
        a = srv.submit(big, 0, e)
        b = srv.submit(s1, 0, e)
        srv.drain()
        st = srv.stats()
        assert st["completed"] == 2 and st["failed"] == 0
        assert st["parts_requeued"] >= 6 and st["batches"] >= 7, st
        ra, rb = srv.poll(a), srv.poll(b)
        for res, cat in ((ra, big), (rb, s1)):
            dd, dr, rr = _alone(cat, R, e)
            assert res["DD"].tolist() == dd.tolist() and res["DR"].tolist() == dr.tolist()
            assert res["RR"].tolist() == rr.tolist()
            w = pc.pc_wtheta(dd[1:-1], dr[1:-1], rr[1:-1], cat[0].size, R[0].size)
            assert np.array_equal(res["w"], w, equal_nan=True)
        assert rb["DR"].tolist() == oracle.count(s1, e, B=R, auto=False).tolist()
        assert rb["latency_s"] < ra["latency_s"]
    finally:
        srv.close()
