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
