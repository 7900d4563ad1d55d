"""pc_count_batch_static -- the batch entry point that allocates no device
memory (its work area is a fixed device array of the library) -- against
pc_count_batch and the oracle, through the C ABI: two calls in a row, the
second on a smaller input, in every kernel; no library allocation is made
(every allocation the library would make is set to fail); a batch larger
than the fixed area is refused before anything runs."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
import paper_1208_3658_amd as pc  # noqa: E402

pytestmark = pytest.mark.gpu

MODES = {"mixed": pc.PC_MIXED, "matrix_cores": pc.PC_MIXED | pc.PC_MATRIX_CORES, "fp64": pc.PC_FP64_PLAIN,
         "tuned": pc.PC_MIXED | pc.PC_TUNED}


def dev(cat):
    return tuple(torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in cat)


def ddrrr(D, R, e):
    return [{"A": D, "edges": e}, {"A": D, "B": R, "edges": e, "auto": False}, {"A": R, "edges": e}]


def oracle_ddrrr(D, R, e):
    return [oracle.count(D, e), oracle.count(D, e, B=R, auto=False), oracle.count(R, e)]


@pytest.fixture(scope="module")
def inputs():
    big = synth.config_small()                 # 10,000 clustered + 10,000 random, 30 log bins
    small = synth.config_small(scale=0.23)     # 2,300 + 2,300
    e_small = synth.log_edges(0.005, 15.0, 61)
    return {
        "big": (big, oracle_ddrrr(big["D"], big["R"], big["edges"])),
        "small": (small, e_small, oracle_ddrrr(small["D"], small["R"], e_small)),
    }


@pytest.mark.parametrize("mode", list(MODES))
def test_static_two_calls_equal_pc_count_batch_and_oracle(inputs, mode):
    big, want_big = inputs["big"]
    small, e_small, want_small = inputs["small"]
    m = MODES[mode]
    jobs_big = ddrrr(dev(big["D"]), dev(big["R"]), big["edges"])
    ref_big = pc.pc_count_batch(jobs_big, mode=m)
    got_big = pc.pc_count_batch_static(jobs_big, mode=m)
    # the second call: fewer points, another edge set, host inputs for one
    # catalogue (copied into the fixed area)
    jobs_small = ddrrr(dev(small["D"]), small["R"], e_small)
    got_small = pc.pc_count_batch_static(jobs_small, mode=m)
    ref_small = pc.pc_count_batch(jobs_small, mode=m)
    for got, ref, want in zip(got_big, ref_big, want_big):
        assert got.tolist() == ref.tolist() == want.tolist(), mode
    for got, ref, want in zip(got_small, ref_small, want_small):
        assert got.tolist() == ref.tolist() == want.tolist(), mode


def test_static_makes_no_library_allocation(inputs):
    """Every device allocation the library would make fails while the call
    runs (the testing hook that injects allocation failures); the call must
    not notice."""
    small, e_small, want_small = inputs["small"]
    jobs = ddrrr(dev(small["D"]), dev(small["R"]), e_small)
    try:
        pc.pc_debug_fail_allocations(1000)
        got = pc.pc_count_batch_static(jobs)
        # control: the allocating entry point does fail under the same hook
        with pytest.raises(pc.PcError) as ex:
            pc.pc_count_batch(jobs)
        assert ex.value.code == pc.PC_ERR_NOMEM
    finally:
        pc.pc_debug_fail_allocations(0)
    for g, w in zip(got, want_small):
        assert g.tolist() == w.tolist()


def test_static_refuses_a_batch_beyond_its_area(inputs):
    """DR of two catalogues of 10^6 points needs more than the fixed area
    (about 440 MB): PC_ERR_INVALID with the sizes in the message, counts
    untouched, and the next call is exact."""
    n = 1_000_000
    a = pc.as_catalog((torch.zeros(n, dtype=torch.float64, device="cuda"),
                       torch.zeros(n, dtype=torch.float64, device="cuda")))
    b = pc.as_catalog((torch.zeros(n, dtype=torch.float64, device="cuda"),
                       torch.zeros(n, dtype=torch.float64, device="cuda")))
    e = synth.log_edges(0.01, 10.0, 30)
    counts = np.full(e.size + 1, 7, dtype=np.uint64)
    job = (pc.pc_job * 1)()
    job[0] = pc.pc_job(pc.ctypes.pointer(a.c), pc.ctypes.pointer(b.c), e.ctypes.data, e.size, 0, 0, -1,
                       counts.ctypes.data)
    rc = pc.lib().pc_count_batch_static(job, 1, pc.PC_MIXED, None)
    assert rc == pc.PC_ERR_INVALID, rc
    msg = pc.pc_last_error()
    assert "workspace" in msg and str(pc.PC_STATIC_SCRATCH_BYTES) in msg, msg
    assert np.all(counts == 7)
    small, e_small, want_small = inputs["small"]
    got = pc.pc_count_batch_static(ddrrr(dev(small["D"]), dev(small["R"]), e_small))
    for g, w in zip(got, want_small):
        assert g.tolist() == w.tolist()
