// fake_device.cpp -- a CPU stand-in for libpc's device layer, so that the
// library's host sources (server, edge tables, estimators, tuner file parser)
// can be built and run under AddressSanitizer, UndefinedBehaviorSanitizer and
// ThreadSanitizer on a machine without a GPU.  Test infrastructure only.
//
// It defines the symbols those sources take from the device-side files
// (pc_api.cpp) and from the HIP runtime.  Its batch runner is a fake
// executor: it checks its arguments like the real one, sleeps a little in
// proportion to the pairs, and puts every pair of a job's rows into one bin
// chosen from the row range, so pair totals are exact and a request counted
// in several row-range parts shows whether its parts cover every row once.
// Device memory is host memory here.  fake_set_free_bytes() and
// fake_fail_next_batches() let a driver shrink the reported free memory and
// make launches fail with PC_ERR_NOMEM.
#include <hip/hip_runtime_api.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../paper_1208_3658_amd/csrc/pc_runtime.hpp"

namespace {
thread_local std::string t_err;
std::mutex g_mu;
std::map<uint64_t, std::shared_ptr<pc::Resident>> g_cats;
std::atomic<uint64_t> g_next{1};
std::atomic<uint64_t> g_free{uint64_t(64) << 30};
std::atomic<int> g_fail_batches{0};
thread_local bool t_timing = false;
}  // namespace

void fake_set_free_bytes(uint64_t b) { g_free = b; }
void fake_fail_next_batches(int n) { g_fail_batches = n; }

namespace pc {

int fail(int code, const std::string &msg) {
    t_err = msg;
    return code;
}
int hip_fail(hipError_t e, const char *what) { return fail(e == hipErrorOutOfMemory ? PC_ERR_NOMEM : PC_ERR_DEVICE, what); }
void clear_error() { t_err.clear(); }
bool injected_alloc_failure() { return false; }

int device_info(DeviceInfo **out) {
    static DeviceInfo d;
    d.device = 0;
    d.cus = 256;
    d.lds_per_block = 64 * 1024;
    d.lds_per_cu = 160 * 1024;
    d.arch = "gfx950 (fake)";
    d.ok = true;
    *out = &d;
    return PC_OK;
}

Resident::~Resident() {}
DevTable::~DevTable() {}

int validate_catalog(const pc_catalog *c, const char *name) {
    if (!c) return fail(PC_ERR_INVALID, std::string(name) + " is NULL");
    if (c->n < 0) return fail(PC_ERR_INVALID, std::string(name) + ".n < 0");
    if (c->n > 0 && (!c->ra_deg || !c->dec_deg)) return fail(PC_ERR_INVALID, std::string(name) + " NULL arrays");
    for (int64_t i = 0; i < c->n; ++i)
        if (!std::isfinite(c->ra_deg[i]) || !std::isfinite(c->dec_deg[i]) || std::fabs(c->dec_deg[i]) > 90.0)
            return fail(PC_ERR_INVALID, std::string(name) + ": bad coordinate");
    return PC_OK;
}

int upload_catalog(const pc_catalog *c, hipStream_t, uint64_t *handle) {
    int rc = validate_catalog(c, "catalogue");
    if (rc) return rc;
    auto r = std::make_shared<Resident>();
    r->n = c->n;
    const uint64_t h = g_next++;
    std::lock_guard<std::mutex> lk(g_mu);
    g_cats[h] = r;
    *handle = h;
    return PC_OK;
}

int release_catalog(uint64_t h) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_cats.erase(h)) return fail(PC_ERR_INVALID, "unknown catalogue handle");
    return PC_OK;
}

int resident_catalog(uint64_t h, std::shared_ptr<Resident> *out) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cats.find(h);
    if (it == g_cats.end()) return fail(PC_ERR_INVALID, "unknown catalogue handle");
    *out = it->second;
    return PC_OK;
}

bool thread_timing() { return t_timing; }
void set_thread_timing(bool on) { t_timing = on; }

int jobs_from_abi(const pc_job *jobs, int32_t n_jobs, std::vector<BatchJob> *out) {
    if (!jobs || n_jobs < 1) return fail(PC_ERR_INVALID, "jobs is NULL or n_jobs < 1");
    out->assign(static_cast<size_t>(n_jobs), BatchJob());
    for (int32_t q = 0; q < n_jobs; ++q) {
        BatchJob &b = (*out)[q];
        b.A = jobs[q].A;
        b.B = jobs[q].B;
        b.theta = jobs[q].theta_edges_deg;
        b.n_edges = jobs[q].n_edges;
        b.auto_flag = jobs[q].auto_flag;
        b.row_begin = jobs[q].row_begin;
        b.row_end = jobs[q].row_end;
        b.counts = jobs[q].counts;
    }
    return PC_OK;
}

static int64_t size_of(const pc_catalog *c, uint64_t h) {
    if (!h) return c ? c->n : -1;
    std::shared_ptr<Resident> r;
    if (resident_catalog(h, &r) != PC_OK) return -1;
    return r->n;
}

int run_batch_opts(const std::vector<BatchJob> &jobs, int mode, hipStream_t, BatchStats *stats,
                   const BatchOpts &opts) {
    if (jobs.empty()) return fail(PC_ERR_INVALID, "no jobs");
    if ((mode & 0xFF) != PC_MIXED && (mode & 0xFF) != PC_FP64_PLAIN) return fail(PC_ERR_INVALID, "unknown mode");
    double pairs = 0, points = 0;
    std::vector<std::pair<int64_t, int64_t>> rows(jobs.size());
    std::vector<int64_t> nb(jobs.size());
    for (size_t q = 0; q < jobs.size(); ++q) {
        const BatchJob &j = jobs[q];
        std::string err;
        if (!validate_edges(j.theta, j.n_edges, err)) return fail(PC_ERR_INVALID, err);
        if (!j.counts && !opts.plan_bytes) return fail(PC_ERR_INVALID, "counts is NULL");
        int64_t nA = -1;
        if (j.hA) {
            if (opts.plan_bytes && opts.plan_sizes && opts.plan_sizes->count(j.hA)) nA = opts.plan_sizes->at(j.hA);
            else nA = size_of(nullptr, j.hA);
        } else {
            if (!opts.trusted_inputs) {
                const int rc = validate_catalog(j.A, "A");
                if (rc) return rc;
            }
            nA = j.A ? j.A->n : -1;
        }
        if (nA < 0) return fail(PC_ERR_INVALID, "catalogue A missing");
        int64_t nB = 0;
        if (!j.auto_flag) {
            if (j.hB && opts.plan_bytes && opts.plan_sizes && opts.plan_sizes->count(j.hB)) nB = opts.plan_sizes->at(j.hB);
            else nB = size_of(j.B, j.hB);
            if (nB < 0) return fail(PC_ERR_INVALID, "catalogue B missing");
        }
        const int64_t r0 = j.row_begin, r1 = j.row_end < 0 ? nA : j.row_end;
        if (r0 < 0 || r1 > nA || r0 > r1) return fail(PC_ERR_INVALID, "row range outside the catalogue");
        rows[q] = {r0, r1};
        nb[q] = j.auto_flag ? nA : nB;
        const double k = static_cast<double>(r1 - r0);
        pairs += j.auto_flag ? k * static_cast<double>(nA - 1 - r0) - 0.5 * k * (k - 1.0) : k * static_cast<double>(nB);
        points += static_cast<double>(nA + nB);
    }
    if (opts.plan_bytes) {
        *opts.plan_bytes = static_cast<uint64_t>(100.0 * points + pairs / 4096.0);
        return PC_OK;
    }
    if (g_fail_batches > 0 && jobs.size() > 3) {  // a launch of several requests
        --g_fail_batches;
        return fail(PC_ERR_NOMEM, "injected: out of device memory");
    }
    std::this_thread::sleep_for(std::chrono::microseconds(50 + static_cast<int64_t>(pairs / 5e7)));
    for (size_t q = 0; q < jobs.size(); ++q) {
        const BatchJob &j = jobs[q];
        const int64_t r0 = rows[q].first, r1 = rows[q].second, n = nb[q];
        uint64_t total = 0;
        for (int64_t i = r0; i < r1; ++i) total += static_cast<uint64_t>(j.auto_flag ? n - 1 - i : n);
        std::fill(j.counts, j.counts + j.n_edges + 1, 0ull);
        if (total) j.counts[1 + (r0 % (j.n_edges - 1))] = total;
    }
    if (stats) *stats = BatchStats();
    return PC_OK;
}

int run_batch(const std::vector<BatchJob> &jobs, int mode, hipStream_t st, BatchStats *stats,
              const LaunchTune *tune) {
    BatchOpts o;
    o.tune = tune;
    return run_batch_opts(jobs, mode, st, stats, o);
}

}  // namespace pc

extern "C" const char *pc_last_error(void) { return t_err.c_str(); }

extern "C" {
hipError_t hipMemGetInfo(size_t *free_b, size_t *total_b) {
    *free_b = g_free;
    *total_b = size_t(288) << 30;
    return hipSuccess;
}
hipError_t hipMemcpy(void *dst, const void *src, size_t n, hipMemcpyKind) {
    memcpy(dst, src, n);
    return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int) {
    *s = reinterpret_cast<hipStream_t>(new char[16]);
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    delete[] reinterpret_cast<char *>(s);
    return hipSuccess;
}
}
