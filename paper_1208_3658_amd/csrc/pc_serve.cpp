// pc_serve.cpp -- w(theta) request server with continuous batching.
//
// Each request is a data catalogue on one registered sky patch plus theta
// edges; its answer is DD, DR (against the patch's resident random
// catalogue), RR and the Landy-Szalay w(theta) (paper Sec. 2, Eq. 2).
//
//  * Admission: a request enters the device only while the memory it needs
//    (128 bytes per point: its converted catalogue, the spatially ordered
//    copies and the sort's staging)
//    fits in the free device memory minus a configured budget, and while fewer
//    than max_inflight requests are on the device.  A request that can never
//    fit fails with PC_ERR_NOMEM.
//  * Continuous batching: one worker thread per stream.  A worker takes every
//    admitted request waiting at that moment (up to max_batch_pairs), packs
//    their DD, DR and missing RR jobs into one persistent launch on its own
//    stream, and returns for more.  Requests that arrive while a batch runs are
//    picked up by an idle worker, so their work overlaps the running batch on
//    the device.
//  * Random catalogues are converted once per patch and stay resident; RR is
//    cached per (patch, edge set), so a patch's RR is counted once.
//  * Latency = submit -> answer ready, per request; the stats report p50/p99.
//  * A request can be cancelled (queued: dropped at once; running: its batch
//    finishes and its answer is discarded), and an optional queueing deadline
//    fails requests still waiting for admission after that many seconds.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pc_runtime.hpp"

namespace pc {

namespace {

using Clock = std::chrono::steady_clock;

struct ServerCfg {
    uint64_t hbm_budget = 4ull << 30;
    int max_inflight = 64;
    int streams = 2;
    double max_batch_pairs = 2e12;
    int mode = PC_MIXED;
    int max_queue = 1 << 20;
    double deadline_s = 0;  // 0: no queueing deadline
    int policy = 0;         // 0: first come first served; 1: fewest pairs first, with ageing
    double aging_s = 1.0;   // policy 1: requests waiting this long go first, oldest first
    std::string log_path;   // one JSON line per finished request is appended here (empty: none)
    double slice_pairs = 5e11;  // a request with more pairs runs as row-range parts of about this many (0: never)
};

// minimal reader for flat {"key": number, ...} objects
bool parse_cfg(const char *s, ServerCfg &c, std::string &err) {
    if (const char *env = getenv("PC_HBM_BUDGET_BYTES")) {
        char *end = nullptr;
        const double v = strtod(env, &end);
        if (end == env || !(v >= 0.0)) { err = "PC_HBM_BUDGET_BYTES must be a number >= 0"; return false; }
        c.hbm_budget = static_cast<uint64_t>(std::min(v, 0x1p63));
    }
    if (!s) return true;
    std::string j(s);
    size_t p = 0;
    auto skip = [&]() { while (p < j.size() && isspace(static_cast<unsigned char>(j[p]))) ++p; };
    skip();
    if (p >= j.size() || j[p] != '{') { err = "config must be a JSON object"; return false; }
    ++p;
    while (true) {
        skip();
        if (p < j.size() && j[p] == '}') break;
        if (p >= j.size() || j[p] != '"') { err = "config: expected a key"; return false; }
        const size_t q = j.find('"', p + 1);
        if (q == std::string::npos) { err = "config: bad key"; return false; }
        const std::string key = j.substr(p + 1, q - p - 1);
        p = q + 1;
        skip();
        if (p >= j.size() || j[p] != ':') { err = "config: expected ':'"; return false; }
        ++p;
        skip();
        if (key == "log_path") {
            if (p >= j.size() || j[p] != '"') { err = "config: log_path must be a string"; return false; }
            const size_t q2 = j.find('"', p + 1);
            if (q2 == std::string::npos) { err = "config: bad log_path"; return false; }
            c.log_path = j.substr(p + 1, q2 - p - 1);
            p = q2 + 1;
            skip();
            if (p < j.size() && j[p] == ',') { ++p; continue; }
            if (p < j.size() && j[p] == '}') break;
            err = "config: expected ',' or '}'";
            return false;
        }
        char *end = nullptr;
        const double v = strtod(j.c_str() + p, &end);
        if (end == j.c_str() + p) { err = "config: value of " + key + " must be a number"; return false; }
        p = static_cast<size_t>(end - j.c_str());
        if (key == "hbm_budget_bytes") c.hbm_budget = static_cast<uint64_t>(std::min(std::max(0.0, v), 0x1p63));
        else if (key == "max_inflight") c.max_inflight = std::max(1, static_cast<int>(v));
        else if (key == "streams") c.streams = std::min(8, std::max(1, static_cast<int>(v)));
        else if (key == "max_batch_pairs") c.max_batch_pairs = std::max(1.0, v);
        else if (key == "mode") c.mode = static_cast<int>(v);
        else if (key == "max_queue") c.max_queue = std::max(1, static_cast<int>(v));
        else if (key == "deadline_s") c.deadline_s = std::max(0.0, v);
        else if (key == "policy") c.policy = static_cast<int>(v);
        else if (key == "aging_s") c.aging_s = std::max(0.0, v);
        else if (key == "slice_pairs") c.slice_pairs = std::max(0.0, v);
        else { err = "config: unknown key " + key; return false; }
        skip();
        if (p < j.size() && j[p] == ',') { ++p; continue; }
        skip();
        if (p < j.size() && j[p] == '}') break;
        err = "config: expected ',' or '}'";
        return false;
    }
    if (c.mode != PC_MIXED && c.mode != PC_FP64_PLAIN) { err = "config: mode must be 0 or 1"; return false; }
    if (c.policy != 0 && c.policy != 1) { err = "config: policy must be 0 or 1"; return false; }
    return true;
}

// The rows a request counts in one launch: DD and DR for data rows [a, b)
// (pairs i < j with i in range, and (i, all randoms)), RR for random rows
// [c, d).  Counts over disjoint row ranges add up exactly (Sec. 2.1, the pair
// matrix cut into submatrices), so a large request can run as several parts
// in successive launches while small requests run in between.
struct Part {
    int64_t a = 0, b = 0;  // data rows
    int64_t c = 0, d = 0;  // random rows (RR), empty when RR is not counted here
};

struct Request {
    uint64_t id = 0;
    int32_t patch = 0;
    std::vector<double> ra, dec;
    std::vector<double> edges;
    Clock::time_point t_submit;
    int64_t n_points = 0;
    int64_t n_random = 0;    // the patch's random catalogue when the request was submitted
    uint64_t random_handle = 0;
    uint64_t need_bytes = 0; // device bytes of the next part's launch (planned on the host)
    double pairs = 0;        // pairs of the whole request (DD + DR)
    double part_pairs = 0;   // pairs of the next part (DD + DR + RR rows)
    Part part;               // the next part
    int64_t data_done = 0;   // data rows counted so far
    int64_t rr_done = 0;     // random rows counted so far (RR)
    bool rr_needed = true;   // RR not cached: counted by this request's parts
    bool started = false;    // a part has run: no queueing deadline any more
    int parts_run = 0;
    bool running = false;    // admitted: its batch is on the device
    bool cancelled = false;  // cancelled while running: answer discarded
    std::vector<uint64_t> pDD, pDR, pRR;  // counts of the part on the device
    // results
    int status = PC_OK;
    std::string error;
    std::vector<uint64_t> DD, DR, RR;
    std::vector<double> w;
    double latency = 0;
    bool done = false;
};

struct Patch {
    uint64_t handle = 0;
    int64_t n = 0;
};

// Admission decision for one queued request.
enum AdmitOutcome : int32_t { kAdmit = 0, kNeverFits = 1, kExpired = 2, kWait = 3 };

struct QueuedView {
    uint64_t need;  // device bytes the request needs while it runs
    double pairs;   // pairs its DD and DR jobs count
    double age_s;   // seconds since submission
    bool started = false;  // a part of it has already run (no queueing deadline)
};

// The admission policy, free of device calls (the server feeds it the free
// and total device memory it reads; tests feed it chosen figures).  Walks
// the queue from the front (policy 0; policy 1 visits aged requests first,
// then the rest by fewest pairs):
//  * a request that cannot fit even on an empty device (need + budget >
//    total) fails, wherever it stands;
//  * a request past the queueing deadline fails, wherever it stands;
//  * otherwise requests are admitted in order while the in-flight limit, the
//    free memory (free - budget - bytes reserved by running batches) and the
//    pairs per launch allow (the first request of a batch is exempt from the
//    pairs limit); the first that does not fit ends admission, and it and
//    every later request wait (first come, first served).
// Returns the number admitted; *memory_blocked says whether admission ended
// on free memory.
int plan_admission(const QueuedView *q, int n, uint64_t free_b, uint64_t total_b, uint64_t reserved,
                   int inflight, const ServerCfg &cfg, int32_t *outcome, bool *memory_blocked) {
    const uint64_t held = cfg.hbm_budget + std::min<uint64_t>(reserved, UINT64_MAX - cfg.hbm_budget);
    const uint64_t avail = free_b > held ? free_b - held : 0;
    uint64_t bytes = 0;
    double pairs = 0;
    int admitted = 0;
    bool open = true;
    *memory_blocked = false;
    // visiting order: the queue's, or (policy 1) requests past the ageing
    // limit first, oldest first, then the rest by pairs, fewest first (ties in
    // queue order)
    std::vector<int> order(static_cast<size_t>(n));
    for (int i = 0; i < n; ++i) order[static_cast<size_t>(i)] = i;
    if (cfg.policy == 1)
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            const bool oa = q[a].age_s >= cfg.aging_s, ob = q[b].age_s >= cfg.aging_s;
            if (oa != ob) return oa;
            if (oa) return false;  // both aged: queue order (stable)
            return q[a].pairs < q[b].pairs;
        });
    for (int k = 0; k < n; ++k) {
        const int i = order[static_cast<size_t>(k)];
        if (q[i].need > total_b || cfg.hbm_budget > total_b - q[i].need) {
            outcome[i] = kNeverFits;
            continue;
        }
        if (cfg.deadline_s > 0 && !q[i].started && q[i].age_s > cfg.deadline_s) {
            outcome[i] = kExpired;
            continue;
        }
        if (open) {
            const bool slot = inflight + admitted < cfg.max_inflight;
            const bool mem = q[i].need <= avail - bytes;  // bytes <= avail: only fitting requests add to it
            const bool fits_launch = admitted == 0 || pairs + q[i].pairs <= cfg.max_batch_pairs;
            if (slot && mem && fits_launch) {
                outcome[i] = kAdmit;
                bytes += q[i].need;
                pairs += q[i].pairs;
                ++admitted;
                continue;
            }
            open = false;
            *memory_blocked = slot && !mem;
        }
        outcome[i] = kWait;
    }
    return admitted;
}

// RR cache key: the random catalogue's handle (unique per upload, so counts
// of a replaced catalogue never match) and the edges.
std::string rr_key(uint64_t random_handle, const std::vector<double> &e) {
    std::string k(reinterpret_cast<const char *>(&random_handle), sizeof(random_handle));
    k.append(reinterpret_cast<const char *>(e.data()), sizeof(double) * e.size());
    return k;
}

// DD pairs of data rows [a, b) of an n-point catalogue (pairs i < j with i in
// the range): sum over i of n - 1 - i.
double auto_rows_pairs(int64_t n, int64_t a, int64_t b) {
    const double k = static_cast<double>(b - a);
    return k * static_cast<double>(n - 1 - a) - 0.5 * k * (k - 1.0);
}

// The next part of request r: all that is left when that is at most `slice`
// pairs (or slicing is off); else data rows from where the last part ended
// whose DD + DR pairs first reach `slice`, and once the data rows are done,
// random rows for RR likewise.  *pairs receives the part's pairs.
Part next_part(const Request &r, double slice, double *pairs) {
    const int64_t n = r.n_points, nr = r.n_random;
    const int64_t c = r.rr_needed ? r.rr_done : nr, d = nr;
    const double data_left = auto_rows_pairs(n, r.data_done, n) +
                             static_cast<double>(n - r.data_done) * static_cast<double>(nr);
    const double rr_left = auto_rows_pairs(nr, c, d);
    Part p;
    if (slice <= 0 || data_left + rr_left <= slice) {
        p.a = r.data_done;
        p.b = n;
        p.c = c;
        p.d = d;
        *pairs = data_left + rr_left;
        return p;
    }
    if (r.data_done < n) {
        const int64_t a = r.data_done;
        auto rows_pairs = [&](int64_t b) {
            return auto_rows_pairs(n, a, b) + static_cast<double>(b - a) * static_cast<double>(nr);
        };
        int64_t lo = a + 1, hi = n;  // the first b whose pairs reach `slice`
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (rows_pairs(mid) >= slice) hi = mid;
            else lo = mid + 1;
        }
        p.a = a;
        p.b = lo;
        p.c = p.d = 0;
        *pairs = rows_pairs(lo);
        return p;
    }
    int64_t lo = c + 1, hi = d;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (auto_rows_pairs(nr, c, mid) >= slice) hi = mid;
        else lo = mid + 1;
    }
    p.a = p.b = n;
    p.c = c;
    p.d = lo;
    *pairs = auto_rows_pairs(nr, c, lo);
    return p;
}

// The jobs of one part: DD and DR over data rows [a, b) (left out when the
// range is empty and the part counts RR rows), RR over random rows [c, d).
// `cat` describes the request's host copy of its catalogue.
void part_jobs(const Request &r, const Part &p, const pc_catalog *cat, std::vector<BatchJob> *jobs,
               uint64_t *dd, uint64_t *dr, uint64_t *rr) {
    const int32_t ne = static_cast<int32_t>(r.edges.size());
    const bool has_rr = p.c < p.d;
    if (p.a < p.b || !has_rr) {
        BatchJob j;
        j.A = cat;
        j.theta = r.edges.data();
        j.n_edges = ne;
        j.auto_flag = 1;
        j.row_begin = p.a;
        j.row_end = p.b;
        j.counts = dd;
        jobs->push_back(j);
        j.hB = r.random_handle;
        j.auto_flag = 0;
        j.counts = dr;
        jobs->push_back(j);
    }
    if (has_rr) {
        BatchJob j;
        j.hA = r.random_handle;
        j.theta = r.edges.data();
        j.n_edges = ne;
        j.auto_flag = 1;
        j.row_begin = p.c;
        j.row_end = p.d;
        j.counts = rr;
        jobs->push_back(j);
    }
}

// Device bytes the launch of part p needs on its own, planned on the host by
// the batch runner itself (its workspace: converted and ordered copies, sort
// scratch, survivor lists, results).  `sizes` describes resident catalogues
// that need not exist (tests).
int part_need_bytes(const Request &r, const Part &p, int mode, const std::map<uint64_t, int64_t> *sizes,
                    uint64_t *bytes) {
    pc_catalog cat;
    cat.ra_deg = r.ra.empty() ? reinterpret_cast<const double *>(&r) : r.ra.data();
    cat.dec_deg = r.dec.empty() ? reinterpret_cast<const double *>(&r) : r.dec.data();
    cat.n = r.n_points;
    cat.on_device = 0;
    cat.reserved = 0;
    std::vector<BatchJob> jobs;
    part_jobs(r, p, &cat, &jobs, nullptr, nullptr, nullptr);
    BatchOpts o;
    uint64_t b = 0;
    o.plan_bytes = &b;
    o.trusted_inputs = true;
    o.plan_sizes = sizes;
    const int rc = run_batch_opts(jobs, mode, nullptr, nullptr, o);
    if (rc) return rc;
    *bytes = b + (1u << 20);  // plus the launch's tables and descriptors, generously
    return PC_OK;
}

}  // namespace

struct Server {
    ServerCfg cfg;
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> jobs;  // submitted, not yet polled
    std::map<int32_t, Patch> patches;
    std::map<std::string, std::vector<uint64_t>> rr_cache;
    std::vector<uint64_t> retired;  // replaced random catalogues, released once no launch runs
    uint64_t next_id = 1;
    int inflight = 0;
    uint64_t reserved = 0;
    bool stop = false;
    bool hold = false;  // debug gate: admitted batches wait before their launch
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    // stats
    uint64_t n_submitted = 0, n_done = 0, n_failed = 0, n_batches = 0, n_admit_waits = 0;
    uint64_t n_cancelled = 0, n_expired = 0, n_requeued = 0, n_split_batches = 0;
    int running_batches = 0, max_running_batches = 0;
    double pairs_done = 0, busy_s = 0;
    std::vector<double> latencies;
    Clock::time_point t0 = Clock::now();
    std::string stats_buf;
    std::vector<std::string> log_pending;  // request log lines not yet written (mu)
    std::mutex log_mu;                     // serialises appends to cfg.log_path

    void worker(int k);
    int take_batch(std::vector<std::shared_ptr<Request>> &out, uint64_t &bytes);
    void prepare(Request &r);                                            // mu held
    int launch_parts(const std::vector<std::shared_ptr<Request>> &reqs, hipStream_t st, std::string *err);
    void finish_part(Request &r, int rc, const std::string &err);        // mu held
    void release_retired();                                              // mu held
    void finish_unrun(Request &r, int status, const std::string &msg);  // mu held
    void log_request(const Request &r, int64_t batch);                  // mu held
    void write_log();                                                    // mu not held
};

void Server::log_request(const Request &r, int64_t batch) {
    if (cfg.log_path.empty()) return;
    std::string err;
    for (char ch : r.error) {
        if (ch == '"' || ch == '\\') err += '\\';
        if (static_cast<unsigned char>(ch) >= 0x20) err += ch;
    }
    std::ostringstream o;
    o.precision(9);
    o << "{\"id\": " << r.id << ", \"patch\": " << r.patch << ", \"n\": " << r.n_points
      << ", \"n_edges\": " << r.edges.size() << ", \"pairs\": " << r.pairs << ", \"status\": " << r.status
      << ", \"error\": \"" << err << "\", \"batch\": " << batch
      << ", \"submit_s\": " << std::chrono::duration<double>(r.t_submit - t0).count()
      << ", \"latency_s\": " << r.latency << "}\n";
    log_pending.push_back(o.str());
}

void Server::write_log() {
    if (cfg.log_path.empty()) return;
    std::vector<std::string> lines;
    {
        std::lock_guard<std::mutex> lk(mu);
        lines.swap(log_pending);
    }
    if (lines.empty()) return;
    std::lock_guard<std::mutex> lk(log_mu);
    if (FILE *f = fopen(cfg.log_path.c_str(), "a")) {
        for (const auto &l : lines) fwrite(l.data(), 1, l.size(), f);
        fclose(f);
    }
}

void Server::finish_unrun(Request &r, int status, const std::string &msg) {
    r.status = status;
    r.error = msg;
    r.latency = std::chrono::duration<double>(Clock::now() - r.t_submit).count();
    r.done = true;
    std::vector<double>().swap(r.ra);
    std::vector<double>().swap(r.dec);
    ++n_failed;
    if (status == PC_ERR_CANCELLED) ++n_cancelled;
    log_request(r, -1);
}

int Server::take_batch(std::vector<std::shared_ptr<Request>> &out, uint64_t &bytes) {
    // called with mu held
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = total_b = 0;
    bytes = 0;
    if (queue.empty()) return 0;
    const auto now = Clock::now();
    std::vector<QueuedView> view(queue.size());
    std::vector<int32_t> outcome(queue.size());
    for (size_t i = 0; i < queue.size(); ++i)
        view[i] = {queue[i]->need_bytes, queue[i]->part_pairs,
                   std::chrono::duration<double>(now - queue[i]->t_submit).count(), queue[i]->started};
    bool mem_blocked = false;
    plan_admission(view.data(), static_cast<int>(view.size()), free_b, total_b, reserved, inflight, cfg,
                   outcome.data(), &mem_blocked);
    if (mem_blocked) ++n_admit_waits;
    std::deque<std::shared_ptr<Request>> keep;
    bool failed = false;
    for (size_t i = 0; i < queue.size(); ++i) {
        auto &r = queue[i];
        switch (outcome[i]) {
            case kAdmit:
                if (r->rr_needed && r->rr_done == 0 && r->part.c < r->part.d) {
                    // RR counted (and cached) since the part was planned
                    auto it = rr_cache.find(rr_key(r->random_handle, r->edges));
                    if (it != rr_cache.end()) {
                        r->RR = it->second;
                        r->rr_needed = false;
                        r->part.c = r->part.d = 0;
                    }
                }
                r->running = true;
                bytes += r->need_bytes;
                ++inflight;
                out.push_back(r);
                break;
            case kNeverFits:
                finish_unrun(*r, PC_ERR_NOMEM,
                             "request needs " + std::to_string(r->need_bytes) + " bytes; device has " +
                                 std::to_string(total_b) + " with a budget of " + std::to_string(cfg.hbm_budget));
                failed = true;
                break;
            case kExpired:
                ++n_expired;
                finish_unrun(*r, PC_ERR_CANCELLED, "queueing deadline passed before admission");
                failed = true;
                break;
            default:
                keep.push_back(r);
        }
    }
    queue.swap(keep);
    reserved += bytes;
    if (failed) cv_done.notify_all();
    return static_cast<int>(out.size());
}

// Replaced random catalogues are released once no launch runs and no request
// that has been counted in part still refers to them (mu held).
void Server::release_retired() {
    if (running_batches != 0 || retired.empty()) return;
    std::vector<uint64_t> keep;
    for (uint64_t h : retired) {
        const bool used = std::any_of(queue.begin(), queue.end(), [&](const std::shared_ptr<Request> &q) {
            return q->random_handle == h;
        });
        if (used) keep.push_back(h);
        else release_catalog(h);
    }
    retired.swap(keep);
}

// The next part of r and the device bytes its launch needs (mu held).
void Server::prepare(Request &r) {
    r.part = next_part(r, cfg.slice_pairs, &r.part_pairs);
    uint64_t b = 0;
    if (part_need_bytes(r, r.part, cfg.mode, nullptr, &b) != PC_OK) {
        // planning only fails for arguments that were checked at submission;
        // fall back to a generous figure rather than refusing the request
        const double pts = static_cast<double>(r.n_points) + static_cast<double>(r.n_random);
        b = static_cast<uint64_t>(std::min(0x1p62, 200.0 * pts + 16.0 * r.part_pairs / 65536.0)) + (1u << 20);
    }
    r.need_bytes = b;
}

// One launch for the current parts of `reqs` on stream st: each request's
// part counts land in its pDD, pDR, pRR.  RR over the same rows of the same
// random catalogue and edges is counted once.
int Server::launch_parts(const std::vector<std::shared_ptr<Request>> &reqs, hipStream_t st, std::string *err) {
    std::vector<pc_catalog> cats(reqs.size());
    std::vector<BatchJob> jobs;
    std::map<std::tuple<std::string, int64_t, int64_t>, size_t> rr_of;
    std::vector<std::vector<uint64_t>> rr_store;
    std::vector<size_t> rr_job(reqs.size(), SIZE_MAX);
    std::vector<size_t> rr_first;  // jobs index of each RR job
    for (size_t q = 0; q < reqs.size(); ++q) {
        Request &r = *reqs[q];
        const size_t ne = r.edges.size();
        r.pDD.assign(ne + 1, 0);
        r.pDR.assign(ne + 1, 0);
        r.pRR.assign(ne + 1, 0);
        cats[q].ra_deg = r.ra.data();
        cats[q].dec_deg = r.dec.data();
        cats[q].n = r.n_points;
        cats[q].on_device = 0;
        cats[q].reserved = 0;
        Part p = r.part;
        const bool has_rr = p.c < p.d;
        std::tuple<std::string, int64_t, int64_t> key;
        bool shared = false;
        if (has_rr) {
            key = std::make_tuple(rr_key(r.random_handle, r.edges), p.c, p.d);
            auto it = rr_of.find(key);
            if (it != rr_of.end()) {
                rr_job[q] = it->second;
                shared = true;
                p.c = p.d = 0;  // counted by an earlier request of this launch
            }
        }
        const size_t before = jobs.size();
        part_jobs(r, p, &cats[q], &jobs, r.pDD.data(), r.pDR.data(), nullptr);
        if (has_rr && !shared) {
            rr_job[q] = rr_store.size();
            rr_of.emplace(key, rr_store.size());
            rr_store.emplace_back(ne + 1, 0);
            for (size_t k = before; k < jobs.size(); ++k)
                if (jobs[k].hA) rr_first.push_back(k);
        }
    }
    for (size_t s = 0; s < rr_first.size(); ++s) jobs[rr_first[s]].counts = rr_store[s].data();
    BatchOpts o;
    o.trusted_inputs = true;  // checked point by point at submission
    const int rc = run_batch_opts(jobs, cfg.mode, st, nullptr, o);
    if (rc) {
        *err = pc_last_error();
        return rc;
    }
    for (size_t q = 0; q < reqs.size(); ++q)
        if (rr_job[q] != SIZE_MAX) reqs[q]->pRR = rr_store[rr_job[q]];
    return PC_OK;
}

// A part of r has run (status rc): add its counts, then either requeue r
// for its next part or finish it (mu held).
void Server::finish_part(Request &r, int rc, const std::string &err) {
    r.running = false;
    --inflight;
    bool done = true;
    if (r.cancelled) {
        r.status = PC_ERR_CANCELLED;
        r.error = "request cancelled";
        ++n_failed;
        ++n_cancelled;
    } else if (rc != PC_OK) {
        r.status = rc;
        r.error = err;
        ++n_failed;
    } else {
        const size_t ne = r.edges.size();
        for (size_t k = 0; k <= ne; ++k) {
            r.DD[k] += r.pDD[k];
            r.DR[k] += r.pDR[k];
        }
        if (r.part.c < r.part.d)
            for (size_t k = 0; k <= ne; ++k) r.RR[k] += r.pRR[k];
        r.data_done = r.part.b;
        if (r.part.c < r.part.d) r.rr_done = r.part.d;
        r.started = true;
        ++r.parts_run;
        const bool rr_left = r.rr_needed && r.rr_done < r.n_random;
        if (r.data_done < r.n_points || rr_left) {
            done = false;
        } else {
            if (r.rr_needed) {
                // cache RR unless the patch's random catalogue was replaced meanwhile
                const bool current = std::any_of(patches.begin(), patches.end(),
                                                 [&](const std::pair<const int32_t, Patch> &pp) {
                                                     return pp.second.handle == r.random_handle;
                                                 });
                if (current) rr_cache.emplace(rr_key(r.random_handle, r.edges), r.RR);
            }
            const int32_t nb = static_cast<int32_t>(r.edges.size()) - 1;
            r.w.assign(nb, 0.0);
            if (r.n_points >= 2 && r.n_random >= 2)
                landy_szalay(r.DD.data() + 1, r.DR.data() + 1, r.RR.data() + 1, nb, r.n_points, r.n_random,
                             r.w.data());
            else
                std::fill(r.w.begin(), r.w.end(), std::nan(""));
            pairs_done += r.pairs;
            ++n_done;
        }
    }
    std::vector<uint64_t>().swap(r.pDD);
    std::vector<uint64_t>().swap(r.pDR);
    std::vector<uint64_t>().swap(r.pRR);
    if (!done) {
        // back to the front of the queue, ahead of requests submitted later
        prepare(r);
        auto pos = std::find_if(queue.begin(), queue.end(),
                                [&](const std::shared_ptr<Request> &x) { return x->t_submit > r.t_submit; });
        queue.insert(pos, jobs.at(r.id));
        ++n_requeued;
        return;
    }
    r.latency = std::chrono::duration<double>(Clock::now() - r.t_submit).count();
    if (r.status == PC_OK) latencies.push_back(r.latency);
    r.done = true;
    log_request(r, static_cast<int64_t>(n_batches));
    std::vector<double>().swap(r.ra);
    std::vector<double>().swap(r.dec);
}

void Server::worker(int k) {
    (void)hipSetDevice(device);
    hipStream_t st = streams[k];
    while (true) {
        std::vector<std::shared_ptr<Request>> batch;
        uint64_t bytes = 0;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] {
                if (stop) return true;
                if (queue.empty()) return false;
                return true;
            });
            if (stop && queue.empty()) return;
            take_batch(batch, bytes);
            if (batch.empty()) {
                // nothing admissible now: wait for memory to free up
                cv_work.wait_for(lk, std::chrono::milliseconds(2));
                continue;
            }
            max_running_batches = std::max(max_running_batches, ++running_batches);
            // the batch is admitted (it holds its slots and bytes); a test
            // may hold it here to make the queue's timing deterministic
            cv_work.wait(lk, [&] { return !hold || stop; });
        }
        const auto t_start = Clock::now();
        std::string err;
        std::vector<int> rcs(batch.size(), launch_parts(batch, st, &err));
        std::vector<std::string> errs(batch.size(), err);
        const bool split_up = rcs[0] == PC_ERR_NOMEM && batch.size() > 1;
        if (split_up) {
            // the device had less memory than admission saw: the requests
            // run one launch each rather than fail together
            for (size_t q = 0; q < batch.size(); ++q) {
                errs[q].clear();
                rcs[q] = launch_parts({batch[q]}, st, &errs[q]);
            }
        }
        const double dt = std::chrono::duration<double>(Clock::now() - t_start).count();
        {
            std::lock_guard<std::mutex> lk(mu);
            for (size_t q = 0; q < batch.size(); ++q) finish_part(*batch[q], rcs[q], errs[q]);
            if (split_up) ++n_split_batches;
            reserved -= bytes;
            --running_batches;
            ++n_batches;
            release_retired();
            busy_s += dt;
        }
        write_log();
        cv_done.notify_all();
        cv_work.notify_all();
    }
}

}  // namespace pc

using namespace pc;

extern "C" {

int pc_server_create(const char *json_cfg, void **server) {
    clear_error();
    if (!server) return fail(PC_ERR_INVALID, "server is NULL");
    ServerCfg cfg;
    std::string err;
    if (!parse_cfg(json_cfg, cfg, err)) return fail(PC_ERR_INVALID, err);
    DeviceInfo *di = nullptr;
    int rc = device_info(&di);
    if (rc) return rc;
    auto *s = new Server();
    s->cfg = cfg;
    s->device = di->device;
    for (int k = 0; k < cfg.streams; ++k) {
        hipStream_t st = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) {
            for (auto x : s->streams) (void)hipStreamDestroy(x);
            delete s;
            return hip_fail(e, "hipStreamCreate");
        }
        s->streams.push_back(st);
    }
    for (int k = 0; k < cfg.streams; ++k) s->workers.emplace_back(&Server::worker, s, k);
    *server = s;
    return PC_OK;
}

int pc_server_set_random(void *server, int32_t patch_id, const pc_catalog *randoms) {
    clear_error();
    auto *s = static_cast<Server *>(server);
    if (!s) return fail(PC_ERR_INVALID, "server is NULL");
    (void)hipSetDevice(s->device);
    uint64_t h = 0;
    int rc = upload_catalog(randoms, s->streams[0], &h);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->patches.find(patch_id);
    if (it != s->patches.end()) {
        const uint64_t old = it->second.handle;
        // a running launch may still read the old catalogue: release it once
        // none runs; its cached RR counts are dropped now
        s->retired.push_back(old);
        for (auto c = s->rr_cache.begin(); c != s->rr_cache.end();) {
            uint64_t h;
            memcpy(&h, c->first.data(), sizeof(h));
            if (h == old) c = s->rr_cache.erase(c);
            else ++c;
        }
    }
    Patch p;
    p.handle = h;
    p.n = randoms->n;
    s->patches[patch_id] = p;
    // requests of this patch still waiting for their first launch use the new
    // catalogue; requests already counted in part keep the old one until they
    // finish (it is released once nothing refers to it)
    for (auto &q : s->queue) {
        Request &r = *q;
        if (r.patch != patch_id || r.started) continue;
        r.random_handle = h;
        r.n_random = p.n;
        const double nn = static_cast<double>(r.n_points), nr = static_cast<double>(p.n);
        r.pairs = 0.5 * nn * (nn - 1.0) + nn * nr;
        r.rr_needed = true;
        r.rr_done = 0;
        std::fill(r.RR.begin(), r.RR.end(), 0ull);
        s->prepare(r);
    }
    s->release_retired();
    return PC_OK;
}

int pc_server_submit(void *server, const pc_catalog *data, int32_t patch_id, const double *theta_edges_deg,
                     int32_t n_edges, uint64_t *job_id) {
    clear_error();
    auto *s = static_cast<Server *>(server);
    if (!s || !job_id) return fail(PC_ERR_INVALID, "NULL argument");
    int rc = validate_catalog(data, "data");
    if (rc) return rc;
    HostTable t;
    std::string err;
    if (!theta_edges_deg || !build_table(theta_edges_deg, n_edges, t, err))
        return fail(PC_ERR_INVALID, theta_edges_deg ? err : "theta_edges_deg is NULL");
    auto r = std::make_shared<Request>();
    r->patch = patch_id;
    r->edges.assign(theta_edges_deg, theta_edges_deg + n_edges);
    const size_t n = static_cast<size_t>(data->n);
    r->ra.resize(n);
    r->dec.resize(n);
    if (n) {
        if (data->on_device) {
            (void)hipSetDevice(s->device);
            hipError_t e = hipMemcpy(r->ra.data(), data->ra_deg, sizeof(double) * n, hipMemcpyDeviceToHost);
            if (e == hipSuccess)
                e = hipMemcpy(r->dec.data(), data->dec_deg, sizeof(double) * n, hipMemcpyDeviceToHost);
            if (e != hipSuccess) return hip_fail(e, "copy request catalogue");
            for (size_t i = 0; i < n; ++i)
                if (!std::isfinite(r->ra[i]) || !std::isfinite(r->dec[i]) || r->dec[i] < -90.0 || r->dec[i] > 90.0)
                    return fail(PC_ERR_INVALID, "data: RA must be finite and Dec in [-90, 90]");
        } else {
            memcpy(r->ra.data(), data->ra_deg, sizeof(double) * n);
            memcpy(r->dec.data(), data->dec_deg, sizeof(double) * n);
        }
    }
    r->n_points = static_cast<int64_t>(n);
    r->DD.assign(static_cast<size_t>(n_edges) + 1, 0);
    r->DR.assign(static_cast<size_t>(n_edges) + 1, 0);
    r->RR.assign(static_cast<size_t>(n_edges) + 1, 0);
    std::lock_guard<std::mutex> lk(s->mu);
    auto pit = s->patches.find(patch_id);
    if (pit == s->patches.end()) return fail(PC_ERR_INVALID, "no random catalogue registered for this patch");
    if (static_cast<int>(s->queue.size()) >= s->cfg.max_queue) return fail(PC_ERR_BUSY, "server queue is full");
    r->n_random = pit->second.n;
    r->random_handle = pit->second.handle;
    const double nn = static_cast<double>(n), nr = static_cast<double>(pit->second.n);
    r->pairs = 0.5 * nn * (nn - 1.0) + nn * nr;
    auto cached = s->rr_cache.find(rr_key(r->random_handle, r->edges));
    if (cached != s->rr_cache.end()) {
        r->RR = cached->second;
        r->rr_needed = false;
    }
    // the first part and the device bytes its launch needs (host-only plan)
    s->prepare(*r);
    r->id = s->next_id++;
    r->t_submit = Clock::now();
    s->jobs.emplace(r->id, r);
    s->queue.push_back(r);
    ++s->n_submitted;
    *job_id = r->id;
    s->cv_work.notify_all();
    return PC_OK;
}

int pc_server_poll(void *server, uint64_t job_id, int32_t *done, uint64_t *DD, uint64_t *DR, uint64_t *RR,
                   double *w, double *latency_s) {
    clear_error();
    auto *s = static_cast<Server *>(server);
    if (!s || !done) return fail(PC_ERR_INVALID, "NULL argument");
    std::shared_ptr<Request> r;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->jobs.find(job_id);
        if (it == s->jobs.end()) return fail(PC_ERR_INVALID, "unknown job id");
        Request &q = *it->second;
        if (!q.done && !q.running && !q.started && s->cfg.deadline_s > 0 &&
            std::chrono::duration<double>(Clock::now() - q.t_submit).count() > s->cfg.deadline_s) {
            auto pos = std::find(s->queue.begin(), s->queue.end(), it->second);
            if (pos != s->queue.end()) {
                s->queue.erase(pos);
                ++s->n_expired;
                s->finish_unrun(q, PC_ERR_CANCELLED, "queueing deadline passed before admission");
                s->cv_done.notify_all();
            }
        }
        if (!q.done) {
            *done = 0;
            return PC_OK;
        }
        r = it->second;
        s->jobs.erase(it);
    }
    if (latency_s) *latency_s = r->latency;
    if (r->status != PC_OK) {
        *done = -1;
        return fail(r->status, r->error);
    }
    *done = 1;
    const size_t ne = r->edges.size();
    if (DD) memcpy(DD, r->DD.data(), sizeof(uint64_t) * (ne + 1));
    if (DR) memcpy(DR, r->DR.data(), sizeof(uint64_t) * (ne + 1));
    if (RR) memcpy(RR, r->RR.data(), sizeof(uint64_t) * (ne + 1));
    if (w) memcpy(w, r->w.data(), sizeof(double) * (ne - 1));
    return PC_OK;
}

int pc_server_cancel(void *server, uint64_t job_id, int32_t *cancelled) {
    clear_error();
    auto *s = static_cast<Server *>(server);
    if (!s || !cancelled) return fail(PC_ERR_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return fail(PC_ERR_INVALID, "unknown job id");
    Request &r = *it->second;
    *cancelled = 0;
    if (r.done) return PC_OK;  // finished first: its answer stays pollable
    *cancelled = 1;
    if (r.running) {
        r.cancelled = true;    // the batch runs on; the answer is discarded
        return PC_OK;
    }
    auto pos = std::find(s->queue.begin(), s->queue.end(), it->second);
    if (pos != s->queue.end()) s->queue.erase(pos);
    s->finish_unrun(r, PC_ERR_CANCELLED, "request cancelled");
    s->cv_done.notify_all();
    return PC_OK;
}

int pc_server_drain(void *server) {
    clear_error();
    auto *s = static_cast<Server *>(server);
    if (!s) return fail(PC_ERR_INVALID, "server is NULL");
    {
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.wait(lk, [&] { return s->queue.empty() && s->inflight == 0; });
    }
    s->write_log();
    return PC_OK;
}

const char *pc_server_stats(void *server) {
    clear_error();
    auto *s = static_cast<Server *>(server);
    static thread_local std::string buf;
    if (!s) {
        buf = "{}";
        return buf.c_str();
    }
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<double> l = s->latencies;
    std::sort(l.begin(), l.end());
    auto pct = [&](double p) {
        if (l.empty()) return 0.0;
        const size_t i = std::min(l.size() - 1, static_cast<size_t>(std::ceil(p * l.size())) - (p > 0 ? 1 : 0));
        return l[i];
    };
    std::ostringstream o;
    o.precision(9);
    const double wall = std::chrono::duration<double>(Clock::now() - s->t0).count();
    o << "{\"submitted\": " << s->n_submitted << ", \"completed\": " << s->n_done << ", \"failed\": " << s->n_failed
      << ", \"queued\": " << s->queue.size() << ", \"inflight\": " << s->inflight << ", \"batches\": " << s->n_batches
      << ", \"admission_waits\": " << s->n_admit_waits << ", \"pairs\": " << s->pairs_done
      << ", \"busy_s\": " << s->busy_s << ", \"wall_s\": " << wall << ", \"p50_s\": " << pct(0.50)
      << ", \"p99_s\": " << pct(0.99) << ", \"max_s\": " << (l.empty() ? 0.0 : l.back())
      << ", \"rr_cached\": " << s->rr_cache.size() << ", \"streams\": " << s->cfg.streams
      << ", \"cancelled\": " << s->n_cancelled << ", \"expired\": " << s->n_expired
      << ", \"max_concurrent_batches\": " << s->max_running_batches << ", \"parts_requeued\": " << s->n_requeued
      << ", \"split_batches\": " << s->n_split_batches << ", \"slice_pairs\": " << s->cfg.slice_pairs << "}";
    buf = o.str();
    return buf.c_str();
}

int pc_server_destroy(void *server) {
    clear_error();
    auto *s = static_cast<Server *>(server);
    if (!s) return PC_OK;
    {
        // nobody can poll after this call: requests still waiting are dropped,
        // launches already running finish
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (auto &r : s->queue) s->finish_unrun(*r, PC_ERR_CANCELLED, "server destroyed before admission");
        s->queue.clear();
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
    for (auto &t : s->workers) t.join();
    s->write_log();
    (void)hipSetDevice(s->device);
    for (auto &p : s->patches) release_catalog(p.second.handle);
    for (uint64_t h : s->retired) release_catalog(h);
    for (auto st : s->streams) (void)hipStreamDestroy(st);
    delete s;
    return PC_OK;
}

int pc_debug_request_parts(int64_t n_points, int64_t n_random, int32_t n_edges, int32_t count_rr,
                           double slice_pairs, int32_t max_parts, int64_t *rows, uint64_t *need_bytes,
                           int32_t *n_parts) {
    clear_error();
    if (!n_parts || (max_parts > 0 && (!rows || !need_bytes))) return fail(PC_ERR_INVALID, "NULL argument");
    if (n_points < 0 || n_random < 0 || n_edges < 2 || n_edges > kMaxEdges || !(slice_pairs >= 0))
        return fail(PC_ERR_INVALID, "bad sizes");
    Request r;
    r.n_points = n_points;
    r.n_random = n_random;
    r.random_handle = 1;  // a catalogue described by its size only
    r.rr_needed = count_rr != 0;
    r.edges.resize(static_cast<size_t>(n_edges));
    for (int32_t k = 0; k < n_edges; ++k) r.edges[k] = 0.01 * std::pow(1000.0, k / double(n_edges - 1));
    const std::map<uint64_t, int64_t> sizes{{1, n_random}};
    int32_t np = 0;
    while (true) {
        double pairs = 0;
        const Part p = next_part(r, slice_pairs, &pairs);
        if (np < max_parts) {
            uint64_t b = 0;
            const int rc = part_need_bytes(r, p, PC_MIXED, &sizes, &b);
            if (rc) return rc;
            rows[4 * np + 0] = p.a;
            rows[4 * np + 1] = p.b;
            rows[4 * np + 2] = p.c;
            rows[4 * np + 3] = p.d;
            need_bytes[np] = b;
        }
        ++np;
        r.data_done = p.b;
        if (p.c < p.d) r.rr_done = p.d;
        if (r.data_done >= n_points && (!r.rr_needed || r.rr_done >= n_random)) break;
        if (np > (1 << 24)) return fail(PC_ERR_INVALID, "too many parts");
    }
    *n_parts = np;
    return PC_OK;
}

int pc_debug_server_hold(void *server, int32_t hold) {
    clear_error();
    auto *s = static_cast<Server *>(server);
    if (!s) return fail(PC_ERR_INVALID, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->hold = hold != 0;
    }
    s->cv_work.notify_all();
    return PC_OK;
}

int pc_debug_admission_plan(const uint64_t *need_bytes, const double *pairs, const double *age_s, int32_t n,
                            uint64_t free_bytes, uint64_t total_bytes, uint64_t reserved_bytes, int32_t inflight,
                            const char *json_cfg, int32_t *outcome) {
    clear_error();
    if (n < 0) return fail(PC_ERR_INVALID, "n must be >= 0");
    if (n > 0 && (!need_bytes || !pairs || !age_s || !outcome)) return fail(PC_ERR_INVALID, "NULL argument");
    if (inflight < 0) return fail(PC_ERR_INVALID, "inflight must be >= 0");
    ServerCfg cfg;
    std::string err;
    if (!parse_cfg(json_cfg, cfg, err)) return fail(PC_ERR_INVALID, err);
    std::vector<QueuedView> q(static_cast<size_t>(n));
    for (int32_t i = 0; i < n; ++i) q[i] = {need_bytes[i], pairs[i], age_s[i]};
    bool mem_blocked = false;
    plan_admission(q.data(), n, free_bytes, total_bytes, reserved_bytes, inflight, cfg, outcome, &mem_blocked);
    return PC_OK;
}

}  // extern "C"
