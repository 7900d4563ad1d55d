// pc_tune.cpp -- launch-parameter tuning for batches of a given shape.
//
// The counting launch has parameters that change its speed but not its counts:
// the tile size (the size of the paper's submatrices, Sec. 2.1: 128 or 256
// points; smaller tiles bound sparse catalogues more tightly, so more tile
// pairs are binned whole or against fewer edges, at more work items), the
// mixed kernel's histogram lane columns (LDS per wave, hence waves per CU,
// and lanes sharing a counter word), how many work items a wave takes from the
// queue at a time, and whether far tile pairs go through the matrix cores.
// pc_autotune times every candidate on the caller's own batch, checks that
// all candidates agree, and keeps the fastest per (device, edge count class,
// pair count class); batches run with PC_TUNED then use it.  Entries persist
// as one JSON object per line.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

#include "pc_runtime.hpp"

namespace pc {

namespace {

std::mutex g_tune_mu;
std::map<TuneKey, TuneEntry> g_tune;

int ceil_log2(int64_t x) {
    int k = 0;
    while ((int64_t{1} << k) < x) ++k;
    return k;
}

int floor_log2(uint64_t x) {
    int k = -1;
    while (x) {
        x >>= 1;
        ++k;
    }
    return k;
}

int64_t catalogue_size(const pc_catalog *c, uint64_t h) {
    if (h) {
        std::shared_ptr<Resident> r;
        if (resident_catalog(h, &r) == PC_OK) return r->n;
        return 0;
    }
    return c ? c->n : 0;
}

// value of "key": in a one-line JSON object (numbers or a string)
bool field(const std::string &line, const char *key, std::string *out) {
    const std::string k = std::string("\"") + key + "\"";
    size_t p = line.find(k);
    if (p == std::string::npos) return false;
    p = line.find(':', p + k.size());
    if (p == std::string::npos) return false;
    ++p;
    while (p < line.size() && line[p] == ' ') ++p;
    if (p < line.size() && line[p] == '"') {
        const size_t e = line.find('"', p + 1);
        if (e == std::string::npos) return false;
        *out = line.substr(p + 1, e - p - 1);
        return true;
    }
    size_t e = p;
    while (e < line.size() && line[e] != ',' && line[e] != '}' && line[e] != ' ') ++e;
    *out = line.substr(p, e - p);
    return !out->empty();
}

bool to_int(const std::string &s, int *v) {
    char *end = nullptr;
    const long x = strtol(s.c_str(), &end, 10);
    if (!end || *end || s.empty()) return false;
    *v = static_cast<int>(x);
    return true;
}

std::string entry_json(const TuneKey &k, const TuneEntry &e) {
    char buf[512];
    snprintf(buf, sizeof(buf),
             "{\"device\": \"%s\", \"edges_class\": %d, \"pairs_class\": %d, \"tile\": %d, \"cols\": %d, "
             "\"chunk\": %d, \"matrix_cores\": %d, \"kernel_ms\": %.4f, \"launch_ms\": %.4f}",
             k.device.c_str(), k.edges_class, k.pairs_class, e.tune.tile, e.tune.cols, e.tune.chunk,
             e.tune.matrix_cores ? 1 : 0, e.kernel_ms, e.launch_ms);
    return buf;
}

}  // namespace

TuneKey tune_key_of(const std::vector<BatchJob> &jobs) {
    TuneKey k;
    DeviceInfo *di = nullptr;
    if (device_info(&di) == PC_OK) k.device = di->arch + ":" + std::to_string(di->cus);
    int32_t max_edges = 2;
    uint64_t pairs = 0;
    for (const BatchJob &j : jobs) {
        max_edges = std::max(max_edges, j.n_edges);
        const int64_t nA = catalogue_size(j.A, j.hA);
        const int64_t r0 = std::max<int64_t>(j.row_begin, 0);
        const int64_t r1 = j.row_end < 0 ? nA : std::min(j.row_end, nA);
        if (r1 <= r0) continue;
        const uint64_t rows = static_cast<uint64_t>(r1 - r0);
        if (j.auto_flag) {
            // sum over i in [r0, r1) of (nA - 1 - i)
            pairs += rows * static_cast<uint64_t>(2 * nA - r0 - r1 - 1) / 2;
        } else {
            pairs += rows * static_cast<uint64_t>(catalogue_size(j.B, j.hB));
        }
    }
    k.edges_class = ceil_log2(max_edges);
    k.pairs_class = floor_log2(std::max<uint64_t>(pairs, 1));
    return k;
}

int tune_lookup(const TuneKey &k, TuneEntry *e) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(k);
    if (it == g_tune.end()) return PC_ERR_INVALID;
    *e = it->second;
    return PC_OK;
}

void tune_store(const TuneKey &k, const TuneEntry &e) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[k] = e;
}

namespace {

// entries of a tuning file (one JSON object per line)
int parse_file(const char *path, std::map<TuneKey, TuneEntry> *out) {
    if (!path) return fail(PC_ERR_INVALID, "cache_path is NULL");
    std::ifstream f(path);
    if (!f) return fail(PC_ERR_INVALID, std::string("cannot read ") + path);
    std::string line;
    std::map<TuneKey, TuneEntry> &got = *out;
    while (std::getline(f, line)) {
        if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
        TuneKey k;
        TuneEntry e;
        std::string v;
        int mc = 0;
        bool ok = field(line, "device", &k.device);
        ok = ok && field(line, "edges_class", &v) && to_int(v, &k.edges_class);
        ok = ok && field(line, "pairs_class", &v) && to_int(v, &k.pairs_class);
        ok = ok && field(line, "cols", &v) && to_int(v, &e.tune.cols);
        ok = ok && field(line, "chunk", &v) && to_int(v, &e.tune.chunk);
        ok = ok && field(line, "matrix_cores", &v) && to_int(v, &mc);
        if (ok && field(line, "kernel_ms", &v)) e.kernel_ms = atof(v.c_str());
        if (ok && field(line, "launch_ms", &v)) e.launch_ms = atof(v.c_str());
        // entries written before the tile size was tuned mean 256-point tiles
        if (ok && field(line, "tile", &v)) ok = to_int(v, &e.tune.tile) && (e.tune.tile == 128 || e.tune.tile == 256);
        const bool cols_ok = e.tune.cols == 0 || (e.tune.cols >= 4 && e.tune.cols <= 64 &&
                                                  (e.tune.cols & (e.tune.cols - 1)) == 0);
        if (!ok || !cols_ok || e.tune.chunk < 1 || e.tune.chunk > 64 || (mc != 0 && mc != 1) ||
            (mc && e.tune.tile != 256))
            return fail(PC_ERR_INVALID, std::string("bad tuning entry in ") + path + ": " + line);
        e.tune.matrix_cores = mc != 0;
        got[k] = e;
    }
    return PC_OK;
}

}  // namespace

int tune_load_file(const char *path) {
    std::map<TuneKey, TuneEntry> got;
    const int rc = parse_file(path, &got);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto &kv : got) g_tune[kv.first] = kv.second;
    return PC_OK;
}

int tune_save_file(const char *path) {
    // merge: entries already in the file, overlaid by this process's table
    std::map<TuneKey, TuneEntry> all;
    {
        std::ifstream f(path);
        if (f) {
            f.close();
            const int rc = parse_file(path, &all);
            if (rc) return rc;
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (auto &kv : g_tune) all[kv.first] = kv.second;
    }
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream o(tmp, std::ios::trunc);
        if (!o) return fail(PC_ERR_INVALID, std::string("cannot write ") + tmp);
        for (auto &kv : all) o << entry_json(kv.first, kv.second) << "\n";
        if (!o) return fail(PC_ERR_INVALID, std::string("cannot write ") + tmp);
    }
    if (rename(tmp.c_str(), path) != 0) return fail(PC_ERR_INVALID, std::string("cannot replace ") + path);
    return PC_OK;
}

}  // namespace pc

using namespace pc;

extern "C" int pc_autotune(const pc_job *jobs, int32_t n_jobs, int32_t mode, const char *cache_path, void *stream,
                           char *result, int32_t result_len) {
    clear_error();
    std::vector<BatchJob> v;
    int rc = jobs_from_abi(jobs, n_jobs, &v);
    if (rc) return rc;
    if (mode & (PC_TUNED | PC_MATRIX_CORES))
        return fail(PC_ERR_INVALID, "pc_autotune chooses the launch parameters itself: pass PC_MIXED or PC_FP64_PLAIN "
                                    "(optionally with PC_NO_PRUNE)");
    const bool mixed = (mode & ~PC_NO_PRUNE) == PC_MIXED;
    const bool prune = (mode & PC_NO_PRUNE) == 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // Two stages.  The tile size changes the prune pass and the ordering too
    // (four times as many tile pairs at 128 points, each tighter), so it is
    // chosen first on the whole launch's time with the other parameters at
    // their defaults; then the histogram columns, the queue chunk and (256-point
    // tiles) the matrix-core path on the counting kernel's time at that size.
    std::vector<LaunchTune> stage1;
    for (int tile : {256, 128}) {
        LaunchTune t;
        t.tile = tile;
        stage1.push_back(t);
    }
    // every candidate counts into its own buffers; the first is the reference
    std::vector<std::vector<uint64_t>> ref(v.size()), cur(v.size());
    std::vector<BatchJob> w = v;
    for (size_t q = 0; q < v.size(); ++q) {
        ref[q].assign(static_cast<size_t>(std::max(v[q].n_edges, 0)) + 1, 0);
        cur[q] = ref[q];
    }
    const bool was_timing = thread_timing();
    set_thread_timing(true);
    struct Reset {
        bool on;
        ~Reset() { set_thread_timing(on); }
    } reset{was_timing};
    // one untimed run first (code objects, tables)
    for (size_t q = 0; q < v.size(); ++q) w[q].counts = ref[q].data();
    rc = run_batch(w, mode, st, nullptr, &stage1[0]);
    if (rc) return rc;
    size_t n_cands = 0;
    // times each candidate (counting kernel, whole launch on the host's
    // clock) and checks its counts against the reference
    auto run = [&](const LaunchTune &t, double *kernel_ms, double *launch_ms, bool new_candidate = true) -> int {
        for (size_t q = 0; q < v.size(); ++q) w[q].counts = cur[q].data();
        BatchStats bs;
        const auto t0 = std::chrono::steady_clock::now();
        const int r = run_batch(w, mode, st, &bs, &t);
        if (r) return r;
        *launch_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        *kernel_ms = bs.kernel_ms >= 0.0 ? bs.kernel_ms : 0.0;
        if (new_candidate) ++n_cands;
        for (size_t q = 0; q < v.size(); ++q)
            if (cur[q] != ref[q])
                return fail(PC_ERR_DEVICE, "tuning candidates disagree on the counts (tile " + std::to_string(t.tile) +
                                               ", cols " + std::to_string(t.cols) + ", chunk " +
                                               std::to_string(t.chunk) + ")");
        return PC_OK;
    };
    // Stage 1: the second tile size also gets an untimed run (its kernels'
    // first launch), then the sizes are timed twice each, in the order 256,
    // 128, 128, 256, and each keeps its faster launch: where the two are within
    // a few percent of each other (the batched mocks), one run each left the
    // choice to the first launch's costs and to noise.
    {
        double kms = 0, lms = 0;
        rc = run(stage1[1], &kms, &lms, false);
        if (rc) return rc;
    }
    double stage1_ms[2] = {0.0, 0.0};
    for (int s = 0; s < 4; ++s) {
        const int c = (s == 1 || s == 2) ? 1 : 0;
        double kms = 0, lms = 0;
        rc = run(stage1[static_cast<size_t>(c)], &kms, &lms, s < 2);
        if (rc) return rc;
        if (s < 2 || lms < stage1_ms[c]) stage1_ms[c] = lms;
    }
    const int tile = stage1_ms[1] < stage1_ms[0] ? stage1[1].tile : stage1[0].tile;
    std::vector<LaunchTune> cands;
    for (int mc = 0; mc <= ((mixed && prune && tile == 256) ? 1 : 0); ++mc)
        for (int cols : {4, 8, 16, 32})
            for (int chunk : {2, 4, 8}) {
                if (!mixed && cols != 8) continue;  // the binary64 kernel's columns are fixed
                LaunchTune t;
                t.tile = tile;
                t.cols = mixed ? cols : 0;
                t.chunk = chunk;
                t.matrix_cores = mc != 0;
                cands.push_back(t);
            }
    int best = -1;
    double best_ms = 0.0, best_lms = 0.0;
    for (size_t c = 0; c < cands.size(); ++c) {
        double kms = 0, lms = 0;
        rc = run(cands[c], &kms, &lms);
        if (rc) return rc;
        if (best < 0 || kms < best_ms) {
            best = static_cast<int>(c);
            best_ms = kms;
            best_lms = lms;
        }
    }
    TuneEntry e;
    e.tune = cands[static_cast<size_t>(best)];
    e.kernel_ms = best_ms;
    e.launch_ms = best_lms;
    const TuneKey key = tune_key_of(v);
    tune_store(key, e);
    if (cache_path) {
        rc = tune_save_file(cache_path);
        if (rc) return rc;
    }
    for (size_t q = 0; q < v.size(); ++q) memcpy(v[q].counts, ref[q].data(), sizeof(uint64_t) * ref[q].size());
    if (result && result_len > 0) {
        std::string j = entry_json(key, e);
        j.pop_back();
        j += ", \"candidates\": " + std::to_string(n_cands) + "}";
        snprintf(result, static_cast<size_t>(result_len), "%s", j.c_str());
    }
    return PC_OK;
}

extern "C" int pc_autotune_load(const char *cache_path) {
    clear_error();
    return tune_load_file(cache_path);
}
