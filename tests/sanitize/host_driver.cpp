// host_driver.cpp -- drives libpc's host code (edge tables and guard bands,
// estimators, tuner file parser, admission policy, request planner, and the
// threaded w(theta) server) against the fake device layer in
// fake_device.cpp.  Built under AddressSanitizer + UndefinedBehaviorSanitizer
// and under ThreadSanitizer by tests/test_host_sanitizers.py; exits non-zero
// when a check fails.  Test infrastructure only.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <cmath>
#include <chrono>
#include <mutex>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pc.h"
#include "../../include/pc_debug.h"
#include "../../paper_1208_3658_amd/csrc/pc_runtime.hpp"

void fake_set_free_bytes(uint64_t b);
void fake_fail_next_batches(int n);

static int g_failures = 0;
#define CHECK(c)                                                           \
    do {                                                                   \
        if (!(c)) {                                                        \
            fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #c); \
            ++g_failures;                                                  \
        }                                                                  \
    } while (0)

static std::vector<double> log_edges(double lo, double hi, int n) {
    std::vector<double> e(static_cast<size_t>(n));
    for (int k = 0; k < n; ++k) e[k] = lo * pow(hi / lo, k / double(n - 1));
    e[0] = lo;
    e[n - 1] = hi;
    return e;
}

static void tables_and_estimators(std::mt19937_64 &rng) {
    std::uniform_real_distribution<double> U(0.0, 1.0);
    for (int trial = 0; trial < 200; ++trial) {
        const int n = 2 + static_cast<int>(U(rng) * (trial % 10 == 0 ? 1022 : 60));
        std::vector<double> e;
        if (trial % 3 == 0) {
            e = log_edges(1e-4 + U(rng) * 0.01, 1.0 + U(rng) * 179.0, n);
        } else {
            const double lo = trial % 3 == 1 ? 0.0 : U(rng) * 10.0, hi = lo + 1e-9 + U(rng) * (180.0 - lo);
            for (int k = 0; k < n; ++k) e.push_back(lo + (hi - lo) * k / (n - 1));
        }
        pc::HostTable t;
        std::string err;
        const bool ok = pc::build_table(e.data(), n, t, err, trial % 2 ? 8 : 0);
        CHECK(ok);
        if (ok) {
            CHECK(t.e64.size() == static_cast<size_t>(n));
            for (int k = 0; k < n; ++k) CHECK(t.lo[k] <= t.hi[k]);
        }
    }
    // invalid edge sets are refused
    {
        pc::HostTable t;
        std::string err;
        const double bad1[3] = {1.0, 1.0, 2.0}, bad2[2] = {-1.0, 2.0}, bad3[2] = {0.0, NAN};
        CHECK(!pc::build_table(bad1, 3, t, err));
        CHECK(!pc::build_table(bad2, 2, t, err));
        CHECK(!pc::build_table(bad3, 2, t, err));
    }
    for (int trial = 0; trial < 100; ++trial) {
        const int nb = 1 + trial % 40;
        std::vector<uint64_t> dd(nb), dr(nb), rr(nb);
        for (int k = 0; k < nb; ++k) {
            dd[k] = rng() % 1000;
            dr[k] = rng() % 1000;
            rr[k] = trial % 5 ? rng() % 1000 : 0;
        }
        std::vector<double> w(nb);
        for (int kind = 0; kind < 4; ++kind) pc::estimator(kind, dd.data(), dr.data(), rr.data(), nb, 1000, 2000, w.data());
        pc::landy_szalay(dd.data(), dr.data(), rr.data(), nb, 1000, 2000, w.data());
        // RR = 0: the IEEE quotient (an infinity, or NaN when DD and DR are 0 too)
        for (int k = 0; k < nb; ++k) CHECK(rr[k] == 0 ? !std::isfinite(w[k]) : std::isfinite(w[k]));
    }
}

static void tuner_file(const char *dir) {
    const std::string path = std::string(dir) + "/tune.jsonl";
    FILE *f = fopen(path.c_str(), "w");
    fputs("{\"device\": \"gfx950:256\", \"edges_class\": 6, \"pairs_class\": 40, \"cols\": 16, \"chunk\": 8, "
          "\"matrix_cores\": 0, \"kernel_ms\": 51.5}\n",
          f);
    fputs("\n{\"device\": \"x\", \"edges_class\": 2}\n", f);  // incomplete: refused
    fclose(f);
    const int rc = pc_autotune_load(path.c_str());
    CHECK(rc == PC_OK || rc == PC_ERR_INVALID);
    f = fopen(path.c_str(), "w");
    fputs("{\"device\": \"gfx950:256\", \"edges_class\": \"six\"", f);  // truncated line
    fclose(f);
    CHECK(pc_autotune_load(path.c_str()) != PC_OK);
    CHECK(pc_autotune_load((std::string(dir) + "/missing.jsonl").c_str()) != PC_OK);
}

static void planners(std::mt19937_64 &rng) {
    for (int trial = 0; trial < 200; ++trial) {
        const int n = trial % 17;
        std::vector<uint64_t> need(n);
        std::vector<double> pairs(n), age(n);
        for (int i = 0; i < n; ++i) {
            need[i] = rng() % (uint64_t(8) << 30);
            pairs[i] = static_cast<double>(rng() % 1000000000000ull);
            age[i] = static_cast<double>(rng() % 3000) / 1000.0;
        }
        std::vector<int32_t> out(n + 1, -1);
        const char *cfg = trial % 2 ? "{\"policy\": 1, \"deadline_s\": 1.5, \"max_inflight\": 4}" : nullptr;
        CHECK(pc_debug_admission_plan(need.data(), pairs.data(), age.data(), n, uint64_t(20) << 30,
                                      uint64_t(64) << 30, rng() % (uint64_t(4) << 30), trial % 5, cfg,
                                      out.data()) == PC_OK);
        for (int i = 0; i < n; ++i) CHECK(out[i] >= 0 && out[i] <= 3);
    }
    for (int trial = 0; trial < 40; ++trial) {
        const int64_t np = static_cast<int64_t>(rng() % 3000000), nr = 2 + static_cast<int64_t>(rng() % 2000000);
        const double slice = trial % 4 ? 1e9 * (1 + rng() % 500) : 0.0;
        int32_t parts = 0;
        CHECK(pc_debug_request_parts(np, nr, 2 + trial % 60, trial % 2, slice, 0, nullptr, nullptr, &parts) == PC_OK);
        std::vector<int64_t> rows(4 * static_cast<size_t>(parts));
        std::vector<uint64_t> need(static_cast<size_t>(parts));
        CHECK(pc_debug_request_parts(np, nr, 2 + trial % 60, trial % 2, slice, parts, rows.data(), need.data(),
                                     &parts) == PC_OK);
        int64_t a = 0, c = 0;
        for (int32_t k = 0; k < parts; ++k) {
            if (rows[4 * k] < rows[4 * k + 1]) {
                CHECK(rows[4 * k] == a);
                a = rows[4 * k + 1];
            }
            if (rows[4 * k + 2] < rows[4 * k + 3]) {
                CHECK(rows[4 * k + 2] == c);
                c = rows[4 * k + 3];
            }
        }
        CHECK(a == np || np == 0);
        CHECK(c == (trial % 2 ? nr : 0));
    }
}

struct Submitted {
    uint64_t id;
    int64_t n, nr;
    int n_edges;
};

static void server(std::mt19937_64 &seed_rng, const char *dir) {
    const std::string log = std::string(dir) + "/serve.jsonl";
    const std::string cfg = "{\"streams\": 3, \"slice_pairs\": 4e6, \"max_batch_pairs\": 3e7, \"deadline_s\": 5, "
                            "\"max_inflight\": 24, \"log_path\": \"" + log + "\"}";
    void *srv = nullptr;
    CHECK(pc_server_create(cfg.c_str(), &srv) == PC_OK);
    const int64_t nr[3] = {3000, 1500, 800};
    std::vector<std::vector<double>> rra(3), rdec(3);
    for (int p = 0; p < 3; ++p) {
        std::mt19937_64 rng(100 + p);
        std::uniform_real_distribution<double> U(-5.0, 5.0);
        for (int64_t i = 0; i < nr[p]; ++i) {
            rra[p].push_back(U(rng) + 5.0);
            rdec[p].push_back(U(rng));
        }
        pc_catalog c{rra[p].data(), rdec[p].data(), nr[p], 0, 0};
        CHECK(pc_server_set_random(srv, p, &c) == PC_OK);
    }
    std::mutex mu;
    std::vector<Submitted> sub;
    std::atomic<bool> done_submitting{false};
    std::atomic<int> cancelled_ok{0};
    auto submitter = [&](int t) {
        std::mt19937_64 rng(1000 + t);
        std::uniform_real_distribution<double> U(-5.0, 5.0);
        for (int k = 0; k < 40; ++k) {
            const int64_t n = static_cast<int64_t>(rng() % 4000);
            std::vector<double> ra(static_cast<size_t>(n)), dec(static_cast<size_t>(n));
            for (int64_t i = 0; i < n; ++i) {
                ra[i] = U(rng) + 5.0;
                dec[i] = U(rng);
            }
            const int ne = 2 + static_cast<int>(rng() % 30);
            const std::vector<double> e = log_edges(0.01, 5.0, ne);
            const int patch = static_cast<int>(rng() % 3);
            pc_catalog c{ra.data(), dec.data(), n, static_cast<int32_t>(k % 3 == 0), 0};
            uint64_t id = 0;
            const int rc = pc_server_submit(srv, &c, patch, e.data(), ne, &id);
            CHECK(rc == PC_OK);
            if (rc == PC_OK) {
                std::lock_guard<std::mutex> lk(mu);
                sub.push_back({id, n, nr[patch], ne});
            }
            if (k % 9 == 4) std::this_thread::sleep_for(std::chrono::milliseconds(1));
        }
    };
    auto canceller = [&]() {
        std::mt19937_64 rng(7);
        while (!done_submitting) {
            uint64_t id = 0;
            {
                std::lock_guard<std::mutex> lk(mu);
                if (!sub.empty()) id = sub[rng() % sub.size()].id;
            }
            int32_t c = 0;
            if (id && pc_server_cancel(srv, id, &c) == PC_OK && c) ++cancelled_ok;
            std::this_thread::sleep_for(std::chrono::microseconds(700));
        }
    };
    auto watcher = [&]() {
        while (!done_submitting) {
            const char *s = pc_server_stats(srv);
            CHECK(s && s[0] == '{');
            std::this_thread::sleep_for(std::chrono::microseconds(300));
        }
    };
    std::vector<std::thread> th;
    for (int t = 0; t < 4; ++t) th.emplace_back(submitter, t);
    std::thread tc(canceller), tw(watcher);
    // meanwhile: a held gate, launches that fail for lack of memory (the
    // server splits such batches), a patch's randoms replaced (same size)
    CHECK(pc_debug_server_hold(srv, 1) == PC_OK);
    std::this_thread::sleep_for(std::chrono::milliseconds(5));
    CHECK(pc_debug_server_hold(srv, 0) == PC_OK);
    fake_fail_next_batches(3);
    {
        pc_catalog c{rra[1].data(), rdec[1].data(), nr[1], 0, 0};
        CHECK(pc_server_set_random(srv, 1, &c) == PC_OK);
    }
    for (auto &t : th) t.join();
    done_submitting = true;
    tc.join();
    tw.join();
    CHECK(pc_server_drain(srv) == PC_OK);
    int ok = 0, cancelled = 0, other = 0;
    for (const Submitted &s : sub) {
        std::vector<uint64_t> DD(s.n_edges + 1), DR(s.n_edges + 1), RR(s.n_edges + 1);
        std::vector<double> w(s.n_edges);
        int32_t done = 0;
        double lat = 0;
        const int rc = pc_server_poll(srv, s.id, &done, DD.data(), DR.data(), RR.data(), w.data(), &lat);
        if (rc == PC_OK && done == 1) {
            ++ok;
            uint64_t a = 0, b = 0, c = 0;
            for (int k = 0; k <= s.n_edges; ++k) {
                a += DD[k];
                b += DR[k];
                c += RR[k];
            }
            CHECK(a == static_cast<uint64_t>(s.n * (s.n > 0 ? s.n - 1 : 0) / 2));
            CHECK(b == static_cast<uint64_t>(s.n * s.nr));
            CHECK(c == static_cast<uint64_t>(s.nr * (s.nr - 1) / 2));
            CHECK(lat > 0);
        } else if (rc == PC_ERR_CANCELLED) {
            ++cancelled;
        } else {
            ++other;
            fprintf(stderr, "request %llu: rc %d done %d (%s)\n", (unsigned long long)s.id, rc, done,
                    pc_last_error());
        }
    }
    CHECK(other == 0);
    CHECK(ok + cancelled == static_cast<int>(sub.size()));
    printf("server: %d finished, %d cancelled (%d cancel calls took effect)\n%s\n", ok, cancelled,
           cancelled_ok.load(), pc_server_stats(srv));
    // a second server destroyed with requests still waiting
    void *srv2 = nullptr;
    CHECK(pc_server_create("{\"streams\": 1}", &srv2) == PC_OK);
    {
        pc_catalog c{rra[0].data(), rdec[0].data(), nr[0], 0, 0};
        CHECK(pc_server_set_random(srv2, 0, &c) == PC_OK);
        CHECK(pc_debug_server_hold(srv2, 1) == PC_OK);
        const std::vector<double> e = log_edges(0.01, 5.0, 8);
        for (int k = 0; k < 5; ++k) {
            uint64_t id = 0;
            CHECK(pc_server_submit(srv2, &c, 0, e.data(), 8, &id) == PC_OK);
        }
    }
    CHECK(pc_server_destroy(srv2) == PC_OK);
    CHECK(pc_server_destroy(srv) == PC_OK);
    (void)seed_rng;
}

int main(int argc, char **argv) {
    const char *dir = argc > 1 ? argv[1] : ".";
    std::mt19937_64 rng(20261203);
    tables_and_estimators(rng);
    tuner_file(dir);
    planners(rng);
    server(rng, dir);
    printf("host driver: %d check(s) failed\n", g_failures);
    return g_failures ? 1 : 0;
}
