// pc_api.cpp -- the C ABI of libpc.so: validation, device memory, edge-set
// tables, catalogue conversion and residency, and the batched launch.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/pc.h"
#include "pc_internal.hpp"
#include "pc_math.h"
#include "pc_runtime.hpp"
#include "../../include/pc_debug.h"

namespace pc {

hipError_t launch_convert(const double *ra, const double *dec, int64_t n, double4 *a64, float4 *a32,
                          int *err, hipStream_t st);
hipError_t launch_zero(unsigned long long *p, int64_t n, hipStream_t st);
hipError_t launch_add_copies(unsigned long long *dst, const unsigned long long *src, int64_t n, int32_t n_copies,
                             hipStream_t st);
size_t sort_scratch_words(int64_t n);

// the per-tile-size steps (pc_kernels.hip, pc_prep.hip; one instance per size)
#define PC_TILE_STEPS                                                                                              \
    hipError_t launch_count(bool fp64, bool mc, bool compact, const SegDesc *segs, int32_t n_segs,                 \
                            const TableDesc *tabs,                                                                 \
                            const uint64_t *items, const unsigned long long *n_items, const uint64_t *sub,         \
                            uint64_t total_items, uint32_t lut_lds_off, uint32_t stage_lds_off,                    \
                            unsigned long long *queue, unsigned long long *rechecked, int chunk,                   \
                            uint32_t lds_bytes, int grid, uint64_t flush_cap, hipStream_t st);                     \
    hipError_t launch_sort(const double4 *src, int64_t base, int64_t n, uint32_t *scratch, double4 *a64s,          \
                           float4 *a32s, float4 *g32s, double4 *bounds, hipStream_t st);                           \
    hipError_t launch_prune(const SegDesc *segs, int32_t n_segs, const TableDesc *tabs, int64_t total_rows,        \
                            uint64_t *survivors, uint64_t *sub, unsigned long long *meta, int32_t mfma_ok,         \
                            int32_t split_ok, hipStream_t st);                                                     \
    hipError_t count_occupancy(bool fp64, bool mc, bool compact, uint32_t lds_bytes, int *blocks_per_cu);          \
    hipError_t set_max_lds(uint32_t bytes);
namespace t256 { PC_TILE_STEPS }
namespace t128 { PC_TILE_STEPS }
#undef PC_TILE_STEPS

// One tile size's steps.  tile = points per tile (both axes); 64-point
// sub-blocks, tile / 64 of them per tile; the matrix-core path needs 256.
struct TileOps {
    int tile;
    int subs;
    bool matrix_cores;
    decltype(&t256::launch_count) launch_count;
    decltype(&t256::launch_sort) launch_sort;
    decltype(&t256::launch_prune) launch_prune;
    decltype(&t256::count_occupancy) count_occupancy;
    decltype(&t256::set_max_lds) set_max_lds;
};
static const TileOps kTile256 = {256, 4, true, t256::launch_count, t256::launch_sort, t256::launch_prune,
                                 t256::count_occupancy, t256::set_max_lds};
static const TileOps kTile128 = {128, 2, false, t128::launch_count, t128::launch_sort, t128::launch_prune,
                                 t128::count_occupancy, t128::set_max_lds};
// the tile size resident catalogues are ordered and bounded for
static const TileOps &kResidentTile = kTile256;

#ifndef PC_SPLIT
#define PC_SPLIT 1  // split surviving tile pairs into j sub-blocks in the prune pass
#endif

// ------------------------------------------------------------------ errors

static thread_local std::string t_err;

int fail(int code, const std::string &msg) {
    t_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(PC_ERR_NOMEM, std::string(what) + ": " + hipGetErrorString(e));
    return fail(PC_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define PC_HIP(call, what)                                  \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hip_fail(e_, (what));  \
    } while (0)

void clear_error() { t_err.clear(); }

// per-thread count of device allocations still to fail (testing)
static thread_local int32_t t_fail_allocs = 0;

bool injected_alloc_failure() {
    if (t_fail_allocs <= 0) return false;
    --t_fail_allocs;
    return true;
}

// ------------------------------------------------------------------ device

static std::mutex g_dev_mu;
static std::map<int, DeviceInfo> g_dev;

int device_info(DeviceInfo **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto it = g_dev.find(dev);
    if (it == g_dev.end()) {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
        DeviceInfo d;
        d.device = dev;
        d.cus = prop.multiProcessorCount;
        d.lds_per_block = static_cast<uint32_t>(prop.sharedMemPerBlock);
        d.lds_per_cu = static_cast<uint32_t>(prop.maxSharedMemoryPerMultiProcessor);
        d.arch = prop.gcnArchName;
        d.ok = d.arch.rfind("gfx950", 0) == 0;
        if (d.ok) {
            const uint32_t want = std::max<uint32_t>(d.lds_per_block, 64u * 1024u);
            if (kTile256.set_max_lds(want) == hipSuccess && kTile128.set_max_lds(want) == hipSuccess)
                d.lds_per_block = want;
        }
        it = g_dev.emplace(dev, d).first;
    }
    if (!it->second.ok)
        return fail(PC_ERR_DEVICE, "libpc needs an AMD gfx950 (MI355X) device; current device is " +
                                       it->second.arch);
    *out = &it->second;
    return PC_OK;
}

// ------------------------------------------------------------------ tables

struct TableKey {
    int device;
    int cols;
    std::vector<uint64_t> bits;
    bool operator<(const TableKey &o) const {
        if (device != o.device) return device < o.device;
        if (cols != o.cols) return cols < o.cols;
        return bits < o.bits;
    }
};

static std::mutex g_tab_mu;
// Device tables by (device, cols, edges), least recently used dropped past
// kMaxCachedTables (a launch holds its own references, so dropping an entry
// never frees a table in use).  A server with a new edge set per request
// would otherwise keep every table.
constexpr size_t kMaxCachedTables = 256;
struct CachedTable {
    std::shared_ptr<DevTable> t;
    uint64_t last_use = 0;
};
static std::map<TableKey, CachedTable> g_tabs;
static uint64_t g_tab_tick = 0;

DevTable::~DevTable() {
    if (d_mem) (void)hipFree(d_mem);
}

void table_blob(const HostTable &h, TableBlob *out) {
    // one device block: e64 | band | band_g | fband | fband_g | lut32 | lutc | lut64
    const size_t b_e = sizeof(double) * h.e64.size();
    const size_t b_b = 2 * sizeof(float) * h.e64.size();
    out->o_band = (b_e + 255) & ~size_t(255);
    out->o_band_g = (out->o_band + b_b + 255) & ~size_t(255);
    out->o_fband = (out->o_band_g + b_b + 255) & ~size_t(255);
    out->o_fband_g = (out->o_fband + b_b + 255) & ~size_t(255);
    out->o_lut32 = (out->o_fband_g + b_b + 255) & ~size_t(255);
    const size_t b_l32 = sizeof(LutEntry32) * h.lut32.entries.size();
    out->o_lutc = (out->o_lut32 + b_l32 + 255) & ~size_t(255);
    const size_t b_lc = sizeof(LutEntryC) * h.lut32.compact.size();
    out->o_lut64 = (out->o_lutc + b_lc + 255) & ~size_t(255);
    const size_t b_l64 = sizeof(LutEntry64) * h.lut64.size();
    std::vector<unsigned char> &blob = out->bytes;
    blob.assign(out->o_lut64 + b_l64 + 256, 0);
    memcpy(blob.data(), h.e64.data(), b_e);
    for (size_t k = 0; k < h.e64.size(); ++k) {
        const float bb[4] = {h.lo[k], h.hi[k], h.lo_g[k], h.hi_g[k]};
        memcpy(blob.data() + out->o_band + 8 * k, bb, 8);
        memcpy(blob.data() + out->o_band_g + 8 * k, bb + 2, 8);
        const float fb[4] = {h.fh[k], h.fw[k], h.fh_g[k], h.fw_g[k]};
        memcpy(blob.data() + out->o_fband + 8 * k, fb, 8);
        memcpy(blob.data() + out->o_fband_g + 8 * k, fb + 2, 8);
    }
    if (b_l32) memcpy(blob.data() + out->o_lut32, h.lut32.entries.data(), b_l32);
    if (b_lc) memcpy(blob.data() + out->o_lutc, h.lut32.compact.data(), b_lc);
    if (b_l64) memcpy(blob.data() + out->o_lut64, h.lut64.data(), b_l64);
}

void table_place(DevTable *t, const TableBlob &b, unsigned char *base) {
    t->d_e64 = reinterpret_cast<const double *>(base);
    t->d_band = reinterpret_cast<const float *>(base + b.o_band);
    t->d_band_g = reinterpret_cast<const float *>(base + b.o_band_g);
    t->d_fband = reinterpret_cast<const float *>(base + b.o_fband);
    t->d_fband_g = reinterpret_cast<const float *>(base + b.o_fband_g);
    t->d_lut32 = base + b.o_lut32;
    t->d_lutc = t->host.lut32.compact.empty() ? nullptr : base + b.o_lutc;
    t->d_lut64 = base + b.o_lut64;
}

int get_table(const double *theta, int32_t n_edges, std::shared_ptr<DevTable> *out, int cols) {
    if (!theta) return fail(PC_ERR_INVALID, "theta_edges_deg is NULL");
    if (n_edges < 2) return fail(PC_ERR_INVALID, "n_edges must be >= 2");
    DeviceInfo *di = nullptr;
    int rc = device_info(&di);
    if (rc) return rc;
    TableKey key;
    key.device = di->device;
    key.cols = cols;
    key.bits.resize(static_cast<size_t>(n_edges));
    memcpy(key.bits.data(), theta, sizeof(double) * static_cast<size_t>(n_edges));
    {
        std::lock_guard<std::mutex> lk(g_tab_mu);
        auto it = g_tabs.find(key);
        if (it != g_tabs.end()) {
            it->second.last_use = ++g_tab_tick;
            *out = it->second.t;
            return PC_OK;
        }
    }
    auto t = std::make_shared<DevTable>();
    std::string err;
    if (!build_table(theta, n_edges, t->host, err, cols)) return fail(PC_ERR_INVALID, err);
    TableBlob blob;
    table_blob(t->host, &blob);
    void *d = nullptr;
    PC_HIP(injected_alloc_failure() ? hipErrorOutOfMemory : hipMalloc(&d, blob.bytes.size()), "hipMalloc(tables)");
    t->d_mem = d;
    PC_HIP(hipMemcpy(d, blob.bytes.data(), blob.bytes.size(), hipMemcpyHostToDevice), "hipMemcpy(tables)");
    table_place(t.get(), blob, static_cast<unsigned char *>(d));
    std::lock_guard<std::mutex> lk(g_tab_mu);
    auto it = g_tabs.find(key);
    if (it != g_tabs.end()) {
        it->second.last_use = ++g_tab_tick;
        *out = it->second.t;  // another thread won; ours is freed
        return PC_OK;
    }
    if (g_tabs.size() >= kMaxCachedTables) {
        auto lru = g_tabs.begin();
        for (auto c = g_tabs.begin(); c != g_tabs.end(); ++c)
            if (c->second.last_use < lru->second.last_use) lru = c;
        g_tabs.erase(lru);
    }
    g_tabs.emplace(key, CachedTable{t, ++g_tab_tick});
    *out = t;
    return PC_OK;
}

TableDesc table_desc(const DevTable &t, bool fp64) {
    TableDesc d;
    memset(&d, 0, sizeof(d));
    const HostTable &h = t.host;
    d.e64 = t.d_e64;
    d.n_edges = static_cast<int32_t>(h.e64.size());
    if (fp64) {
        d.cols = h.cols64;
        d.lut = t.d_lut64;
        d.clamp_lo = h.clamp_lo64;
        d.clamp_hi = h.clamp_hi64;
        d.shift = h.shift64;
        d.key0 = h.clamp_lo64 >> h.shift64;
        d.n_cells = static_cast<int32_t>(h.lut64.size());
        d.search = h.search64 ? 1 : 0;
    } else {
        d.cols = h.cols32;
        d.lut = t.d_lut32;
        d.lutc = t.d_lutc;
        d.clamp_lo = h.lut32.clamp_lo;
        d.clamp_hi = h.lut32.clamp_hi;
        d.shift = h.lut32.shift;
        d.key0 = h.lut32.clamp_lo >> h.lut32.shift;
        d.n_cells = static_cast<int32_t>(h.lut32.entries.size());
        d.search = 0;
        d.band = t.d_band;
        d.band_g = t.d_band_g;
        d.fband = t.d_fband;
        d.fband_g = t.d_fband_g;
    }
    return d;
}

// LDS bytes a table needs: histogram rows, then the cell table (or edges;
// compact: the 8-byte cells)
static void table_lds(const DevTable &t, bool fp64, bool compact, uint32_t *hist, uint32_t *lut) {
    const HostTable &h = t.host;
    *hist = static_cast<uint32_t>(h.e64.size() + 3) * (fp64 ? h.row_bytes64 : h.row_bytes32);
    if (fp64) {
        *lut = h.search64 ? static_cast<uint32_t>(8 * h.e64.size())
                          : static_cast<uint32_t>(16 * h.lut64.size());
    } else {
        *lut = static_cast<uint32_t>((compact ? 8 : 16) * h.lut32.entries.size());
    }
}

// ------------------------------------------------------------- catalogues

static std::mutex g_cat_mu;
static std::unordered_map<uint64_t, std::shared_ptr<Resident>> g_cats;
static std::atomic<uint64_t> g_next_handle{1};

Resident::~Resident() {
    if (d_mem) (void)hipFree(d_mem);
}

int validate_catalog(const pc_catalog *c, const char *name) {
    if (!c) return fail(PC_ERR_INVALID, std::string(name) + " is NULL");
    if (c->n < 0) return fail(PC_ERR_INVALID, std::string(name) + ".n < 0");
    if (c->n > 0 && (!c->ra_deg || !c->dec_deg))
        return fail(PC_ERR_INVALID, std::string(name) + " has NULL coordinate pointers");
    if (c->n > (int64_t(1) << 40)) return fail(PC_ERR_INVALID, std::string(name) + ".n too large");
    if (!c->on_device) {
        for (int64_t i = 0; i < c->n; ++i) {
            const double r = c->ra_deg[i], d = c->dec_deg[i];
            if (!std::isfinite(r) || !std::isfinite(d) || d < -90.0 || d > 90.0)
                return fail(PC_ERR_INVALID, std::string(name) + ": RA must be finite and Dec in [-90, 90] (index " +
                                                std::to_string(i) + ")");
        }
    }
    return PC_OK;
}

static int get_resident(uint64_t h, std::shared_ptr<Resident> *out) {
    std::lock_guard<std::mutex> lk(g_cat_mu);
    auto it = g_cats.find(h);
    if (it == g_cats.end()) return fail(PC_ERR_INVALID, "unknown catalogue handle");
    *out = it->second;
    return PC_OK;
}

// Stream-ordered device allocation released when the batch ends.
struct Workspace {
    void *mem = nullptr;
    hipStream_t st = nullptr;
    ~Workspace() {
        if (mem) (void)hipFreeAsync(mem, st);
    }
};

struct Arena {
    size_t size = 0;
    size_t take(size_t bytes) {
        const size_t o = (size_t(size) + 255) & ~size_t(255);
        size = o + bytes;
        return o;
    }
};

static int64_t n_tiles(int64_t n, int tile) { return (n + tile - 1) / tile; }

// ------------------------------------------------------------------- batch

// optional per-thread timing of the counting kernel (HIP events on its stream)
static thread_local bool t_timing = false;

bool thread_timing() { return t_timing; }
void set_thread_timing(bool on) { t_timing = on; }
static thread_local hipEvent_t t_ev0 = nullptr, t_ev1 = nullptr;
// per-thread cap on the counting kernel's histogram flush interval (testing)
static thread_local uint64_t t_flush_cap = 0;
// compact cell tables: 0 when they raise the waves per CU, 1 whenever built, -1 never
static thread_local int t_compact_mode = 0;
// per-thread tile size for launches without explicit parameters (testing; 0: as chosen)
static thread_local int t_force_tile = 0;
static thread_local BatchStats t_last;

int run_batch(const std::vector<BatchJob> &jobs, int mode_flags, hipStream_t st, BatchStats *stats,
              const LaunchTune *tune) {
    BatchOpts o;
    o.tune = tune;
    return run_batch_opts(jobs, mode_flags, st, stats, o);
}

int run_batch_opts(const std::vector<BatchJob> &jobs, int mode_flags, hipStream_t st, BatchStats *stats,
                   const BatchOpts &opts) {
    const LaunchTune *tune = opts.tune;
    const bool plan_only = opts.plan_bytes != nullptr;
    const bool ext = !plan_only && opts.ws != nullptr;  // caller's workspace: allocate nothing
    if (jobs.empty()) return fail(PC_ERR_INVALID, "no jobs");
    const int mode = mode_flags & ~(PC_NO_PRUNE | PC_MATRIX_CORES | PC_TUNED);
    const bool prune = (mode_flags & PC_NO_PRUNE) == 0;
    if (mode != PC_MIXED && mode != PC_FP64_PLAIN) return fail(PC_ERR_INVALID, "unknown mode");
    const bool fp64 = mode == PC_FP64_PLAIN;
    // launch parameters: explicit, tuned for this shape (PC_TUNED), or defaults
    LaunchTune lt;
    if (tune) {
        lt = *tune;
    } else if (mode_flags & PC_TUNED) {
        TuneEntry te;
        if (tune_lookup(tune_key_of(jobs), &te) == PC_OK) lt = te.tune;
        else lt.matrix_cores = (mode_flags & PC_MATRIX_CORES) != 0;
    } else {
        lt.matrix_cores = (mode_flags & PC_MATRIX_CORES) != 0;
    }
    if (!tune && t_force_tile) lt.tile = t_force_tile;
    if (lt.chunk < 1 || lt.chunk > 64) return fail(PC_ERR_INVALID, "work chunk must be in [1, 64]");
    // the matrix-core path needs the prune pass's marks; binary32 only
    if (lt.tile != 0 && lt.tile != 128 && lt.tile != 256) return fail(PC_ERR_INVALID, "tile must be 128 or 256 points");
    const TileOps &T = lt.tile == 128 ? kTile128 : kTile256;
    const int tile = T.tile;
    const bool mc = lt.matrix_cores && prune && !fp64 && T.matrix_cores;
    // host-side validation first, so bad arguments are reported as such
    for (const BatchJob &j : jobs) {
        if (j.auto_flag != 0 && j.auto_flag != 1) return fail(PC_ERR_INVALID, "auto_flag must be 0 or 1");
        std::string err;
        if (!validate_edges(j.theta, j.n_edges, err)) return fail(PC_ERR_INVALID, err);
        if (!j.counts && !plan_only) return fail(PC_ERR_INVALID, "counts is NULL");
        // inputs the caller already checked point by point (the server's
        // copies) skip the per-point scan here
        const pc_catalog *A = j.hA ? nullptr : j.A, *B = (j.auto_flag || j.hB) ? nullptr : j.B;
        if (opts.trusted_inputs) {
            if ((!j.hA && !A) || (!j.auto_flag && !j.hB && !B)) return fail(PC_ERR_INVALID, "catalogue is NULL");
        } else {
            int r = A ? validate_catalog(A, "A") : PC_OK;
            if (r) return r;
            r = B ? validate_catalog(B, "B") : PC_OK;
            if (r) return r;
        }
        if (!j.hA) {
            const int64_t nA = j.A->n;
            const int64_t r0 = j.row_begin, r1 = j.row_end < 0 ? nA : j.row_end;
            if (r0 < 0 || r1 > nA || r0 > r1)
                return fail(PC_ERR_INVALID, "row range [" + std::to_string(r0) + ", " + std::to_string(r1) +
                                                ") outside [0, " + std::to_string(nA) + "]");
        }
    }
    DeviceInfo *di = nullptr;
    int rc = PC_OK;
    if (!plan_only) {
        rc = device_info(&di);
        if (rc) return rc;
    }

    Arena ar;
    // ---- sources: catalogues as binary64 unit vectors in the caller's order
    struct Source {
        const pc_catalog *c = nullptr;
        std::shared_ptr<Resident> res;
        int64_t n = 0;
        size_t o_a64 = 0, o_ra = 0, o_dec = 0;
    };
    std::vector<Source> srcs;
    std::map<std::tuple<const double *, const double *, int64_t>, int> src_of_ptr;
    std::map<uint64_t, int> src_of_handle;
    auto add_source = [&](const pc_catalog *c, uint64_t h, int *out) -> int {
        if (h) {
            auto it = src_of_handle.find(h);
            if (it != src_of_handle.end()) { *out = it->second; return PC_OK; }
            Source sc;
            auto v = plan_only && opts.plan_sizes ? opts.plan_sizes->find(h) : std::map<uint64_t, int64_t>::const_iterator();
            if (plan_only && opts.plan_sizes && v != opts.plan_sizes->end()) {
                // planning against a catalogue described only by its size
                sc.res = std::make_shared<Resident>();
                sc.res->n = v->second;
            } else {
                int r = get_resident(h, &sc.res);
                if (r) return r;
            }
            sc.n = sc.res->n;
            *out = static_cast<int>(srcs.size());
            src_of_handle.emplace(h, *out);
            srcs.push_back(sc);
            return PC_OK;
        }
        auto key = std::make_tuple(c->ra_deg, c->dec_deg, c->n);
        auto it = src_of_ptr.find(key);
        if (it != src_of_ptr.end()) { *out = it->second; return PC_OK; }
        Source sc;
        sc.c = c;
        sc.n = c->n;
        sc.o_a64 = ar.take(sizeof(double4) * static_cast<size_t>(std::max<int64_t>(c->n, 1)));
        if (!c->on_device && c->n > 0) {
            sc.o_ra = ar.take(sizeof(double) * static_cast<size_t>(c->n));
            sc.o_dec = ar.take(sizeof(double) * static_cast<size_t>(c->n));
        }
        *out = static_cast<int>(srcs.size());
        src_of_ptr.emplace(key, *out);
        srcs.push_back(sc);
        return PC_OK;
    };

    // ---- views: spatially ordered copies of source index ranges
    struct View {
        int src = -1;
        int64_t b = 0, e = 0;
        bool resident_full = false;
        size_t o_a64s = 0, o_a32s = 0, o_g32s = 0, o_bounds = 0;
    };
    std::vector<View> views;
    std::map<std::tuple<int, int64_t, int64_t>, int> view_of;
    int64_t max_sort_n = 0;
    auto add_view = [&](int src, int64_t b, int64_t e) -> int {
        auto key = std::make_tuple(src, b, e);
        auto it = view_of.find(key);
        if (it != view_of.end()) return it->second;
        View v;
        v.src = src;
        v.b = b;
        v.e = e;
        const int64_t n = e - b;
        // a resident catalogue's own ordered copy and bounds serve a view of
        // all of it when the launch uses the tile size they were built for
        if (srcs[src].res && b == 0 && e == srcs[src].n && &T == &kResidentTile) {
            v.resident_full = true;
        } else if (n > 0) {
            v.o_a64s = ar.take(sizeof(double4) * static_cast<size_t>(n));
            // binary32 copies padded: the kernel reads a step of j-points ahead
            v.o_a32s = ar.take(sizeof(float4) * static_cast<size_t>(n + kJPad));
            v.o_g32s = ar.take(sizeof(float4) * static_cast<size_t>(n + kJPad));
            v.o_bounds = ar.take(sizeof(double4) * static_cast<size_t>(n_tiles(n, tile) * (1 + T.subs)));
            max_sort_n = std::max(max_sort_n, n);
        }
        const int id = static_cast<int>(views.size());
        view_of.emplace(key, id);
        views.push_back(v);
        return id;
    };

    std::vector<std::shared_ptr<DevTable>> tabs;
    std::map<const DevTable *, int> tab_idx;
    // planning, or the caller's workspace: the batch's own tables by edge set
    // (in the workspace, not the allocating per-device cache)
    std::map<std::pair<int, std::vector<uint64_t>>, int> local_tab;
    std::vector<TableBlob> blobs;
    struct JobPlan {
        int tab = 0;
        size_t o_counts = 0;
        int vi_tri = -1, vi_rect = -1, vj_rect = -1;
    };
    std::vector<JobPlan> plan(jobs.size());
    for (size_t q = 0; q < jobs.size(); ++q) {
        const BatchJob &j = jobs[q];
        int sa = -1, sb = -1;
        rc = add_source(j.A, j.hA, &sa);
        if (rc) return rc;
        if (!j.auto_flag) {
            rc = add_source(j.B, j.hB, &sb);
            if (rc) return rc;
        }
        const int64_t nA = srcs[sa].n;
        const int64_t r0 = j.row_begin, r1 = j.row_end < 0 ? nA : j.row_end;
        if (r0 < 0 || r1 > nA || r0 > r1)
            return fail(PC_ERR_INVALID, "row range [" + std::to_string(r0) + ", " + std::to_string(r1) +
                                            ") outside [0, " + std::to_string(nA) + "]");
        if (plan_only || ext) {
            std::vector<uint64_t> bits(static_cast<size_t>(j.n_edges));
            memcpy(bits.data(), j.theta, sizeof(double) * bits.size());
            auto key = std::make_pair(fp64 ? 0 : lt.cols, std::move(bits));
            auto it = local_tab.find(key);
            if (it == local_tab.end()) {
                auto t = std::make_shared<DevTable>();
                if (ext) {
                    std::string err;
                    if (!build_table(j.theta, j.n_edges, t->host, err, fp64 ? 0 : lt.cols))
                        return fail(PC_ERR_INVALID, err);
                    blobs.emplace_back();
                    table_blob(t->host, &blobs.back());
                }
                it = local_tab.emplace(std::move(key), static_cast<int>(tabs.size())).first;
                tabs.push_back(t);
            }
            plan[q].tab = it->second;
        } else {
            std::shared_ptr<DevTable> t;
            rc = get_table(j.theta, j.n_edges, &t, fp64 ? 0 : lt.cols);
            if (rc) return rc;
            auto it = tab_idx.find(t.get());
            if (it == tab_idx.end()) {
                it = tab_idx.emplace(t.get(), static_cast<int>(tabs.size())).first;
                tabs.push_back(t);
            }
            plan[q].tab = it->second;
        }
        if (j.auto_flag) {
            // pairs i<j with i in [r0, r1): triangle on [r0, r1) + rectangle [r0, r1) x [r1, n)
            plan[q].vi_tri = add_view(sa, r0, r1);
            if (r1 < nA && r1 > r0) {
                plan[q].vi_rect = plan[q].vi_tri;
                plan[q].vj_rect = add_view(sa, r1, nA);
            }
        } else {
            plan[q].vi_rect = add_view(sa, r0, r1);
            plan[q].vj_rect = add_view(sb, 0, srcs[sb].n);
        }
    }
    // results block, read back with one copy: meta[kMetaWords] | each job's counts | conversion flags
    // (meta[0]: survivors, meta[7]: re-check tally, from meta[kPruneStatBase]:
    // the prune pass's statistics in kPruneStripes copies, from
    // meta[kQueueBase]: the counting kernel's work queue, 8 counters
    // kQueueStride words apart)
    constexpr size_t kMetaWords = kQueueBase + 8 * kQueueStride;
    size_t res_words = kMetaWords;
    for (size_t q = 0; q < jobs.size(); ++q) res_words += static_cast<size_t>(jobs[q].n_edges + 1);
    const size_t err_words = (std::max<size_t>(srcs.size(), 1) + 1) / 2;
    const size_t o_res = ar.take(sizeof(unsigned long long) * (res_words + err_words));
    {
        size_t w = kMetaWords;
        for (size_t q = 0; q < jobs.size(); ++q) {
            plan[q].o_counts = o_res + sizeof(unsigned long long) * w;
            w += static_cast<size_t>(jobs[q].n_edges + 1);
        }
    }
    const size_t o_err = o_res + sizeof(unsigned long long) * res_words;
    const size_t o_meta = o_res;
    // the prune pass's copies of every job's counters (zeroed with the results)
    const size_t count_words = res_words - kMetaWords;
    const size_t o_pcopies = ar.take(sizeof(unsigned long long) * kPruneStripes * count_words);
    const size_t zero_words = (o_pcopies - o_res) / sizeof(unsigned long long) + kPruneStripes * count_words;
    const size_t o_scratch = ar.take(sizeof(uint32_t) * (max_sort_n > 0 ? sort_scratch_words(max_sort_n) : 1));

    // ---- segments
    std::vector<SegDesc> segs;
    uint64_t items = 0;
    bool items_overflow = false;  // more tile pairs than an item number holds
    int64_t prune_rows = 0;
    auto view_n = [&](int v) { return views[v].e - views[v].b; };
    for (size_t q = 0; q < jobs.size(); ++q) {
        auto add = [&](bool tri, int vi, int vj) {
            const int64_t ni = view_n(vi), nj = view_n(vj);
            if (ni <= 0 || nj <= 0 || (tri && ni < 2)) return;
            SegDesc sd;
            memset(&sd, 0, sizeof(sd));
            sd.tri = tri ? 1 : 0;
            sd.i0 = 0;
            sd.ni = ni;
            sd.j0 = 0;
            sd.nj = nj;
            sd.tiles_i = n_tiles(ni, tile);
            sd.tiles_j = n_tiles(nj, tile);
            // in 128 bits: up to 2^32 tiles per side, whose products pass 2^64
            const unsigned __int128 n_items =
                tri ? static_cast<unsigned __int128>(sd.tiles_i) * static_cast<unsigned __int128>(sd.tiles_i + 1) / 2
                    : static_cast<unsigned __int128>(sd.tiles_i) * static_cast<unsigned __int128>(sd.tiles_j);
            if (n_items > kItemMask || items + static_cast<uint64_t>(n_items) > kItemMask) items_overflow = true;
            sd.n_items = static_cast<uint64_t>(std::min<unsigned __int128>(n_items, kItemMask));
            sd.item0 = items;
            items = std::min<uint64_t>(items + sd.n_items, kItemMask + 1);
            // rows of the prune pass (see k_prune)
            sd.prow0 = prune_rows;
            prune_rows += tri ? (sd.tiles_i + 1) / 2 : sd.tiles_i;
            sd.tab = plan[q].tab;
            sd.job = static_cast<int32_t>(q);
            // view indices parked in the pointer slots until the workspace exists
            sd.i0 = vi;
            sd.j0 = vj;
            segs.push_back(sd);
        };
        if (plan[q].vi_tri >= 0) add(true, plan[q].vi_tri, plan[q].vi_tri);
        if (plan[q].vi_rect >= 0 && plan[q].vj_rect >= 0) add(false, plan[q].vi_rect, plan[q].vj_rect);
    }
    if (items_overflow || items > kItemMask)
        return fail(PC_ERR_INVALID, "too many tile pairs in one call (more than " + std::to_string(kItemMask) +
                                        "); split the catalogues into row ranges");
    const size_t o_segs = ar.take(sizeof(SegDesc) * std::max<size_t>(segs.size(), 1));
    const size_t o_tabs = ar.take(sizeof(TableDesc) * tabs.size());
    const size_t o_surv = ar.take(sizeof(uint64_t) * std::max<uint64_t>(prune ? items : 1, 1));
    // split survivors: the prune pass looks at the j-tile's sub-blocks too
    // (mixed mode); their descriptions sit beside the survivors
    const bool split = PC_SPLIT && prune && !fp64;
    const size_t o_sub = ar.take(sizeof(uint64_t) * std::max<uint64_t>(split ? items : 1, 1));
    std::vector<size_t> o_blob(blobs.size());
    for (size_t k = 0; k < blobs.size(); ++k) o_blob[k] = ar.take(blobs[k].bytes.size());
    if (plan_only) {
        *opts.plan_bytes = ar.size;
        return PC_OK;
    }

    // ---- the workspace: allocated here, or the caller's
    Workspace ws;
    ws.st = st;
    unsigned char *W = nullptr;
    if (ext) {
        if (ar.size > opts.ws_bytes)
            return fail(PC_ERR_INVALID, "the call needs " + std::to_string(ar.size) +
                                            " bytes of device workspace; the fixed workspace holds " +
                                            std::to_string(opts.ws_bytes));
        W = static_cast<unsigned char *>(opts.ws);
        for (size_t k = 0; k < blobs.size(); ++k) {
            PC_HIP(hipMemcpyAsync(W + o_blob[k], blobs[k].bytes.data(), blobs[k].bytes.size(), hipMemcpyHostToDevice,
                                  st),
                   "H2D tables");
            table_place(tabs[k].get(), blobs[k], W + o_blob[k]);
        }
    } else {
        PC_HIP(injected_alloc_failure() ? hipErrorOutOfMemory : hipMallocAsync(&ws.mem, ar.size, st),
               "hipMallocAsync(workspace)");
        W = static_cast<unsigned char *>(ws.mem);
    }

    // ---- convert the sources (validity flags read back at the end)
    PC_HIP(launch_zero(reinterpret_cast<unsigned long long *>(W + o_res), static_cast<int64_t>(zero_words), st),
           "zero results");
    std::vector<const double4 *> src_a64(srcs.size(), nullptr);
    for (size_t k = 0; k < srcs.size(); ++k) {
        if (srcs[k].res) {
            src_a64[k] = srcs[k].res->a64;
            continue;
        }
        const pc_catalog *c = srcs[k].c;
        src_a64[k] = reinterpret_cast<const double4 *>(W + srcs[k].o_a64);
        if (c->n <= 0) continue;
        const double *ra = c->ra_deg, *dec = c->dec_deg;
        if (!c->on_device) {
            double *dra = reinterpret_cast<double *>(W + srcs[k].o_ra);
            double *ddec = reinterpret_cast<double *>(W + srcs[k].o_dec);
            PC_HIP(hipMemcpyAsync(dra, ra, sizeof(double) * c->n, hipMemcpyHostToDevice, st), "H2D ra");
            PC_HIP(hipMemcpyAsync(ddec, dec, sizeof(double) * c->n, hipMemcpyHostToDevice, st), "H2D dec");
            ra = dra;
            dec = ddec;
        }
        PC_HIP(launch_convert(ra, dec, c->n, reinterpret_cast<double4 *>(W + srcs[k].o_a64), nullptr,
                              reinterpret_cast<int *>(W + o_err) + k, st),
               "convert");
    }

    // ---- spatially ordered views and their tile bounds
    struct ViewPtrs {
        const double4 *a64s = nullptr;
        const float4 *a32s = nullptr;
        const float4 *g32s = nullptr;
        const double4 *bounds = nullptr;
        const double4 *sub_bounds = nullptr;  // T.subs per tile, after the tiles' own
    };
    std::vector<ViewPtrs> vp(views.size());
    for (size_t v = 0; v < views.size(); ++v) {
        const View &vw = views[v];
        if (vw.resident_full) {
            const Resident &r = *srcs[vw.src].res;
            vp[v].a64s = r.a64s;
            vp[v].a32s = r.a32s;
            vp[v].g32s = r.g32s;
            vp[v].bounds = r.bounds;
            vp[v].sub_bounds = r.bounds + n_tiles(r.n, tile);
            continue;
        }
        const int64_t n = vw.e - vw.b;
        if (n <= 0) continue;
        double4 *a64s = reinterpret_cast<double4 *>(W + vw.o_a64s);
        float4 *a32s = reinterpret_cast<float4 *>(W + vw.o_a32s);
        float4 *g32s = reinterpret_cast<float4 *>(W + vw.o_g32s);
        double4 *bnd = reinterpret_cast<double4 *>(W + vw.o_bounds);
        PC_HIP(T.launch_sort(src_a64[vw.src], vw.b, n, reinterpret_cast<uint32_t *>(W + o_scratch), a64s, a32s, g32s,
                           bnd, st),
               "sort");
        vp[v].a64s = a64s;
        vp[v].a32s = a32s;
        vp[v].g32s = g32s;
        vp[v].bounds = bnd;
        vp[v].sub_bounds = bnd + n_tiles(n, tile);
    }

    // ---- descriptors
    for (SegDesc &sd : segs) {
        const int vi = static_cast<int>(sd.i0), vj = static_cast<int>(sd.j0);
        sd.i0 = 0;
        sd.j0 = 0;
        sd.i32 = vp[vi].a32s;
        sd.i64 = vp[vi].a64s;
        sd.ib = vp[vi].bounds;
        sd.j32 = vp[vj].a32s;
        sd.j64 = vp[vj].a64s;
        sd.jb = vp[vj].bounds;
        sd.jg = vp[vj].g32s;
        sd.jb_sub = vp[vj].sub_bounds;
        sd.counts = reinterpret_cast<unsigned long long *>(W + plan[static_cast<size_t>(sd.job)].o_counts);
        sd.pcounts = reinterpret_cast<unsigned long long *>(W + o_pcopies + plan[static_cast<size_t>(sd.job)].o_counts -
                                                            o_res - sizeof(unsigned long long) * kMetaWords);
        sd.pstride = static_cast<int64_t>(count_words);
    }
    std::vector<TableDesc> tds;
    bool compact_ok = !fp64 && !mc;
    for (auto &t : tabs) {
        tds.push_back(table_desc(*t, fp64));
        compact_ok = compact_ok && t->d_lutc != nullptr;
    }
    // LDS: histogram | cell table (or edges) | matrix-core A operands
    auto layout = [&](bool compact, uint32_t *lut_off, uint32_t *stage_off, uint32_t *lds) {
        uint32_t hist_max = 0, lut_max = 0;
        for (auto &t : tabs) {
            uint32_t h, l;
            table_lds(*t, fp64, compact, &h, &l);
            hist_max = std::max(hist_max, h);
            lut_max = std::max(lut_max, l);
        }
        *lut_off = (hist_max + 15u) & ~15u;
        *stage_off = *lut_off + ((std::max<uint32_t>(lut_max, 16u) + 15u) & ~15u);
        *lds = *stage_off + (mc ? 16u * kWave * 4u : 0u);
    };
    uint32_t lut_off = 0, stage_off = 0, lds_bytes = 0;
    layout(false, &lut_off, &stage_off, &lds_bytes);
    // the compact cell table costs one instruction per cell-table chord; it
    // is taken when its smaller LDS footprint lets more waves share a CU
    bool compact = false;
    if (compact_ok && t_compact_mode >= 0 && items > 0) {
        uint32_t lo_c = 0, so_c = 0, lds_c = 0;
        layout(true, &lo_c, &so_c, &lds_c);
        bool take = t_compact_mode > 0;
        if (!take && lds_bytes <= di->lds_per_block) {
            int full = 0, small = 0;
            PC_HIP(T.count_occupancy(false, false, false, lds_bytes, &full), "occupancy");
            PC_HIP(T.count_occupancy(false, false, true, lds_c, &small), "occupancy");
            take = small > full;
        } else if (!take) {
            take = true;  // only the compact table fits
        }
        if (take) {
            compact = true;
            lut_off = lo_c;
            stage_off = so_c;
            lds_bytes = lds_c;
        }
    }
    if (lds_bytes > di->lds_per_block)
        return fail(PC_ERR_INVALID, "edge set needs " + std::to_string(lds_bytes) +
                                        " bytes of LDS per wave; the device allows " +
                                        std::to_string(di->lds_per_block));
    if (!segs.empty())
        PC_HIP(hipMemcpyAsync(W + o_segs, segs.data(), sizeof(SegDesc) * segs.size(), hipMemcpyHostToDevice, st),
               "H2D segments");
    PC_HIP(hipMemcpyAsync(W + o_tabs, tds.data(), sizeof(TableDesc) * tds.size(), hipMemcpyHostToDevice, st),
           "H2D tables");
    unsigned long long *meta = reinterpret_cast<unsigned long long *>(W + o_meta);

    // ---- whole-tile-pair binning, then the counting kernel over the rest
    const SegDesc *d_segs = reinterpret_cast<const SegDesc *>(W + o_segs);
    const TableDesc *d_tabs = reinterpret_cast<const TableDesc *>(W + o_tabs);
    uint64_t *surv = reinterpret_cast<uint64_t *>(W + o_surv);
    uint64_t *sub_words = reinterpret_cast<uint64_t *>(W + o_sub);
    int grid = 0;
    if (items > 0) {
        if (prune) {
            PC_HIP(T.launch_prune(d_segs, static_cast<int32_t>(segs.size()), d_tabs, prune_rows, surv,
                                split ? sub_words : nullptr, meta, mc ? 1 : 0, split ? 1 : 0, st),
                   "prune");
            PC_HIP(launch_add_copies(reinterpret_cast<unsigned long long *>(W + o_res) + kMetaWords,
                                     reinterpret_cast<const unsigned long long *>(W + o_pcopies),
                                     static_cast<int64_t>(count_words), kPruneStripes, st),
                   "add prune counts");
        }
        int per_cu = 0;
        PC_HIP(T.count_occupancy(fp64, mc, compact, lds_bytes, &per_cu), "occupancy");
        per_cu = std::max(per_cu, 1);
        int64_t g = static_cast<int64_t>(di->cus) * per_cu;
        g = std::min<int64_t>(g, static_cast<int64_t>(items));
        if (g >= 8) g -= g % 8;
        grid = static_cast<int>(std::max<int64_t>(g, 1));
        const bool timed = t_timing && !ext;  // events are not created in the caller's-workspace mode
        if (timed) {
            if (!t_ev0) {
                PC_HIP(hipEventCreate(&t_ev0), "hipEventCreate");
                PC_HIP(hipEventCreate(&t_ev1), "hipEventCreate");
            }
            PC_HIP(hipEventRecord(t_ev0, st), "hipEventRecord");
        }
        PC_HIP(T.launch_count(fp64, mc, compact, d_segs, static_cast<int32_t>(segs.size()), d_tabs, prune ? surv : nullptr,
                            prune ? meta : nullptr, split ? sub_words : nullptr, items, lut_off, stage_off, meta + kQueueBase,
                            meta + 7, lt.chunk, lds_bytes, grid, t_flush_cap, st),
               "count kernel");
        if (timed) PC_HIP(hipEventRecord(t_ev1, st), "hipEventRecord");
    }

    // ---- results: counts, validity flags and pruning figures under one sync
    std::vector<unsigned long long> hres(res_words + err_words, 0ull);
    PC_HIP(hipMemcpyAsync(hres.data(), W + o_res, sizeof(unsigned long long) * hres.size(), hipMemcpyDeviceToHost, st),
           "D2H results");
    PC_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
    const int *flags = reinterpret_cast<const int *>(hres.data() + res_words);
    for (size_t k = 0; k < srcs.size(); ++k)
        if (flags[k]) return fail(PC_ERR_INVALID, "catalogue has non-finite RA/Dec or |Dec| > 90");
    for (size_t q = 0; q < jobs.size(); ++q)
        memcpy(jobs[q].counts, hres.data() + (plan[q].o_counts - o_res) / sizeof(unsigned long long),
               sizeof(uint64_t) * static_cast<size_t>(jobs[q].n_edges + 1));
    const unsigned long long *hmeta = hres.data();
    uint64_t ps[kPruneStats] = {};  // the prune pass's statistics, stripes added up
    for (int c = 0; c < kPruneStripes; ++c)
        for (int k = 1; k < kPruneStats; ++k) ps[k] += hmeta[kPruneStatBase + c * kPruneStripeWords + k];

    uint64_t total_pairs = 0;
    for (const SegDesc &sd : segs) {
        const uint64_t ni = static_cast<uint64_t>(sd.ni), nj = static_cast<uint64_t>(sd.nj);
        total_pairs += sd.tri ? ni * (ni - 1) / 2 : ni * nj;
    }
    t_last = BatchStats();
    t_last.items = items;
    t_last.grid = grid;
    t_last.lds_bytes = lds_bytes;
    t_last.segments = static_cast<int>(segs.size());
    t_last.kernel_ms = -1.0;
    t_last.survivors = prune ? hmeta[0] : items;
    t_last.pairs_total = total_pairs;
    t_last.pairs_computed = prune ? ps[1] : total_pairs;
    t_last.mfma_items = prune ? ps[2] : 0;
    t_last.few_items = prune ? ps[3] : 0;
    t_last.gram_items = prune ? ps[4] : 0;
    t_last.split_items = prune ? ps[5] : 0;
    t_last.rechecked = hmeta[7];
    for (int m = 0; m < 4; ++m) t_last.pairs_by_m[m] = prune ? ps[6 + m] : 0;
    t_last.pairs_gram = prune ? ps[10] : 0;
    if (!prune || fp64) {
        // every computed pair through the cell table (the binary64 kernel
        // ignores the few-edge tags)
        t_last.pairs_by_m[0] = t_last.pairs_computed;
        for (int m = 1; m < 4; ++m) t_last.pairs_by_m[m] = 0;
        t_last.pairs_gram = 0;
    }
    t_last.pairs_mfma = prune ? ps[11] : 0;
    t_last.workspace_bytes = ar.size;
    if (t_timing && !ext && items > 0) {
        float ms = 0.0f;
        PC_HIP(hipEventElapsedTime(&ms, t_ev0, t_ev1), "hipEventElapsedTime");
        t_last.kernel_ms = ms;
    }
    if (stats) *stats = t_last;
    return PC_OK;
}

int upload_catalog(const pc_catalog *c, hipStream_t st, uint64_t *handle) {
    int rc = validate_catalog(c, "catalogue");
    if (rc) return rc;
    if (!handle) return fail(PC_ERR_INVALID, "handle is NULL");
    DeviceInfo *di = nullptr;
    rc = device_info(&di);
    if (rc) return rc;
    auto r = std::make_shared<Resident>();
    r->n = c->n;
    r->device = di->device;
    const size_t n = static_cast<size_t>(std::max<int64_t>(c->n, 1));
    Arena ar;
    const size_t o64 = ar.take(sizeof(double4) * n);
    const size_t o32 = ar.take(sizeof(float4) * n);
    const size_t o64s = ar.take(sizeof(double4) * n);
    const size_t o32s = ar.take(sizeof(float4) * (n + kJPad));  // padded as in run_batch
    const size_t og32s = ar.take(sizeof(float4) * (n + kJPad));
    const size_t ob = ar.take(sizeof(double4) * static_cast<size_t>(n_tiles(static_cast<int64_t>(n), kResidentTile.tile) *
                                                                     (1 + kResidentTile.subs)));
    const size_t oerr = ar.take(sizeof(int));
    const size_t osc = ar.take(sizeof(uint32_t) * sort_scratch_words(static_cast<int64_t>(n)));
    size_t ora = 0, odec = 0;
    if (!c->on_device) {
        ora = ar.take(sizeof(double) * n);
        odec = ar.take(sizeof(double) * n);
    }
    PC_HIP(injected_alloc_failure() ? hipErrorOutOfMemory : hipMalloc(&r->d_mem, ar.size), "hipMalloc(catalogue)");
    unsigned char *W = static_cast<unsigned char *>(r->d_mem);
    r->a64 = reinterpret_cast<double4 *>(W + o64);
    r->a32 = reinterpret_cast<float4 *>(W + o32);
    r->a64s = reinterpret_cast<double4 *>(W + o64s);
    r->a32s = reinterpret_cast<float4 *>(W + o32s);
    r->g32s = reinterpret_cast<float4 *>(W + og32s);
    r->bounds = reinterpret_cast<double4 *>(W + ob);
    PC_HIP(hipMemsetAsync(W + oerr, 0, sizeof(int), st), "hipMemsetAsync");
    if (c->n > 0) {
        const double *ra = c->ra_deg, *dec = c->dec_deg;
        if (!c->on_device) {
            PC_HIP(hipMemcpyAsync(W + ora, ra, sizeof(double) * c->n, hipMemcpyHostToDevice, st), "H2D ra");
            PC_HIP(hipMemcpyAsync(W + odec, dec, sizeof(double) * c->n, hipMemcpyHostToDevice, st), "H2D dec");
            ra = reinterpret_cast<const double *>(W + ora);
            dec = reinterpret_cast<const double *>(W + odec);
        }
        PC_HIP(launch_convert(ra, dec, c->n, r->a64, r->a32, reinterpret_cast<int *>(W + oerr), st), "convert");
        PC_HIP(kResidentTile.launch_sort(r->a64, 0, c->n, reinterpret_cast<uint32_t *>(W + osc), r->a64s, r->a32s, r->g32s,
                           r->bounds, st),
               "sort");
    }
    int flag = 0;
    PC_HIP(hipMemcpyAsync(&flag, W + oerr, sizeof(int), hipMemcpyDeviceToHost, st), "D2H flag");
    PC_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
    if (flag) return fail(PC_ERR_INVALID, "catalogue has non-finite RA/Dec or |Dec| > 90");
    const uint64_t h = g_next_handle.fetch_add(1);
    {
        std::lock_guard<std::mutex> lk(g_cat_mu);
        g_cats.emplace(h, r);
    }
    *handle = h;
    return PC_OK;
}

int release_catalog(uint64_t h) {
    std::shared_ptr<Resident> r;
    {
        std::lock_guard<std::mutex> lk(g_cat_mu);
        auto it = g_cats.find(h);
        if (it == g_cats.end()) return fail(PC_ERR_INVALID, "unknown catalogue handle");
        r = it->second;
        g_cats.erase(it);
    }
    // the allocation goes when the last user (a running batch) drops it
    return PC_OK;
}

int resident_catalog(uint64_t h, std::shared_ptr<Resident> *out) { return get_resident(h, out); }

int jobs_from_abi(const pc_job *jobs, int32_t n_jobs, std::vector<BatchJob> *out) {
    if (!jobs || n_jobs < 1) return fail(PC_ERR_INVALID, "jobs is NULL or n_jobs < 1");
    std::vector<BatchJob> &v = *out;
    v.assign(static_cast<size_t>(n_jobs), BatchJob());
    for (int32_t q = 0; q < n_jobs; ++q) {
        v[q].A = jobs[q].A;
        v[q].B = jobs[q].B;
        v[q].theta = jobs[q].theta_edges_deg;
        v[q].n_edges = jobs[q].n_edges;
        v[q].auto_flag = jobs[q].auto_flag;
        v[q].row_begin = jobs[q].row_begin;
        v[q].row_end = jobs[q].row_end;
        v[q].counts = jobs[q].counts;
    }
    return PC_OK;
}

}  // namespace pc

// ===================================================================== C ABI

using namespace pc;

extern "C" {

const char *pc_last_error(void) { return t_err.c_str(); }

const char *pc_version(void) { return "pc 0.1 gfx950"; }

int pc_count_ex(const pc_catalog *A, const pc_catalog *B, const double *theta_edges_deg, int32_t n_edges,
                int32_t auto_flag, int32_t mode, int64_t row_begin, int64_t row_end, uint64_t *counts,
                void *stream) {
    clear_error();
    BatchJob j;
    j.A = A;
    j.B = B;
    j.theta = theta_edges_deg;
    j.n_edges = n_edges;
    j.auto_flag = auto_flag;
    j.row_begin = row_begin;
    j.row_end = row_end;
    j.counts = counts;
    std::vector<BatchJob> v(1, j);
    return run_batch(v, mode, static_cast<hipStream_t>(stream), nullptr);
}

int pc_count(const pc_catalog *A, const pc_catalog *B, const double *theta_edges_deg, int32_t n_edges,
             int32_t auto_flag, uint64_t *counts, void *stream) {
    return pc_count_ex(A, B, theta_edges_deg, n_edges, auto_flag, PC_MIXED, 0, -1, counts, stream);
}

int pc_count_batch(const pc_job *jobs, int32_t n_jobs, int32_t mode, void *stream) {
    clear_error();
    std::vector<BatchJob> v;
    const int rc = jobs_from_abi(jobs, n_jobs, &v);
    if (rc) return rc;
    return run_batch(v, mode, static_cast<hipStream_t>(stream), nullptr);
}

int pc_wtheta(const uint64_t *DD, const uint64_t *DR, const uint64_t *RR, int32_t n_bins, int64_t nD, int64_t nR,
              double *w) {
    clear_error();
    if (!DD || !DR || !RR || !w) return fail(PC_ERR_INVALID, "NULL argument");
    if (n_bins < 1) return fail(PC_ERR_INVALID, "n_bins must be >= 1");
    if (nD < 2 || nR < 2) return fail(PC_ERR_INVALID, "nD and nR must be >= 2");
    landy_szalay(DD, DR, RR, n_bins, nD, nR, w);
    return PC_OK;
}

int pc_estimator(int32_t kind, const uint64_t *DD, const uint64_t *DR, const uint64_t *RR, int32_t n_bins,
                 int64_t nD, int64_t nR, double *w) {
    clear_error();
    if (kind < PC_EST_LANDY_SZALAY || kind > PC_EST_HAMILTON) return fail(PC_ERR_INVALID, "unknown estimator");
    const bool need_dr = kind != PC_EST_NATURAL, need_rr = kind != PC_EST_DAVIS_PEEBLES;
    if (!DD || !w || (need_dr && !DR) || (need_rr && !RR)) return fail(PC_ERR_INVALID, "NULL argument");
    if (n_bins < 1) return fail(PC_ERR_INVALID, "n_bins must be >= 1");
    if (nD < 2 || nR < 2) return fail(PC_ERR_INVALID, "nD and nR must be >= 2");
    estimator(kind, DD, DR, RR, n_bins, nD, nR, w);
    return PC_OK;
}

int pc_catalog_upload(const pc_catalog *c, void *stream, uint64_t *handle) {
    clear_error();
    return upload_catalog(c, static_cast<hipStream_t>(stream), handle);
}

int pc_catalog_release(uint64_t handle) {
    clear_error();
    return release_catalog(handle);
}

int pc_count_h(uint64_t hA, uint64_t hB, const double *theta_edges_deg, int32_t n_edges, int32_t auto_flag,
               int32_t mode, int64_t row_begin, int64_t row_end, uint64_t *counts, void *stream) {
    clear_error();
    if (!hA || (!auto_flag && !hB)) return fail(PC_ERR_INVALID, "catalogue handle is 0");
    BatchJob j;
    j.hA = hA;
    j.hB = auto_flag ? 0 : hB;
    j.theta = theta_edges_deg;
    j.n_edges = n_edges;
    j.auto_flag = auto_flag;
    j.row_begin = row_begin;
    j.row_end = row_end;
    j.counts = counts;
    std::vector<BatchJob> v(1, j);
    return run_batch(v, mode, static_cast<hipStream_t>(stream), nullptr);
}

int pc_unit_vectors(const pc_catalog *c, double *xyz64, float *xyz32, void *stream) {
    clear_error();
    uint64_t h = 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int rc = upload_catalog(c, st, &h);
    if (rc) return rc;
    std::shared_ptr<Resident> r;
    get_resident(h, &r);
    release_catalog(h);
    const size_t n = static_cast<size_t>(c->n);
    if (n > 0) {
        std::vector<double4> v64(n);
        std::vector<float4> v32(n);
        PC_HIP(hipMemcpyAsync(v64.data(), r->a64, sizeof(double4) * n, hipMemcpyDeviceToHost, st), "D2H a64");
        PC_HIP(hipMemcpyAsync(v32.data(), r->a32, sizeof(float4) * n, hipMemcpyDeviceToHost, st), "D2H a32");
        PC_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
        for (size_t i = 0; i < n; ++i) {
            if (xyz64) {
                xyz64[3 * i + 0] = v64[i].x;
                xyz64[3 * i + 1] = v64[i].y;
                xyz64[3 * i + 2] = v64[i].z;
            }
            if (xyz32) {
                xyz32[3 * i + 0] = v32[i].x;
                xyz32[3 * i + 1] = v32[i].y;
                xyz32[3 * i + 2] = v32[i].z;
            }
        }
    }
    return PC_OK;
}

int pc_chord2_edges(const double *theta_edges_deg, int32_t n_edges, double *e) {
    clear_error();
    if (!theta_edges_deg || !e) return fail(PC_ERR_INVALID, "NULL argument");
    HostTable t;
    std::string err;
    if (!build_table(theta_edges_deg, n_edges, t, err)) return fail(PC_ERR_INVALID, err);
    memcpy(e, t.e64.data(), sizeof(double) * static_cast<size_t>(n_edges));
    return PC_OK;
}

int pc_guard_band(const double *theta_edges_deg, int32_t n_edges, float *lo, float *hi) {
    clear_error();
    if (!theta_edges_deg || !lo || !hi) return fail(PC_ERR_INVALID, "NULL argument");
    HostTable t;
    std::string err;
    if (!build_table(theta_edges_deg, n_edges, t, err)) return fail(PC_ERR_INVALID, err);
    memcpy(lo, t.lo.data(), sizeof(float) * static_cast<size_t>(n_edges));
    memcpy(hi, t.hi.data(), sizeof(float) * static_cast<size_t>(n_edges));
    return PC_OK;
}

}  // extern "C"

extern "C" int pc_debug_lut32(const double *theta_edges_deg, int32_t n_edges, int64_t *info, uint32_t *entries,
                              int64_t max_cells) {
    clear_error();
    if (!theta_edges_deg || !info) return fail(PC_ERR_INVALID, "NULL argument");
    HostTable t;
    std::string err;
    if (!build_table(theta_edges_deg, n_edges, t, err)) return fail(PC_ERR_INVALID, err);
    const Lut32 &L = t.lut32;
    info[0] = static_cast<int64_t>(L.entries.size());
    info[1] = L.shift;
    info[2] = L.clamp_lo;
    info[3] = L.clamp_hi;
    info[4] = t.row_bytes32;
    info[5] = t.cols32;
    info[6] = L.multi;
    info[7] = 0;
    if (entries && static_cast<int64_t>(L.entries.size()) <= max_cells)
        memcpy(entries, L.entries.data(), sizeof(LutEntry32) * L.entries.size());
    return PC_OK;
}

extern "C" int pc_debug_fused_band(const double *theta_edges_deg, int32_t n_edges, int32_t gram, float *h,
                                   float *w) {
    clear_error();
    if (!theta_edges_deg || !h || !w) return fail(PC_ERR_INVALID, "NULL argument");
    HostTable t;
    std::string err;
    if (!build_table(theta_edges_deg, n_edges, t, err)) return fail(PC_ERR_INVALID, err);
    memcpy(h, (gram ? t.fh_g : t.fh).data(), sizeof(float) * static_cast<size_t>(n_edges));
    memcpy(w, (gram ? t.fw_g : t.fw).data(), sizeof(float) * static_cast<size_t>(n_edges));
    return PC_OK;
}

extern "C" int pc_debug_guard_band_gram(const double *theta_edges_deg, int32_t n_edges, float *lo, float *hi) {
    clear_error();
    if (!theta_edges_deg || !lo || !hi) return fail(PC_ERR_INVALID, "NULL argument");
    HostTable t;
    std::string err;
    if (!build_table(theta_edges_deg, n_edges, t, err)) return fail(PC_ERR_INVALID, err);
    memcpy(lo, t.lo_g.data(), sizeof(float) * static_cast<size_t>(n_edges));
    memcpy(hi, t.hi_g.data(), sizeof(float) * static_cast<size_t>(n_edges));
    return PC_OK;
}

extern "C" int pc_debug_fail_allocations(int32_t n) {
    clear_error();
    if (n < 0) return fail(PC_ERR_INVALID, "n must be >= 0");
    t_fail_allocs = n;
    return PC_OK;
}

extern "C" int pc_debug_set_tile(int32_t tile) {
    clear_error();
    if (tile != 0 && tile != 128 && tile != 256) return fail(PC_ERR_INVALID, "tile must be 0, 128 or 256");
    t_force_tile = tile;
    return PC_OK;
}

extern "C" int pc_debug_set_flush_every(uint64_t items) {
    clear_error();
    t_flush_cap = items;
    return PC_OK;
}

extern "C" int pc_debug_set_compact_table(int32_t mode) {
    clear_error();
    if (mode < -1 || mode > 1) return fail(PC_ERR_INVALID, "mode must be -1, 0 or 1");
    t_compact_mode = mode;
    return PC_OK;
}

extern "C" int pc_debug_set_timing(int32_t on) {
    clear_error();
    t_timing = on != 0;
    return PC_OK;
}

extern "C" int pc_debug_last_pruning(uint64_t *survivors, uint64_t *pairs_computed, uint64_t *pairs_total,
                                     uint64_t *mfma_items, uint64_t *few_items, uint64_t *gram_items,
                                     uint64_t *split_items) {
    clear_error();
    if (split_items) *split_items = t_last.split_items;
    if (gram_items) *gram_items = t_last.gram_items;
    if (few_items) *few_items = t_last.few_items;
    if (mfma_items) *mfma_items = t_last.mfma_items;
    if (survivors) *survivors = t_last.survivors;
    if (pairs_computed) *pairs_computed = t_last.pairs_computed;
    if (pairs_total) *pairs_total = t_last.pairs_total;
    return PC_OK;
}

extern "C" int pc_debug_last_paths(uint64_t *pairs_by_edges, uint64_t *gram_pairs, uint64_t *mfma_pairs) {
    clear_error();
    if (pairs_by_edges)
        for (int m = 0; m < 4; ++m) pairs_by_edges[m] = t_last.pairs_by_m[m];
    if (gram_pairs) *gram_pairs = t_last.pairs_gram;
    if (mfma_pairs) *mfma_pairs = t_last.pairs_mfma;
    return PC_OK;
}

extern "C" int pc_debug_last_rechecks(uint64_t *pairs_rechecked) {
    clear_error();
    if (!pairs_rechecked) return fail(PC_ERR_INVALID, "pairs_rechecked is NULL");
    *pairs_rechecked = t_last.rechecked;
    return PC_OK;
}

extern "C" int pc_debug_last_launch(double *kernel_ms, uint64_t *items, int32_t *grid, uint32_t *lds_bytes) {
    clear_error();
    if (kernel_ms) *kernel_ms = t_last.kernel_ms;
    if (items) *items = t_last.items;
    if (grid) *grid = t_last.grid;
    if (lds_bytes) *lds_bytes = t_last.lds_bytes;
    return PC_OK;
}
