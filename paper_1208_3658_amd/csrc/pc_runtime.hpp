// pc_runtime.hpp -- host runtime internals shared by the C ABI and the server.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/pc.h"
#include "pc_internal.hpp"

namespace pc {

int fail(int code, const std::string &msg);
// true when a test asked this thread's next device allocation to fail
// (pc_debug_fail_allocations); the caller then reports it as out of memory
bool injected_alloc_failure();
int hip_fail(hipError_t e, const char *what);
void clear_error();

struct DeviceInfo {
    int device = 0;
    int cus = 0;
    uint32_t lds_per_block = 0;
    uint32_t lds_per_cu = 0;
    std::string arch;
    bool ok = false;
};
int device_info(DeviceInfo **out);

// An edge set uploaded to one device.
struct DevTable {
    HostTable host;
    void *d_mem = nullptr;
    const double *d_e64 = nullptr;
    const float *d_band = nullptr;    // (lo, hi) per edge, binary32 guard band
    const float *d_band_g = nullptr;  // the same for the matrix-core path
    const float *d_fband = nullptr;   // (h, W) per edge, the vector few-edge paths' fused thresholds
    const float *d_fband_g = nullptr; // the same for tile-centred Gram chords
    const void *d_lut32 = nullptr;
    const void *d_lutc = nullptr;
    const void *d_lut64 = nullptr;
    ~DevTable();
};
// cols: histogram lane columns of the mixed kernel's tables (0 = default)
int get_table(const double *theta, int32_t n_edges, std::shared_ptr<DevTable> *out, int cols = 0);

// A table's device image: e64 | band | band_g | fband | fband_g | lut32 |
// lutc | lut64 at the offsets below (256-byte aligned), built on the host.
struct TableBlob {
    std::vector<unsigned char> bytes;
    size_t o_band = 0, o_band_g = 0, o_fband = 0, o_fband_g = 0, o_lut32 = 0, o_lutc = 0, o_lut64 = 0;
};
void table_blob(const HostTable &h, TableBlob *out);
// points t's device pointers into a copy of the blob at `base` (t does not own it)
void table_place(DevTable *t, const TableBlob &b, unsigned char *base);

// A converted catalogue kept on the device.
struct Resident {
    void *d_mem = nullptr;
    double4 *a64 = nullptr;     // caller order
    float4 *a32 = nullptr;      // caller order
    double4 *a64s = nullptr;    // spatially ordered copy
    float4 *a32s = nullptr;
    float4 *g32s = nullptr;     // ordered copy in Gram form, centred on its tile
    double4 *bounds = nullptr;  // tile bounds of the ordered copy
    int64_t n = 0;
    int device = 0;
    ~Resident();
};
int validate_catalog(const pc_catalog *c, const char *name);
int upload_catalog(const pc_catalog *c, hipStream_t st, uint64_t *handle);
int release_catalog(uint64_t h);
int resident_catalog(uint64_t h, std::shared_ptr<Resident> *out);

// One counting job: catalogues by pointer (A/B) or by resident handle (hA/hB).
struct BatchJob {
    const pc_catalog *A = nullptr;
    const pc_catalog *B = nullptr;
    uint64_t hA = 0, hB = 0;
    const double *theta = nullptr;
    int32_t n_edges = 0;
    int32_t auto_flag = 1;
    int64_t row_begin = 0;
    int64_t row_end = -1;
    uint64_t *counts = nullptr;  // host, n_edges + 1
};

struct BatchStats {
    uint64_t items = 0;
    int grid = 0;
    uint32_t lds_bytes = 0;
    int segments = 0;
    double kernel_ms = -1.0;
    uint64_t survivors = 0;       // work items left after whole-tile-pair binning
    uint64_t pairs_total = 0;     // pairs counted by the launch
    uint64_t pairs_computed = 0;  // pairs visited one by one
    uint64_t mfma_items = 0;      // of the survivors, tile pairs done on the matrix cores
    uint64_t few_items = 0;       // work units (survivors, or open sub-blocks of split ones) with few edges inside
    uint64_t gram_items = 0;      // work units with Gram-form chords on the vector path
    uint64_t split_items = 0;     // survivors visited as sub-blocks of the j-tile
    uint64_t rechecked = 0;       // pairs whose binary32 chord fell in a guard band (re-checked in binary64)
    // computed pairs by the counting kernel's path: [m] binned against m edges
    // one by one (m = 1..3), [0] through the cell table (or binary64 kernel)
    uint64_t pairs_by_m[4] = {0, 0, 0, 0};
    uint64_t pairs_gram = 0;      // of the few-edge pairs, chords in tile-centred Gram form
    uint64_t pairs_mfma = 0;      // pairs on the matrix cores
    uint64_t workspace_bytes = 0; // device workspace of the launch
};

// Launch parameters a tuner may choose (all give the same counts):
// histogram lane columns of the mixed kernel (0 = the table's default), work
// items taken from the queue at a time, the matrix-core chord path (256-point
// tiles only) and the tile size.
struct LaunchTune {
    int cols = 0;
    int chunk = 4;
    bool matrix_cores = false;
    int tile = 256;  // points per tile, 128 or 256 (0: 256)
};

// Runs the jobs in one persistent launch on `st` and blocks until the host
// counts are written.  `tune` (may be null) overrides the launch parameters;
// with PC_TUNED in `mode` and no `tune`, a tuned entry for the batch's shape
// is used when one exists.
int run_batch(const std::vector<BatchJob> &jobs, int mode, hipStream_t st, BatchStats *stats,
              const LaunchTune *tune = nullptr);

// Further options of a batch:
//  * ws / ws_bytes: run in this caller-provided device workspace instead of
//    allocating one; the batch's edge-set tables are placed in it too (not
//    taken from the per-device cache, which allocates).  PC_ERR_INVALID when
//    the batch needs more than ws_bytes (nothing is launched then).
//  * plan_bytes: only plan -- write the workspace bytes the batch needs
//    (tables excluded; they are cached per device) and return, with no device
//    call.  Catalogue arguments are validated as for a real run.
//  * trusted_inputs: the host catalogues were already checked point by point
//    (finite RA, |Dec| <= 90); only their shape is checked here.
//  * plan_sizes (planning only): resident-catalogue handles that need not
//    exist, given by their number of points.
struct BatchOpts {
    const LaunchTune *tune = nullptr;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    uint64_t *plan_bytes = nullptr;
    bool trusted_inputs = false;
    const std::map<uint64_t, int64_t> *plan_sizes = nullptr;
};
int run_batch_opts(const std::vector<BatchJob> &jobs, int mode, hipStream_t st, BatchStats *stats,
                   const BatchOpts &opts);

// Tuned entries: keyed by device, edge count class and pair count class.
struct TuneKey {
    std::string device;
    int edges_class = 0;  // ceil(log2(max n_edges over the jobs))
    int pairs_class = 0;  // floor(log2(pairs in the batch))
    bool operator<(const TuneKey &o) const {
        return std::tie(device, edges_class, pairs_class) < std::tie(o.device, o.edges_class, o.pairs_class);
    }
};
struct TuneEntry {
    LaunchTune tune;
    double kernel_ms = 0.0;  // counting kernel (HIP events)
    double launch_ms = 0.0;  // the whole launch (host clock)
};
TuneKey tune_key_of(const std::vector<BatchJob> &jobs);
int tune_lookup(const TuneKey &k, TuneEntry *e);
void tune_store(const TuneKey &k, const TuneEntry &e);
int tune_load_file(const char *path);
int tune_save_file(const char *path);

// pc_job array -> BatchJob list (validates the pointer and count only)
int jobs_from_abi(const pc_job *jobs, int32_t n_jobs, std::vector<BatchJob> *out);
// per-thread HIP-event timing of the counting kernel (see pc_debug_set_timing)
bool thread_timing();
void set_thread_timing(bool on);

// Landy-Szalay in binary64, fixed operation order, no contraction.
// kind: 0 Landy-Szalay, 1 natural, 2 Davis-Peebles, 3 Hamilton (see pc.h)
void estimator(int32_t kind, const uint64_t *DD, const uint64_t *DR, const uint64_t *RR, int32_t n_bins,
               int64_t nD, int64_t nR, double *w);
void landy_szalay(const uint64_t *DD, const uint64_t *DR, const uint64_t *RR, int32_t n_bins, int64_t nD,
                  int64_t nR, double *w);

}  // namespace pc
