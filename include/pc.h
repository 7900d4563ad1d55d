/*
 * pc.h -- exact angular pair counting on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libpc.so.  Plain pointers and sizes only.
 *
 * The problem (Bard et al., "Cosmological calculations on the GPU", Sec. 2):
 * given catalogues of sky positions (RA, Dec), count pairs of points by their
 * great-circle separation theta (Appendix A) in user-chosen bins (Sec. 2.1,
 * binning presets): DD and RR over the n(n-1)/2 unordered pairs of one
 * catalogue (no self-pairs, no double counting), DR over all n*n_r pairs of
 * two catalogues; then form the Landy-Szalay estimate w(theta) (Eq. 2).
 *
 * Counts are exact: every pair is binned as the binary64 reference
 * definition bins it (unit vectors from RA/Dec by an exactly specified
 * degree sine/cosine, squared chord c = (dx*dx + dy*dy) + dz*dz with no fused
 * multiply-add, compared with edges 4*sin^2(theta_k/2)).  The fast path
 * computes c in binary32 and re-computes in binary64 only the pairs that fall
 * inside a proven error band around an edge.
 *
 * Conventions for every call:
 *  - Return value: PC_OK (0) or a pc_status error code.  On error the
 *    outputs are left untouched and pc_last_error() describes the cause.
 *  - Ownership: the caller owns every buffer it passes in; the library never
 *    frees caller memory.  Catalogue handles own only library allocations.
 *  - Streams: `stream` is a hipStream_t (NULL = the null stream).  Device
 *    inputs must be ready on that stream; calls return when their host
 *    outputs are written.
 *  - Threads: calls are thread-safe; concurrent calls should use distinct
 *    streams.
 */
#ifndef PC_H
#define PC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum pc_status {
    PC_OK = 0,
    PC_ERR_INVALID = 1,   /* bad argument: NaN/Inf, |Dec| > 90, n < 0, bad edges, ... */
    PC_ERR_NOMEM = 2,     /* device or host allocation failed, or admission refused   */
    PC_ERR_DEVICE = 3,    /* HIP runtime error or no usable gfx950 device               */
    PC_ERR_BUSY = 4,      /* server queue full                                          */
    PC_ERR_CANCELLED = 5  /* job cancelled                                              */
};

enum pc_mode {
    PC_MIXED = 0,      /* binary32 chord^2 + binary64 re-check in the guard band (default) */
    PC_FP64_PLAIN = 1, /* binary64 chord^2 for every pair (baseline kernel)                */
    /* flag, or-ed into a mode: visit every pair even where a whole pair of
       tiles provably falls into one bin (same counts; for testing and timing) */
    PC_NO_PRUNE = 0x100,
    /* flag, or-ed into PC_MIXED: full tile pairs whose chords are all at least
       twice the smaller tile's radius get their binary32 chords from the
       matrix cores (the Gram form |a'|^2 + |b'|^2 - 2 a'.b' of tile-centred
       coordinates, with its own guard band); same counts.  Ignored with
       PC_FP64_PLAIN or PC_NO_PRUNE. */
    PC_MATRIX_CORES = 0x200,
    /* flag: use the launch parameters pc_autotune chose for a batch of this
       shape (device, edge count class, pair count class), if there is one;
       otherwise the defaults.  Same counts. */
    PC_TUNED = 0x400
};

/* A catalogue of n points: RA and Dec in degrees, binary64.  Paper Sec. 2.2
 * (input is a list of RA, Dec per galaxy).  RA: any finite value.  Dec: finite
 * and in [-90, 90].  on_device = 1: ra_deg/dec_deg are device pointers (e.g.
 * torch data_ptr() of float64 CUDA tensors); 0: host pointers. */
typedef struct {
    const double *ra_deg;
    const double *dec_deg;
    int64_t n;
    int32_t on_device;
    int32_t reserved;
} pc_catalog;

/*
 * pc_count -- pair counts of one catalogue (auto) or of two (cross).
 * Paper Sec. 2: DD/RR count the n(n-1)/2 pairs i<j of one catalogue; DR counts
 * all n_A*n_B pairs.  Sec. 2.1: histogram of separations over user edges.
 *
 *   A, B            catalogues; B is ignored (may be NULL) when auto_flag = 1.
 *   theta_edges_deg n_edges >= 2 host binary64 values, strictly increasing,
 *                   in [0, 180] degrees.
 *   auto_flag       1: unordered pairs of A; 0: all pairs of A x B.
 *   counts          host array of n_edges + 1 uint64, written on success:
 *                   counts[0]         pairs with theta <  edges[0] (underflow)
 *                   counts[k], 1<=k<n_edges: edges[k-1] <= theta < edges[k]
 *                   counts[n_edges]   pairs with theta >= edges[n_edges-1]
 *                   (theta compared through the binary64 squared chord).
 *                   The entries sum to n(n-1)/2 (auto) or n_A*n_B (cross).
 *   stream          hipStream_t or NULL.
 * n = 0 or 1 (auto) gives all-zero counts.  Mode PC_MIXED.
 * Limits (PC_ERR_INVALID beyond them): n_edges <= 1024; n <= 2^40 points per
 * catalogue; at most 2^40 - 1 tile pairs of 256 points in one call (one auto
 * job of up to ~3.8e8 points, or the sum over a batch's jobs).  Device memory:
 * about 100-130 bytes per point plus 16 bytes per tile pair; PC_ERR_NOMEM
 * when it is not available.  Returns PC_OK, PC_ERR_INVALID (bad argument; nothing
 * launched), PC_ERR_NOMEM or PC_ERR_DEVICE (pc_last_error() has the text).
 */
int pc_count(const pc_catalog *A, const pc_catalog *B, const double *theta_edges_deg,
             int32_t n_edges, int32_t auto_flag, uint64_t *counts, void *stream);

/*
 * pc_count_ex -- pc_count with an explicit mode and a row range.
 *   mode            PC_MIXED or PC_FP64_PLAIN (identical counts, different kernels).
 *   row_begin/end   count only pairs whose A-side index i is in [row_begin,
 *                   row_end) (auto: pairs i<j with i in range; cross: (i, j) for
 *                   all j).  row_end = -1 means n_A.  Rows outside [0, n_A] are
 *                   PC_ERR_INVALID.  Disjoint row ranges add up to the full count
 *                   (the paper's submatrix decomposition, Sec. 2.1).
 */
int pc_count_ex(const pc_catalog *A, const pc_catalog *B, const double *theta_edges_deg,
                int32_t n_edges, int32_t auto_flag, int32_t mode, int64_t row_begin,
                int64_t row_end, uint64_t *counts, void *stream);

/* One counting job inside a batch; fields as in pc_count_ex.  counts is a host
 * array of n_edges + 1 uint64 owned by the caller. */
typedef struct {
    const pc_catalog *A;
    const pc_catalog *B;
    const double *theta_edges_deg;
    int32_t n_edges;
    int32_t auto_flag;
    int64_t row_begin;
    int64_t row_end;
    uint64_t *counts;
} pc_job;

/*
 * pc_count_batch -- many counting jobs in one persistent kernel launch (the
 * paper's DD, DR and RR of one estimate; or many mock catalogues against a
 * shared random catalogue for Monte Carlo errors, Sec. 4).  Catalogues passed
 * with identical (ra_deg, dec_deg, n) pointers are converted once.  Jobs may use
 * different edge sets.  All jobs use `mode`.  Results are the same as running
 * each job alone.  n_jobs >= 1.
 */
int pc_count_batch(const pc_job *jobs, int32_t n_jobs, int32_t mode, void *stream);

/*
 * pc_count_batch_static -- pc_count_batch without any device allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * kernels and counts as pc_count_batch.  Every device buffer of the call --
 * converted and spatially ordered catalogue copies, sort scratch, survivor
 * lists, descriptors, edge-set tables, results -- is placed in one fixed
 * device array of PC_STATIC_SCRATCH_BYTES bytes that the library holds on each
 * GPU it has run this call on, from the first such call until the process
 * ends.  Host catalogues are copied into that array as well.
 *   Limit: a batch whose work area exceeds PC_STATIC_SCRATCH_BYTES returns
 *   PC_ERR_INVALID with the needed size in pc_last_error(), before anything
 *   is launched (roughly: about 200 bytes per point of every distinct
 *   catalogue plus 16 bytes per pair of 256-point tiles; e.g. DD, DR and RR
 *   of 2 x 300,000 points fit).
 *   Sharing: all calls on one GPU use that GPU's array, which keeps the last
 *   call's contents (each call clears what it needs cleared).  Calls from one
 *   process are serialised by a per-device lock; calls of different processes,
 *   or graph replays of a captured call, that overlap on one GPU race on the
 *   array and must be ordered by the caller.
 *   PC_TUNED is honoured; the counting kernel is not timed by HIP events here.
 */
#define PC_STATIC_SCRATCH_BYTES (256ull * 1024ull * 1024ull)
int pc_count_batch_static(const pc_job *jobs, int32_t n_jobs, int32_t mode, void *stream);

/*
 * pc_bin_edges -- theta edges from the paper's binning presets (Sec. 2.1: the
 * histogram's low and high limits and one of three preset bin widths),
 * host only; the counting calls take the edges it writes.
 *   preset      PC_BINS_EVEN (equal widths in theta), PC_BINS_LN (in ln theta)
 *               or PC_BINS_LOG10 (in log10 theta; the same edges as PC_BINS_LN
 *               for the same number of bins, up to rounding).
 *   lo_deg, hi_deg  0 <= lo < hi <= 180 degrees (lo > 0 for the log presets);
 *               the first and last edges are exactly lo and hi.
 *   n_bins      > 0: that many bins of equal width in the preset's scale;
 *               0: bins of `width` (in the preset's scale: degrees, natural
 *               log or decades), the last one narrower when the range is not a
 *               whole number of widths.
 *   edges       host array of max_edges doubles, written with the n_edges
 *               edges (may be NULL to ask only for *n_edges).
 *   n_edges     written: number of edges (bins + 1, at most 1024).
 * In the preset's scale F: edge k = F^-1(F(lo) + k w) in binary64 (libm),
 * k = 1 .. n-1.  PC_ERR_INVALID for bad limits, a bad preset or width, more
 * than 1023 bins, or a buffer that is too small.
 */
enum pc_bin_preset { PC_BINS_EVEN = 0, PC_BINS_LN = 1, PC_BINS_LOG10 = 2 };
int pc_bin_edges(int32_t preset, double lo_deg, double hi_deg, int32_t n_bins, double width, int32_t max_edges,
                 double *edges, int32_t *n_edges);

/*
 * pc_wtheta -- Landy-Szalay estimator (Eq. 2) from in-range bin counts.
 *   DD, DR, RR   host arrays of n_bins uint64 (pass counts + 1 of pc_count).
 *   nD, nR       catalogue sizes, each >= 2.
 *   w            host array of n_bins binary64, written:
 *                w[k] = ((dd - 2 dr) + rr) / rr with dd = DD[k]/(nD(nD-1)/2),
 *                dr = DR[k]/(nD nR), rr = RR[k]/(nR(nR-1)/2)  (binary64, this
 *                order, no fused multiply-add).  RR[k] = 0 gives the IEEE
 *                quotient: an infinity, or NaN when DD[k] and DR[k] are 0 too.
 * Host computation; no device needed.
 */
int pc_wtheta(const uint64_t *DD, const uint64_t *DR, const uint64_t *RR, int32_t n_bins,
              int64_t nD, int64_t nR, double *w);

/*
 * pc_estimator -- w(theta) by one of several estimators from in-range bin
 * counts.  Sec. 2 uses Landy-Szalay and notes that other estimators are easy
 * to try with the same counts; these are the usual ones, all on counts
 * normalised as in pc_wtheta (dd = DD/(nD(nD-1)/2), dr = DR/(nD nR),
 * rr = RR/(nR(nR-1)/2)), binary64, this operation order, no fused multiply-add:
 *   PC_EST_LANDY_SZALAY   ((dd - 2 dr) + rr) / rr      (same as pc_wtheta)
 *   PC_EST_NATURAL        dd / rr - 1                  (DR unused, may be NULL)
 *   PC_EST_DAVIS_PEEBLES  dd / dr - 1                  (RR unused, may be NULL)
 *   PC_EST_HAMILTON       (dd * rr) / (dr * dr) - 1
 * A zero denominator gives IEEE inf or NaN.  nD, nR >= 2; n_bins >= 1.
 * Host computation; no device needed.
 */
enum pc_estimator_kind {
    PC_EST_LANDY_SZALAY = 0,
    PC_EST_NATURAL = 1,
    PC_EST_DAVIS_PEEBLES = 2,
    PC_EST_HAMILTON = 3
};
int pc_estimator(int32_t kind, const uint64_t *DD, const uint64_t *DR, const uint64_t *RR, int32_t n_bins,
                 int64_t nD, int64_t nR, double *w);

/*
 * pc_autotune -- time the batch (as pc_count_batch would run it in `mode`)
 * under candidate launch configurations, check that every candidate gives the
 * same counts, and remember the fastest for batches of this shape (device,
 * ceil(log2(max n_edges)), floor(log2(pairs))); later calls with PC_TUNED use
 * it.  First the tile size -- the size of the submatrices the pair matrix is
 * cut into (Sec. 2.1): 128 or 256 points -- on the whole launch's time (each
 * size launched once untimed, then timed twice, its faster run kept); then,
 * at that size, histogram lane columns {4, 8, 16, 32}, work items taken from the
 * queue at a time {2, 4, 8} and matrix cores off/on (PC_MIXED with 256-point
 * tiles only) on the counting kernel's time.  Each job's counts are written
 * as pc_count_batch writes them.
 *   cache_path   NULL, or a file of tuned entries (one JSON object per line)
 *                that the result is added to (created if missing).
 *   result       NULL, or a host buffer of result_len bytes receiving a JSON
 *                object {"device", "edges_class", "pairs_class", "tile",
 *                "cols", "chunk", "matrix_cores", "kernel_ms", "launch_ms",
 *                "candidates"}.
 * Returns PC_ERR_DEVICE if two candidates disagree (a library fault).
 */
int pc_autotune(const pc_job *jobs, int32_t n_jobs, int32_t mode, const char *cache_path, void *stream,
                char *result, int32_t result_len);

/* pc_autotune_load -- add the tuned entries of a file written by pc_autotune
 * (for any device) to this process's table.  Host only. */
int pc_autotune_load(const char *cache_path);

/* Thread-local description of the last error on this thread ("" if none).
 * Valid until the next pc_* call on the same thread. */
const char *pc_last_error(void);

/* Library version string, e.g. "pc 0.1 gfx950". */
const char *pc_version(void);

/* ------------------------------------------------------------ residency */

/*
 * pc_catalog_upload -- convert a catalogue once (RA/Dec -> binary64 and
 * binary32 unit vectors in caller order and in a spatially ordered copy with
 * its tile bounds, about 112 bytes per point) and keep it resident on the
 * current device.  *handle receives a nonzero id.  Paper Sec. 2.1: positions
 * are copied to GPU global memory once and reused for every submatrix.
 */
int pc_catalog_upload(const pc_catalog *c, void *stream, uint64_t *handle);

/* Release a resident catalogue (waits for work on the device to finish). */
int pc_catalog_release(uint64_t handle);

/* pc_count_ex on resident catalogues (hB ignored when auto_flag = 1). */
int pc_count_h(uint64_t hA, uint64_t hB, const double *theta_edges_deg, int32_t n_edges,
               int32_t auto_flag, int32_t mode, int64_t row_begin, int64_t row_end,
               uint64_t *counts, void *stream);

/*
 * pc_unit_vectors -- the conversion step alone, for verification.
 *   c        catalogue (host or device).
 *   xyz64    host array of 3n binary64 (x, y, z per point), written;
 *   xyz32    host array of 3n binary32 (round-to-nearest of xyz64), written;
 *            either may be NULL.
 * x = cos(dec) cos(ra), y = cos(dec) sin(ra), z = sin(dec) (Appendix A
 * coordinates), computed on the device.
 */
int pc_unit_vectors(const pc_catalog *c, double *xyz64, float *xyz32, void *stream);

/* ------------------------------------------------------------- tables */

/*
 * pc_chord2_edges -- e[k] = 4 sin^2(theta_k/2) in binary64 (host), the squared
 * chord of each edge separation; n_edges values.  Appendix A separation
 * expressed through the chord.  No device needed.
 */
int pc_chord2_edges(const double *theta_edges_deg, int32_t n_edges, double *e);

/*
 * pc_guard_band -- the binary32 band around each squared-chord edge inside
 * which the mixed kernel re-checks a pair in binary64.  Host, no device.
 *   lo[k], hi[k]  written (n_edges floats): a binary32 chord^2 above hi[k]
 *                 proves the binary64 chord^2 is >= e[k]; one below lo[k]
 *                 proves it is < e[k].
 */
int pc_guard_band(const double *theta_edges_deg, int32_t n_edges, float *lo, float *hi);

/* ------------------------------------------------------------- serving */

/*
 * A w(theta) server: requests (a data catalogue on one of the caller's sky
 * patches, plus theta edges) are admitted while free device memory minus a
 * budget allows, their DD/DR/RR work is packed into persistent launches on
 * several streams so that new requests overlap running ones, random catalogues
 * are resident per patch and RR counts are cached per (patch, edges).
 *
 * pc_server_create: json_cfg (may be NULL) keys:
 *   "hbm_budget_bytes"  bytes of device memory to leave free (default 4 GiB)
 *   "max_inflight"      requests on the device at once (default 64)
 *   "streams"           number of streams (default 2)
 *   "max_batch_pairs"   pairs packed into one launch (default 2e12)
 *   "mode"              0 mixed, 1 fp64 plain
 *   "max_queue"         requests waiting at once (default 2^20)
 *   "deadline_s"        a request still waiting for admission this many
 *                       seconds after submission fails with PC_ERR_CANCELLED
 *                       (default 0: no deadline)
 *   "policy"            0 (default): first come, first served; 1: requests
 *                       waiting at least "aging_s" seconds (default 1) go
 *                       first, oldest first, then the others with the fewest
 *                       pairs first
 *   "log_path"          (a string) file to which one JSON line per finished
 *                       request is appended: id, patch, n, n_edges, pairs,
 *                       status, error, batch (-1 if it never ran), submit_s
 *                       (since the server started), latency_s.  Lines are
 *                       written after each launch and by pc_server_drain.
 * The environment variable PC_HBM_BUDGET_BYTES, if set, replaces the default
 * of "hbm_budget_bytes" (the key still wins).
 * Admission (policy 0) is first come, first served: requests enter in submission order
 * while max_inflight, the free device memory minus the budget and the bytes
 * held by running batches, and max_batch_pairs per launch allow.  A request
 * (or its next part) reserves the device work area its launch needs as the
 * batch runner plans it on the host -- converted and ordered copies, sort
 * scratch, 16 bytes per tile pair of survivor lists, results -- plus 1 MiB
 * for tables and descriptors.  A request that could not fit even on an empty
 * device fails with PC_ERR_NOMEM; a launch of several requests that still
 * runs out of device memory is retried one request per launch.
 *   "slice_pairs"       requests of more pairs than this (DD + DR + RR) run
 *                       as row-range parts of about this many pairs, one per
 *                       launch, between other requests (default 5e11; 0:
 *                       whole requests).  Counts add up exactly over the
 *                       parts (the paper's submatrices, Sec. 2.1).
 */
int pc_server_create(const char *json_cfg, void **server);

/* Register the random catalogue of sky patch `patch_id` (converted and kept
 * resident; copied, so the caller may free its arrays afterwards).  Replacing
 * a patch's catalogue drops its cached RR counts; launches already running
 * keep using the old copy, which is released when none runs; requests not yet
 * launched use the new one. */
int pc_server_set_random(void *server, int32_t patch_id, const pc_catalog *randoms);

/* Submit a request.  The data arrays are copied before return.  *job_id
 * receives the request id.  PC_ERR_BUSY when the queue is full. */
int pc_server_submit(void *server, const pc_catalog *data, int32_t patch_id,
                     const double *theta_edges_deg, int32_t n_edges, uint64_t *job_id);

/*
 * Poll a request.  *done = 1 when finished (then DD, DR, RR (n_edges+1 uint64
 * each, any may be NULL) and w (n_edges-1 binary64, may be NULL) are written and
 * the request is forgotten), 0 while queued or running, -1 if it failed (the
 * status is returned and the request forgotten).  latency_s (may be NULL)
 * receives submit-to-completion seconds.
 */
int pc_server_poll(void *server, uint64_t job_id, int32_t *done, uint64_t *DD, uint64_t *DR,
                   uint64_t *RR, double *w, double *latency_s);

/*
 * Cancel a request.  *cancelled = 1 when the request will report
 * PC_ERR_CANCELLED from pc_server_poll: a waiting request leaves the queue at
 * once; a running one finishes its launch and its answer is discarded.
 * *cancelled = 0 when it had already finished (its answer stays pollable).
 * PC_ERR_INVALID for an unknown (or already polled) id.
 */
int pc_server_cancel(void *server, uint64_t job_id, int32_t *cancelled);

/* Block until every submitted request has finished. */
int pc_server_drain(void *server);

/* Server statistics as a JSON string (thread-local buffer, valid until the
 * next call on this thread). */
const char *pc_server_stats(void *server);

/* Stop the server: requests still waiting for admission are dropped, running
 * launches finish, then the streams and resident catalogues are released.
 * Unpolled answers are lost. */
int pc_server_destroy(void *server);

#ifdef __cplusplus
}
#endif

#endif /* PC_H */
