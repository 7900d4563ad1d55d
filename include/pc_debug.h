/*
 * pc_debug.h -- verification hooks of libpc.so (host only, no device needed).
 *
 * They expose the host-built tables that the mixed-precision kernel uses to
 * place a binary32 squared chord into a bin, so that the table logic can be
 * checked on a CPU against the binary64 definition, facts about the last
 * launches, and the server's admission policy.
 */
#ifndef PC_DEBUG_H
#define PC_DEBUG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * pc_debug_lut32 -- the binary32 cell table of an edge set.
 *   theta_edges_deg, n_edges  as for pc_count.
 *   info      host int64[8], written: {n_cells, shift, clamp_lo_bits,
 *             clamp_hi_bits, row_bytes, cols, multi_band_cells, 0}.
 *   entries   host uint32[4 * max_cells] or NULL; written with n_cells entries
 *             {row offset if c <= hi, bits(lo), bits(hi), row offset if c > hi}
 *             when n_cells <= max_cells.
 * A binary32 chord c in [0, 4.0001] is looked up as: key = clamp(bits(c),
 * clamp_lo, clamp_hi); cell = (key >> shift) - (clamp_lo >> shift); bin row =
 * (c > hi ? off_hi : off_lo) / row_bytes; lo <= c <= hi means re-check.  A
 * finite hi implies off_hi = off_lo + row_bytes (the kernel relies on it).
 * Returns PC_OK or PC_ERR_INVALID (bad edges).
 */
int pc_debug_lut32(const double *theta_edges_deg, int32_t n_edges, int64_t *info,
                   uint32_t *entries, int64_t max_cells);

/*
 * pc_debug_guard_band_gram -- the per-edge guard band of the matrix-core path
 * (lo, hi: host arrays of n_edges floats, written), with the meaning of
 * pc_guard_band for binary32 chords formed by the matrix cores from
 * coordinates centred on the tile of smaller bounding radius r, in tile pairs
 * whose chords are all at least 2 r (a relative error bound).
 */
int pc_debug_guard_band_gram(const double *theta_edges_deg, int32_t n_edges, float *lo, float *hi);

/*
 * pc_debug_fused_band -- the thresholds of the vector few-edge paths (h, w:
 * host arrays of n_edges floats, written).  Those paths form d = h - c for
 * the smallest edge of a work item in one chain of binary32 roundings (gram !=
 * 0: tile-centred Gram chords; 0: differences of binary32 unit vectors), and
 * for its other edges d_t = RN32(d + RN32(h_t - h)) (at most three edges, so
 * the reference is at most two edges down); then d_t < 0 proves the binary64
 * chord is at or above edge t, d_t > w_t proves it below, and 0 <= d_t <= w_t
 * sends the pair to the binary64 re-check.  An edge at 0 gets h = -FLT_MAX,
 * w = 0.  Returns PC_OK or PC_ERR_INVALID (bad edges).
 */
int pc_debug_fused_band(const double *theta_edges_deg, int32_t n_edges, int32_t gram, float *h, float *w);

/*
 * pc_debug_set_timing -- on != 0: the calling thread's later counting calls
 * record HIP events around the counting kernel on the call's stream.
 */
int pc_debug_set_timing(int32_t on);

/*
 * pc_debug_set_flush_every -- items > 0: the calling thread's later counting
 * launches flush each wave's 32-bit LDS histogram into the 64-bit global
 * counts at least every `items` work items (normally only when a word could
 * otherwise wrap, about 10^6 items, at a change of job or edge set, and at the
 * end), so that tests reach the wrap-guard flush; 0 restores the default.
 * Counts are unchanged (Sec. 2.1: per-block histograms summed into global
 * memory).
 */
int pc_debug_set_flush_every(uint64_t items);

/*
 * pc_debug_set_compact_table -- the calling thread's later mixed-precision
 * counting launches (not the matrix-core one) hold the binary32 cell table in
 * its 8-byte form: mode 0 (default) when that lets more waves share a CU than
 * the 16-byte form, 1 whenever every table of the launch has it (row offsets
 * within 14 bits), -1 never.  Counts are unchanged (the same cells and
 * re-check decisions, Sec. 2.1 binning); PC_ERR_INVALID for another mode.
 */
int pc_debug_set_compact_table(int32_t mode);

/*
 * pc_debug_set_tile -- tile = 128 or 256: the calling thread's later counting
 * launches (except pc_autotune's own candidates) cut the pair matrix into
 * tiles of that many points whatever the tuner chose; 0 restores the default
 * (256, or the tuned size with PC_TUNED).  Counts do not depend on it.
 * PC_ERR_INVALID for other values.
 */
int pc_debug_set_tile(int32_t tile);

/*
 * pc_debug_fail_allocations -- the calling thread's next n device
 * allocations made by the library (workspaces, edge-set tables, resident
 * catalogues, aperture-map work space) fail as if the device were out of
 * memory: the call reports PC_ERR_NOMEM, leaves its outputs untouched and
 * keeps nothing it had allocated.  n = 0 turns it off.  PC_ERR_INVALID for
 * n < 0.  For testing failure handling.
 */
int pc_debug_fail_allocations(int32_t n);

/*
 * pc_debug_last_launch -- facts about the calling thread's last counting
 * launch: kernel time in ms from the HIP events (-1 if timing was off),
 * number of tile-pair work items, grid size (single-wave workgroups) and LDS
 * bytes per workgroup.  Any pointer may be NULL.
 */
int pc_debug_last_launch(double *kernel_ms, uint64_t *items, int32_t *grid, uint32_t *lds_bytes);

/*
 * pc_debug_last_pruning -- the calling thread's last counting launch: work
 * items (tile pairs) left for the pair kernel after whole-tile-pair binning,
 * pairs visited one by one, all pairs counted, and how many of the left items
 * went through the matrix cores.  A left item of the mixed mode may be split:
 * the j-tile's four sub-blocks of 64 points are looked at one by one, some
 * binned whole, the others visited with their own edges (split_items counts
 * those items).  few_items counts the work units (items, or open sub-blocks
 * of split items) with at most 3 edges inside their chord interval (binned by
 * comparing with those edges alone), gram_items those whose vector-path
 * chords are formed in tile-centred Gram form.  Any pointer may be NULL.
 */
int pc_debug_last_pruning(uint64_t *survivors, uint64_t *pairs_computed, uint64_t *pairs_total,
                          uint64_t *mfma_items, uint64_t *few_items, uint64_t *gram_items,
                          uint64_t *split_items);

/*
 * pc_debug_last_paths -- the calling thread's last counting launch: how the
 * pairs visited one by one were binned, as the prune pass assigned them.
 *   pairs_by_edges  host uint64[4] or NULL, written: [m] for m = 1..3 the pairs
 *                   binned by comparing with the m edges inside their tile
 *                   pair's (or sub-block's) chord interval; [0] the pairs
 *                   binned through the cell table (every computed pair of the
 *                   binary64 kernel and of launches with PC_NO_PRUNE).
 *   gram_pairs      of the few-edge pairs, those whose chords the vector path
 *                   forms in tile-centred Gram form (NULL allowed).
 *   mfma_pairs      pairs whose chords came from the matrix cores (NULL allowed).
 * Sec. 2.1 (binning) is the operation; these figures let a reader count the
 * comparisons a pair needs on its path.
 */
int pc_debug_last_paths(uint64_t *pairs_by_edges, uint64_t *gram_pairs, uint64_t *mfma_pairs);

/*
 * pc_debug_last_rechecks -- the calling thread's last counting launch: how many
 * pairs had a binary32 squared chord inside the guard band of an edge and were
 * recomputed in binary64 (Appendix A separation; the mixed kernel only: the
 * binary64 kernel and whole-binned tile pairs report none).  Counted on the
 * device in a histogram row of its own.  PC_ERR_INVALID for NULL.
 */
int pc_debug_last_rechecks(uint64_t *pairs_rechecked);

/*
 * pc_debug_request_parts -- how the w(theta) server would run one request,
 * host only: the request (n_points data points, a patch of n_random randoms,
 * n_edges log-spaced edges, RR counted by it when count_rr != 0) is cut into
 * parts of about slice_pairs pairs (the "slice_pairs" key; 0: one part), each
 * a launch over data rows [a, b) (DD and DR) and random rows [c, d) (RR);
 * counts over disjoint row ranges add up exactly (Sec. 2.1 submatrices).
 *   rows        host int64[4 * max_parts], written: {a, b, c, d} per part.
 *   need_bytes  host uint64[max_parts], written: device bytes each part's
 *               launch needs, as the server's admission reserves them (planned
 *               by the batch runner without a device).
 *   n_parts     written: the number of parts (may exceed max_parts; only the
 *               first max_parts are described).
 */
int pc_debug_request_parts(int64_t n_points, int64_t n_random, int32_t n_edges, int32_t count_rr,
                           double slice_pairs, int32_t max_parts, int64_t *rows, uint64_t *need_bytes,
                           int32_t *n_parts);

/*
 * pc_debug_server_hold -- hold != 0: the server's workers keep each batch they
 * admit (its requests hold their device slots and bytes) from launching until
 * the hold is released (hold = 0); other requests keep waiting or expire as
 * usual.  Makes queueing tests independent of kernel durations.
 * PC_ERR_INVALID for a NULL server.
 */
int pc_debug_server_hold(void *server, int32_t hold);

/*
 * pc_debug_admission_plan -- the w(theta) server's admission policy applied to
 * a queue described by the caller, with no device involved (the server applies
 * the same function to its own queue and to the free and total device memory
 * it reads).
 *   need_bytes, pairs, age_s   host arrays of n: device bytes each queued
 *                  request needs, the pairs it counts, seconds since it was
 *                  submitted; index 0 is the front of the queue.
 *   free_bytes, total_bytes    device memory figures to decide with.
 *   reserved_bytes bytes held by batches already running.
 *   inflight       requests already on the device.
 *   json_cfg       server configuration as for pc_server_create (may be NULL).
 *   outcome        host int32[n] (in queue order), written: 0 admitted into the next batch,
 *                  1 fails (can never fit: PC_ERR_NOMEM), 2 fails (queueing
 *                  deadline passed: PC_ERR_CANCELLED), 3 keeps waiting.
 * Returns PC_OK, or PC_ERR_INVALID (NULL arrays with n > 0, n < 0, bad config).
 */
int pc_debug_admission_plan(const uint64_t *need_bytes, const double *pairs, const double *age_s, int32_t n,
                            uint64_t free_bytes, uint64_t total_bytes, uint64_t reserved_bytes,
                            int32_t inflight, const char *json_cfg, int32_t *outcome);

#ifdef __cplusplus
}
#endif

#endif /* PC_DEBUG_H */
