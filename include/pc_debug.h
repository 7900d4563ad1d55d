/*
 * pc_debug.h -- verification hooks of libpc.so (host only, no device needed).
 *
 * They expose the host-built tables that the mixed-precision kernel uses to
 * place a binary32 squared chord into a bin, so that the table logic can be
 * checked on a CPU against the binary64 definition.
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
 *             {row offset if c <= hi, row offset if c > hi, bits(lo), bits(hi)}
 *             when n_cells <= max_cells.
 * A binary32 chord c in [0, 4.0001] is looked up as: key = clamp(bits(c),
 * clamp_lo, clamp_hi); cell = (key >> shift) - (clamp_lo >> shift); bin row =
 * (c > hi ? off_hi : off_lo) / row_bytes; lo <= c <= hi means re-check.
 * Returns PC_OK or PC_ERR_INVALID (bad edges).
 */
int pc_debug_lut32(const double *theta_edges_deg, int32_t n_edges, int64_t *info,
                   uint32_t *entries, int64_t max_cells);

/*
 * pc_debug_set_timing -- on != 0: the calling thread's later counting calls
 * record HIP events around the counting kernel on the call's stream.
 */
int pc_debug_set_timing(int32_t on);

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
 * pairs visited one by one, and all pairs counted.  Any pointer may be NULL.
 */
int pc_debug_last_pruning(uint64_t *survivors, uint64_t *pairs_computed, uint64_t *pairs_total);

#ifdef __cplusplus
}
#endif

#endif /* PC_DEBUG_H */
