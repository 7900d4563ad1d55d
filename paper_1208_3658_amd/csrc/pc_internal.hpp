// pc_internal.hpp -- descriptors shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace pc {

// The counting path is compiled for two tile sizes: 256 points (4 i-points
// per lane, namespace pc::t256) and 128 points (2 per lane, pc::t128); the
// launch picks one at run time (a tuned launch parameter).  A translation
// unit sees one of them through PC_R.
#ifndef PC_R
#define PC_R 4              // i-points held per lane
#endif
#if PC_R == 4
#define PC_TILE_NS t256
#elif PC_R == 2
#define PC_TILE_NS t128
#else
#error "PC_R must be 2 or 4"
#endif
#ifndef PC_COLS32
#define PC_COLS32 16        // widest histogram of the mixed kernel (lane columns)
#endif
#ifndef PC_COLS64
#define PC_COLS64 16        // widest histogram of the binary64 kernel
#endif

constexpr int kWave = 64;                 // gfx950 wavefront
constexpr int kR = PC_R;                  // i-points held per lane
constexpr int kTile = kWave * kR;         // points per tile, both axes (square tiles)
constexpr int kMaxEdges = 1024;       // theta edges per table
// The prune pass's statistics (12 words) are added into kPruneStripes copies
// of kPruneStripeWords words at word kPruneStatBase of the launch's results
// block, a copy per group of workgroups; the host adds the copies up.  Its
// whole-tile-pair counts go to kPruneStripes copies of the jobs' counters in
// the same way, which one small kernel adds into the counters.  Device-wide
// atomics on one address serialise, and every workgroup has some to add.
constexpr int kPruneStats = 12;
constexpr int kPruneStripes = 16;
constexpr int kPruneStripeWords = 16;
constexpr int kPruneStatBase = 32;
// The counting kernel's work queue: eight counters (one per XCD slice), each
// in its own cache line, after the prune statistics.
constexpr int kQueueStride = 16;
constexpr int kQueueBase = kPruneStatBase + kPruneStripes * kPruneStripeWords;
constexpr int kJPad = 16;               // readable points past the end of an ordered binary32 copy
constexpr int kMaxLutCells = 1024;        // per table, 16 bytes each
constexpr uint32_t kLdsTarget = 16 * 1024;  // per-wave histogram bytes aimed for at most

// Histogram layout in LDS: n_edges + 3 rows (under/overflow bins, one
// discard row for masked pairs, and one row tallying the pairs re-checked in
// binary64) of `cols` lane columns.  Lane l adds to column
// l & (cols - 1); a row is exactly `cols` words, so the columns of one add sit
// in distinct banks whatever their rows, and only the 64 / cols lanes that
// share a column meet on a word (with cols = 64, none).
inline uint32_t row_bytes_for(int cols) { return static_cast<uint32_t>(cols) * 4u; }

// Cell lookup entry of the mixed (binary32) kernel.  For a squared chord c in
// the cell: row offset off_lo, plus one row when c > hi; lo <= c <= hi ->
// re-check in binary64.  Offsets are byte offsets of histogram rows.  A
// finite hi only occurs in a cell that one band meets (the next row is then
// that band's edge's).  wbits = the bits of RN32(hi - lo) in a one-band cell
// (a chord in the band has 0 <= RN32(hi - c) <= RN32(hi - lo)), 0 in a cell
// without a band (lo = hi = +inf: RN32(hi - c) = +inf is never in), all ones
// in a cell that several bands meet (lo = -inf, hi = +inf: always re-checked).
struct LutEntry32 {
    uint32_t off_lo;
    float lo, hi;
    uint32_t wbits;
};

// The same cell in 8 bytes, for launches whose LDS would otherwise limit
// the waves per CU: bits(hi), and wc = wbits rounded up to a multiple of
// kCtOffMask + 1 (all ones stay all ones) with off_lo in the low bits.  wc >=
// wbits, so the flag test against it takes every chord the full entry's
// does; the kernel re-checks every flagged chord (provisional row off_lo), so
// lo is not needed.  Only built when every off_lo is at most kCtOffMask.
constexpr uint32_t kCtOffMask = 0x3FFFu;
struct LutEntryC {
    uint32_t hi_bits, wc;
};

// Cell lookup entry of the binary64 kernel: c >= e -> off_hi, else off_lo.
struct LutEntry64 {
    uint32_t off_lo, off_hi;
    double e;
};

// One edge set as the kernels see it.
struct TableDesc {
    const void *lut;        // LutEntry32[] (mixed) or LutEntry64[] (fp64); device
    const void *lutc;       // LutEntryC[] (mixed, when built) or null; device
    const double *e64;      // n_edges binary64 squared-chord edges; device
    uint32_t clamp_lo;      // cell key clamp (binary32 bits, or high word of binary64)
    uint32_t clamp_hi;
    uint32_t shift;         // cell = clamped key >> shift
    uint32_t key0;          // first cell = clamp_lo >> shift
    int32_t n_cells;
    int32_t n_edges;
    int32_t search;         // fp64 only: 1 = no exact cell table, binary search per pair
    int32_t cols;           // histogram lane columns (power of two <= 64)
    // guard bands as (lo, hi) binary32 pairs per edge, plain (kept for
    // inspection; the cell tables hold its values and no kernel reads it) and
    // matrix-core, and the vector few-edge paths' fused (h, W) pairs, plain
    // and Gram (mixed only; device)
    const float *band, *band_g, *fband, *fband_g;
};

// A survivor work item (one tile pair left after whole-tile-pair binning), as
// the prune pass writes it for the counting kernel:
//   bits  0..39  item number within the launch
//   bits 40..50  k0: edges at or below the item's whole chord interval
//   bits 51..52  m: edges inside the interval when at most kFewMax, else 0
//   bit  53      split: the j-tile is visited as kSubs blocks of kSub points,
//                each described by 16 bits of the item's sub-block word
//   bit  61      vector path, chords in Gram form centred on the j-tile
//   bit  62      matrix-core path centred on the j-tile
//   bit  63      matrix-core path
constexpr int kItemBits = 40;
constexpr int kFewMax = 3;  // at most 3: m has two bits
#ifndef PC_FEWCUT
#define PC_FEWCUT 3         // items with at most this many edges use few-edge binning (<= kFewMax)
#endif
constexpr uint64_t kItemMask = (1ull << kItemBits) - 1;
constexpr int kSplitBit = 53;

// Sub-blocks of a split item.  A full, off-diagonal tile pair that the prune
// pass cannot bin whole is looked at again as kSubs pairs (i-tile, 64 points
// of the j-tile), each with its own chord interval: some of them fall in one
// bin and are binned whole, the others often meet fewer edges than the whole
// tile pair.  Sub-block s of an item is described by bits 16s..16s+15 of the
// item's sub-block word:
//   bits  0..10  k0: edges at or below its chord interval (its bin if whole)
//   bits 11..12  m: edges inside when at most PC_FEWCUT, else 0 (cell table)
//   bit  13      binned whole by the prune pass (the kernel skips it)
//   bit  14      vector path with Gram-form chords centred on the j-tile
constexpr int kSub = 64;
constexpr int kSubs = kTile / kSub;
static_assert(kSubs >= 1 && kSubs <= 4, "at most four 16-bit sub-block fields per 64-bit word");
constexpr uint32_t kSubWhole = 1u << 13;
constexpr uint32_t kSubGram = 1u << 14;

// A binary32 cell table (see pc_tables.cpp).
struct Lut32 {
    uint32_t clamp_lo = 0, clamp_hi = 0, shift = 0;
    std::vector<LutEntry32> entries;
    std::vector<LutEntryC> compact;  // the same cells, 8 bytes each; empty when off_lo does not fit
    int multi = 0;  // cells that always re-check (bands closer than the cell width)
};

// A block of tile pairs of one job: a triangle (unordered pairs i<j inside
// one index range of one catalogue) or a rectangle (all pairs of two ranges).
struct SegDesc {
    uint64_t item0;         // first global work item of the segment
    uint64_t n_items;
    const float4 *i32, *j32;          // spatially ordered binary32 points
    const double4 *i64, *j64;         // the same points in binary64
    const double4 *ib, *jb;           // tile bounds (centre, radius) of each side
    const float4 *jg;                 // j side in Gram form, centred on its own tile
                                      // (-2 b'_x, -2 b'_y, -2 b'_z, |b'|^2)
    const double4 *jb_sub;            // bounds of the j side's sub-blocks, kSubs per tile
    int64_t i0, ni, j0, nj;
    int64_t tiles_i, tiles_j;
    int64_t prow0;          // first row of the segment in the prune pass's row space
    int32_t tri, tab, job, pad;
    unsigned long long *counts;  // the job's n_edges+1 device counters
    // the prune pass's copies of the job's counters: copy c at pcounts + c *
    // pstride, c < kPruneStripes (added into counts after the pass)
    unsigned long long *pcounts;
    int64_t pstride;
};

// Host-side form of an edge set.
struct HostTable {
    // histogram columns and row size of each kernel's layout (the cell tables
    // hold byte offsets of rows, so each kernel has its own)
    int cols32 = 32, cols64 = 16;
    uint32_t row_bytes32 = 128, row_bytes64 = 64;
    std::vector<double> theta;
    std::vector<double> e64;
    std::vector<float> lo, hi;
    // mixed kernel: direct chords (binary32 unit vectors) and tile-centred
    // chords formed by the matrix cores, each with its own guard band
    std::vector<float> lo_g, hi_g;
    // vector few-edge paths: thresholds h and flag widths W of the fused
    // differences d = h - c (fused_bands), direct and tile-centred chords
    std::vector<float> fh, fw, fh_g, fw_g;
    Lut32 lut32;
    // fp64 kernel
    uint32_t clamp_lo64 = 0, clamp_hi64 = 0, shift64 = 0;
    std::vector<LutEntry64> lut64;
    bool search64 = false;
};

// Checks theta edges: 2..1024 values, finite, in [0, 180], strictly increasing.
bool validate_edges(const double *theta_deg, int n_edges, std::string &err);

// Validates theta edges; fills e64, the guard bands and both cell tables.
// cols32 > 0 fixes the mixed kernel's histogram lane columns (a power of two
// in [4, 64]); 0 picks the widest up to PC_COLS32 whose histogram and cell
// table fit the LDS target together.
bool build_table(const double *theta_deg, int n_edges, HostTable &t, std::string &err, int cols32 = 0);

// The guard band of one squared-chord edge e (binary64): binary32 lo, hi with
//   c32 > hi  =>  c64 >= e,     c32 < lo  =>  c64 < e.
void guard_band(double e, float *lo, float *hi);

// The same for chords formed from tile-centred binary32 coordinates by the
// matrix cores (coordinates centred on the tile of smaller bounding radius r,
// every pair of the tile pair at chord >= 2 r).
void guard_band_gram(double e, float *lo, float *hi);

// Thresholds h and flag widths W of the vector few-edge paths, which form d =
// h - c for the item's smallest edge in one chain of roundings and the other
// edges' d from it (gram: tile-centred Gram chords, else differences of
// binary32 unit vectors): d < 0 => c64 >= e; d > W => c64 < e; an edge at 0
// gets h = -FLT_MAX, W = 0.
void fused_bands(const std::vector<double> &e64, bool gram, std::vector<float> &h, std::vector<float> &w);

}  // namespace pc
