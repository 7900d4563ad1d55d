// pc_kernels.hip -- gfx950 kernels for exact angular pair counting.
//
// Work decomposition (paper Sec. 2.1 splits the n x n pair matrix into
// submatrices, one launch each; here one persistent launch covers every
// submatrix of every job):
//   * a tile is kTile = 256 consecutive points; a work item is one pair of
//     tiles (I, J), all 256 x 256 pairs, processed by one wavefront;
//   * the i-tile sits in registers (4 points per lane, lanes on consecutive
//     points), the j-tile is streamed one point at a time through scalar
//     loads (the same j for the whole wave), so each lane forms 4 pairs per j;
//   * auto pairs use only tile pairs I <= J (triangle), and on the diagonal
//     tile only i < j: every unordered pair exactly once, no self-pairs
//     (Sec. 2, n(n-1)/2 pairs); cross pairs use every tile pair (n_A n_B);
//   * each workgroup is a single wave that owns its LDS: a private cell
//     table for the current edge set (16-byte entries, or 8-byte ones when
//     that lets more waves share a CU) and a histogram of `cols` lane columns
//     (4 to 32: only the 64 / cols lanes of one wave that share a column can
//     meet on a word, never lanes of other waves, so the paper's same-bin
//     atomic contention across threads, Sec. 2.1, is bounded), flushed into
//     64-bit global counters when the job changes and at the end; the
//     few-edge paths count in registers and touch LDS once per item.
#include "pc_internal.hpp"
#include "pc_math.h"

namespace pc {

#if PC_R == 4
// ------------------- tile-independent part (compiled once, 256-point build)

// -------------------------------------------------------------- conversion

// RA/Dec (degrees, binary64) -> unit vectors: binary64 (x, y, z, 0) and its
// round-to-nearest binary32 copy.  Invalid inputs (non-finite, |Dec| > 90) set
// *err and produce the vector of (0, 0).
__global__ void __launch_bounds__(256) k_convert(const double *__restrict__ ra,
                                                 const double *__restrict__ dec, int64_t n,
                                                 double4 *__restrict__ a64,
                                                 float4 *__restrict__ a32,
                                                 int *__restrict__ err) {
#pragma clang fp contract(off)
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double r = ra[i], d = dec[i];
    const bool ok = isfinite(r) && isfinite(d) && d >= -90.0 && d <= 90.0;
    if (!ok) {
        atomicOr(err, 1);
        r = 0.0;
        d = 0.0;
    }
    double sa, ca, sd, cd;
    sincosd(r, &sa, &ca);
    sincosd(d, &sd, &cd);
    const double x = cd * ca;
    const double y = cd * sa;
    const double z = sd;
    a64[i] = make_double4(x, y, z, 0.0);
    if (a32) a32[i] = make_float4(static_cast<float>(x), static_cast<float>(y), static_cast<float>(z), 0.0f);
}

__global__ void __launch_bounds__(256) k_zero_u64(unsigned long long *p, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// ---------------------------------------------------------------- launchers

hipError_t launch_convert(const double *ra, const double *dec, int64_t n, double4 *a64, float4 *a32,
                          int *err, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    k_convert<<<dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, st>>>(ra, dec, n, a64, a32, err);
    return hipGetLastError();
}

hipError_t launch_zero(unsigned long long *p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    k_zero_u64<<<dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, st>>>(p, n);
    return hipGetLastError();
}

#endif  // tile-independent part

// ------------------------------------------------ per tile size

namespace PC_TILE_NS {

struct KParams {
    const SegDesc *segs;
    const TableDesc *tabs;
    const uint64_t *items;                 // work items to visit (survivors), or null: all items
    const unsigned long long *n_items;     // device count of `items`
    const uint64_t *sub;                   // sub-block words beside `items` (split items), or null
    uint64_t total_items;                  // number of items when `items` is null
    int32_t n_segs;
    uint32_t lut_lds_off;   // byte offset of the cell table in LDS (after the histogram)
    uint32_t stage_lds_off; // byte offset of the matrix-core path's A-operand block (16 x 64 floats)
    unsigned long long *queue;  // 8 zeroed chunk counters kQueueStride words apart, one per slice of the items
    unsigned long long *rechecked;  // zeroed; pairs re-checked in binary64 are added here
    uint32_t chunk;             // items taken from the queue at a time
    uint64_t flush_cap;         // > 0: flush the histogram at least every flush_cap items (testing)
};

#ifndef PC_SPLIT
#define PC_SPLIT 1  // split items (sub-blocks of the j-tile) from the prune pass
#endif
#ifndef PC_EARLY_GRAM
#define PC_EARLY_GRAM 0  // 1: Gram-form items load their binary64 i-points first too (more registers)
#endif

// ------------------------------------------------------------ helpers

// Loads through the constant address space: the addresses below are the
// same for every lane, so these become scalar loads (the data is read-only
// for the whole launch).
__device__ __forceinline__ float4 ld_const(const float4 *p) {
    using CF = const __attribute__((address_space(4))) float;
    CF *q = (CF *)(p);
    return make_float4(q[0], q[1], q[2], q[3]);
}

__device__ __forceinline__ float2 ld_const_f2(const float *p) {
    using CF = const __attribute__((address_space(4))) float;
    CF *q = (CF *)(p);
    return make_float2(q[0], q[1]);
}

__device__ __forceinline__ double4 ld_const(const double4 *p) {
    using CD = const __attribute__((address_space(4))) double;
    CD *q = (CD *)(p);
    return make_double4(q[0], q[1], q[2], q[3]);
}

__device__ __forceinline__ uint64_t ld_const(const uint64_t *p) {
    using CU = const __attribute__((address_space(4))) unsigned long long;
    return static_cast<uint64_t>(*(CU *)(p));
}

// A descriptor read through the constant address space (scalar loads), so
// its fields live in scalar registers.
template <typename T>
__device__ __forceinline__ T ld_const_struct(const T *p) {
    static_assert(sizeof(T) % 4 == 0, "descriptor size");
    using CU = const __attribute__((address_space(4))) uint32_t;
    CU *q = (CU *)(p);
    T out;
    uint32_t *o = reinterpret_cast<uint32_t *>(&out);
#pragma unroll
    for (int i = 0; i < static_cast<int>(sizeof(T) / 4); ++i) o[i] = q[i];
    return out;
}

__device__ __forceinline__ double chord2_64(double ax, double ay, double az, double bx, double by,
                                            double bz) {
#pragma clang fp contract(off)
    const double dx = ax - bx;
    const double dy = ay - by;
    const double dz = az - bz;
    double c = dx * dx;
    c = c + dy * dy;
    c = c + dz * dz;
    return c;
}

// number of edges <= c
template <typename P>
__device__ __forceinline__ uint32_t bin_search(P e, int32_t n, double c) {
    int32_t lo = 0, hi = n;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (e[mid] <= c) lo = mid + 1;
        else hi = mid;
    }
    return static_cast<uint32_t>(lo);
}

// LDS accessed by absolute byte address (address space 3), so that no base
// register has to be added per access.
using lds_u32 = __attribute__((address_space(3))) uint32_t;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
using lds_u4 = __attribute__((address_space(3))) const u32x4;

__device__ __forceinline__ uint32_t lds_addr(const unsigned char *p) {
    return static_cast<uint32_t>(reinterpret_cast<uintptr_t>(
        (__attribute__((address_space(3))) const unsigned char *)(p)));
}

__device__ __forceinline__ void lds_add(unsigned char *, uint32_t addr, uint32_t v) {
    __hip_atomic_fetch_add((lds_u32 *)(uintptr_t)(addr), v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}

typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));
using lds_u3 = __attribute__((address_space(3))) const u32x3;

// first 12 bytes of a 16-byte aligned cell entry: (off_lo, bits(lo), bits(hi))
__device__ __forceinline__ uint3 lds_read3(uint32_t addr) {
    const u32x3 v = *(lds_u3 *)(uintptr_t)(addr);
    return make_uint3(v.x, v.y, v.z);
}

__device__ __forceinline__ uint4 lds_read4(uint32_t addr) {
    const u32x4 v = *(lds_u4 *)(uintptr_t)(addr);
    return make_uint4(v.x, v.y, v.z, v.w);
}

// max(a - b, 0) for unsigned a, b: one subtract with its clamp bit.
__device__ __forceinline__ uint32_t sub_sat(uint32_t a, uint32_t b) {
    uint32_t r;
    asm("v_sub_u32_e64 %0, %1, %2 clamp" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

__device__ __forceinline__ uint32_t umed3(uint32_t x, uint32_t lo, uint32_t hi) {
    return min(max(x, lo), hi);
}

// Sum the histogram rows [0, n_rows) over the lane columns into the job's
// 64-bit counters and the re-check tally row (row n_rows + 1, after the
// discard row) into *rechecked, then clear every row.  Lane r sums row r,
// visiting the columns in a lane-rotated order so that the lanes of one read
// touch distinct banks.
__device__ void flush_hist(unsigned char *lds, int32_t n_rows, int32_t cols, int32_t clear_words,
                           unsigned long long *counts, unsigned long long *rechecked) {
    __syncthreads();
    const uint32_t lane = threadIdx.x;
    uint32_t *h = reinterpret_cast<uint32_t *>(lds);
    for (int32_t r = lane; r < n_rows; r += kWave) {
        unsigned long long s = 0;
        const uint32_t *row = h + r * cols;
        for (int c = 0; c < cols; ++c) s += row[(c + r) & (cols - 1)];
        if (s) atomicAdd(counts + r, s);
    }
    if (lane == kWave - 1) {
        unsigned long long s = 0;
        const uint32_t *row = h + (n_rows + 1) * cols;
        for (int c = 0; c < cols; ++c) s += row[c];
        if (s) atomicAdd(rechecked, s);
    }
    __syncthreads();
    for (int32_t w = lane; w < clear_words; w += kWave) h[w] = 0u;
    __syncthreads();
}

__device__ __forceinline__ void map_item(const SegDesc &sd, uint64_t q, int64_t &t, int64_t &u) {
    if (sd.tri) {
        // fold the triangle {t <= u < T} into a (ceil(T/2)) x (T+1) rectangle:
        // row r holds (r, r..T-1) followed by (T-1-r, T-1-r..T-1)
        const int64_t T = sd.tiles_i;
        const int64_t r = static_cast<int64_t>(q / static_cast<uint64_t>(T + 1));
        const int64_t c = static_cast<int64_t>(q % static_cast<uint64_t>(T + 1));
        if (c < T - r) {
            t = r;
            u = r + c;
        } else {
            t = T - 1 - r;
            u = t + (c - (T - r));
        }
    } else {
        t = static_cast<int64_t>(q / static_cast<uint64_t>(sd.tiles_j));
        u = static_cast<int64_t>(q % static_cast<uint64_t>(sd.tiles_j));
    }
}

__device__ __forceinline__ int find_seg(const SegDesc *segs, int n, uint64_t item) {
    int lo = 0, hi = n - 1;  // last segment with item0 <= item
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].item0 <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ------------------------------------------------------- mixed precision

__device__ __forceinline__ uint32_t uniform(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// A wave-uniform binary32 value kept in a scalar register (the band limits
// of the few-edge compares: without this the compiler may not prove them
// uniform and keeps them in vector registers, which then spill).
__device__ __forceinline__ float uniform_f(float x) { return __uint_as_float(uniform(__float_as_uint(x))); }

__device__ __forceinline__ uint64_t uniform_u64(uint64_t x) {
    return static_cast<uint64_t>(uniform(static_cast<uint32_t>(x))) |
           (static_cast<uint64_t>(uniform(static_cast<uint32_t>(x >> 32))) << 32);
}

template <typename T>
__device__ __forceinline__ const T *uniform_ptr(const T *p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint64_t lo = uniform(static_cast<uint32_t>(v));
    const uint64_t hi = uniform(static_cast<uint32_t>(v >> 32));
    return reinterpret_cast<const T *>(lo | (hi << 32));
}

// LDS byte address of the cell-table entry for key: ((key >> shift) << 4) +
// base, or << 3 for the compact 8-byte entries
template <int ES = 4>
__device__ __forceinline__ uint32_t cell_addr(uint32_t key, uint32_t shift, uint32_t base) {
    uint32_t r;
    asm("v_lshl_add_u32 %0, %1, %3, %2" : "=v"(r) : "v"(key >> shift), "v"(base), "i"(ES));
    return r;
}

__device__ __forceinline__ uint2 lds_read2(uint32_t addr) {
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    const u32x2 v = *(__attribute__((address_space(3))) const u32x2 *)(uintptr_t)(addr);
    return make_uint2(v.x, v.y);
}

// Cell key of a binary32 squared chord: its bits, clamped to the table range
// (c >= 0, so float order and bit order agree).
__device__ __forceinline__ uint32_t key32(float c2, float lo, float hi) {
    return __float_as_uint(__builtin_amdgcn_fmed3f(c2, lo, hi));
}

__device__ __forceinline__ float chord2_32(float ax, float ay, float az, float4 b) {
    const float dx = ax - b.x;
    const float dy = ay - b.y;
    const float dz = az - b.z;
    return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}

struct TileCtx {
    uint32_t shift, lut_base, lane_off, trash_off, row_bytes, row_shift;
    float klo, khi;  // key clamp as floats
    int32_t n_edges;
    const double *e64;
};

#ifndef PC_JUNROLL
#define PC_JUNROLL 2        // j-points per inner iteration
#endif

// The j-points of one step (wave-uniform, scalar loads), issued a step ahead
// of their use.  The ordered binary32 copies are allocated kJPad points
// longer than the catalogue, so a read-ahead past the last j-point of the
// last tile stays inside the allocation (its values are not used).
template <int NJ>
__device__ __forceinline__ void load_j(const float4 *__restrict__ J, float4 (&b)[NJ]) {
    static_assert(NJ <= kJPad, "read-ahead beyond the padding");
#pragma unroll
    for (int q = 0; q < NJ; ++q) b[q] = ld_const(J + q);
}

// NJ consecutive j-points against the lane's kR i-points: all chords first,
// then all cell-table reads, then all histogram adds, so the LDS latency of
// NJ * kR lookups overlaps.  Slot r of lane l holds i = ibeg + r*64 + l.
//
// CT: the compact cell table, 8 bytes per entry (bits(hi), wc), wc = the
// width bits rounded up to a multiple of kCtOffMask + 1 with off_lo in its low
// bits: the flag test against wc is a superset of the one against the width
// bits, and the re-check takes every flagged chord (its provisional row is
// off_lo), so no lo is needed.
template <bool MASKED, int NJ, bool CT = false>
__device__ __forceinline__ void step32(unsigned char *lds, const float4 (&b)[NJ],
                                       const double4 *__restrict__ J64t, int32_t jj,
                                       const float (&ax)[kR], const float (&ay)[kR],
                                       const float (&az)[kR], const double4 *__restrict__ I64,
                                       int64_t ibeg, int32_t i_lim, int32_t j_rel, bool diag,
                                       const TileCtx &k) {
    const int32_t lane = static_cast<int32_t>(threadIdx.x);
    float c2[NJ][kR];
    uint32_t a[NJ][kR];
#pragma unroll
    for (int q = 0; q < NJ; ++q)
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            c2[q][r] = chord2_32(ax[r], ay[r], az[r], b[q]);
            a[q][r] = cell_addr<CT ? 3 : 4>(key32(c2[q][r], k.klo, k.khi), k.shift, k.lut_base);
        }
    uint4 e[NJ][kR];
#pragma unroll
    for (int q = 0; q < NJ; ++q)
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            if (CT) {
                const uint2 v = lds_read2(a[q][r]);
                e[q][r] = make_uint4(v.y & kCtOffMask, 0u, v.x, v.y);
            } else {
                e[q][r] = lds_read4(a[q][r]);
            }
        }
    // As in the few-edge paths, without compares: d = RN(hi - c) has the sign
    // of hi - c, so its sign bit adds the cell's next row when c > hi; a chord
    // in the cell's band has 0 <= d <= RN(hi - lo), whose bits the entry holds
    // (all ones where several bands meet, 0 where none does), so the step's
    // minimum of max(bits(d) - wbits, 0) is 0 when some chord may be in a band.
    uint32_t mn = 0xFFFFFFFFu;
#pragma unroll
    for (int q = 0; q < NJ; ++q)
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const uint32_t bd = __float_as_uint(__uint_as_float(e[q][r].z) - c2[q][r]);
            uint32_t off = e[q][r].x + ((bd >> 31) << k.row_shift) + k.lane_off;
            uint32_t t = sub_sat(bd, e[q][r].w);
            if (MASKED) {
                // i slot valid, and on a diagonal tile i < j (positions
                // relative to the tile start: i = r*64 + lane, j = j_rel + jj + q)
                const int32_t ir = r * kWave + lane;
                const bool ok = ir < i_lim && (!diag || ir < j_rel + jj + q);
                off = ok ? off : k.trash_off;
                t = ok ? t : 1u;
            }
            mn = min(mn, t);
            lds_add(lds, off, 1u);
        }
    if (__builtin_expect(__builtin_amdgcn_ballot_w64(mn == 0u) != 0, 0)) {
        // rare: a binary32 chord is within the error band of an edge;
        // recompute such pairs in binary64 exactly as the reference does and
        // move their count from the provisional row to the exact one
#pragma unroll
        for (int q = 0; q < NJ; ++q) {
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                float c = chord2_32(ax[r], ay[r], az[r], b[q]);
                asm volatile("" : "+v"(c));
                uint3 en;
                bool band;
                if (CT) {
                    const uint2 v = lds_read2(cell_addr<3>(key32(c, k.klo, k.khi), k.shift, k.lut_base));
                    en = make_uint3(v.y & kCtOffMask, 0u, v.x);
                    band = __float_as_uint(__uint_as_float(v.x) - c) <= v.y;
                } else {
                    en = lds_read3(cell_addr(key32(c, k.klo, k.khi), k.shift, k.lut_base));
                    band = !(c > __uint_as_float(en.z)) && (c >= __uint_as_float(en.y));
                }
                if (MASKED) {
                    const int32_t ir = r * kWave + lane;
                    band &= ir < i_lim && (!diag || ir < j_rel + jj + q);
                }
                if (band) {
                    const double4 b64 = J64t[jj + q];
                    const double4 a64 = I64[ibeg + r * kWave + lane];
                    const double c64 = chord2_64(a64.x, a64.y, a64.z, b64.x, b64.y, b64.z);
                    const uint32_t exact = bin_search(k.e64, k.n_edges, c64) * k.row_bytes + k.lane_off;
                    const uint32_t prov = en.x + k.lane_off;
                    lds_add(lds, k.trash_off + k.row_bytes, 1u);  // re-check tally row
                    if (exact != prov) {
                        lds_add(lds, exact, 1u);
                        lds_add(lds, prov, 0xFFFFFFFFu);
                    }
                }
            }
        }
    }
}

// One tile pair in binary32 with binary64 re-check of in-band pairs.
// MASKED: some i slots are past the end of the range (i_lim < kTile), or this
// is a diagonal tile (only i < j counts); masked-out pairs go to the discard
// row.  j_rel = first j of the tile minus first i of the tile.
template <bool MASKED, bool CT = false>
__device__ __forceinline__ void tile32(unsigned char *lds, const float4 *__restrict__ Jt,
                                       const double4 *__restrict__ J64t, int32_t jn,
                                       const float (&ax)[kR], const float (&ay)[kR],
                                       const float (&az)[kR], const double4 *__restrict__ I64,
                                       int64_t ibeg, int32_t i_lim, int32_t j_rel, bool diag,
                                       const TileCtx &k) {
    constexpr int NJ = PC_JUNROLL;
    int32_t jj = 0;
    // two j buffers in turn: the next step's points load while this step runs
    float4 b0[NJ], b1[NJ];
    load_j<NJ>(Jt, b0);
    for (; jj + 2 * NJ <= jn; jj += 2 * NJ) {
        load_j<NJ>(Jt + jj + NJ, b1);
        step32<MASKED, NJ, CT>(lds, b0, J64t, jj, ax, ay, az, I64, ibeg, i_lim, j_rel, diag, k);
        load_j<NJ>(Jt + jj + 2 * NJ, b0);
        step32<MASKED, NJ, CT>(lds, b1, J64t, jj + NJ, ax, ay, az, I64, ibeg, i_lim, j_rel, diag, k);
    }
    if (jj + NJ <= jn) {
        step32<MASKED, NJ, CT>(lds, b0, J64t, jj, ax, ay, az, I64, ibeg, i_lim, j_rel, diag, k);
        jj += NJ;
    }
    for (; jj < jn; ++jj) {
        float4 bt[1];
        load_j<1>(Jt + jj, bt);
        step32<MASKED, 1, CT>(lds, bt, J64t, jj, ax, ay, az, I64, ibeg, i_lim, j_rel, diag, k);
    }
}

// ------------------------------------------------------- few-edge items
//
// When the whole chord interval of a tile pair contains only M <= kFewMax
// edges (k0 .. k0+M-1; the prune pass proved every exact chord to lie above
// edge k0-1 and below edge k0+M), a chord's row is k0 + #{k < M : chord above
// edge k0+k}, and only those M edges need checking.  Each lane counts, per k,
// its chords above edge k in a register over the whole item and adds the
// counts to its histogram column at the end: no cell table read and no
// histogram atomic per pair.  Chords that binary32 cannot place are
// re-checked in binary64; their correction (+1 on the exact row, -1 on the
// provisional one) goes to the histogram directly.

struct FewCtx {
    float lo[kFewMax], hi[kFewMax];  // bands of edges k0 .. k0+M-1 (matrix-core path), or
                                     // hi: the vector paths' thresholds h
    uint32_t w[kFewMax];             // bits of RN(hi - lo) per band, or of the flag width W
    float del[kFewMax];              // vector paths: RN(h_t - h_0), t >= 1
    uint32_t k0;
};

// The M bands of an item, wave-uniform, and the width bits w.  An edge at 0
// has the band (-inf, -inf): every chord lies above it.  Its hi is taken as
// -FLT_MAX, which orders every chord the same way, so that hi - c is never
// -inf - (-inf) for a chord marked -infinity (see few_tally2).
__device__ __forceinline__ void few_band(FewCtx &f, int q, float2 v) {
    const float hi = fmaxf(v.y, -__FLT_MAX__);
    f.lo[q] = uniform_f(v.x);
    f.hi[q] = uniform_f(hi);
    f.w[q] = uniform(__float_as_uint(hi - v.x));
}

// The vector few-edge paths (thresholds from fused_bands): chords are never
// rounded themselves.  For the item's smallest edge the path forms d_0 = h_0 -
// c in one chain of binary32 roundings, and for edge t >= 1 d_t = RN(d_0 +
// del_t), del_t = RN(h_t - h_0): d_t < 0 proves the binary64 chord at or above
// edge t, d_t > W_t proves it below, and 0 <= d_t <= W_t sends the chord to
// the binary64 re-check.  A pair that counts nowhere has d = +infinity.  The
// prune pass never puts an edge at 0 into a few-edge item.
__device__ __forceinline__ void few_band_fused(FewCtx &f, int q, float2 v) {
    f.hi[q] = uniform_f(v.x);
    f.w[q] = uniform(__float_as_uint(v.y));
}

__device__ __forceinline__ void few_fused_ref(FewCtx &f) {
#pragma unroll
    for (int q = 1; q < kFewMax; ++q) f.del[q] = uniform_f(f.hi[q] - f.hi[0]);
}

// Two chords' d against the smallest edge: the sign bits are added to n, the
// bits of d (unsigned) to the step's minimum mn.  Four vector instructions.
__device__ __forceinline__ void tally_d2(float d1, float d2, uint32_t &n, uint32_t &mn) {
    uint32_t s1, s2;
    asm volatile(
        "v_lshrrev_b32 %[s1], 31, %[d1]\n\t"
        "v_lshrrev_b32 %[s2], 31, %[d2]\n\t"
        "v_add3_u32 %[n], %[n], %[s1], %[s2]\n\t"
        "v_min3_u32 %[mn], %[mn], %[d1], %[d2]"
        : [n] "+v"(n), [mn] "+v"(mn), [s1] "=&v"(s1), [s2] "=&v"(s2)
        : [d1] "v"(d1), [d2] "v"(d2));
}

// The same for a higher edge of the item: d = RN(d_0 + del).  Six vector
// instructions, as many as one subtract per chord and edge needs.
__device__ __forceinline__ void tally_add2(float d1, float d2, float del, uint32_t &n, uint32_t &mn) {
    uint32_t e1, e2, s1, s2;
    asm volatile(
        "v_add_f32 %[e1], %[del], %[d1]\n\t"
        "v_add_f32 %[e2], %[del], %[d2]\n\t"
        "v_lshrrev_b32 %[s1], 31, %[e1]\n\t"
        "v_lshrrev_b32 %[s2], 31, %[e2]\n\t"
        "v_add3_u32 %[n], %[n], %[s1], %[s2]\n\t"
        "v_min3_u32 %[mn], %[mn], %[e1], %[e2]"
        : [n] "+v"(n), [mn] "+v"(mn), [e1] "=&v"(e1), [e2] "=&v"(e2), [s1] "=&v"(s1), [s2] "=&v"(s2)
        : [d1] "v"(d1), [d2] "v"(d2), [del] "s"(del));
}

template <int M>
__device__ __forceinline__ void few_tally_fused(float d1, float d2, const FewCtx &f, uint32_t (&ngt)[M],
                                                uint32_t (&mn)[M]) {
    tally_d2(d1, d2, ngt[0], mn[0]);
#pragma unroll
    for (int t = 1; t < M; ++t) tally_add2(d1, d2, f.del[t], ngt[t], mn[t]);
}

// A pair whose d_0 a flagged step recomputes: true if some d_t lies in its
// flag window; prov = k0 + #{t : d_t < 0}, the row the step counted it in.
template <int M>
__device__ __forceinline__ bool few_in_window(float d0, const FewCtx &f, uint32_t &prov) {
    bool in = false;
    prov = f.k0;
#pragma unroll
    for (int t = 0; t < M; ++t) {
        const uint32_t b = __float_as_uint(t == 0 ? d0 : d0 + f.del[t]);
        prov += b >> 31;
        in |= b <= f.w[t];
    }
    return in;
}

// binary64 re-check of one flagged pair counted in row prov
__device__ __forceinline__ void few_recheck_row(unsigned char *lds, uint32_t prov, const double4 &a64,
                                                const double4 &b64, const TileCtx &k) {
    const double c64 = chord2_64(a64.x, a64.y, a64.z, b64.x, b64.y, b64.z);
    const uint32_t exact = bin_search(k.e64, k.n_edges, c64);
    lds_add(lds, k.trash_off + k.row_bytes, 1u);  // re-check tally row
    if (exact != prov) {
        lds_add(lds, exact * k.row_bytes + k.lane_off, 1u);
        lds_add(lds, prov * k.row_bytes + k.lane_off, 0xFFFFFFFFu);
    }
}

// d_0 of a pair in the difference form: d_0 = RN(-s_z^2 + RN(-s_y^2 +
// RN(h_0 - s_x^2))) with s = RN(a - b) per component
__device__ __forceinline__ float fused_d_diff(float ax, float ay, float az, float4 b, float h0) {
    const float dx = ax - b.x;
    const float dy = ay - b.y;
    const float dz = az - b.z;
    return __builtin_fmaf(-dz, dz, __builtin_fmaf(-dy, dy, __builtin_fmaf(-dx, dx, h0)));
}

// Two chords against one band, in plain arithmetic (no compare, no scalar
// instruction).  d = RN(hi - c) has the sign of hi - c, so its sign bit is
// (c > hi): added to n, the lane's count of chords above the band.  A chord
// inside the band (lo <= c <= hi) has 0 <= hi - c <= hi - lo, hence, rounding
// being monotone, 0 <= d <= RN(hi - lo): the bits of d, read as an unsigned
// integer (a negative d has the sign bit set), are at most w.  mn keeps the
// minimum of those bits over a step; a step whose minimum is at most w in some
// lane is re-checked (a superset of its in-band chords).  Chords that must
// count nowhere (masked pairs) are -infinity: d = +infinity adds nothing and
// is never at most w.  Six vector instructions for two chords; written out so
// that the compiler keeps the two differences short-lived.
__device__ __forceinline__ void few_tally2(float c1, float c2, float hi, uint32_t &n, uint32_t &mn) {
    uint32_t d1, d2, s1, s2;
    asm volatile(
        "v_sub_f32 %[d1], %[hi], %[c1]\n\t"
        "v_sub_f32 %[d2], %[hi], %[c2]\n\t"
        "v_lshrrev_b32 %[s1], 31, %[d1]\n\t"
        "v_lshrrev_b32 %[s2], 31, %[d2]\n\t"
        "v_add3_u32 %[n], %[n], %[s1], %[s2]\n\t"
        "v_min3_u32 %[mn], %[mn], %[d1], %[d2]"
        : [n] "+v"(n), [mn] "+v"(mn), [d1] "=&v"(d1), [d2] "=&v"(d2), [s1] "=&v"(s1), [s2] "=&v"(s2)
        : [c1] "v"(c1), [c2] "v"(c2), [hi] "s"(hi));
}

template <int M>
__device__ __forceinline__ void few_tally(float c1, float c2, const FewCtx &f, uint32_t (&ngt)[M], uint32_t (&mn)[M]) {
#pragma unroll
    for (int t = 0; t < M; ++t) few_tally2(c1, c2, f.hi[t], ngt[t], mn[t]);
}

template <int M>
__device__ __forceinline__ void few_step_start(uint32_t (&mn)[M]) {
#pragma unroll
    for (int t = 0; t < M; ++t) mn[t] = 0xFFFFFFFFu;
}

template <int M>
__device__ __forceinline__ bool few_step_band(const uint32_t (&mn)[M], const FewCtx &f) {
    bool b = false;
#pragma unroll
    for (int t = 0; t < M; ++t) b |= mn[t] <= f.w[t];
    return __builtin_amdgcn_ballot_w64(b) != 0;
}

// Add a lane's few-edge register counts to its histogram column: rows k0 ..
// k0+M get (chords above band t-1) - (chords above band t), with `total`
// valid chords above "band -1".
template <int M>
__device__ __forceinline__ void few_flush(unsigned char *lds, const uint32_t (&ngt)[M], uint32_t total,
                                          const FewCtx &f, const TileCtx &k) {
    uint32_t prev = total;
#pragma unroll
    for (int t = 0; t <= M; ++t) {
        const uint32_t above = t < M ? ngt[t] : 0u;
        const uint32_t cnt = prev - above;
        if (cnt) lds_add(lds, (f.k0 + static_cast<uint32_t>(t)) * k.row_bytes + k.lane_off, cnt);
        prev = above;
    }
}

// binary64 re-check of one in-band chord (provisional row k0 + #{c > hi_k})
template <int M>
__device__ __forceinline__ void few_recheck(unsigned char *lds, float c, const double4 &a64, const double4 &b64,
                                            const FewCtx &f, const TileCtx &k) {
    uint32_t prov = f.k0;
#pragma unroll
    for (int t = 0; t < M; ++t) prov += c > f.hi[t] ? 1u : 0u;
    const double c64 = chord2_64(a64.x, a64.y, a64.z, b64.x, b64.y, b64.z);
    const uint32_t exact = bin_search(k.e64, k.n_edges, c64);
    lds_add(lds, k.trash_off + k.row_bytes, 1u);  // re-check tally row
    if (exact != prov) {
        lds_add(lds, exact * k.row_bytes + k.lane_off, 1u);
        lds_add(lds, prov * k.row_bytes + k.lane_off, 0xFFFFFFFFu);
    }
}

// A chord inside one of the item's bands.  -infinity marks a pair that
// counts nowhere (a Gram-form i slot past a ragged end), which a band with
// lo = -infinity (an edge at or near 0) would otherwise take in.
template <int M>
__device__ __forceinline__ bool few_in_band(float c, const FewCtx &f) {
    bool band = false;
#pragma unroll
    for (int t = 0; t < M; ++t) band |= !(c > f.hi[t]) & (c >= f.lo[t]);
    return band & (c > -__builtin_inff());
}

template <bool MASKED, int M, int NJ>
__device__ __forceinline__ void step32_few(unsigned char *lds, const float4 (&b)[NJ],
                                           const double4 *__restrict__ J64t, int32_t jj,
                                           const float (&ax)[kR], const float (&ay)[kR],
                                           const float (&az)[kR], const double4 *__restrict__ I64,
                                           int64_t ibeg, int32_t i_lim, int32_t j_rel, bool diag,
                                           const TileCtx &k, const FewCtx &f, uint32_t (&ngt)[M]) {
    const int32_t lane = static_cast<int32_t>(threadIdx.x);
    uint32_t mn[M];
    few_step_start<M>(mn);
    static_assert(kR % 2 == 0, "chords are tallied in pairs");
#pragma unroll
    for (int q = 0; q < NJ; ++q)
#pragma unroll
        for (int r = 0; r < kR; r += 2) {
            float d[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                d[h] = fused_d_diff(ax[r + h], ay[r + h], az[r + h], b[q], f.hi[0]);
                if (MASKED) {
                    // a masked-out pair gets d = +infinity, which counts nowhere
                    const int32_t ir = (r + h) * kWave + lane;
                    const bool ok = ir < i_lim && (!diag || ir < j_rel + jj + q);
                    d[h] = ok ? d[h] : __builtin_inff();
                }
            }
            few_tally_fused<M>(d[0], d[1], f, ngt, mn);
        }
    if (__builtin_expect(few_step_band<M>(mn, f), 0)) {
#pragma unroll
        for (int q = 0; q < NJ; ++q)
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                float d = fused_d_diff(ax[r], ay[r], az[r], b[q], f.hi[0]);
                asm volatile("" : "+v"(d));
                uint32_t prov;
                bool in = few_in_window<M>(d, f, prov);
                if (MASKED) {
                    const int32_t ir = r * kWave + lane;
                    in &= ir < i_lim && (!diag || ir < j_rel + jj + q);
                }
                if (in) few_recheck_row(lds, prov, I64[ibeg + r * kWave + lane], J64t[jj + q], k);
            }
    }
}

// One tile pair of a few-edge item in binary32 (masking as in tile32).
template <bool MASKED, int M>
__device__ __forceinline__ void tile32_few(unsigned char *lds, const float4 *__restrict__ Jt,
                                           const double4 *__restrict__ J64t, int32_t jn,
                                           const float (&ax)[kR], const float (&ay)[kR],
                                           const float (&az)[kR], const double4 *__restrict__ I64,
                                           int64_t ibeg, int32_t i_lim, int32_t j_rel, bool diag,
                                           const TileCtx &k, const FewCtx &f) {
    uint32_t ngt[M];
#pragma unroll
    for (int t = 0; t < M; ++t) ngt[t] = 0u;
    constexpr int NJ = PC_JUNROLL;
    int32_t jj = 0;
    // two j buffers in turn: the next step's points load while this step runs
    float4 b0[NJ], b1[NJ];
    load_j<NJ>(Jt, b0);
    for (; jj + 2 * NJ <= jn; jj += 2 * NJ) {
        load_j<NJ>(Jt + jj + NJ, b1);
        step32_few<MASKED, M, NJ>(lds, b0, J64t, jj, ax, ay, az, I64, ibeg, i_lim, j_rel, diag, k, f, ngt);
        load_j<NJ>(Jt + jj + 2 * NJ, b0);
        step32_few<MASKED, M, NJ>(lds, b1, J64t, jj + NJ, ax, ay, az, I64, ibeg, i_lim, j_rel, diag, k, f, ngt);
    }
    if (jj + NJ <= jn) {
        step32_few<MASKED, M, NJ>(lds, b0, J64t, jj, ax, ay, az, I64, ibeg, i_lim, j_rel, diag, k, f, ngt);
        jj += NJ;
    }
    for (; jj < jn; ++jj) {
        float4 bt[1];
        load_j<1>(Jt + jj, bt);
        step32_few<MASKED, M, 1>(lds, bt, J64t, jj, ax, ay, az, I64, ibeg, i_lim, j_rel, diag, k, f, ngt);
    }
    // valid chords of this lane: slot r holds i = r*64 + lane; on a diagonal
    // tile only j with i < j count
    uint32_t total = 0;
    const int32_t lane = static_cast<int32_t>(threadIdx.x);
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int32_t ir = r * kWave + lane;
        if (!MASKED) {
            total += static_cast<uint32_t>(jn);
        } else if (ir < i_lim) {
            const int32_t skip = diag ? min(max(ir - j_rel + 1, 0), jn) : 0;
            total += static_cast<uint32_t>(jn - skip);
        }
    }
    few_flush<M>(lds, ngt, total, f, k);
}

// Few-edge items whose j-tile radius r satisfies 2 r <= the chord lower
// bound: chords in Gram form centred on the j-tile's centre o, on the vector
// ALU.  The j side comes precomputed per point as (-2 b'_x, -2 b'_y, -2 b'_z,
// |b'|^2) with b' = RN32(b - o); the lane's i-points are centred here, a' =
// RN32(a - o), kept negated, with |a'|^2 in binary32 and, per run of edges,
// S = RN(h_0 - |a'|^2).  Then d_0 = h_0 - |a' - b'|^2 comes as
// (-a'_x) B_x + ((-a'_y) B_y + ((-a'_z) B_z + (S - |b'|^2))): one subtract and
// three fused multiply-adds, against six instructions for the difference
// form; fused_bands bounds its error (same centring condition).  i slots past
// the end of the range get |a'|^2 = -infinity, so S and every d are
// +infinity and count nowhere.
template <int M, int NJ>
__device__ __forceinline__ void step32_gram(unsigned char *lds, const float4 (&b)[NJ],
                                            const double4 *__restrict__ J64t, int32_t jj, const float (&nx)[kR],
                                            const float (&ny)[kR], const float (&nz)[kR], const float (&S)[kR],
                                            const double4 *__restrict__ I64, int64_t ibeg, const TileCtx &k,
                                            const FewCtx &f, uint32_t (&ngt)[M]) {
    const int32_t lane = static_cast<int32_t>(threadIdx.x);
    uint32_t mn[M];
    few_step_start<M>(mn);
#pragma unroll
    for (int q = 0; q < NJ; ++q)
#pragma unroll
        for (int r = 0; r < kR; r += 2) {
            float d[2];
#pragma unroll
            for (int h = 0; h < 2; ++h)
                d[h] = __builtin_fmaf(nx[r + h], b[q].x, __builtin_fmaf(ny[r + h], b[q].y,
                                      __builtin_fmaf(nz[r + h], b[q].z, S[r + h] - b[q].w)));
            few_tally_fused<M>(d[0], d[1], f, ngt, mn);
        }
    if (__builtin_expect(few_step_band<M>(mn, f), 0)) {
#pragma unroll
        for (int q = 0; q < NJ; ++q)
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                float d = __builtin_fmaf(nx[r], b[q].x, __builtin_fmaf(ny[r], b[q].y,
                                         __builtin_fmaf(nz[r], b[q].z, S[r] - b[q].w)));
                asm volatile("" : "+v"(d));
                uint32_t prov;
                if (few_in_window<M>(d, f, prov)) few_recheck_row(lds, prov, I64[ibeg + r * kWave + lane], J64t[jj + q], k);
            }
    }
}

// The lane's i-points centred on the j-tile's centre o, in binary32 and
// negated, with |a'|^2; slots past a ragged end get -infinity so their pairs
// count nowhere.
struct GramI {
    float nx[kR], ny[kR], nz[kR], na[kR];
    uint32_t valid;
};

__device__ __forceinline__ void centre_i_gram(GramI &g, const double4 (&pts)[kR], int32_t i_lim, double ox,
                                              double oy, double oz) {
    const int32_t lane = static_cast<int32_t>(threadIdx.x);
    g.valid = 0;
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int32_t ir = r * kWave + lane;
        const bool ok = ir < i_lim;
        const double4 p = pts[r];
        const float x = static_cast<float>(p.x - ox);
        const float y = static_cast<float>(p.y - oy);
        const float z = static_cast<float>(p.z - oz);
        g.nx[r] = -x;
        g.ny[r] = -y;
        g.nz[r] = -z;
        const float n2 = __builtin_fmaf(z, z, __builtin_fmaf(y, y, x * x));
        g.na[r] = ok ? n2 : -__builtin_inff();
        g.valid += ok ? 1u : 0u;
    }
}

template <int M>
__device__ __forceinline__ void tile32_gram(unsigned char *lds, const float4 *__restrict__ Jg,
                                            const double4 *__restrict__ J64t, int32_t jn, const GramI &g,
                                            const double4 *__restrict__ I64, int64_t ibeg, const TileCtx &k,
                                            const FewCtx &f) {
    uint32_t ngt[M];
#pragma unroll
    for (int t = 0; t < M; ++t) ngt[t] = 0u;
    // S = RN(h_0 - |a'|^2) per slot, for this run's edges
    float S[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) S[r] = f.hi[0] - g.na[r];
    constexpr int NJ = PC_JUNROLL;
    int32_t jj = 0;
    // two j buffers in turn: the next step's points load while this step runs
    float4 b0[NJ], b1[NJ];
    load_j<NJ>(Jg, b0);
    for (; jj + 2 * NJ <= jn; jj += 2 * NJ) {
        load_j<NJ>(Jg + jj + NJ, b1);
        step32_gram<M, NJ>(lds, b0, J64t, jj, g.nx, g.ny, g.nz, S, I64, ibeg, k, f, ngt);
        load_j<NJ>(Jg + jj + 2 * NJ, b0);
        step32_gram<M, NJ>(lds, b1, J64t, jj + NJ, g.nx, g.ny, g.nz, S, I64, ibeg, k, f, ngt);
    }
    if (jj + NJ <= jn) {
        step32_gram<M, NJ>(lds, b0, J64t, jj, g.nx, g.ny, g.nz, S, I64, ibeg, k, f, ngt);
        jj += NJ;
    }
    for (; jj < jn; ++jj) {
        float4 bt[1];
        load_j<1>(Jg + jj, bt);
        step32_gram<M, 1>(lds, bt, J64t, jj, g.nx, g.ny, g.nz, S, I64, ibeg, k, f, ngt);
    }
    few_flush<M>(lds, ngt, g.valid * static_cast<uint32_t>(jn), f, k);
}

// ----------------------------------------------------------- matrix cores
// (256-point tiles only: a tile pair is 16 x 16 blocks of 16 x 16 pairs)

constexpr bool kMatrixCores = kTile == 256;

typedef float f32x4 __attribute__((ext_vector_type(4)));

#ifndef PC_MB
#define PC_MB 1             // 16x16 blocks binned together (4 chords per lane each)
#endif

// Few-edge binning of the chords one lane holds after MB matrix multiplies
// (see the few-edge items above).
template <int MB, int M>
__device__ __forceinline__ void bin_mfma_few(unsigned char *lds, const f32x4 (&D)[MB], const double4 *__restrict__ I64t,
                                             const double4 *__restrict__ J64t, int bi0, int bj, const TileCtx &g,
                                             const FewCtx &f, uint32_t (&ngt)[M]) {
    const int lane = static_cast<int>(threadIdx.x);
    const int l16 = lane & 15, kq = lane >> 4;
    float c[4 * MB];
#pragma unroll
    for (int m = 0; m < MB; ++m) {
        c[4 * m + 0] = D[m].x;
        c[4 * m + 1] = D[m].y;
        c[4 * m + 2] = D[m].z;
        c[4 * m + 3] = D[m].w;
    }
    uint32_t mn[M];
    few_step_start<M>(mn);
#pragma unroll
    for (int v = 0; v < 4 * MB; v += 2) few_tally<M>(c[v], c[v + 1], f, ngt, mn);
    if (__builtin_expect(few_step_band<M>(mn, f), 0)) {
#pragma unroll
        for (int v = 0; v < 4 * MB; ++v) {
            // an opaque copy: the compares are redone here rather than their
            // results kept live (in scalar registers) through the main path
            float cv = c[v];
            asm volatile("" : "+v"(cv));
            if (few_in_band<M>(cv, f)) {
                int row = (bi0 + v / 4) * 16 + 4 * kq + (v & 3);
                asm volatile("" : "+v"(row));
                few_recheck<M>(lds, cv, I64t[row], J64t[bj * 16 + l16], f, g);
            }
        }
    }
}

// One full 256 x 256 tile pair through the matrix cores.  Coordinates are
// centred on o (the bounding-sphere centre of the tile with the smaller
// radius) in binary64 and rounded to binary32: a' = a - o, b' = b - o.  With
// A_i = (a'_x, a'_y, a'_z, |a'_i|^2), B_j = (-2 b'_x, -2 b'_y, -2 b'_z, 1) and
// the addend |b'_j|^2, one v_mfma_f32_16x16x4f32 gives |a'_i - b'_j|^2 for a
// 16 x 16 block of pairs (operand layout: lane l holds row l%16, k = l/16 of
// A and column l%16, k = l/16 of B).  The lane's A operands of the 16
// i-blocks are staged in the wave's LDS block `a_stage` (16 x 64 floats) and
// read one binning step ahead of their multiply; the j-block loop loads the
// next block's point one iteration ahead.  Only tile pairs whose chord lower
// bound is at least twice that radius, and with M <= kFewMax edges inside
// their chord interval, come here; f holds those edges' matrix-core bands.
template <int M>
__device__ __forceinline__ void tile_mfma(unsigned char *lds, uint32_t a_stage, const double4 *__restrict__ I64t,
                                          const double4 *__restrict__ J64t, double ox, double oy, double oz,
                                          const TileCtx &g, const FewCtx &f) {
    const int lane = static_cast<int>(threadIdx.x);
    const int l16 = lane & 15, kq = lane >> 4;
    constexpr int MB = PC_MB;
    constexpr int NB = 16 / MB;  // binning steps per j-block
    static_assert(16 % (2 * MB) == 0, "blocks per binning step");
    using lds_f32 = __attribute__((address_space(3))) float;
    static_assert(M >= 1 && M <= kFewMax, "few-edge items only");
    uint32_t ngt[M];
#pragma unroll
    for (int t = 0; t < M; ++t) ngt[t] = 0u;
#pragma unroll 4
    for (int bi = 0; bi < 16; ++bi) {
        const double4 p = I64t[bi * 16 + l16];
        const float x = static_cast<float>(p.x - ox);
        const float y = static_cast<float>(p.y - oy);
        const float z = static_cast<float>(p.z - oz);
        const float na = __builtin_fmaf(z, z, __builtin_fmaf(y, y, x * x));
        *(lds_f32 *)(uintptr_t)(a_stage + (bi * kWave + lane) * 4u) = kq == 0 ? x : kq == 1 ? y : kq == 2 ? z : na;
    }
    // A operands of binning step s (blocks s*MB .. s*MB+MB-1); steps past the
    // last re-read the last one (their products are not used)
    auto load_a = [&](int step, float (&out)[MB]) {
        const int s0 = min(step, NB - 1) * MB;
#pragma unroll
        for (int m = 0; m < MB; ++m) out[m] = *(const lds_f32 *)(uintptr_t)(a_stage + ((s0 + m) * kWave + lane) * 4u);
    };
    // only x, y, z of the j-points are loaded (the prefetched one stays live
    // through a whole iteration)
    auto load_j = [&](int blk, double &x, double &y, double &z) {
        const double *pj = reinterpret_cast<const double *>(J64t + blk * 16 + l16);
        x = pj[0];
        y = pj[1];
        z = pj[2];
    };
    double qx, qy, qz;
    load_j(0, qx, qy, qz);
#pragma unroll 1
    for (int bj = 0; bj < 16; ++bj) {
        double nx, ny, nz;
        load_j(min(bj + 1, 15), nx, ny, nz);
        const double4 q = make_double4(qx, qy, qz, 0.0);
        const float x = static_cast<float>(q.x - ox);
        const float y = static_cast<float>(q.y - oy);
        const float z = static_cast<float>(q.z - oz);
        const float nb = __builtin_fmaf(z, z, __builtin_fmaf(y, y, x * x));
        const float B = kq == 0 ? -2.0f * x : kq == 1 ? -2.0f * y : kq == 2 ? -2.0f * z : 1.0f;
        const f32x4 C = {nb, nb, nb, nb};
        // two binning steps per iteration with two product buffers: the
        // products of step s+1 are issued before step s is binned, and the A
        // operands of step s+2 are read meanwhile
        float Ap[MB];
        f32x4 DA[MB], DB[MB];
        load_a(0, Ap);
#pragma unroll
        for (int m = 0; m < MB; ++m) DA[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(Ap[m], B, C, 0, 0, 0);
        load_a(1, Ap);
#pragma unroll 1
        for (int st = 0; st < NB; st += 2) {
#pragma unroll
            for (int m = 0; m < MB; ++m) DB[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(Ap[m], B, C, 0, 0, 0);
            load_a(st + 2, Ap);
            bin_mfma_few<MB, M>(lds, DA, I64t, J64t, st * MB, bj, g, f, ngt);
#pragma unroll
            for (int m = 0; m < MB; ++m) DA[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(Ap[m], B, C, 0, 0, 0);
            load_a(st + 3, Ap);
            bin_mfma_few<MB, M>(lds, DB, I64t, J64t, (st + 1) * MB, bj, g, f, ngt);
        }
        qx = nx;
        qy = ny;
        qz = nz;
    }
    few_flush<M>(lds, ngt, 16u * 16u * 4u, f, g);
}

// ------------------------------------------------------------------ fp64

template <bool MASKED, bool SEARCH>
__device__ __forceinline__ void tile64(unsigned char *lds, const double4 *__restrict__ J64t, int32_t jn,
                                       const double (&ax)[kR], const double (&ay)[kR],
                                       const double (&az)[kR], int32_t i_lim, int32_t j_rel, bool diag,
                                       uint32_t kclo, uint32_t kchi, const TileCtx &k) {
    const int32_t lane = static_cast<int32_t>(threadIdx.x);
    for (int32_t jj = 0; jj < jn; ++jj) {
        const double4 b = ld_const(J64t + jj);
        double c[kR];
        uint32_t off[kR];
        if (SEARCH) {
            const __attribute__((address_space(3))) double *e =
                (const __attribute__((address_space(3))) double *)(uintptr_t)(k.lut_base);
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                c[r] = chord2_64(ax[r], ay[r], az[r], b.x, b.y, b.z);
                off[r] = bin_search(e, k.n_edges, c[r]) * k.row_bytes + k.lane_off;
            }
        } else {
            uint32_t a[kR];
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                c[r] = chord2_64(ax[r], ay[r], az[r], b.x, b.y, b.z);
                const uint32_t hw = static_cast<uint32_t>(__double_as_longlong(c[r]) >> 32);
                a[r] = cell_addr(min(max(hw, kclo), kchi), k.shift, k.lut_base);
            }
            uint4 e[kR];
#pragma unroll
            for (int r = 0; r < kR; ++r) e[r] = lds_read4(a[r]);
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                const double ev = __hiloint2double(static_cast<int>(e[r].w), static_cast<int>(e[r].z));
                off[r] = (c[r] >= ev ? e[r].y : e[r].x) + k.lane_off;
            }
        }
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            uint32_t o = off[r];
            if (MASKED) {
                const int32_t ir = r * kWave + lane;
                const bool ok = ir < i_lim && (!diag || ir < j_rel + jj);
                o = ok ? o : k.trash_off;
            }
            lds_add(lds, o, 1u);
        }
    }
}

// ------------------------------------------------------- persistent kernel

// Waves per SIMD asked of the register allocator.  The counting loops wait
// on scalar loads of j-points, LDS and the i-point loads of each item, and
// more resident waves hide that, while fewer leave more registers and fewer
// spills to scratch (mostly around the rarely taken binary64 re-check
// branches).  The 256-point instance (4 i-points per lane, a Gram run's S
// per slot) is built for 6 (80 VGPRs, 96 bytes of scratch per lane): on the
// 1M workload it takes 43.6, 43.9, 45.9 and 47.2 ms at 6, 5, 7 and 8 waves per
// SIMD on one box.  The 128-point instance keeps 8 (64 VGPRs): on the
// batched workload 730 ms, against 765 ms for the best launch at 6.  The
// binary64 instance keeps 7, the matrix-core one 3.
#ifdef PC_WAVES_PER_EU
#define PC_OCCUPANCY __attribute__((amdgpu_waves_per_eu(PC_WAVES_PER_EU)))
#elif defined(PC_NO_OCCUPANCY_HINT)
#define PC_OCCUPANCY
#else
#define PC_OCCUPANCY __attribute__((amdgpu_waves_per_eu(MC ? 3 : (FP64 ? 7 : (kR == 4 ? 6 : 8)))))
#endif

// MC: tile pairs marked by the prune pass go through the matrix cores (a
// separate instance, so the binary32-only instance keeps its lower register
// count and occupancy).
// CT: the cell table in its compact form (mixed kernel only; see step32).
template <bool FP64, bool MC, bool CT = false>
__global__ void __launch_bounds__(kWave) PC_OCCUPANCY k_count(KParams p) {
    extern __shared__ __align__(16) unsigned char lds[];
    const uint32_t lds0 = lds_addr(lds);
    const uint32_t lane = threadIdx.x;
    const uint32_t b = blockIdx.x;
    const uint64_t total = p.items ? static_cast<uint64_t>(*(const __attribute__((address_space(4))) unsigned long long *)(p.n_items))
                                   : p.total_items;
    // Work queue: the items are cut into 8 contiguous slices, one per XCD
    // (consecutive workgroups are dispatched to different XCDs, so each XCD's
    // L2 sees neighbouring tiles); a wave takes kChunk items at a time from its
    // own XCD's slice, then from the others.  Waves that become resident late
    // simply find less work, so the launch ends evenly whatever the residency.
    const uint64_t kChunk = p.chunk;
    const uint32_t x0 = b & 7u;
    uint32_t xs = 0;
    uint64_t wi = 0, end = 0;

    // Carried from item to item: the queue position, the current segment's
    // descriptor, the histogram's owner (table, job, counters, words to
    // clear, items since the last flush) and the table's layout.
    int s = 0;
    int cur_tab = -1, cur_job = -1;
    int32_t clear_words = 0;
    unsigned long long *cur_counts = nullptr;
    uint64_t since_flush = 0;
    SegDesc sd = ld_const_struct(p.segs);
    int32_t n_edges = 0, cols = 64;
    uint32_t row_bytes = 0, lane_off = 0, clo = 0, chi = 0, shift = 0, lut_base = 0, trash_off = 0;
    bool search = false;
    const double *e64 = nullptr;
    const float *band_g = nullptr, *fband = nullptr, *fband_g = nullptr;
    uint64_t flush_every = 1;

    for (;; ++wi) {
        if (wi >= end) {
            bool got = false;
            for (; xs < 8u; ++xs) {
                const uint32_t x = (x0 + xs) & 7u;
                const uint64_t s0 = total * x / 8u, s1 = total * (x + 1u) / 8u;
                unsigned long long c = 0;
                if (lane == 0) c = atomicAdd(p.queue + x * kQueueStride, static_cast<unsigned long long>(kChunk));
                c = uniform_u64(c);
                if (s0 + c < s1) {
                    wi = s0 + c;
                    end = min<uint64_t>(s1, s0 + c + kChunk);
                    got = true;
                    break;
                }
            }
            if (!got) break;
        }
        const uint64_t raw = p.items ? static_cast<uint64_t>(uniform_u64(p.items[wi])) : wi;
        // marked by the prune pass (layout next to kItemBits)
        const bool to_mfma = !FP64 && (raw >> 63) != 0;
        const bool centre_j = ((raw >> 62) & 1u) != 0;
        const bool gram_j = !FP64 && ((raw >> 61) & 1u) != 0;
        const uint32_t few_m = FP64 ? 0u : static_cast<uint32_t>((raw >> (kItemBits + 11)) & 3u);
        const uint32_t few_k0 = static_cast<uint32_t>((raw >> kItemBits) & 2047u);

        const bool split = PC_SPLIT && !FP64 && ((raw >> kSplitBit) & 1u) != 0;
        // a split item's sub-block word, and the chord form of the item: a
        // split item takes the Gram form when every open part allows it
        const uint64_t sub = split ? ld_const(p.sub + wi) : 0ull;
        bool gram_all = true;
#pragma unroll
        for (int q = 0; q < kSubs; ++q) {
            const uint32_t w = static_cast<uint32_t>(sub >> (16 * q)) & 0xFFFFu;
            if (!(w & kSubWhole) && !(w & kSubGram)) gram_all = false;
        }
        const bool use_gram = !FP64 && !(MC && to_mfma) && (split ? gram_all : (gram_j && few_m != 0u));
        const uint64_t it = raw & kItemMask;
        if (it < sd.item0 || it >= sd.item0 + sd.n_items) {
            s = find_seg(p.segs, p.n_segs, it);
            sd = ld_const_struct(p.segs + s);
        }
        // a lane adds at most kTile * kR per item to a word it shares with
        // kWave / cols - 1 other lanes: flush before a 32-bit word can wrap
        if (sd.tab != cur_tab || sd.job != cur_job || since_flush >= flush_every) {
            if (cur_job >= 0) flush_hist(lds, n_edges + 1, cols, clear_words, cur_counts, p.rechecked);
            if (sd.tab != cur_tab) {
                const TableDesc td = ld_const_struct(p.tabs + sd.tab);
                n_edges = td.n_edges;
                band_g = td.band_g;
                fband = td.fband;
                fband_g = td.fband_g;
                clo = td.clamp_lo;
                chi = td.clamp_hi;
                shift = td.shift;
                search = td.search != 0;
                e64 = td.e64;
                cols = td.cols;
                flush_every = 0xFFFFFFFFull / (static_cast<uint64_t>(kTile) * kR * static_cast<uint64_t>(kWave / cols));
                if (p.flush_cap) flush_every = min(flush_every, p.flush_cap);
                row_bytes = static_cast<uint32_t>(cols) * 4u;
                lane_off = lds0 + (lane & static_cast<uint32_t>(cols - 1)) * 4u;
                trash_off = static_cast<uint32_t>(n_edges + 1) * row_bytes + lane_off;
                lut_base = (FP64 && search) ? lds0 + p.lut_lds_off
                                            : lds0 + p.lut_lds_off - (td.key0 << (CT ? 3 : 4));
                // copy the cell table (or, for a search table, the edges) into LDS
                if (FP64 && search) {
                    double *dst = reinterpret_cast<double *>(lds + p.lut_lds_off);
                    for (int32_t k = lane; k < n_edges; k += kWave) dst[k] = td.e64[k];
                } else if (CT) {
                    const uint2 *src = reinterpret_cast<const uint2 *>(td.lutc);
                    uint2 *dst = reinterpret_cast<uint2 *>(lds + p.lut_lds_off);
                    for (int32_t k = lane; k < td.n_cells; k += kWave) dst[k] = src[k];
                } else {
                    const uint4 *src = reinterpret_cast<const uint4 *>(td.lut);
                    uint4 *dst = reinterpret_cast<uint4 *>(lds + p.lut_lds_off);
                    for (int32_t k = lane; k < td.n_cells; k += kWave) dst[k] = src[k];
                }
                const int32_t words = (n_edges + 3) * cols;
                uint32_t *h = reinterpret_cast<uint32_t *>(lds);
                for (int32_t x = lane + (cur_job < 0 ? 0 : clear_words); x < words; x += kWave) h[x] = 0u;
                clear_words = max(clear_words, words);
                cur_tab = sd.tab;
                __syncthreads();
            }
            cur_job = sd.job;
            cur_counts = sd.counts;
            since_flush = 0;
        }
        ++since_flush;
        int64_t t, u;
        map_item(sd, it - sd.item0, t, u);
        const int64_t iend = sd.i0 + sd.ni;
        const int64_t ibeg = sd.i0 + t * kTile;
        const int32_t i_lim = static_cast<int32_t>(uniform(static_cast<uint32_t>(min<int64_t>(kTile, iend - ibeg))));
        // the lane's i-points, reloaded per item (4 loads against 1024 pairs)
        // and issued first, so that their latency passes while the item is
        // set up: binary64 for that kernel and for the Gram form (centred on
        // the j-tile once the loads are in), binary32 for the difference form
        double dx[kR], dy[kR], dz[kR];
        float fx[kR], fy[kR], fz[kR];
        double4 gi[kR];
        auto load_gi = [&]() {
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                const int32_t ir = r * kWave + static_cast<int32_t>(lane);
                gi[r] = sd.i64[ibeg + (ir < i_lim ? ir : 0)];
            }
        };
        if (use_gram) {
            if (PC_EARLY_GRAM) load_gi();
        } else if (FP64 || !(MC && to_mfma)) {
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                const int32_t ir = r * kWave + static_cast<int32_t>(lane);
                const int64_t g = ibeg + (ir < i_lim ? ir : 0);
                if (FP64) {
                    const double4 v = sd.i64[g];
                    dx[r] = v.x;
                    dy[r] = v.y;
                    dz[r] = v.z;
                } else {
                    const float4 v = sd.i32[g];
                    fx[r] = v.x;
                    fy[r] = v.y;
                    fz[r] = v.z;
                }
            }
        }
        const int64_t jbeg = sd.j0 + u * kTile;
        const int32_t jn = static_cast<int32_t>(uniform(static_cast<uint32_t>(min<int64_t>(kTile, sd.j0 + sd.nj - jbeg))));
        const bool diag = uniform((sd.tri && t == u) ? 1u : 0u) != 0u;
        const bool masked = diag || i_lim < kTile;
        const int32_t j_rel = static_cast<int32_t>(uniform(static_cast<uint32_t>(jbeg - ibeg)));
        const double4 *J64t = uniform_ptr(sd.j64 + jbeg);
        TileCtx k;
        k.shift = shift;
        k.lut_base = lut_base;
        k.lane_off = lane_off;
        k.trash_off = trash_off;
        k.row_bytes = row_bytes;
        k.row_shift = static_cast<uint32_t>(__builtin_ctz(row_bytes));
        k.klo = __uint_as_float(clo);
        k.khi = __uint_as_float(chi);
        k.n_edges = n_edges;
        k.e64 = e64;
        if (FP64) {
            if (search) {
                if (masked)
                    tile64<true, true>(lds, J64t, jn, dx, dy, dz, i_lim, j_rel, diag, clo, chi, k);
                else
                    tile64<false, true>(lds, J64t, jn, dx, dy, dz, i_lim, j_rel, diag, clo, chi, k);
            } else {
                if (masked)
                    tile64<true, false>(lds, J64t, jn, dx, dy, dz, i_lim, j_rel, diag, clo, chi, k);
                else
                    tile64<false, false>(lds, J64t, jn, dx, dy, dz, i_lim, j_rel, diag, clo, chi, k);
            }
        } else if (MC && to_mfma) {
            // the prune pass marks only few-edge items for the matrix cores
            FewCtx f;
            f.k0 = uniform(few_k0);
#pragma unroll
            for (int q = 0; q < kFewMax; ++q) {
                const uint32_t e = min(few_k0 + static_cast<uint32_t>(q), static_cast<uint32_t>(n_edges - 1));
                few_band(f, q, ld_const_f2(band_g + 2u * e));
            }
            const double4 o = ld_const(centre_j ? sd.jb + u : sd.ib + t);
            const double4 *I64t = uniform_ptr(sd.i64 + ibeg);
            const uint32_t st = lds0 + p.stage_lds_off;
            if (few_m == 1) tile_mfma<1>(lds, st, I64t, J64t, o.x, o.y, o.z, k, f);
            else if (few_m == 2) tile_mfma<2>(lds, st, I64t, J64t, o.x, o.y, o.z, k, f);
            else tile_mfma<3>(lds, st, I64t, J64t, o.x, o.y, o.z, k, f);
        } else if (!split) {
            // one part: the whole j-tile with the item's own edges
            FewCtx f;
            f.k0 = uniform(few_k0);
            if (few_m) {
                const float *bd = gram_j ? fband_g : fband;
#pragma unroll
                for (int q = 0; q < kFewMax; ++q) {
                    const uint32_t e = min(few_k0 + static_cast<uint32_t>(q), static_cast<uint32_t>(n_edges - 1));
                    few_band_fused(f, q, ld_const_f2(bd + 2u * e));
                }
                few_fused_ref(f);
            }
            if (use_gram) {
                // not a diagonal tile; i slots past a ragged end are -infinity
                const double4 o = ld_const(sd.jb + u);
                GramI g;
                if (!PC_EARLY_GRAM) load_gi();
                centre_i_gram(g, gi, i_lim, o.x, o.y, o.z);
                const float4 *Jg = uniform_ptr(sd.jg + jbeg);
                if (few_m == 1) tile32_gram<1>(lds, Jg, J64t, jn, g, sd.i64, ibeg, k, f);
                else if (few_m == 2) tile32_gram<2>(lds, Jg, J64t, jn, g, sd.i64, ibeg, k, f);
                else tile32_gram<3>(lds, Jg, J64t, jn, g, sd.i64, ibeg, k, f);
            } else {
                const float4 *Jt = uniform_ptr(sd.j32 + jbeg);
                if (masked) {
                    if (few_m == 1) tile32_few<true, 1>(lds, Jt, J64t, jn, fx, fy, fz, sd.i64, ibeg, i_lim, j_rel, diag, k, f);
                    else if (few_m == 2) tile32_few<true, 2>(lds, Jt, J64t, jn, fx, fy, fz, sd.i64, ibeg, i_lim, j_rel, diag, k, f);
                    else if (few_m == 3) tile32_few<true, 3>(lds, Jt, J64t, jn, fx, fy, fz, sd.i64, ibeg, i_lim, j_rel, diag, k, f);
                    else tile32<true, CT>(lds, Jt, J64t, jn, fx, fy, fz, sd.i64, ibeg, i_lim, j_rel, diag, k);
                } else {
                    if (few_m == 1) tile32_few<false, 1>(lds, Jt, J64t, jn, fx, fy, fz, sd.i64, ibeg, i_lim, j_rel, diag, k, f);
                    else if (few_m == 2) tile32_few<false, 2>(lds, Jt, J64t, jn, fx, fy, fz, sd.i64, ibeg, i_lim, j_rel, diag, k, f);
                    else if (few_m == 3) tile32_few<false, 3>(lds, Jt, J64t, jn, fx, fy, fz, sd.i64, ibeg, i_lim, j_rel, diag, k, f);
                    else tile32<false, CT>(lds, Jt, J64t, jn, fx, fy, fz, sd.i64, ibeg, i_lim, j_rel, diag, k);
                }
            }
        } else {
            // A split item (full, off-diagonal) visits its open sub-blocks of
            // kSub j-points, each with its own edges.  The lane's i-points
            // are loaded once, in one chord form for all its parts: Gram form
            // when every part allows it, else the difference form (its guard
            // band holds for any pair, so a Gram-eligible part may use it too).
            // the next run of parts from `part` on: consecutive open parts
            // with the same description go in one call; its edges
            // k0 .. k0+m-1 (m = 0: cell table) and j range.  False when no
            // part is left (the prune pass binned the rest whole).
            auto next_run = [&](int &part, uint32_t &m, uint32_t &k0, int64_t &jb, int32_t &nj) -> bool {
                uint32_t w = 0;
                for (; part < kSubs; ++part) {
                    w = static_cast<uint32_t>(sub >> (16 * part)) & 0xFFFFu;
                    if (!(w & kSubWhole)) break;
                }
                if (part >= kSubs) return false;
                int len = 1;
                while (part + len < kSubs && (static_cast<uint32_t>(sub >> (16 * (part + len))) & 0xFFFFu) == w) ++len;
                k0 = w & 2047u;
                m = (w >> 11) & 3u;
                jb = jbeg + part * kSub;
                nj = len * kSub;
                part += len;
                return true;
            };
            auto bands = [&](FewCtx &f, uint32_t m, uint32_t k0, const float *bd) {
                f.k0 = uniform(k0);
                if (m) {
#pragma unroll
                    for (int q = 0; q < kFewMax; ++q) {
                        const uint32_t e = min(k0 + static_cast<uint32_t>(q), static_cast<uint32_t>(n_edges - 1));
                        few_band_fused(f, q, ld_const_f2(bd + 2u * e));
                    }
                    few_fused_ref(f);
                }
            };
            if (use_gram) {
                // not a diagonal tile; i slots past a ragged end are -infinity
                const double4 o = ld_const(sd.jb + u);
                GramI g;
                if (!PC_EARLY_GRAM) load_gi();
                centre_i_gram(g, gi, i_lim, o.x, o.y, o.z);
                uint32_t m, k0;
                int64_t jb;
                int32_t nj;
                for (int part = 0; next_run(part, m, k0, jb, nj);) {
                    FewCtx f;
                    bands(f, m, k0, fband_g);
                    const float4 *Jg = uniform_ptr(sd.jg + jb);
                    const double4 *J64p = uniform_ptr(sd.j64 + jb);
                    if (m == 1) tile32_gram<1>(lds, Jg, J64p, nj, g, sd.i64, ibeg, k, f);
                    else if (m == 2) tile32_gram<2>(lds, Jg, J64p, nj, g, sd.i64, ibeg, k, f);
                    else tile32_gram<3>(lds, Jg, J64p, nj, g, sd.i64, ibeg, k, f);
                }
            } else {
                uint32_t m, k0;
                int64_t jb;
                int32_t nj;
                for (int part = 0; next_run(part, m, k0, jb, nj);) {
                    FewCtx f;
                    bands(f, m, k0, fband);
                    const float4 *Jt = uniform_ptr(sd.j32 + jb);
                    const double4 *J64p = uniform_ptr(sd.j64 + jb);
                    if (m == 1) tile32_few<false, 1>(lds, Jt, J64p, nj, fx, fy, fz, sd.i64, ibeg, i_lim, j_rel, false, k, f);
                    else if (m == 2) tile32_few<false, 2>(lds, Jt, J64p, nj, fx, fy, fz, sd.i64, ibeg, i_lim, j_rel, false, k, f);
                    else if (m == 3) tile32_few<false, 3>(lds, Jt, J64p, nj, fx, fy, fz, sd.i64, ibeg, i_lim, j_rel, false, k, f);
                    else tile32<false, CT>(lds, Jt, J64p, nj, fx, fy, fz, sd.i64, ibeg, i_lim, j_rel, false, k);
                }
            }
        }
    }
    if (cur_job >= 0) flush_hist(lds, n_edges + 1, cols, clear_words, cur_counts, p.rechecked);
}

hipError_t launch_count(bool fp64, bool mc, bool compact, const SegDesc *segs, int32_t n_segs, const TableDesc *tabs,
                        const uint64_t *items, const unsigned long long *n_items, const uint64_t *sub,
                        uint64_t total_items, uint32_t lut_lds_off, uint32_t stage_lds_off,
                        unsigned long long *queue, unsigned long long *rechecked, int chunk, uint32_t lds_bytes,
                        int grid, uint64_t flush_cap, hipStream_t st) {
    KParams p;
    p.flush_cap = flush_cap;
    p.queue = queue;
    p.rechecked = rechecked;
    p.chunk = static_cast<uint32_t>(chunk);
    p.segs = segs;
    p.tabs = tabs;
    p.items = items;
    p.n_items = n_items;
    p.sub = sub;
    p.total_items = total_items;
    p.n_segs = n_segs;
    p.lut_lds_off = lut_lds_off;
    p.stage_lds_off = stage_lds_off;
    if (fp64)
        k_count<true, false><<<dim3(grid), dim3(kWave), lds_bytes, st>>>(p);
    else if (mc)
        k_count<false, kMatrixCores><<<dim3(grid), dim3(kWave), lds_bytes, st>>>(p);
    else if (compact)
        k_count<false, false, true><<<dim3(grid), dim3(kWave), lds_bytes, st>>>(p);
    else
        k_count<false, false><<<dim3(grid), dim3(kWave), lds_bytes, st>>>(p);
    return hipGetLastError();
}

hipError_t count_occupancy(bool fp64, bool mc, bool compact, uint32_t lds_bytes, int *blocks_per_cu) {
    if (fp64)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_count<true, false>, kWave, lds_bytes);
    if (mc)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_count<false, kMatrixCores>, kWave,
                                                             lds_bytes);
    if (compact)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_count<false, false, true>, kWave,
                                                             lds_bytes);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_count<false, false>, kWave, lds_bytes);
}

hipError_t set_max_lds(uint32_t bytes) {
    const void *fs[4] = {reinterpret_cast<const void *>(k_count<true, false>),
                         reinterpret_cast<const void *>(k_count<false, false>),
                         reinterpret_cast<const void *>(k_count<false, false, true>),
                         reinterpret_cast<const void *>(k_count<false, kMatrixCores>)};
    for (const void *f : fs) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace PC_TILE_NS

}  // namespace pc
