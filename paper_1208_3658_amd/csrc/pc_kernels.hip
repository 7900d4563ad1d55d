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
//     table for the current edge set and a histogram with one column per lane
//     (no two lanes ever add to the same LDS word, so the paper's same-bin
//     atomic contention, Sec. 2.1, cannot arise), flushed into 64-bit global
//     counters when the job changes and at the end.
#include "pc_internal.hpp"
#include "pc_math.h"

namespace pc {

struct KParams {
    const SegDesc *segs;
    const TableDesc *tabs;
    const uint64_t *items;                 // work items to visit (survivors), or null: all items
    const unsigned long long *n_items;     // device count of `items`
    uint64_t total_items;                  // number of items when `items` is null
    int32_t n_segs;
    uint32_t lut_lds_off;  // byte offset of the cell table in LDS (after the histogram)
};

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

// ------------------------------------------------------------ helpers

// Loads through the constant address space: the addresses below are the
// same for every lane, so these become scalar loads (the data is read-only
// for the whole launch).
__device__ __forceinline__ float4 ld_const(const float4 *p) {
    using CF = const __attribute__((address_space(4))) float;
    CF *q = (CF *)(p);
    return make_float4(q[0], q[1], q[2], q[3]);
}

__device__ __forceinline__ double4 ld_const(const double4 *p) {
    using CD = const __attribute__((address_space(4))) double;
    CD *q = (CD *)(p);
    return make_double4(q[0], q[1], q[2], q[3]);
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

__device__ __forceinline__ uint4 lds_read4(uint32_t addr) {
    const u32x4 v = *(lds_u4 *)(uintptr_t)(addr);
    return make_uint4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ uint32_t umed3(uint32_t x, uint32_t lo, uint32_t hi) {
    return min(max(x, lo), hi);
}

// Sum the histogram rows [0, n_rows) over the lane columns into the job's
// 64-bit counters, then clear every row (including the discard row).  Lane r
// sums row r, visiting the columns in a lane-rotated order so that the lanes
// of one read touch distinct banks.
__device__ void flush_hist(unsigned char *lds, int32_t n_rows, int32_t cols, int32_t clear_words,
                           unsigned long long *counts) {
    __syncthreads();
    const uint32_t lane = threadIdx.x;
    uint32_t *h = reinterpret_cast<uint32_t *>(lds);
    for (int32_t r = lane; r < n_rows; r += kWave) {
        unsigned long long s = 0;
        const uint32_t *row = h + r * cols;
        for (int c = 0; c < cols; ++c) s += row[(c + r) & (cols - 1)];
        if (s) atomicAdd(counts + r, s);
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

// LDS byte address of the cell-table entry for key: ((key >> shift) << 4) + base
__device__ __forceinline__ uint32_t cell_addr(uint32_t key, uint32_t shift, uint32_t base) {
    uint32_t r;
    asm("v_lshl_add_u32 %0, %1, 4, %2" : "=v"(r) : "v"(key >> shift), "v"(base));
    return r;
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
    uint32_t shift, lut_base, lane_off, trash_off, row_bytes;
    float klo, khi;  // key clamp as floats
    int32_t n_edges;
    const double *e64;
};

#ifndef PC_JUNROLL
#define PC_JUNROLL 2        // j-points per inner iteration
#endif

// NJ consecutive j-points against the lane's kR i-points: all chords first,
// then all cell-table reads, then all histogram adds, so the LDS latency of
// NJ * kR lookups overlaps.  Slot r of lane l holds i = ibeg + r*64 + l.
template <bool MASKED, int NJ>
__device__ __forceinline__ void step32(unsigned char *lds, const float4 *__restrict__ Jt,
                                       const double4 *__restrict__ J64t, int32_t jj,
                                       const float (&ax)[kR], const float (&ay)[kR],
                                       const float (&az)[kR], const double4 *__restrict__ I64,
                                       int64_t ibeg, int32_t i_lim, int32_t j_rel, bool diag,
                                       const TileCtx &k) {
    const int32_t lane = static_cast<int32_t>(threadIdx.x);
    float4 b[NJ];
#pragma unroll
    for (int q = 0; q < NJ; ++q) b[q] = ld_const(Jt + jj + q);
    float c2[NJ][kR];
    uint32_t a[NJ][kR];
#pragma unroll
    for (int q = 0; q < NJ; ++q)
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            c2[q][r] = chord2_32(ax[r], ay[r], az[r], b[q]);
            a[q][r] = cell_addr(key32(c2[q][r], k.klo, k.khi), k.shift, k.lut_base);
        }
    uint4 e[NJ][kR];
#pragma unroll
    for (int q = 0; q < NJ; ++q)
#pragma unroll
        for (int r = 0; r < kR; ++r) e[q][r] = lds_read4(a[q][r]);
    bool any_band = false;
#pragma unroll
    for (int q = 0; q < NJ; ++q)
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const bool gt = c2[q][r] > __uint_as_float(e[q][r].w);
            const bool band = !gt & (c2[q][r] >= __uint_as_float(e[q][r].z));
            uint32_t off = (gt ? e[q][r].y : e[q][r].x) + k.lane_off;
            if (MASKED) {
                // i slot valid, and on a diagonal tile i < j (positions
                // relative to the tile start: i = r*64 + lane, j = j_rel + jj + q)
                const int32_t ir = r * kWave + lane;
                const bool ok = ir < i_lim && (!diag || ir < j_rel + jj + q);
                off = ok ? off : k.trash_off;
                any_band |= ok & band;
            } else {
                any_band |= band;
            }
            lds_add(lds, off, 1u);
        }
    if (__builtin_expect(any_band, 0)) {
        // rare: a binary32 chord is within the error band of an edge;
        // recompute such pairs in binary64 exactly as the reference does and
        // move their count from the provisional row to the exact one
#pragma unroll
        for (int q = 0; q < NJ; ++q) {
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                const float c = chord2_32(ax[r], ay[r], az[r], b[q]);
                const uint4 en = lds_read4(cell_addr(key32(c, k.klo, k.khi), k.shift, k.lut_base));
                bool band = !(c > __uint_as_float(en.w)) && (c >= __uint_as_float(en.z));
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
template <bool MASKED>
__device__ __forceinline__ void tile32(unsigned char *lds, const float4 *__restrict__ Jt,
                                       const double4 *__restrict__ J64t, int32_t jn,
                                       const float (&ax)[kR], const float (&ay)[kR],
                                       const float (&az)[kR], const double4 *__restrict__ I64,
                                       int64_t ibeg, int32_t i_lim, int32_t j_rel, bool diag,
                                       const TileCtx &k) {
    int32_t jj = 0;
    for (; jj + PC_JUNROLL <= jn; jj += PC_JUNROLL)
        step32<MASKED, PC_JUNROLL>(lds, Jt, J64t, jj, ax, ay, az, I64, ibeg, i_lim, j_rel, diag, k);
    for (; jj < jn; ++jj)
        step32<MASKED, 1>(lds, Jt, J64t, jj, ax, ay, az, I64, ibeg, i_lim, j_rel, diag, k);
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

#ifdef PC_WAVES_PER_EU
#define PC_OCCUPANCY __attribute__((amdgpu_waves_per_eu(PC_WAVES_PER_EU)))
#else
#define PC_OCCUPANCY
#endif

template <bool FP64>
__global__ void __launch_bounds__(kWave) PC_OCCUPANCY k_count(KParams p) {
    extern __shared__ __align__(16) unsigned char lds[];
    const uint32_t lds0 = lds_addr(lds);
    const uint32_t lane = threadIdx.x;
    const uint32_t nb = gridDim.x;
    const uint32_t b = blockIdx.x;
    // consecutive blocks land on different XCDs; give each XCD a contiguous
    // run of work items so its L2 sees neighbouring tiles
    const uint32_t w = (nb % 8u == 0u) ? (b % 8u) * (nb / 8u) + b / 8u : b;
    const uint64_t total = p.items ? static_cast<uint64_t>(*(const __attribute__((address_space(4))) unsigned long long *)(p.n_items))
                                   : p.total_items;
    const uint64_t per = total / nb, rem = total % nb;
    const uint64_t beg = per * w + min<uint64_t>(w, rem);
    const uint64_t end = beg + per + (w < rem ? 1u : 0u);
    if (beg >= end) return;

    const uint64_t it0 = p.items ? p.items[beg] : beg;
    int s = find_seg(p.segs, p.n_segs, it0);
    SegDesc sd = ld_const_struct(p.segs + s);
    int cur_tab = -1, cur_job = -1;
    int32_t n_edges = 0, cols = 64, clear_words = 0;
    uint32_t row_bytes = 0, lane_off = 0;
    unsigned long long *cur_counts = nullptr;
    uint32_t clo = 0, chi = 0, shift = 0, lut_base = 0, trash_off = 0;
    bool search = false;
    const double *e64 = nullptr;
    uint64_t since_flush = 0;

    int64_t cur_t = -1;
    int cur_t_seg = -1;
    float fx[kR], fy[kR], fz[kR];
    double dx[kR], dy[kR], dz[kR];

    for (uint64_t wi = beg; wi < end; ++wi) {
        const uint64_t it = p.items ? static_cast<uint64_t>(uniform_u64(p.items[wi])) : wi;
        if (it < sd.item0 || it >= sd.item0 + sd.n_items) {
            s = find_seg(p.segs, p.n_segs, it);
            sd = ld_const_struct(p.segs + s);
        }
        if (sd.tab != cur_tab || sd.job != cur_job || since_flush >= (1ull << 21)) {
            if (cur_job >= 0) flush_hist(lds, n_edges + 1, cols, clear_words, cur_counts);
            if (sd.tab != cur_tab) {
                const TableDesc td = ld_const_struct(p.tabs + sd.tab);
                n_edges = td.n_edges;
                clo = td.clamp_lo;
                chi = td.clamp_hi;
                shift = td.shift;
                search = td.search != 0;
                e64 = td.e64;
                cols = td.cols;
                row_bytes = static_cast<uint32_t>(cols) * 4u;
                // absolute LDS addresses: histogram at lds0, cell table at lds0 + lut_lds_off
                lane_off = lds0 + (lane & static_cast<uint32_t>(cols - 1)) * 4u;
                trash_off = static_cast<uint32_t>(n_edges + 1) * row_bytes + lane_off;
                lut_base = lds0 + p.lut_lds_off - (td.key0 << 4);
                // copy the cell table (or, for a search table, the edges) into LDS
                if (FP64 && search) {
                    lut_base = lds0 + p.lut_lds_off;
                    double *dst = reinterpret_cast<double *>(lds + p.lut_lds_off);
                    for (int32_t k = lane; k < n_edges; k += kWave) dst[k] = td.e64[k];
                } else {
                    const uint4 *src = reinterpret_cast<const uint4 *>(td.lut);
                    uint4 *dst = reinterpret_cast<uint4 *>(lds + p.lut_lds_off);
                    for (int32_t k = lane; k < td.n_cells; k += kWave) dst[k] = src[k];
                }
                // histogram words this table uses; anything beyond what was
                // cleared before is cleared now
                const int32_t words = (n_edges + 2) * cols;
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
        if (t != cur_t || s != cur_t_seg) {
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
            cur_t = t;
            cur_t_seg = s;
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
        } else {
            const float4 *Jt = uniform_ptr(sd.j32 + jbeg);
            if (masked)
                tile32<true>(lds, Jt, J64t, jn, fx, fy, fz, sd.i64, ibeg, i_lim, j_rel, diag, k);
            else
                tile32<false>(lds, Jt, J64t, jn, fx, fy, fz, sd.i64, ibeg, i_lim, j_rel, diag, k);
        }
    }
    flush_hist(lds, n_edges + 1, cols, clear_words, cur_counts);
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

hipError_t launch_count(bool fp64, const SegDesc *segs, int32_t n_segs, const TableDesc *tabs,
                        const uint64_t *items, const unsigned long long *n_items, uint64_t total_items,
                        uint32_t lut_lds_off, uint32_t lds_bytes, int grid, hipStream_t st) {
    KParams p;
    p.segs = segs;
    p.tabs = tabs;
    p.items = items;
    p.n_items = n_items;
    p.total_items = total_items;
    p.n_segs = n_segs;
    p.lut_lds_off = lut_lds_off;
    if (fp64)
        k_count<true><<<dim3(grid), dim3(kWave), lds_bytes, st>>>(p);
    else
        k_count<false><<<dim3(grid), dim3(kWave), lds_bytes, st>>>(p);
    return hipGetLastError();
}

hipError_t count_occupancy(bool fp64, uint32_t lds_bytes, int *blocks_per_cu) {
    if (fp64)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_count<true>, kWave, lds_bytes);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_count<false>, kWave, lds_bytes);
}

hipError_t set_max_lds(uint32_t bytes) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_count<true>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(k_count<false>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

}  // namespace pc
