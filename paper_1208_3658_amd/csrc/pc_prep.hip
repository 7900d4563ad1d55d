// pc_prep.hip -- per-launch preparation kernels: spatial ordering of the
// catalogues, tile bounding spheres, and exact whole-tile-pair binning.
//
// Counts do not depend on the order of a catalogue, so each index range a job
// uses is copied in a spatial order (counting sort on a cube-face Hilbert key
// of the unit vector; the order inside a key bucket is arbitrary).  Consecutive
// tiles of 256 points are then compact, each gets a bounding sphere (centre,
// radius), and a tile pair whose squared-chord interval lies inside one bin
// is binned as a whole without visiting its pairs (the paper, Sec. 2.2: time
// is saved by not computing separations outside the binned range).
#include "pc_internal.hpp"

namespace pc {

#if PC_R == 4
// ------------------- tile-independent part (compiled once, 256-point build)


// ---------------------------------------------------------- ordering keys
// Cube-face Hilbert key: the face of the cube the unit vector points through
// (axis and sign of its largest component), then the 2-D Hilbert index of the
// two other components divided by the largest one, quantised to 2^bits per
// axis.  Points close on the sphere get close keys, without the long jumps of
// a Morton order.

__device__ __forceinline__ uint32_t quantize(double x, uint32_t bits) {
    // x in [-1, 1] -> [0, 2^bits)
    const double s = static_cast<double>(1u << bits) * 0.5;
    double q = (x + 1.0) * s;
    q = q < 0.0 ? 0.0 : q;
    uint32_t v = static_cast<uint32_t>(q);
    const uint32_t m = (1u << bits) - 1u;
    return v > m ? m : v;
}

__device__ __forceinline__ uint32_t hilbert2d(uint32_t bits, uint32_t x, uint32_t y) {
    const uint32_t n = 1u << bits;
    uint32_t d = 0;
    for (uint32_t s = n >> 1; s > 0; s >>= 1) {
        const uint32_t rx = (x & s) ? 1u : 0u;
        const uint32_t ry = (y & s) ? 1u : 0u;
        d += s * s * ((3u * rx) ^ ry);
        if (ry == 0u) {
            if (rx == 1u) {
                x = n - 1u - x;
                y = n - 1u - y;
            }
            const uint32_t t = x;
            x = y;
            y = t;
        }
    }
    return d;
}

__device__ __forceinline__ uint32_t order_key(double4 v, uint32_t bits) {
    const double ax = fabs(v.x), ay = fabs(v.y), az = fabs(v.z);
    uint32_t face;
    double major, u, w;
    if (ax >= ay && ax >= az) { face = 0; major = v.x; u = v.y; w = v.z; }
    else if (ay >= az) { face = 2; major = v.y; u = v.x; w = v.z; }
    else { face = 4; major = v.z; u = v.x; w = v.y; }
    if (major < 0.0) face += 1;
    const double inv = 1.0 / fmax(fabs(major), 1e-300);
    return (face << (2u * bits)) | hilbert2d(bits, quantize(u * inv, bits), quantize(w * inv, bits));
}

__global__ void __launch_bounds__(256) k_keys(const double4 *__restrict__ src, int64_t base, int64_t n,
                                              uint32_t bits, uint32_t *__restrict__ keys,
                                              uint32_t *__restrict__ hist) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = order_key(src[base + i], bits);
    keys[i] = k;
    atomicAdd(hist + k, 1u);
}

// ------------------------------------------------------------------ scan
// Exclusive prefix sum of m uint32 counters, in three passes: per-block
// scans (1024 values per block) with block totals, a scan of the totals,
// and the add-back.

constexpr int kScanBlock = 256;
constexpr int kScanPer = 4;
constexpr int kScanChunk = kScanBlock * kScanPer;

__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *sh, uint32_t *total) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        const uint32_t x = t >= off ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += x;
        __syncthreads();
    }
    const uint32_t incl = sh[t];
    if (total) *total = sh[kScanBlock - 1];
    __syncthreads();
    return incl - v;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_local(uint32_t *__restrict__ a, int64_t m,
                                                           uint32_t *__restrict__ block_sums) {
    __shared__ uint32_t sh[kScanBlock];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanChunk + threadIdx.x * kScanPer;
    uint32_t v[kScanPer];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        v[k] = base + k < m ? a[base + k] : 0u;
        s += v[k];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, sh, &total);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < m) a[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_sums(uint32_t *__restrict__ s, int64_t nb) {
    __shared__ uint32_t sh[kScanBlock];
    uint32_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kScanBlock) {
        const int64_t i = b0 + threadIdx.x;
        const uint32_t v = i < nb ? s[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_exclusive_scan(v, sh, &total);
        if (i < nb) s[i] = ex + carry;
        carry += total;
    }
}

__global__ void __launch_bounds__(kScanBlock) k_scan_add(uint32_t *__restrict__ a, int64_t m,
                                                         const uint32_t *__restrict__ block_sums) {
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanChunk + threadIdx.x * kScanPer;
    const uint32_t add = block_sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanPer; ++k)
        if (base + k < m) a[base + k] += add;
}

// --------------------------------------------------------------- scatter

__global__ void __launch_bounds__(256) k_scatter(const double4 *__restrict__ src, int64_t base, int64_t n,
                                                 const uint32_t *__restrict__ keys,
                                                 uint32_t *__restrict__ cursor, double4 *__restrict__ a64s,
                                                 float4 *__restrict__ a32s) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t pos = atomicAdd(cursor + keys[i], 1u);
    const double4 v = src[base + i];
    a64s[pos] = v;
    a32s[pos] = make_float4(static_cast<float>(v.x), static_cast<float>(v.y), static_cast<float>(v.z), 0.0f);
}

// --------------------------------------------------------------- launchers

__global__ void __launch_bounds__(256) k_zero_u32(uint32_t *p, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Key bits per face axis for n points: 4^(bits+1) * 4 <= n, between 2 and 9
// (at most 6 * 4^9 buckets).
uint32_t order_bits(int64_t n) {
    uint32_t b = 2;
    while (b < 9 && (int64_t(1) << (2 * (b + 1))) * 4 <= n) ++b;
    return b;
}

static int64_t n_buckets(uint32_t bits) { return int64_t(6) << (2 * bits); }

size_t sort_scratch_words(int64_t n) {
    const int64_t m = n_buckets(order_bits(n));
    return static_cast<size_t>(n + m + (m + kScanChunk - 1) / kScanChunk + 64);
}

size_t scan_sums_words(int64_t m) { return static_cast<size_t>((m + kScanChunk - 1) / kScanChunk); }

hipError_t launch_zero_u32(uint32_t *p, int64_t m, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    k_zero_u32<<<dim3(static_cast<uint32_t>((m + 255) / 256)), dim3(256), 0, st>>>(p, m);
    return hipGetLastError();
}

// dst[w] += sum over s < n_copies of src[s * n + w], w < n (one thread per word)
__global__ void __launch_bounds__(256) k_add_copies(unsigned long long *__restrict__ dst,
                                                    const unsigned long long *__restrict__ src, int64_t n,
                                                    int32_t n_copies) {
    const int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (w >= n) return;
    unsigned long long v = 0;
    for (int32_t s = 0; s < n_copies; ++s) v += src[static_cast<int64_t>(s) * n + w];
    dst[w] += v;
}

hipError_t launch_add_copies(unsigned long long *dst, const unsigned long long *src, int64_t n, int32_t n_copies,
                             hipStream_t st) {
    if (n <= 0 || n_copies <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    k_add_copies<<<dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, st>>>(dst, src, n, n_copies);
    return hipGetLastError();
}

// In-place exclusive prefix sum of a[0, m); sums: scan_sums_words(m) words.
hipError_t launch_exclusive_scan(uint32_t *a, int64_t m, uint32_t *sums, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    const int64_t nb = (m + kScanChunk - 1) / kScanChunk;
    k_scan_local<<<dim3(static_cast<uint32_t>(nb)), dim3(kScanBlock), 0, st>>>(a, m, sums);
    k_scan_sums<<<dim3(1), dim3(kScanBlock), 0, st>>>(sums, nb);
    k_scan_add<<<dim3(static_cast<uint32_t>(nb)), dim3(kScanBlock), 0, st>>>(a, m, sums);
    return hipGetLastError();
}

// Spatially ordered copy of src[base, base+n) into a64s/a32s, and the tile
// bounds: bounds[0, T) for the T tiles, then bounds[T, T + kSubs T) for their
// sub-blocks.  scratch: sort_scratch_words(n) uint32 words.
hipError_t launch_order(const double4 *src, int64_t base, int64_t n, uint32_t *scratch, double4 *a64s,
                        float4 *a32s, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const uint32_t bits = order_bits(n);
    const int64_t m = n_buckets(bits);
    const int64_t nb = (m + kScanChunk - 1) / kScanChunk;
    uint32_t *keys = scratch;
    uint32_t *hist = scratch + n;
    uint32_t *sums = hist + m;
    const uint32_t gn = static_cast<uint32_t>((n + 255) / 256);
    k_zero_u32<<<dim3(static_cast<uint32_t>((m + 255) / 256)), dim3(256), 0, st>>>(hist, m);
    k_keys<<<dim3(gn), dim3(256), 0, st>>>(src, base, n, bits, keys, hist);
    k_scan_local<<<dim3(static_cast<uint32_t>(nb)), dim3(kScanBlock), 0, st>>>(hist, m, sums);
    k_scan_sums<<<dim3(1), dim3(kScanBlock), 0, st>>>(sums, nb);
    k_scan_add<<<dim3(static_cast<uint32_t>(nb)), dim3(kScanBlock), 0, st>>>(hist, m, sums);
    k_scatter<<<dim3(gn), dim3(256), 0, st>>>(src, base, n, keys, hist, a64s, a32s);
    return hipGetLastError();
}

#else
// tile-independent steps, compiled once (with the 256-point instance)
size_t sort_scratch_words(int64_t n);
hipError_t launch_order(const double4 *src, int64_t base, int64_t n, uint32_t *scratch, double4 *a64s,
                        float4 *a32s, hipStream_t st);
#endif  // tile-independent part

// ------------------------------------------------ per tile size

namespace PC_TILE_NS {

// ---------------------------------------------------------------- bounds

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

// One wave per tile of kTile sorted points: centre = normalised mean, radius
// = largest distance from the centre, rounded outward.  Written as
// (cx, cy, cz, r).  The same for each of the tile's kSubs sub-blocks of kSub
// points (the r-th point of every lane: sub-block r), into sub[kSubs t + r].
// Each point is also written in Gram form centred on the tile's centre:
// b' = RN32(b - c) (difference in binary64), (-2 b'_x, -2 b'_y, -2 b'_z,
// |b'|^2) with |b'|^2 formed in binary32 as z*z + (y*y + x*x) by fused
// multiply-adds.
__device__ __forceinline__ double4 ball_of(const double4 *p, const bool *ok, int rows, double sx, double sy,
                                           double sz, double4 fallback) {
    const double norm = sqrt(sx * sx + sy * sy + sz * sz);
    double cx, cy, cz;
    if (norm > 1e-6) {
        cx = sx / norm;
        cy = sy / norm;
        cz = sz / norm;
    } else {
        cx = fallback.x;
        cy = fallback.y;
        cz = fallback.z;
    }
    double m = 0.0;
    for (int r = 0; r < rows; ++r) {
        if (ok[r]) {
            const double dx = p[r].x - cx, dy = p[r].y - cy, dz = p[r].z - cz;
            m = fmax(m, dx * dx + dy * dy + dz * dz);
        }
    }
    m = wave_max(m);
    return make_double4(cx, cy, cz, sqrt(m) * (1.0 + 0x1p-40) + 0x1p-60);
}

__global__ void __launch_bounds__(kWave) k_bounds(const double4 *__restrict__ a64s, int64_t n,
                                                  double4 *__restrict__ bounds, double4 *__restrict__ sub,
                                                  float4 *__restrict__ g32s) {
    static_assert(kSub == kWave, "a sub-block is one point per lane");
    const int64_t t = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t b = t * kTile;
    double sx = 0, sy = 0, sz = 0;
    double4 p[kR];
    bool ok[kR];
    double4 rs[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int64_t i = b + r * kWave + lane;
        ok[r] = i < n;
        p[r] = a64s[ok[r] ? i : b];
        // every lane takes part in the reductions; lanes past the end add 0
        rs[r] = make_double4(wave_sum(ok[r] ? p[r].x : 0.0), wave_sum(ok[r] ? p[r].y : 0.0),
                             wave_sum(ok[r] ? p[r].z : 0.0), 0.0);
        sx += rs[r].x;
        sy += rs[r].y;
        sz += rs[r].z;
    }
    const double4 first = a64s[b];
    const double4 tb = ball_of(p, ok, kR, sx, sy, sz, first);
    if (lane == 0) bounds[t] = tb;
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        // an empty sub-block (past a ragged end) gets the tile's ball; it is
        // never split from
        const bool any = __ballot(ok[r]) != 0ull;
        const double4 sb = any ? ball_of(&p[r], &ok[r], 1, rs[r].x, rs[r].y, rs[r].z, first) : tb;
        if (lane == 0) sub[t * kSubs + r] = sb;
    }
    const double cx = tb.x, cy = tb.y, cz = tb.z;
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        if (ok[r]) {
            const float x = static_cast<float>(p[r].x - cx);
            const float y = static_cast<float>(p[r].y - cy);
            const float z = static_cast<float>(p[r].z - cz);
            g32s[b + r * kWave + lane] =
                make_float4(-2.0f * x, -2.0f * y, -2.0f * z, __builtin_fmaf(z, z, __builtin_fmaf(y, y, x * x)));
        }
    }
}

// ----------------------------------------------------------------- prune


template <typename P>
__device__ __forceinline__ uint32_t count_le(P e, int32_t n, double c) {
    int32_t lo = 0, hi = n;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (e[mid] <= c) lo = mid + 1;
        else hi = mid;
    }
    return static_cast<uint32_t>(lo);
}

// The prune decision for one tile pair.  The chord of every pair of a tile
// pair lies in [d - rI - rJ, d + rI + rJ] (triangle inequality in R^3, d =
// distance of the centres); when the squared interval, widened by 1e-12
// relative for the rounding of these bounds and of the binary64 chord itself,
// sits inside one bin, all the item's pairs belong to that bin (bin >= 0).
// Otherwise the item survives (bin = -1) with its tags: k0 = edges at or below
// the interval, m = edges inside (kept when m <= PC_FEWCUT), and the Gram /
// matrix-core eligibility.
struct PruneOut {
    int32_t bin;
    uint64_t pairs;
    uint64_t tags;  // bits 40..63 of the survivor entry
    uint64_t sub;   // sub-block word of a split item, else 0
};

// Squared-chord interval of the pairs between two balls (centre, radius):
// [c_lo, c_hi], and the chord lower bound lo.
__device__ __forceinline__ void chord_interval(const double4 &bi, const double4 &bj, double &lo, double &c_lo,
                                               double &c_hi) {
    // outward-rounded bounds: distance of the centres (+-2^-45 relative),
    // radii (+2^-45), absolute 2^-50 for the subtraction, then the squared
    // chord interval widened by 1e-12 relative and 1e-300 absolute
    const double dx = bi.x - bj.x, dy = bi.y - bj.y, dz = bi.z - bj.z;
    const double d = sqrt(dx * dx + dy * dy + dz * dz);
    const double rs = (bi.w + bj.w) * (1.0 + 0x1p-45);
    lo = fmax(0.0, d * (1.0 - 0x1p-45) - rs - 0x1p-50);
    const double hi = d * (1.0 + 0x1p-45) + rs + 0x1p-50;
    // (a squared chord is never negative, so an edge at 0 always lies at or
    // below the interval: few-edge items never hold it)
    c_lo = fmax(lo * lo * (1.0 - 1e-12) - 1e-300, 0.0);
    c_hi = hi * hi * (1.0 + 1e-12) + 1e-300;
}

// far_l: a chord length past the last edge, sqrt(e[n_edges - 1]) * (1 +
// 1e-12) in binary64.  A tile pair whose squared centre distance d2 exceeds
// (far_l + r_I + r_J)^2 (1 + 1e-12) has every chord past the last edge: the
// computed d2 is at most 5 ulp above the true squared distance D^2 and the
// bound at most 4 ulp below its value, so D - r_I - r_J > far_l (1 + 0.49e-12);
// every pair is at least that far apart, and its binary64 squared chord
// (5 ulp) stays above e[n_edges - 1].
template <typename P>
__device__ __forceinline__ PruneOut prune_item(const SegDesc &sd, int64_t t, int64_t u, const double4 &bi,
                                               const double4 &bj, P e, int32_t n_edges, double far_l,
                                               int32_t mfma_ok, int32_t split_ok) {
    PruneOut o;
    o.sub = 0;
    const int64_t ni = min<int64_t>(kTile, sd.ni - t * kTile);
    const int64_t nj = min<int64_t>(kTile, sd.nj - u * kTile);
    const bool diag = sd.tri && t == u;
    o.pairs = diag ? static_cast<uint64_t>(ni * (ni - 1) / 2) : static_cast<uint64_t>(ni * nj);
    {
        // past the last edge without the square root (most tile pairs of a
        // wide field)
        const double dx = bi.x - bj.x, dy = bi.y - bj.y, dz = bi.z - bj.z;
        const double reach = far_l + (bi.w + bj.w);
        if (dx * dx + dy * dy + dz * dz > reach * reach * (1.0 + 1e-12)) {
            o.bin = n_edges;
            o.tags = 0;
            return o;
        }
    }
    double lo, c_lo, c_hi;
    chord_interval(bi, bj, lo, c_lo, c_hi);
    if (c_lo > e[n_edges - 1]) {
        // the whole interval lies past the last edge (most tile pairs of a
        // wide field): the bin above it, without the two searches
        o.bin = n_edges;
        o.tags = 0;
        return o;
    }
    const uint32_t k_lo = count_le(e, n_edges, c_lo);
    const uint32_t k_hi = count_le(e, n_edges, c_hi);
    if (k_lo == k_hi) {
        o.bin = static_cast<int32_t>(k_lo);
        o.tags = 0;
        return o;
    }
    o.bin = -1;
    // edges inside the interval: k_lo .. k_hi-1; few of them are compared one
    // by one instead of through the cell table
    const uint32_t m = k_hi - k_lo;
    static_assert(PC_FEWCUT >= 1 && PC_FEWCUT <= kFewMax, "few-edge cut");
    const bool is_few = m <= static_cast<uint32_t>(PC_FEWCUT);
    // few-edge full tiles whose chord lower bound is at least twice the
    // smaller bounding radius: eligible for the matrix-core path (bit 63),
    // centred on the j-tile when that one is smaller (bit 62); otherwise the
    // vector path forms Gram chords centred on the j-tile (bit 61) under the
    // same condition on the j radius
    const bool full = ni == kTile && nj == kTile;
    const bool mfma = mfma_ok && is_few && !diag && full && 2.0 * fmin(bi.w, bj.w) <= lo;
    const bool gram_j = !mfma && is_few && !diag && 2.0 * bj.w <= lo;
    o.tags = (static_cast<uint64_t>(k_lo) << kItemBits) |
             (static_cast<uint64_t>(is_few ? m : 0u) << (kItemBits + 11)) | (mfma ? (1ull << 63) : 0ull) |
             ((mfma && bj.w < bi.w) ? (1ull << 62) : 0ull) | (gram_j ? (1ull << 61) : 0ull);
    if (split_ok && !mfma && !diag && full) {
        // the same decision for each sub-block of the j-tile; the Gram form
        // stays centred on the whole j-tile, so its condition keeps the
        // j-tile's radius against the sub-block's chord lower bound
        uint64_t w = 0;
#pragma unroll
        for (int s = 0; s < kSubs; ++s) {
            const double4 bs = sd.jb_sub[u * kSubs + s];
            double lo_s, cl, ch;
            chord_interval(bi, bs, lo_s, cl, ch);
            const uint32_t kl = count_le(e, n_edges, cl);
            const uint32_t kh = count_le(e, n_edges, ch);
            uint32_t f;
            if (kl == kh) {
                f = kl | kSubWhole;
            } else {
                const uint32_t ms = kh - kl;
                const bool few = ms <= static_cast<uint32_t>(PC_FEWCUT);
                f = kl | ((few ? ms : 0u) << 11) | ((few && 2.0 * bj.w <= lo_s) ? kSubGram : 0u);
            }
            w |= static_cast<uint64_t>(f) << (16 * s);
        }
        o.sub = w;
        o.tags |= 1ull << kSplitBit;
    }
    return o;
}

// Sub-blocks of a split item left for the counting kernel.
__device__ __forceinline__ uint32_t open_subs(uint64_t w) {
    uint32_t n = 0;
#pragma unroll
    for (int s = 0; s < kSubs; ++s) n += (((w >> (16 * s)) & kSubWhole) == 0u) ? 1u : 0u;
    return n;
}

// (t, u) and item number of column c of prune row r (map_item's fold for a
// triangle: row r holds (r, r..T-1) then (T-1-r, T-1-r..T-1))
__device__ __forceinline__ bool row_item(const SegDesc &sd, int64_t r, int64_t c, int64_t &t, int64_t &u,
                                         uint64_t &q) {
    const int64_t T = sd.tiles_i;
    if (sd.tri) {
        q = static_cast<uint64_t>(r * (T + 1) + c);
        if (c < T - r) {
            t = r;
            u = r + c;
        } else {
            t = T - 1 - r;
            u = t + (c - (T - r));
        }
        return c < T + 1 && q < sd.n_items;
    }
    t = r;
    u = c;
    q = static_cast<uint64_t>(r * sd.tiles_j + c);
    return c < sd.tiles_j;
}

constexpr int kPruneThreads = 256;     // threads per prune workgroup
constexpr int kPruneMaskSteps = 128;  // steps of 256 columns whose survivor ballots are kept (4 KB)

// Column c of prune row r with the bounds of its two tiles; a column past the
// row's end (valid false) loads the bounds of tile 0, which every segment has.
struct PruneCol {
    int64_t t, u;
    uint64_t q;
    bool valid;
    double4 bi, bj;
};

__device__ __forceinline__ void load_col(const SegDesc &sd, int64_t r, int64_t c, PruneCol &k) {
    k.valid = row_item(sd, r, c, k.t, k.u, k.q);
    k.bi = sd.ib[k.valid ? k.t : 0];
    k.bj = sd.jb[k.valid ? k.u : 0];
}

// One workgroup per row of tile pairs (one i-tile, or the two i-tiles of a
// folded triangle row), threads across its columns: (t, u) and the item
// number come without divisions, and the edges of the row's table sit in LDS.
// Whole tile pairs are added to an LDS histogram and survivors counted in a
// first pass; the workgroup then reserves its survivors' slots with one global
// atomic and writes them in a second pass (the decision is recomputed), and
// flushes its histogram and statistics with one atomic per non-zero entry --
// global atomics on a few shared counters would otherwise serialise the pass.
__global__ void __launch_bounds__(kPruneThreads) k_prune(const SegDesc *__restrict__ segs, int32_t n_segs,
                                               const TableDesc *__restrict__ tabs,
                                               uint64_t *__restrict__ survivors, uint64_t *__restrict__ sub_out,
                                               unsigned long long *__restrict__ meta, int32_t mfma_ok,
                                               int32_t split_ok) {
    // meta[0] = survivors (the slot counter).  Statistics, summed over the
    // kPruneStripes stripes at meta[kPruneStatBase + stripe * kPruneStripeWords
    // + k] (k as in s_stat): k = 1 pairs left for the counting kernel, 2
    // survivors marked for the matrix cores; work units (a survivor, or an
    // open sub-block of a split one): 3 with at most PC_FEWCUT edges in their
    // chord interval, 4 with vector-path chords in Gram form; 5 split
    // survivors; pairs left for the counting kernel by the path it takes them
    // through (the same decisions as k_count): 6 + m binned against m edges
    // one by one (m = 1..3), 6 through the cell table; 10 pairs whose chords
    // the vector path forms in Gram form, 11 pairs on the matrix cores.
    __shared__ double e_lds[kMaxEdges];
    __shared__ unsigned long long h_lds[kMaxEdges + 1];
    // survivors, pairs, matrix-core, few-edge, Gram, split; pairs by m (4),
    // Gram-form pairs, matrix-core pairs
    static_assert(kPruneStats <= kPruneStripeWords, "statistics per stripe");
    constexpr int kStats = kPruneStats;
    __shared__ unsigned long long s_stat[kStats];
    __shared__ unsigned long long s_base;
    __shared__ unsigned int s_cursor;
    // survivor ballots of the first kPruneMaskSteps steps of each wave
    __shared__ uint64_t s_mask[kPruneMaskSteps][kPruneThreads / kWave];
    const int64_t row_g = blockIdx.x;
    int s = 0;  // last segment with prow0 <= row_g
    {
        int lo = 0, hi = n_segs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (segs[mid].prow0 <= row_g) lo = mid;
            else hi = mid - 1;
        }
        s = lo;
    }
    const SegDesc &sd = segs[s];
    const TableDesc &td = tabs[sd.tab];
    const int32_t n_edges = td.n_edges;
    const int tid = static_cast<int>(threadIdx.x);
    const int lane = tid & (kWave - 1);
    for (int32_t k = tid; k < n_edges; k += blockDim.x) e_lds[k] = td.e64[k];
    for (int32_t k = tid; k <= n_edges; k += blockDim.x) h_lds[k] = 0ull;
    if (tid < kStats) s_stat[tid] = 0ull;
    if (tid == 0) s_cursor = 0u;
    __syncthreads();
    const int64_t r = row_g - sd.prow0;
    const int64_t cols = sd.tri ? sd.tiles_i + 1 : sd.tiles_j;
    const double far_l = sqrt(e_lds[n_edges - 1]) * (1.0 + 1e-12);
    constexpr unsigned long long kSubPairs = static_cast<unsigned long long>(kTile) * kSub;

    // pass 1: histogram of whole tile pairs and sub-blocks, statistics of
    // survivors.  Whole tile pairs past the last edge (most of them in a wide
    // field) and the statistics add up in registers over the row and are
    // reduced once at its end; other whole tile pairs go to the LDS histogram.
    unsigned long long above = 0;
    // survivors, pairs left, matrix-core items, few-edge work units, Gram
    // work units, split items; pairs by the counting kernel's path: by edges
    // compared one by one (index m, 0 = cell table), Gram-form chords, matrix
    // cores (the layout of s_stat)
    unsigned long long st[kStats];
#pragma unroll
    for (int k = 0; k < kStats; ++k) st[k] = 0ull;
    // the next column's tiles load while this one is judged; each wave keeps
    // the ballot of its survivors per step for the second pass
    PruneCol cur, nxt;
    load_col(sd, r, tid, cur);
    nxt = cur;
    const int wave = tid / kWave;
    for (int64_t c0 = 0, it = 0; c0 < cols; c0 += kPruneThreads, ++it) {
        if (c0 + kPruneThreads < cols) load_col(sd, r, c0 + kPruneThreads + tid, nxt);
        bool survive = false;
        if (cur.valid) {
            const PruneOut o = prune_item(sd, cur.t, cur.u, cur.bi, cur.bj, e_lds, n_edges, far_l, mfma_ok, split_ok);
            survive = o.bin < 0;
            if (o.bin == n_edges) {
                above += o.pairs;
            } else if (o.bin >= 0) {
                atomicAdd(&h_lds[o.bin], static_cast<unsigned long long>(o.pairs));
            } else if (o.sub) {
                // the kernel forms a split item's chords in Gram form when
                // every open sub-block allows it
                bool gram_all = true;
#pragma unroll
                for (int k = 0; k < kSubs; ++k) {
                    const uint32_t f = static_cast<uint32_t>(o.sub >> (16 * k)) & 0xFFFFu;
                    if (!(f & kSubWhole) && !(f & kSubGram)) gram_all = false;
                }
                unsigned long long left = 0;
#pragma unroll
                for (int k = 0; k < kSubs; ++k) {
                    const uint32_t f = static_cast<uint32_t>(o.sub >> (16 * k)) & 0xFFFFu;
                    if (f & kSubWhole) {
                        atomicAdd(&h_lds[f & 2047u], kSubPairs);
                    } else {
                        const uint32_t m = (f >> 11) & 3u;
                        left += kSubPairs;
                        st[3] += m != 0u ? 1ull : 0ull;
                        st[4] += (f & kSubGram) != 0u ? 1ull : 0ull;
                        st[6 + m] += kSubPairs;
                        st[10] += gram_all ? kSubPairs : 0ull;
                    }
                }
                st[0] += left != 0 ? 1ull : 0ull;
                st[1] += left;
                st[5] += left != 0 ? 1ull : 0ull;
                survive = left != 0;
            } else {
                const uint32_t m = static_cast<uint32_t>((o.tags >> (kItemBits + 11)) & 3u);
                const bool mc = (o.tags >> 63) != 0;
                const bool gram = ((o.tags >> 61) & 1u) != 0;
                st[0] += 1ull;
                st[1] += o.pairs;
                st[2] += mc ? 1ull : 0ull;
                st[3] += m != 0u ? 1ull : 0ull;
                st[4] += gram ? 1ull : 0ull;
                st[6 + m] += o.pairs;
                st[10] += (!mc && gram && m != 0u) ? o.pairs : 0ull;
                st[11] += mc ? o.pairs : 0ull;
            }
        }
        const uint64_t sm = __ballot(survive);
        if (it < kPruneMaskSteps && lane == 0) s_mask[it][wave] = sm;
        cur = nxt;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        above += __shfl_xor(above, o, kWave);
#pragma unroll
        for (int k = 0; k < kStats; ++k) st[k] += __shfl_xor(st[k], o, kWave);
    }
    if (lane == 0) {
        if (above) atomicAdd(&h_lds[n_edges], above);
#pragma unroll
        for (int k = 0; k < kStats; ++k)
            if (st[k]) atomicAdd(&s_stat[k], st[k]);
    }
    __syncthreads();
    if (tid == 0) s_base = s_stat[0] ? atomicAdd(meta + 0, s_stat[0]) : 0ull;
    __syncthreads();

    // pass 2: the survivors, written into the workgroup's reserved slots
    if (s_stat[0]) {
        const int wave = tid / kWave;
        for (int64_t c0 = 0, it = 0; c0 < cols; c0 += kPruneThreads, ++it) {
            // steps whose ballot the first pass kept: only their survivors
            // are judged again
            const uint64_t kept = it < kPruneMaskSteps ? s_mask[it][wave] : ~0ull;
            if (kept == 0) continue;
            bool survive = false;
            uint64_t tags = 0, sub = 0, q = 0;
            if ((kept >> lane) & 1u) {
                PruneCol k;
                load_col(sd, r, c0 + tid, k);
                if (k.valid) {
                    const PruneOut o = prune_item(sd, k.t, k.u, k.bi, k.bj, e_lds, n_edges, far_l, mfma_ok, split_ok);
                    survive = o.bin < 0 && (o.sub == 0 || open_subs(o.sub) != 0);
                    tags = o.tags;
                    sub = o.sub;
                    q = k.q;
                }
            }
            const uint64_t sm = __ballot(survive);
            if (sm) {
                const uint64_t below = sm & ((lane == 0) ? 0ull : (~0ull >> (kWave - lane)));
                unsigned int at = 0;
                if (lane == __ffsll(static_cast<long long>(sm)) - 1)
                    at = atomicAdd(&s_cursor, static_cast<unsigned int>(__popcll(sm)));
                at = __shfl(at, __ffsll(static_cast<long long>(sm)) - 1, kWave);
                if (survive) {
                    const uint64_t slot = s_base + at + __popcll(below);
                    survivors[slot] = (sd.item0 + q) | tags;
                    if (sub_out) sub_out[slot] = sub;
                }
            }
        }
    }

    // flush: one atomic per non-zero bin and per statistic, into one of
    // kPruneStripes copies (by workgroup) of the counters and statistics
    unsigned long long *pc = sd.pcounts + static_cast<int64_t>(blockIdx.x % kPruneStripes) * sd.pstride;
    for (int32_t k = tid; k <= n_edges; k += blockDim.x) {
        const unsigned long long v = h_lds[k];
        if (v) atomicAdd(pc + k, v);
    }
    if (tid > 0 && tid < kStats && s_stat[0] && s_stat[tid])
        atomicAdd(meta + kPruneStatBase + (blockIdx.x % kPruneStripes) * kPruneStripeWords + tid, s_stat[tid]);
}

// Spatially ordered copy of src[base, base+n) into a64s/a32s, and the tile
// bounds: bounds[0, T) for the T tiles, then bounds[T, T + kSubs T) for their
// sub-blocks, and the Gram-form copy g32s.  scratch: sort_scratch_words(n)
// uint32 words.
hipError_t launch_sort(const double4 *src, int64_t base, int64_t n, uint32_t *scratch, double4 *a64s,
                       float4 *a32s, float4 *g32s, double4 *bounds, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipError_t e = launch_order(src, base, n, scratch, a64s, a32s, st);
    if (e != hipSuccess) return e;
    const int64_t tiles = (n + kTile - 1) / kTile;
    k_bounds<<<dim3(static_cast<uint32_t>(tiles)), dim3(kWave), 0, st>>>(a64s, n, bounds, bounds + tiles, g32s);
    return hipGetLastError();
}

hipError_t launch_prune(const SegDesc *segs, int32_t n_segs, const TableDesc *tabs, int64_t total_rows,
                        uint64_t *survivors, uint64_t *sub, unsigned long long *meta, int32_t mfma_ok,
                        int32_t split_ok, hipStream_t st) {
    if (total_rows <= 0) return hipSuccess;
    if (total_rows > 0x7FFFFFFF) return hipErrorInvalidValue;
    k_prune<<<dim3(static_cast<uint32_t>(total_rows)), dim3(kPruneThreads), 0, st>>>(segs, n_segs, tabs, survivors, sub, meta,
                                                                          mfma_ok, split_ok);
    return hipGetLastError();
}

}  // namespace PC_TILE_NS

}  // namespace pc
