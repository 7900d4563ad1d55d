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
// (cx, cy, cz, r).  Each point is also written in Gram form centred on that
// centre: b' = RN32(b - c) (difference in binary64), (-2 b'_x, -2 b'_y,
// -2 b'_z, |b'|^2) with |b'|^2 formed in binary32 as z*z + (y*y + x*x) by
// fused multiply-adds.
__global__ void __launch_bounds__(kWave) k_bounds(const double4 *__restrict__ a64s, int64_t n,
                                                  double4 *__restrict__ bounds, float4 *__restrict__ g32s) {
    const int64_t t = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t b = t * kTile;
    double sx = 0, sy = 0, sz = 0;
    double4 p[kR];
    bool ok[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int64_t i = b + r * kWave + lane;
        ok[r] = i < n;
        p[r] = a64s[ok[r] ? i : b];
        if (ok[r]) {
            sx += p[r].x;
            sy += p[r].y;
            sz += p[r].z;
        }
    }
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    sz = wave_sum(sz);
    const double norm = sqrt(sx * sx + sy * sy + sz * sz);
    double cx, cy, cz;
    if (norm > 1e-6) {
        cx = sx / norm;
        cy = sy / norm;
        cz = sz / norm;
    } else {
        const double4 f = a64s[b];
        cx = f.x;
        cy = f.y;
        cz = f.z;
    }
    double m = 0.0;
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        if (ok[r]) {
            const double dx = p[r].x - cx, dy = p[r].y - cy, dz = p[r].z - cz;
            m = fmax(m, dx * dx + dy * dy + dz * dz);
        }
    }
    m = wave_max(m);
    if (lane == 0) bounds[t] = make_double4(cx, cy, cz, sqrt(m) * (1.0 + 0x1p-40) + 0x1p-60);
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

__device__ __forceinline__ int find_seg_p(const SegDesc *segs, int n, uint64_t item) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].item0 <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ uint32_t count_le(const double *e, int32_t n, double c) {
    int32_t lo = 0, hi = n;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (e[mid] <= c) lo = mid + 1;
        else hi = mid;
    }
    return static_cast<uint32_t>(lo);
}

// One thread per work item.  The chord of every pair of a tile pair lies in
// [d - rI - rJ, d + rI + rJ] (triangle inequality in R^3, d = distance of the
// centres); when the squared interval, widened by 1e-12 relative for the
// rounding of these bounds and of the binary64 chord itself, sits inside one
// bin, all the item's pairs are added to that bin here.  Other items are
// appended to the survivor list.  Lanes adding to the same counter are summed
// first (one atomic per distinct counter per wave).
__global__ void __launch_bounds__(256) k_prune(const SegDesc *__restrict__ segs, int32_t n_segs,
                                               const TableDesc *__restrict__ tabs, uint64_t total_items,
                                               uint64_t *__restrict__ survivors,
                                               unsigned long long *__restrict__ meta, int32_t mfma_ok) {
    // meta[0] = survivors, meta[1] = pairs in survivors, meta[2] = pairs binned
    // whole, meta[3] = survivors marked for the matrix cores, meta[4] =
    // survivors with at most kFewMax edges in their chord interval, meta[5] =
    // survivors whose vector-path chords are formed in Gram form
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t base = static_cast<uint64_t>(blockIdx.x) * blockDim.x; base < total_items; base += stride) {
        const uint64_t it = base + threadIdx.x;
        const bool valid = it < total_items;
        unsigned long long *dst = nullptr;
        unsigned long long cnt = 0;
        bool survive = false;
        bool mfma = false, centre_j = false, gram_j = false;
        uint64_t pairs = 0, few = 0;
        if (valid) {
            const int s = find_seg_p(segs, n_segs, it);
            const SegDesc &sd = segs[s];
            const uint64_t q = it - sd.item0;
            int64_t t, u;
            if (sd.tri) {
                const int64_t T = sd.tiles_i;
                const int64_t r = static_cast<int64_t>(q / static_cast<uint64_t>(T + 1));
                const int64_t c = static_cast<int64_t>(q % static_cast<uint64_t>(T + 1));
                if (c < T - r) { t = r; u = r + c; }
                else { t = T - 1 - r; u = t + (c - (T - r)); }
            } else {
                t = static_cast<int64_t>(q / static_cast<uint64_t>(sd.tiles_j));
                u = static_cast<int64_t>(q % static_cast<uint64_t>(sd.tiles_j));
            }
            const int64_t ni = min<int64_t>(kTile, sd.ni - t * kTile);
            const int64_t nj = min<int64_t>(kTile, sd.nj - u * kTile);
            const bool diag = sd.tri && t == u;
            pairs = diag ? static_cast<uint64_t>(ni * (ni - 1) / 2) : static_cast<uint64_t>(ni * nj);
            const double4 bi = sd.ib[t];
            const double4 bj = sd.jb[u];
            // outward-rounded bounds: distance of the centres (+-2^-45 relative),
            // radii (+2^-45), absolute 2^-50 for the subtraction, then the squared
            // chord interval widened by 1e-12 relative and 1e-300 absolute
            const double dx = bi.x - bj.x, dy = bi.y - bj.y, dz = bi.z - bj.z;
            const double d = sqrt(dx * dx + dy * dy + dz * dz);
            const double rs = (bi.w + bj.w) * (1.0 + 0x1p-45);
            const double lo = fmax(0.0, d * (1.0 - 0x1p-45) - rs - 0x1p-50);
            const double hi = d * (1.0 + 0x1p-45) + rs + 0x1p-50;
            const double c_lo = lo * lo * (1.0 - 1e-12) - 1e-300;
            const double c_hi = hi * hi * (1.0 + 1e-12) + 1e-300;
            const TableDesc &td = tabs[sd.tab];
            const uint32_t k_lo = count_le(td.e64, td.n_edges, c_lo);
            const uint32_t k_hi = count_le(td.e64, td.n_edges, c_hi);
            if (k_lo == k_hi) {
                dst = sd.counts + k_lo;
                cnt = pairs;
            } else {
                survive = true;
                // edges inside the interval: k_lo .. k_hi-1; few of them are
                // compared one by one instead of through the cell table
                const uint32_t m = k_hi - k_lo;
                static_assert(PC_FEWCUT >= 1 && PC_FEWCUT <= kFewMax, "few-edge cut");
                const bool is_few = m <= static_cast<uint32_t>(PC_FEWCUT);
                few = (static_cast<uint64_t>(k_lo) << kItemBits) |
                      (static_cast<uint64_t>(is_few ? m : 0u) << (kItemBits + 11));
                // few-edge full tiles whose chord lower bound is at least twice
                // the smaller bounding radius: eligible for the matrix-core path
                // (bit 63), centred on the j-tile when that one is smaller
                // (bit 62)
                centre_j = bj.w < bi.w;
                mfma = mfma_ok && is_few && !diag && ni == kTile && nj == kTile && 2.0 * fmin(bi.w, bj.w) <= lo;
                // otherwise the vector path forms Gram chords centred on the
                // j-tile (bit 61) under the same condition on the j radius
                gram_j = !mfma && is_few && !diag && 2.0 * bj.w <= lo;
            }
        }
        // survivors: one atomic per wave
        const uint64_t sm = __ballot(survive);
        if (sm) {
            const int lane = threadIdx.x & (kWave - 1);
            const uint64_t below = sm & ((lane == 0) ? 0ull : (~0ull >> (kWave - lane)));
            unsigned long long at = 0;
            if (lane == __ffsll(static_cast<long long>(sm)) - 1) {
                at = atomicAdd(meta + 0, static_cast<unsigned long long>(__popcll(sm)));
            }
            at = __shfl(at, __ffsll(static_cast<long long>(sm)) - 1, kWave);
            if (survive)
                survivors[at + __popcll(below)] = it | few | (mfma ? (1ull << 63) : 0ull) |
                                                  ((mfma && centre_j) ? (1ull << 62) : 0ull) |
                                                  (gram_j ? (1ull << 61) : 0ull);
            // pairs in survivors, and survivors for the matrix cores
            unsigned long long p = survive ? pairs : 0ull;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) p += __shfl_xor(p, o, kWave);
            const uint64_t mm = __ballot(survive && mfma);
            const uint64_t mf = __ballot(survive && (few >> (kItemBits + 11)) != 0);
            const uint64_t mg = __ballot(survive && gram_j);
            if (lane == 0) {
                atomicAdd(meta + 1, p);
                if (mm) atomicAdd(meta + 3, static_cast<unsigned long long>(__popcll(mm)));
                if (mf) atomicAdd(meta + 4, static_cast<unsigned long long>(__popcll(mf)));
                if (mg) atomicAdd(meta + 5, static_cast<unsigned long long>(__popcll(mg)));
            }
        }
        // whole-item counts: sum lanes with equal destinations
        uint64_t pend = __ballot(dst != nullptr);
        while (pend) {
            const int lead = __ffsll(static_cast<long long>(pend)) - 1;
            const uint64_t key = __shfl(reinterpret_cast<uint64_t>(dst), lead, kWave);
            const bool mine = dst != nullptr && reinterpret_cast<uint64_t>(dst) == key;
            unsigned long long c = mine ? cnt : 0ull;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, kWave);
            const int lane = threadIdx.x & (kWave - 1);
            if (lane == lead) {
                atomicAdd(reinterpret_cast<unsigned long long *>(key), c);
                atomicAdd(meta + 2, c);
            }
            if (mine) dst = nullptr;
            pend = __ballot(dst != nullptr);
        }
    }
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

// Spatially ordered copy of src[base, base+n) into a64s/a32s, and the tile
// bounds.  scratch: sort_scratch_words(n) uint32 words.
hipError_t launch_sort(const double4 *src, int64_t base, int64_t n, uint32_t *scratch, double4 *a64s,
                       float4 *a32s, float4 *g32s, double4 *bounds, hipStream_t st) {
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
    const int64_t tiles = (n + kTile - 1) / kTile;
    k_bounds<<<dim3(static_cast<uint32_t>(tiles)), dim3(kWave), 0, st>>>(a64s, n, bounds, g32s);
    return hipGetLastError();
}

hipError_t launch_prune(const SegDesc *segs, int32_t n_segs, const TableDesc *tabs, uint64_t total_items,
                        uint64_t *survivors, unsigned long long *meta, int32_t mfma_ok, hipStream_t st) {
    if (total_items == 0) return hipSuccess;
    const uint64_t want = (total_items + 255) / 256;
    const uint32_t grid = static_cast<uint32_t>(want < 16384 ? want : 16384);
    k_prune<<<dim3(grid), dim3(256), 0, st>>>(segs, n_segs, tabs, total_items, survivors, meta, mfma_ok);
    return hipGetLastError();
}

}  // namespace pc
