// pc_aperture.hip -- aperture-mass maps (Sec. 3, Eq. 3-5) on gfx950.
//
// The paper's GPU method gives each reconstruction point its own thread,
// which loops over the galaxies near that point.  Here a wavefront owns an
// 8 x 8 block of grid points (one per lane) and streams the galaxies near the
// block through scalar loads: every galaxy is wave-uniform, so it reaches all
// 64 lanes from SGPRs with no LDS and no vector memory traffic.  Galaxies are
// first ordered by the cell of a square search lattice; the galaxies a block
// can see lie, row of cells by row of cells, in one contiguous range each,
// trimmed to the filter disc around the block.
//
// Arithmetic per (point, galaxy) pair:
//   - the aperture cut in binary64, exactly as the definition states it
//     (dx, dy, |d|^2 = dx*dx + dy*dy, 0 < |d|^2 < theta_max^2, no fused
//     multiply-add), so the set of galaxies in each aperture is exact;
//   - for galaxies inside, x = |d| / theta_max from one reciprocal square
//     root in binary32, and the filter Q(x) (Eq. 4), a function of x alone,
//     from a table in LDS: 1024 cells over [0, 1], each a cubic in the
//     position inside the cell fitted on the host in binary64 (no
//     exponential, reciprocal or series per pair);
//   - the tangential ellipticity in binary32 from dx, dy rounded to binary32;
//   - the products Q eps_t and Q^2 |eps|^2 summed in binary32 over at most 64
//     galaxies and then in binary64.
#include <float.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pc_aperture.h"
#include "pc_runtime.hpp"

namespace pc {

hipError_t launch_zero_u32(uint32_t *p, int64_t m, hipStream_t st);
hipError_t launch_exclusive_scan(uint32_t *a, int64_t m, uint32_t *sums, hipStream_t st);
size_t scan_sums_words(int64_t m);

namespace {

constexpr int kApWaves = 4;            // waves per workgroup: 2 x 2 blocks sharing one filter table
constexpr int kQCells = 1024;          // filter table cells over x in [0, 1], and one at x = 1
constexpr int kApFlush = 64;           // galaxies summed in binary32 before the binary64 add
constexpr uint32_t kNoCell = 0xFFFFFFFFu;
constexpr int64_t kMaxCells = int64_t(1) << 22;
constexpr double kMaxExtent = 1e15;     // lattice extent limit (binary32 offsets stay finite)
thread_local int t_ap_force_p = 0;      // points per lane forced for testing (0: chosen per launch)

// One galaxy as the map kernel reads it (32 bytes, one scalar load).
struct alignas(32) ApGal {
    double x, y;  // position
    float a;      // -e1
    float a2;     // 2 e1
    float b2;     // -2 e2
    float ee;     // e1^2 + e2^2 (binary64, rounded once)
};

// Square search lattice: cell (cx, cy) covers [ox + cx s, ox + (cx+1) s) x ...
struct Lattice {
    double ox, oy;
    double s, inv_s;
    int32_t ncx, ncy;
};

struct ApParams {
    const ApGal *gal;
    const uint32_t *start;  // ncx * ncy + 1 cell starts
    const float4 *qtab;     // kQCells + 1 cubics (c0, c1, c2, c3): Q = c0 + t (c1 + t (c2 + t c3))
    Lattice lat;
    double x0, y0, gdx, gdy;
    int32_t nx, ny, tiles_x, n_tiles, per_xcd;  // tiles: groups of 2 x 2 blocks
    double theta;     // filter radius
    double r2;        // theta^2 (binary64), the cut
    double reach;     // theta with a relative margin for the cell search
    float k_x;        // x = r k_x = r / theta, clamped to [0, 1]; table position s = kQCells x
    float r2f;        // theta^2 rounded to binary32: the provisional cut
    float band;       // |f2 - r2f| <= band: the binary32 |d|^2 cannot decide the cut
    float near0;      // f2 <= near0: a galaxy near the point, decided and weighted in binary64
    float nbig;       // -1 / band: clamp(fma(f2 - r2f, nbig, 1/2)) is 1 inside, 0 outside
    float f2_in, f2_out;  // r2f -+ 2 band: where a pair decided in binary64 is moved
    double n_gal;
    double *map;
    double *snr;
    uint32_t *n_in;
    unsigned long long *stats;  // [pairs tested, pairs inside]
};

__device__ __forceinline__ int32_t cell_index(double v, double o, double inv_s, int32_t n) {
    const double t = floor((v - o) * inv_s);
    if (!(t >= 0.0)) return 0;
    return t >= static_cast<double>(n) ? n - 1 : static_cast<int32_t>(t);
}

// ----------------------------------------------------------- cell ordering

__global__ void __launch_bounds__(256) k_ap_keys(const double *__restrict__ X, const double *__restrict__ Y,
                                                 const double *__restrict__ E1, const double *__restrict__ E2,
                                                 int64_t n, Lattice lat, uint32_t *__restrict__ keys,
                                                 uint32_t *__restrict__ count, uint32_t *__restrict__ flag) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = X[i], y = Y[i], e1 = E1[i], e2 = E2[i];
    if (!isfinite(x) || !isfinite(y) || !isfinite(e1) || !isfinite(e2)) {
        atomicOr(flag, 1u);
        keys[i] = kNoCell;
        return;
    }
    const double tx = (x - lat.ox) * lat.inv_s;
    const double ty = (y - lat.oy) * lat.inv_s;
    // outside the lattice: farther than theta_max + one cell from every grid point
    if (!(tx >= 0.0 && tx < static_cast<double>(lat.ncx) && ty >= 0.0 && ty < static_cast<double>(lat.ncy))) {
        keys[i] = kNoCell;
        return;
    }
    const uint32_t key = static_cast<uint32_t>(static_cast<int32_t>(floor(ty))) * static_cast<uint32_t>(lat.ncx) +
                         static_cast<uint32_t>(static_cast<int32_t>(floor(tx)));
    keys[i] = key;
    atomicAdd(count + key, 1u);
}

__global__ void __launch_bounds__(256) k_ap_scatter(const uint32_t *__restrict__ keys, int64_t n,
                                                    uint32_t *__restrict__ cursor, uint32_t *__restrict__ idx) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t key = keys[i];
    if (key == kNoCell) return;
    idx[atomicAdd(cursor + key, 1u)] = static_cast<uint32_t>(i);
}

// The scatter leaves each cell's galaxies in arbitrary order; place each one
// at its rank by catalogue index inside the cell, so the summation order of
// the map kernel, and with it every output bit, is reproducible.
__global__ void __launch_bounds__(256) k_ap_place(const double *__restrict__ X, const double *__restrict__ Y,
                                                  const double *__restrict__ E1, const double *__restrict__ E2,
                                                  const uint32_t *__restrict__ keys, const uint32_t *__restrict__ idx,
                                                  const uint32_t *__restrict__ start, int64_t n_cells, int64_t n,
                                                  ApGal *__restrict__ gal) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= n || p >= static_cast<int64_t>(start[n_cells])) return;
    const uint32_t i = idx[p];
    const uint32_t key = keys[i];
    const uint32_t lo = start[key], hi = start[key + 1];
    uint32_t rank = 0;
    for (uint32_t q = lo; q < hi; ++q) rank += idx[q] < i ? 1u : 0u;
    const double e1 = E1[i], e2 = E2[i];
    ApGal g;
    g.x = X[i];
    g.y = Y[i];
    g.a = static_cast<float>(-e1);
    g.a2 = static_cast<float>(2.0 * e1);
    g.b2 = static_cast<float>(-2.0 * e2);
    g.ee = static_cast<float>(e1 * e1 + e2 * e2);
    gal[lo + rank] = g;
}

// ------------------------------------------------------------------ map

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Constants held in VGPRs (an instruction reads at most one SGPR).
struct ApConsts {
    float k_x, r2f, band, near0, nbig, f2_in, f2_out;
    uint32_t tab;  // LDS byte address of the filter table
};

// clamp(e * m + 1/2) to [0, 1] in one fused multiply-add (its clamp bit).
__device__ __forceinline__ float fma_clamp01(float e, float m) {
    float r;
    asm("v_fma_f32 %0, %1, %2, 0.5 clamp" : "=v"(r) : "v"(e), "v"(m));
    return r;
}

// max(a, b) of two finite values, one instruction (fmaxf would first quiet
// signalling NaNs, which cannot occur here).
__device__ __forceinline__ float max_f32(float a, float b) {
    float r;
    asm("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// The table position of a separation r: x = RN(r k_x) clamped to [0, 1] by
// the multiply's clamp bit (a full-rate instruction, where a min is not),
// then s = kQCells x, exact.  For x below 1 this is RN(r kQCells / theta)
// rounded once, as kQCells is a power of two.
__device__ __forceinline__ float table_pos(float r, float k_x) {
    float x;
    asm("v_mul_f32_e64 %0, %1, %2 clamp" : "=v"(x) : "v"(r), "v"(k_x));
    return x * static_cast<float>(kQCells);
}

// The filter Q(x) of Eq. 4 at table position s = kQCells x (0 <= s <=
// kQCells): cell i = floor(s), t = s - i, Q = c0 + t (c1 + t (c2 + t c3));
// s = kQCells reads the last cell, the constant Q(1).
__device__ __forceinline__ float q_table(float s, uint32_t tab) {
    const uint32_t i = static_cast<uint32_t>(s);
    const float t = __builtin_amdgcn_fractf(s);
    typedef float f32x4 __attribute__((ext_vector_type(4)));
    using lds_f4 = __attribute__((address_space(3))) const f32x4;
    const f32x4 c = *(lds_f4 *)(uintptr_t)(tab + (i << 4));
    return fmaf(fmaf(fmaf(c.w, t, c.z), t, c.y), t, c.x);
}

// One wave owns a block of (8P) x (8P) grid points: lane (lx, ly) = (lane % 8,
// lane / 8) holds the P x P points (lx + 8a, ly + 8b), so every galaxy read
// (wave-uniform, scalar loads) is used for P^2 independent pairs per lane.
// Four waves (2 x 2 blocks) per workgroup share the filter table in LDS.
// Groups are dealt to the eight XCDs in contiguous strips (the hardware
// assigns workgroup b to XCD b mod 8), so neighbouring blocks, which read
// mostly the same galaxies, share an L2.
//
// Per pair, in binary32: the galaxy and the point relative to a reference
// point of the block (the galaxy's offset is formed once per galaxy in
// binary64 and rounded), dx, dy and f2 = dx^2 + dy^2.  The cut is decided
// from f2 against theta^2 wherever a proven bound on |f2 - |d|^2| (host code
// below, `cut_bands`) allows it; pairs with f2 within `band` of theta^2 are
// decided by the binary64 definition, so the set of galaxies in each aperture
// is exact.  A galaxy very near its point (f2 <= near0) is decided by the
// binary64 definition too and, when inside, weighted from its binary64 offset:
// the binary32 offsets, good to a few units in the last place of the block's
// size, would not resolve its direction.  For the other pairs inside: x =
// |d| / theta_max from one reciprocal square root, the filter from the table,
// and
//   eps_t = -(e1 cos 2phi + e2 sin 2phi) = -e1 + (2 / f2) (e1 dy^2 - e2 dx dy)
// (cos 2phi = 1 - 2 dy^2 / f2, sin 2phi = 2 dx dy / f2); the products
// Q eps_t and Q^2 |eps|^2 are summed in binary32 over at most 64 galaxies and
// then in binary64.
//
// RAISE: f2 is raised to near0 before the reciprocal square root.  Every f2
// that reaches the binary32 step is positive and normal when r2f - 2 band is
// (a pair left there has f2 > near0 >= 2^-100, a pair moved there r2f +- 2
// band), and the host then takes the instance without it; with the band
// widened to decide every pair in binary64 (grid spacing far beyond theta)
// r2f - 2 band is negative, and the raise keeps the weights of such moved
// pairs finite.
template <int P, bool RAISE>
__global__ void __launch_bounds__(64 * kApWaves) __attribute__((amdgpu_waves_per_eu(P == 2 ? 4 : 7)))
k_ap_map(const ApParams p) {
    constexpr int BS = 8 * P;   // block side in points
    constexpr int K = P * P;    // points per lane
    __shared__ float4 qtab[kQCells + 1];
    const int lane = static_cast<int>(threadIdx.x) & 63;
    // wave-uniform (a scalar register): the block, its galaxy ranges and the
    // galaxy loop are the same for every lane of the wave
    const int wave = static_cast<int>(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6));
    const int b = static_cast<int>(blockIdx.x);
    const int tile = (b & 7) * p.per_xcd + (b >> 3);
    if (tile >= p.n_tiles) return;  // the whole workgroup: before any barrier
    for (int k = static_cast<int>(threadIdx.x); k <= kQCells; k += 64 * kApWaves) qtab[k] = p.qtab[k];
    __syncthreads();
    const int tx = tile % p.tiles_x, ty = tile / p.tiles_x;
    const int ix0 = tx * 2 * BS + (wave & 1) * BS, iy0 = ty * 2 * BS + (wave >> 1) * BS;
    // a block of the group past the grid's edge has no points
    if (ix0 >= p.nx || iy0 >= p.ny) return;
    const int ix1 = min(ix0 + BS - 1, p.nx - 1), iy1 = min(iy0 + BS - 1, p.ny - 1);
    // the block's reference point: its centre (any binary64 value serves)
    const double xb = p.x0 + (static_cast<double>(ix0) + 0.5 * (BS - 1)) * p.gdx;
    const double yb = p.y0 + (static_cast<double>(iy0) + 0.5 * (BS - 1)) * p.gdy;
    int ixk[K], iyk[K];
    bool valid[K];
    float Xg[K], Yg[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int ixl = ix0 + (lane & 7) + 8 * (k % P), iyl = iy0 + (lane >> 3) + 8 * (k / P);
        valid[k] = ixl <= ix1 && iyl <= iy1;
        ixk[k] = min(ixl, ix1);  // lanes past the grid edge repeat a point
        iyk[k] = min(iyl, iy1);
        // the grid point as the definition forms it (product, then sum)
        const double xg = p.x0 + static_cast<double>(ixk[k]) * p.gdx;
        const double yg = p.y0 + static_cast<double>(iyk[k]) * p.gdy;
        Xg[k] = static_cast<float>(xg - xb);
        Yg[k] = static_cast<float>(yg - yb);
    }
    const double gxl = p.x0 + static_cast<double>(ix0) * p.gdx, gxh = p.x0 + static_cast<double>(ix1) * p.gdx;
    const double gyl = p.y0 + static_cast<double>(iy0) * p.gdy, gyh = p.y0 + static_cast<double>(iy1) * p.gdy;
    const Lattice L = p.lat;
    ApConsts C{p.k_x, p.r2f, p.band, p.near0, p.nbig, p.f2_in, p.f2_out,
               static_cast<uint32_t>(reinterpret_cast<uintptr_t>(
                   (__attribute__((address_space(3))) const float4 *)(qtab)))};
    asm("" : "+v"(C.k_x), "+v"(C.r2f), "+v"(C.band), "+v"(C.near0), "+v"(C.nbig), "+v"(C.f2_in), "+v"(C.f2_out));
    const double slack = L.s * 1e-9;  // covers rounding of the cell coordinates

    double S1[K], S2[K];
    uint32_t cnt[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        S1[k] = 0.0;
        S2[k] = 0.0;
        cnt[k] = 0u;
    }
    uint64_t tested = 0;
    const int cy0 = cell_index(gyl - p.reach - slack, L.oy, L.inv_s, L.ncy);
    const int cy1 = cell_index(gyh + p.reach + slack, L.oy, L.inv_s, L.ncy);
    for (int cy = cy0; cy <= cy1; ++cy) {
        // vertical gap between this row of cells and the block; the row's
        // galaxies within reach of the block lie within w of it horizontally
        const double rlo = L.oy + static_cast<double>(cy) * L.s;
        const double dv = fmax(0.0, fmax(rlo - gyh, gyl - (rlo + L.s)) - slack);
        const double w2 = p.reach * p.reach - dv * dv;
        if (!(w2 > 0.0)) continue;
        const double w = sqrt(w2) + slack;
        const int cx0 = cell_index(gxl - w, L.ox, L.inv_s, L.ncx);
        const int cx1 = cell_index(gxh + w, L.ox, L.inv_s, L.ncx);
        const uint32_t row = static_cast<uint32_t>(cy) * static_cast<uint32_t>(L.ncx);
        const uint32_t g_begin = p.start[row + static_cast<uint32_t>(cx0)];
        const uint32_t g_end = p.start[row + static_cast<uint32_t>(cx1) + 1u];
        tested += g_end - g_begin;
        for (uint32_t c0 = g_begin; c0 < g_end; c0 += kApFlush) {
            const uint32_t c1 = min(c0 + static_cast<uint32_t>(kApFlush), g_end);
            float a1[K], a2[K], cntf[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                a1[k] = 0.0f;
                a2[k] = 0.0f;
                cntf[k] = 0.0f;
            }
            // galaxies go through scalar registers, each loaded one galaxy
            // ahead of its use
            ApGal Gn = p.gal[c0];
            for (uint32_t g = c0; g < c1; ++g) {
                const ApGal G = Gn;
                Gn = p.gal[min(g + 1u, c1 - 1u)];
                const float X = static_cast<float>(G.x - xb), Y = static_cast<float>(G.y - yb);
                float fdx[K], fdy[K], py[K], f2[K];
                float near = FLT_MAX, low = FLT_MAX;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    fdx[k] = X - Xg[k];
                    fdy[k] = Y - Yg[k];
                    py[k] = fdy[k] * fdy[k];
                    f2[k] = fmaf(fdx[k], fdx[k], py[k]);
                    near = fminf(near, fabsf(f2[k] - C.r2f));
                    low = fminf(low, f2[k]);
                }
                if (__builtin_expect(__builtin_amdgcn_ballot_w64(near <= C.band || low <= C.near0) != 0, 0)) {
                    // rare: a pair of the wave that f2 cannot decide is
                    // decided by the binary64 definition (0 < dx*dx + dy*dy <
                    // theta^2, no fused multiply-add, grid point formed as
                    // above) and its f2 moved to the matching side of r2f (by
                    // at most `band`); a galaxy near its point, if inside, is
                    // weighted here from its binary64 offset and left out of
                    // the binary32 step below
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        const double xg = p.x0 + static_cast<double>(ixk[k]) * p.gdx;
                        const double yg = p.y0 + static_cast<double>(iyk[k]) * p.gdy;
                        const double ddx = G.x - xg, ddy = G.y - yg;
                        const double d2 = ddx * ddx + ddy * ddy;
                        const bool inside = d2 < p.r2 && d2 > 0.0;
                        const bool near_point = f2[k] <= C.near0;
                        if (near_point && inside) {
                            const double c2 = (ddx * ddx - ddy * ddy) / d2, s2 = (ddx * ddy) / d2;
                            const float et = static_cast<float>(static_cast<double>(G.a) * c2 +
                                                                static_cast<double>(G.b2) * s2);
                            const float qn = q_table(table_pos(static_cast<float>(sqrt(d2)), C.k_x), C.tab);
                            a1[k] = fmaf(qn, et, a1[k]);
                            a2[k] = fmaf(qn * qn, G.ee, a2[k]);
                            cnt[k] += 1u;
                        }
                        const bool undecided = fabsf(f2[k] - C.r2f) <= C.band || near_point;
                        const float moved = (inside && !near_point) ? C.f2_in : C.f2_out;
                        f2[k] = undecided ? moved : f2[k];
                    }
                }
                // inside: w = 1, outside: w = 0, exactly (|f2 - r2f| > band
                // here, or f2 was moved to 2 band from r2f); plain
                // arithmetic, no compare.  Every value below is finite: f2 is
                // positive and normal (see RAISE).
                float rinv[K], q[K], wt[K];
                uint32_t addr[K];
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    wt[k] = fma_clamp01(f2[k] - C.r2f, C.nbig);
                    cntf[k] += wt[k];
                    const float f2c = RAISE ? max_f32(f2[k], C.near0) : f2[k];
                    rinv[k] = __builtin_amdgcn_rsqf(f2c);
                    const float sk = table_pos(f2c * rinv[k], C.k_x);
                    addr[k] = C.tab + (static_cast<uint32_t>(sk) << 4);
                    q[k] = __builtin_amdgcn_fractf(sk);  // position in the cell, for now
                }
                typedef float f32x4 __attribute__((ext_vector_type(4)));
                using lds_f4 = __attribute__((address_space(3))) const f32x4;
                f32x4 cq[K];
#pragma unroll
                for (int k = 0; k < K; ++k) cq[k] = *(lds_f4 *)(uintptr_t)(addr[k]);
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const float t = q[k];
                    float qk = fmaf(fmaf(fmaf(cq[k].w, t, cq[k].z), t, cq[k].y), t, cq[k].x);
                    qk *= wt[k];
                    const float rr = rinv[k] * rinv[k];
                    const float inner = fmaf(G.a2, py[k], G.b2 * (fdx[k] * fdy[k]));
                    const float et = fmaf(rr, inner, G.a);
                    a1[k] = fmaf(qk, et, a1[k]);
                    a2[k] = fmaf(qk * qk, G.ee, a2[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                S1[k] += static_cast<double>(a1[k]);
                S2[k] += static_cast<double>(a2[k]);
                cnt[k] += static_cast<uint32_t>(cntf[k]);  // at most 64, exact
            }
        }
    }
    uint32_t in_lane = 0, lanes = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (valid[k]) {
            const int64_t o = static_cast<int64_t>(iyk[k]) * p.nx + ixk[k];
            p.map[o] = S1[k] / p.n_gal;
            if (p.snr) p.snr[o] = S2[k] > 0.0 ? (1.4142135623730951 * S1[k]) / sqrt(S2[k]) : __builtin_nan("");
            if (p.n_in) p.n_in[o] = cnt[k];
            in_lane += cnt[k];
            lanes += 1u;
        }
    }
    if (p.stats) {
        const uint32_t in_wave = wave_sum_u32(in_lane);
        const uint32_t pts = wave_sum_u32(lanes);
        if (lane == 0) {
            atomicAdd(p.stats + 0, static_cast<unsigned long long>(tested) * pts);
            atomicAdd(p.stats + 1, static_cast<unsigned long long>(in_wave));
        }
    }
}

// ------------------------------------------------------------------- host

struct ApLast {
    double kernel_ms = -1.0;
    uint64_t tested = 0;
    uint64_t in = 0;
    double cell = 0.0;
};
thread_local ApLast t_ap;

struct DevMem {
    void *mem = nullptr;
    hipStream_t st = nullptr;
    ~DevMem() {
        if (mem) (void)hipFreeAsync(mem, st);
    }
};

struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

size_t take(size_t *size, size_t bytes) {
    const size_t o = (*size + 255) & ~size_t(255);
    *size = o + bytes;
    return o;
}

#define AP_HIP(call, what)                                 \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hip_fail(e_, (what)); \
    } while (0)

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Eq. 4 in binary64: Q(x) = 1 / (1 + e^(6 - 150 x) + e^(-47 + 50 x)) *
// tanh(x / 0.15) / (x / 0.15), with tanh(u)/u = 1 at u = 0.
double q_filter(double x) {
    const double u = x / 0.15;
    const double th = u == 0.0 ? 1.0 : std::tanh(u) / u;
    return th / (1.0 + std::exp(6.0 - 150.0 * x) + std::exp(-47.0 + 50.0 * x));
}

// The filter table: cell k < kQCells covers x in [k, k+1] / kQCells; its
// cubic in t = kQCells x - k interpolates Q at the four Chebyshev points of
// [0, 1] (solved in binary64, coefficients rounded to binary32 once).  Cell
// kQCells holds the constant Q(1), for x = 1 (t = 0).  Built once.
const float4 *filter_table() {
    static float4 tab[kQCells + 1];
    static std::once_flag once;
    std::call_once(once, [] {
        const double kPi = 3.14159265358979323846;
        for (int k = 0; k < kQCells; ++k) {
            double A[4][5];
            for (int j = 0; j < 4; ++j) {
                const double t = 0.5 - 0.5 * std::cos((2 * j + 1) * kPi / 8.0);
                double tp = 1.0;
                for (int m = 0; m < 4; ++m, tp *= t) A[j][m] = tp;
                A[j][4] = q_filter((k + t) / kQCells);
            }
            // Gaussian elimination with partial pivoting on the 4 x 4 system
            for (int c = 0; c < 4; ++c) {
                int piv = c;
                for (int r = c + 1; r < 4; ++r)
                    if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
                for (int m = 0; m < 5; ++m) std::swap(A[c][m], A[piv][m]);
                for (int r = 0; r < 4; ++r) {
                    if (r == c) continue;
                    const double f = A[r][c] / A[c][c];
                    for (int m = c; m < 5; ++m) A[r][m] -= f * A[c][m];
                }
            }
            tab[k] = make_float4(static_cast<float>(A[0][4] / A[0][0]), static_cast<float>(A[1][4] / A[1][1]),
                                 static_cast<float>(A[2][4] / A[2][2]), static_cast<float>(A[3][4] / A[3][3]));
        }
        tab[kQCells] = make_float4(static_cast<float>(q_filter(1.0)), 0.0f, 0.0f, 0.0f);
    });
    return tab;
}

int check_args(const pc_shear_catalog *cat, const pc_grid *grid, double theta_max, double n_gal, const double *map) {
    if (!cat || !grid || !map) return fail(PC_ERR_INVALID, "NULL catalogue, grid or map");
    if (cat->n < 0 || cat->n >= (int64_t(1) << 31)) return fail(PC_ERR_INVALID, "catalogue n outside [0, 2^31)");
    if (cat->n > 0 && (!cat->x || !cat->y || !cat->e1 || !cat->e2))
        return fail(PC_ERR_INVALID, "catalogue has NULL arrays");
    if (!finite_pos(theta_max)) return fail(PC_ERR_INVALID, "theta_max must be finite and > 0");
    if (!finite_pos(n_gal)) return fail(PC_ERR_INVALID, "n_gal must be finite and > 0");
    if (!std::isfinite(grid->x0) || !std::isfinite(grid->y0) || !finite_pos(grid->dx) || !finite_pos(grid->dy))
        return fail(PC_ERR_INVALID, "grid origin must be finite and spacings finite and > 0");
    if (grid->nx < 0 || grid->ny < 0 || int64_t(grid->nx) * grid->ny >= (int64_t(1) << 31))
        return fail(PC_ERR_INVALID, "grid size outside [0, 2^31)");
    const double span_x = (grid->nx > 0 ? grid->nx - 1 : 0) * grid->dx, span_y = (grid->ny > 0 ? grid->ny - 1 : 0) * grid->dy;
    if (!std::isfinite(grid->x0 + span_x) || !std::isfinite(grid->y0 + span_y))
        return fail(PC_ERR_INVALID, "grid extent overflows");
    if (!cat->on_device) {
        for (int64_t i = 0; i < cat->n; ++i)
            if (!std::isfinite(cat->x[i]) || !std::isfinite(cat->y[i]) || !std::isfinite(cat->e1[i]) ||
                !std::isfinite(cat->e2[i]))
                return fail(PC_ERR_INVALID, "non-finite galaxy position or ellipticity (index " +
                                                std::to_string(i) + ")");
    }
    return PC_OK;
}

// Cell side theta/16 (coarser if the lattice would exceed kMaxCells), one
// spare cell beyond theta on every side of the grid.
int make_lattice(const pc_grid *g, double theta, Lattice *L) {
    const double span_x = (g->nx - 1) * g->dx + 2.0 * theta;
    const double span_y = (g->ny - 1) * g->dy + 2.0 * theta;
    // every galaxy the map kernel looks at lies in the lattice, so its
    // binary32 offsets from a block (at most the lattice's extent) stay
    // finite, and so do their squares
    if (!(span_x < kMaxExtent && span_y < kMaxExtent))
        return fail(PC_ERR_INVALID, "grid extent plus twice theta_max must be below 1e15 units");
    double s = theta / 16.0;
    for (int it = 0; it < 200; ++it) {
        const double cx = std::ceil(span_x / s) + 3.0, cy = std::ceil(span_y / s) + 3.0;
        if (cx * cy <= static_cast<double>(kMaxCells)) {
            L->s = s;
            L->inv_s = 1.0 / s;
            L->ncx = static_cast<int32_t>(cx);
            L->ncy = static_cast<int32_t>(cy);
            L->ox = g->x0 - theta - s;
            L->oy = g->y0 - theta - s;
            return PC_OK;
        }
        s *= 2.0;
    }
    return fail(PC_ERR_INVALID, "grid extent too large for the search lattice");
}

// Grid points per lane along each axis (blocks of 8P x 8P points per wave):
// 2 when the 16 x 16 block is small beside the filter disc (a quarter of its
// radius), so that the extra galaxies visited by the larger block stay few,
// and the grid gives at least 16 such blocks per CU (four waves per SIMD, the
// instance's occupancy); else 1.
int points_per_lane(const pc_grid *g, double theta, int cus) {
    if (t_ap_force_p == 1 || t_ap_force_p == 2) return t_ap_force_p;
    const double blocks16 = (static_cast<double>(g->nx) * g->ny) / 256.0;
    return 16.0 * std::max(g->dx, g->dy) <= 0.25 * theta && blocks16 >= 16.0 * cus ? 2 : 1;
}

// The binary32 cut and its guard bands.  Notation: u = 2^-24, v = 2^-53;
// (xb, yb) a block's reference point, every point of the block within hx
// (hy) of it; D = |d| exactly, DX = x_i - x_p exactly.  The kernel forms
//   X = RN32(RN64(x_i - xb)), Xg = RN32(RN64(x_p - xb)), fdx = RN32(X - Xg)
// (likewise in y), py = RN32(fdy^2), f2 = RN32(fdx^2 + py) (one fused
// multiply-add).  |x_i - xb| <= D + hx, so |X - Xg - DX| <= u1 (D + 2 hx)
// with u1 = u + 2v, and
//   |fdx - DX| <= ex = c1 D + cx,  c1 = u1 (1 + u) + u,  cx = 2 u1 (1 + u) hx,
//   |f2 - D^2| <= B(D) = 2 D (ex + ey) + ex^2 + ey^2 + w (D + ex + ey)^2,
// w = u (2 + u): a quadratic a D^2 + b D + c with non-negative coefficients.
// The binary64 definition d2 = RN64(RN64(ddx^2) + RN64(ddy^2)), ddx =
// RN64(DX), is within 4.0001 v D^2 of D^2, and r2f = RN32(r2) within u r2 of
// r2 = RN64(theta^2).  Then
//   * d2 < r2 gives D < theta (1 + 3v) and f2 <= D^2 + B(D) < r2f + G with
//     G = (u + 8v) r2 + B(theta (1 + 1e-6));
//   * d2 >= r2 gives D >= theta0 = theta (1 - 3v) and f2 >= D^2 - B(D); when
//     D^2 - B(D) is increasing from theta0 on (2 (1 - a) theta0 >= b), f2 >
//     r2f - G;
//   * d2 = 0 needs ddx = ddy = 0 up to underflow, D below 1e-161, and then f2
//     <= B(D), about c;
//   * the offset (fdx, fdy) is within e(D) = sqrt(ex^2 + ey^2) <= e0 + sqrt(2)
//     c1 D of (DX, DY), e0 = sqrt(cx^2 + cy^2), so its direction is within
//     about e(D) / D radians: at most 2^-17 + 2 c1 once D >= Dn = 2^17 e0, and
//     cos 2phi, sin 2phi within twice that, a relative 3e-5 of |eps| in eps_t.
// So with band >= G, |f2 - r2f| > band decides the cut as the definition
// does; near0 >= Dn^2 + B(Dn) (and >= 2c) catches every pair with D <= Dn,
// among them every pair with d2 = 0.  Both are doubled, raised by 2^-100
// (absolute: it also covers binary32 results below the normal range) and
// rounded up to binary32.  hx includes the binary64 rounding of the grid
// points and of the reference point.  Where the increasing condition fails
// (grid spacing beyond ~1e6 theta), band is made large enough that every pair
// with f2 below r2f + band is decided in binary64.
void cut_bands(const pc_grid *g, double theta, double r2, int P, float *r2f, float *band, float *near0) {
    const double u = std::ldexp(1.0, -24), v = std::ldexp(1.0, -53), u1 = u + 2.0 * v, w = u * (2.0 + u);
    const double ext_x = std::fabs(g->x0) + (g->nx + 8.0 * P) * g->dx;
    const double ext_y = std::fabs(g->y0) + (g->ny + 8.0 * P) * g->dy;
    const double hx = 4.0 * P * g->dx + 8.0 * v * ext_x, hy = 4.0 * P * g->dy + 8.0 * v * ext_y;
    const double c1 = u1 * (1.0 + u) + u, cx = 2.0 * u1 * (1.0 + u) * hx, cy = 2.0 * u1 * (1.0 + u) * hy;
    const double qa = 4.0 * c1 + 2.0 * c1 * c1 + w * (1.0 + 2.0 * c1) * (1.0 + 2.0 * c1);
    const double qb = 2.0 * (cx + cy) * (1.0 + c1 + w * (1.0 + 2.0 * c1));
    const double qc = cx * cx + cy * cy + w * (cx + cy) * (cx + cy);
    auto B = [&](double D) { return (qa * D + qb) * D + qc; };
    const double floor_abs = std::ldexp(1.0, -100);
    const double theta0 = theta * (1.0 - 3.0 * v);
    double G = (u + 8.0 * v) * r2 + B(theta * (1.0 + 1e-6));
    if (!(2.0 * (1.0 - qa) * theta0 >= qb)) G = std::max(G, 4.0 * r2);
    auto up = [](double x) {
        float f = static_cast<float>(x);
        if (static_cast<double>(f) < x) f = std::nextafter(f, FLT_MAX);
        return f;
    };
    *r2f = static_cast<float>(r2);
    *band = up(2.0 * G + floor_abs);
    const double dn = std::ldexp(std::sqrt(cx * cx + cy * cy), 17);
    *near0 = up(2.0 * std::max(dn * dn + B(dn), B(1e-150)) + floor_abs);
}

}  // namespace
}  // namespace pc

using namespace pc;

extern "C" int pc_debug_ap_points_per_lane(int32_t points) {
    clear_error();
    if (points < 0 || points > 2) return fail(PC_ERR_INVALID, "points per lane must be 0 (automatic), 1 or 2");
    t_ap_force_p = points;
    return PC_OK;
}

extern "C" int pc_aperture_mass(const pc_shear_catalog *cat, const pc_grid *grid, double theta_max, double n_gal,
                                double *map, double *snr, uint32_t *n_in, int32_t out_on_device, void *stream) {
    clear_error();
    int rc = check_args(cat, grid, theta_max, n_gal, map);
    if (rc) return rc;
    DeviceInfo *di = nullptr;
    rc = device_info(&di);
    if (rc) return rc;
    const int64_t n = cat->n;
    const int64_t m = int64_t(grid->nx) * grid->ny;
    t_ap = ApLast();
    if (m == 0) return PC_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);

    Lattice L;
    rc = make_lattice(grid, theta_max, &L);
    if (rc) return rc;
    const int64_t n_cells = int64_t(L.ncx) * L.ncy;

    // work space
    const bool host_in = !cat->on_device, host_out = !out_on_device;
    const size_t nn = static_cast<size_t>(n > 0 ? n : 1);
    size_t size = 0;
    const size_t o_in = host_in ? take(&size, 4 * sizeof(double) * nn) : 0;
    const size_t o_keys = take(&size, sizeof(uint32_t) * nn);
    const size_t o_idx = take(&size, sizeof(uint32_t) * nn);
    const size_t o_gal = take(&size, sizeof(ApGal) * nn);
    const size_t o_start = take(&size, sizeof(uint32_t) * static_cast<size_t>(n_cells + 1));
    const size_t o_cursor = take(&size, sizeof(uint32_t) * static_cast<size_t>(n_cells));
    const size_t o_sums = take(&size, sizeof(uint32_t) * scan_sums_words(n_cells + 1));
    const size_t o_flag = take(&size, 4 * sizeof(uint32_t));
    const size_t o_stats = take(&size, 2 * sizeof(unsigned long long));
    const size_t o_qtab = take(&size, sizeof(float4) * (kQCells + 1));
    const size_t o_out = host_out ? take(&size, (2 * sizeof(double) + sizeof(uint32_t)) * static_cast<size_t>(m)) : 0;
    DevMem ws;
    ws.st = st;
    AP_HIP(injected_alloc_failure() ? hipErrorOutOfMemory : hipMallocAsync(&ws.mem, size, st),
           "hipMallocAsync(aperture work space)");
    char *base = static_cast<char *>(ws.mem);

    const double *X = cat->x, *Y = cat->y, *E1 = cat->e1, *E2 = cat->e2;
    if (host_in && n > 0) {
        double *d = reinterpret_cast<double *>(base + o_in);
        const size_t b = sizeof(double) * static_cast<size_t>(n);
        AP_HIP(hipMemcpyAsync(d, cat->x, b, hipMemcpyHostToDevice, st), "H2D x");
        AP_HIP(hipMemcpyAsync(d + n, cat->y, b, hipMemcpyHostToDevice, st), "H2D y");
        AP_HIP(hipMemcpyAsync(d + 2 * n, cat->e1, b, hipMemcpyHostToDevice, st), "H2D e1");
        AP_HIP(hipMemcpyAsync(d + 3 * n, cat->e2, b, hipMemcpyHostToDevice, st), "H2D e2");
        X = d;
        Y = d + n;
        E1 = d + 2 * n;
        E2 = d + 3 * n;
    }
    uint32_t *keys = reinterpret_cast<uint32_t *>(base + o_keys);
    uint32_t *idx = reinterpret_cast<uint32_t *>(base + o_idx);
    ApGal *gal = reinterpret_cast<ApGal *>(base + o_gal);
    uint32_t *start = reinterpret_cast<uint32_t *>(base + o_start);
    uint32_t *cursor = reinterpret_cast<uint32_t *>(base + o_cursor);
    uint32_t *sums = reinterpret_cast<uint32_t *>(base + o_sums);
    uint32_t *flag = reinterpret_cast<uint32_t *>(base + o_flag);
    unsigned long long *stats = reinterpret_cast<unsigned long long *>(base + o_stats);
    float4 *qtab = reinterpret_cast<float4 *>(base + o_qtab);
    AP_HIP(hipMemcpyAsync(qtab, filter_table(), sizeof(float4) * (kQCells + 1), hipMemcpyHostToDevice, st),
           "H2D filter table");

    // order the galaxies by cell
    AP_HIP(launch_zero_u32(start, n_cells + 1, st), "zero cell counts");
    AP_HIP(launch_zero_u32(flag, 4, st), "zero flags");
    AP_HIP(launch_zero_u32(reinterpret_cast<uint32_t *>(stats), 4, st), "zero stats");
    if (n > 0) {
        const uint32_t gn = static_cast<uint32_t>((n + 255) / 256);
        k_ap_keys<<<dim3(gn), dim3(256), 0, st>>>(X, Y, E1, E2, n, L, keys, start, flag);
        AP_HIP(hipGetLastError(), "k_ap_keys");
        AP_HIP(launch_exclusive_scan(start, n_cells + 1, sums, st), "cell scan");
        AP_HIP(hipMemcpyAsync(cursor, start, sizeof(uint32_t) * static_cast<size_t>(n_cells),
                              hipMemcpyDeviceToDevice, st),
               "cell cursors");
        k_ap_scatter<<<dim3(gn), dim3(256), 0, st>>>(keys, n, cursor, idx);
        AP_HIP(hipGetLastError(), "k_ap_scatter");
        k_ap_place<<<dim3(gn), dim3(256), 0, st>>>(X, Y, E1, E2, keys, idx, start, n_cells, n, gal);
        AP_HIP(hipGetLastError(), "k_ap_place");
    }
    uint32_t h_flag = 0;
    AP_HIP(hipMemcpyAsync(&h_flag, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, st), "D2H flag");
    AP_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
    if (h_flag) return fail(PC_ERR_INVALID, "non-finite galaxy position or ellipticity in the device catalogue");

    double *d_map = map, *d_snr = snr;
    uint32_t *d_nin = n_in;
    if (host_out) {
        d_map = reinterpret_cast<double *>(base + o_out);
        d_snr = d_map + m;
        d_nin = reinterpret_cast<uint32_t *>(d_snr + m);
    }
    ApParams p;
    p.gal = gal;
    p.start = start;
    p.lat = L;
    p.x0 = grid->x0;
    p.y0 = grid->y0;
    p.gdx = grid->dx;
    p.gdy = grid->dy;
    p.nx = grid->nx;
    p.ny = grid->ny;
    const int P = points_per_lane(grid, theta_max, di->cus);
    const int group_side = 16 * P;  // 2 x 2 blocks of 8P x 8P points
    p.tiles_x = (grid->nx + group_side - 1) / group_side;
    const int tiles_y = (grid->ny + group_side - 1) / group_side;
    p.n_tiles = p.tiles_x * tiles_y;
    p.per_xcd = (p.n_tiles + 7) / 8;
    p.theta = theta_max;
    p.r2 = theta_max * theta_max;
    p.reach = theta_max * (1.0 + 1e-9);
    // RN32(kQCells / theta) / kQCells: exact (a power of two, no subnormal
    // for theta below the extent limit)
    p.k_x = static_cast<float>(static_cast<double>(kQCells) / theta_max) / static_cast<float>(kQCells);
    cut_bands(grid, theta_max, p.r2, P, &p.r2f, &p.band, &p.near0);
    p.nbig = -1.0f / p.band;
    p.f2_in = p.r2f - 2.0f * p.band;
    p.f2_out = p.r2f + 2.0f * p.band;
    p.qtab = qtab;
    p.n_gal = n_gal;
    p.map = d_map;
    p.snr = (snr || host_out) ? d_snr : nullptr;
    p.n_in = (n_in || host_out) ? d_nin : nullptr;
    p.stats = stats;

    Events ev;
    const bool timing = thread_timing();
    if (timing) {
        AP_HIP(hipEventCreate(&ev.a), "hipEventCreate");
        AP_HIP(hipEventCreate(&ev.b), "hipEventCreate");
        AP_HIP(hipEventRecord(ev.a, st), "hipEventRecord");
    }
    // f2 needs no raise when every value it can take in the binary32 step is
    // positive and normal (see k_ap_map)
    const bool raise = !(p.f2_in >= FLT_MIN);
    const dim3 grid_dim(static_cast<uint32_t>(8 * p.per_xcd)), block_dim(64 * kApWaves);
    if (P == 2 && !raise)
        k_ap_map<2, false><<<grid_dim, block_dim, 0, st>>>(p);
    else if (P == 2)
        k_ap_map<2, true><<<grid_dim, block_dim, 0, st>>>(p);
    else if (!raise)
        k_ap_map<1, false><<<grid_dim, block_dim, 0, st>>>(p);
    else
        k_ap_map<1, true><<<grid_dim, block_dim, 0, st>>>(p);
    AP_HIP(hipGetLastError(), "k_ap_map");
    if (timing) AP_HIP(hipEventRecord(ev.b, st), "hipEventRecord");

    unsigned long long h_stats[2] = {0, 0};
    AP_HIP(hipMemcpyAsync(h_stats, stats, sizeof(h_stats), hipMemcpyDeviceToHost, st), "D2H stats");
    if (host_out) {
        AP_HIP(hipMemcpyAsync(map, d_map, sizeof(double) * static_cast<size_t>(m), hipMemcpyDeviceToHost, st),
               "D2H map");
        if (snr)
            AP_HIP(hipMemcpyAsync(snr, d_snr, sizeof(double) * static_cast<size_t>(m), hipMemcpyDeviceToHost, st),
                   "D2H snr");
        if (n_in)
            AP_HIP(hipMemcpyAsync(n_in, d_nin, sizeof(uint32_t) * static_cast<size_t>(m), hipMemcpyDeviceToHost,
                                  st),
                   "D2H n_in");
    }
    AP_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
    ApLast last;
    if (timing) {
        float ms = 0.0f;
        AP_HIP(hipEventElapsedTime(&ms, ev.a, ev.b), "hipEventElapsedTime");
        last.kernel_ms = ms;
    }
    last.tested = h_stats[0];
    last.in = h_stats[1];
    last.cell = L.s;
    t_ap = last;
    return PC_OK;
}

extern "C" int pc_debug_last_aperture(double *kernel_ms, uint64_t *pairs_tested, uint64_t *pairs_in,
                                      double *cell_side) {
    clear_error();
    if (kernel_ms) *kernel_ms = t_ap.kernel_ms;
    if (pairs_tested) *pairs_tested = t_ap.tested;
    if (pairs_in) *pairs_in = t_ap.in;
    if (cell_side) *cell_side = t_ap.cell;
    return PC_OK;
}

extern "C" int pc_debug_ap_filter(const double *x, int64_t n, double *q) {
    clear_error();
    if (n < 0 || (n > 0 && (!x || !q))) return fail(PC_ERR_INVALID, "NULL argument or n < 0");
    const float4 *tab = filter_table();
    for (int64_t k = 0; k < n; ++k) {
        // the kernel's steps in binary32: x clamped to [0, 1], s = kQCells x,
        // cell floor(s) (kQCells at x = 1), t = s - floor(s), Horner with
        // fused multiply-adds
        const float xf = std::fmin(std::fmax(static_cast<float>(x[k]), 0.0f), 1.0f);
        const float sv = xf * static_cast<float>(kQCells);
        const uint32_t i = static_cast<uint32_t>(sv);
        const float t = sv - std::floor(sv);
        const float4 c = tab[i];
        q[k] = std::fma(std::fma(std::fma(c.w, t, c.z), t, c.y), t, c.x);
    }
    return PC_OK;
}
