// pc_tables.cpp -- host construction of the per-edge-set tables.
//
// Binning is done on the squared chord c = |a - b|^2 = 4 sin^2(theta/2) of the
// unit vectors a, b (the separation of Appendix A, through a monotone map), so
// an edge theta_k becomes e_k = 4 sin^2(theta_k/2).
//
// The mixed kernel computes c in binary32 (c32) and must still bin every pair
// exactly as the binary64 definition (c64) does.  guard_band() gives, for each
// edge, binary32 limits lo <= hi such that c32 > hi proves c64 >= e and c32 < lo
// proves c64 < e; only pairs with lo <= c32 <= hi are re-computed in binary64.
//
// Error bound (u = 2^-24, v = 2^-53, t = 2^-126 for underflow or flush-to-zero,
// c = |a-b|^2 exactly for the binary64 unit vectors a, b, |a|, |b| <= 1 + 2^-40):
//   * rounding a, b to binary32 moves each component by <= u|a_i| + t, and the
//     binary32 difference adds <= u|d_i| + t, so the computed difference vector
//     s satisfies |s - d| <= d0 + u sqrt(c),  d0 = 2u(1+u)^2(1+2^-40) + 6t;
//   * |(|s|^2) - c| <= D (2 sqrt(c) + D) with D = d0 + u sqrt(c);
//   * the sum of three squares, with or without fused multiply-add, has
//     relative error <= g3 = 3u/(1-3u), plus <= 5t absolute from underflow;
//   => |c32 - c| <= E(c) = D(2 sqrt c + D) + g3 (sqrt c + D)^2 + 5t.
//   * the binary64 chord (3 subtractions, 3 products, 2 sums) has
//     |c64 - c| <= g5 c + 5*2^-1074, g5 = 5v/(1-5v).
// If c64 < e then c < e+ = (e + 5*2^-1074)/(1 - g5) and c32 <= e+ + E(e+) since E
// is increasing: hi = RU32(e+ + K E(e+)).  If c64 >= e then c >= e- =
// (e - 5*2^-1074)/(1 + g5) and c32 >= e- - E(e-) because c - E(c) increases for
// sqrt(c) beyond ~d0: lo = RD32(e- - K E(e-)) when sqrt(e-) >= 4 K d0, else
// -inf (every c32 <= hi is re-checked).  K = 2 is a safety factor that also
// covers the binary64 rounding of these host formulas.  e = 0 needs no band
// (c64 >= 0 always): lo = hi = -inf.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <string>
#include <vector>

#include "pc_internal.hpp"
#include "pc_math.h"
#include "pc_runtime.hpp"

namespace pc {

namespace {

constexpr double kU = 0x1p-24;
constexpr double kV = 0x1p-53;
constexpr double kTau = 0x1p-126;
constexpr double kK = 2.0;

inline uint32_t f2u(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
inline float u2f(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }
inline uint64_t d2u(double d) { uint64_t u; memcpy(&u, &d, 8); return u; }
inline double u2d(uint64_t u) { double d; memcpy(&d, &u, 8); return d; }

double delta0() { return 2.0 * kU * (1.0 + kU) * (1.0 + kU) * (1.0 + 0x1p-40) + 6.0 * kTau; }

// |c32 - c| <= E(c)
double err32(double c) {
    const double r = std::sqrt(c);
    const double D = delta0() + kU * r;
    const double g3 = 3.0 * kU / (1.0 - 3.0 * kU);
    return D * (2.0 * r + D) + g3 * (r + D) * (r + D) + 5.0 * kTau;
}

float round_up32(double x) {
    float f = static_cast<float>(x);
    if (static_cast<double>(f) < x) f = std::nextafter(f, std::numeric_limits<float>::infinity());
    return f;
}

float round_down32(double x) {
    float f = static_cast<float>(x);
    if (static_cast<double>(f) > x) f = std::nextafter(f, -std::numeric_limits<float>::infinity());
    return f;
}

}  // namespace

// Band from an error bound E(c) that is increasing in c with E(c)/c
// decreasing: hi from e+ ; lo from e- when K E(e-) <= e-/2 (then c - K E(c)
// is increasing for c >= e-, since E'(c) <= E(c)/c), else -inf.
template <typename ErrFn>
void band_from(double e, ErrFn err, float *lo, float *hi) {
    const float ninf = -std::numeric_limits<float>::infinity();
    if (e <= 0.0) {
        *lo = ninf;
        *hi = ninf;
        return;
    }
    const double g5 = 5.0 * kV / (1.0 - 5.0 * kV);
    // outward by a further 8v for the rounding of these expressions
    const double ep = (e + 5.0 * 0x1p-1074) / (1.0 - g5) * (1.0 + 8.0 * kV);
    const double em = (e - 5.0 * 0x1p-1074) / (1.0 + g5) * (1.0 - 8.0 * kV);
    *hi = round_up32(ep + kK * err(ep));
    const double ke = kK * err(em);
    if (em > 0.0 && ke <= 0.5 * em) *lo = round_down32(em - ke);
    else *lo = ninf;
}

void guard_band(double e, float *lo, float *hi) { band_from(e, err32, lo, hi); }

// Tile-centred chords (the matrix-core path).  o = centre of whichever tile
// of the pair has the smaller bounding radius r; say the i-tile (the other
// case swaps the roles of a and b).  A = a - o with |A| <= r, B = b - o with
// |B| <= |b - a| + |a - o| <= sqrt(c) + r.  The binary32 copies a' = RN(A),
// b' = RN(B) (A, B formed in binary64) move by alpha <= u r (1+2^-52) +
// sqrt(3) t and beta <= u (sqrt(c) + r)(1+2^-52) + sqrt(3) t; |a'|^2 and
// |b'|^2 are formed in binary32 (3 roundings each, g3); the matrix core sums
// |a'|^2 + |b'|^2 - 2 a'.b' from 4 products and an addend, bounded here by 8
// roundings on the sum of absolute terms, <= g8 (|a'| + |b'|)^2 (1 + g3)
// (denormal operands flushed to zero are covered by the t terms).  Then
//   |c32 - c| <= 2 sqrt(c)(alpha + beta) + (alpha + beta)^2
//                + g3 (|a'|^2 + |b'|^2) + g8 (|a'| + |b'|)^2 (1 + g3) + 20 t.
// The path only takes tile pairs whose chord lower bound is at least 2r, so
// r <= sqrt(c)/2 for every pair it sees; the bound grows with r and is taken
// at r = sqrt(c)/2, which makes it relative (about 50 u c) plus underflow
// terms: increasing in c, with E(c)/c decreasing, as band_from needs.
double err_gram(double c) {
    const double sc = std::sqrt(c);
    const double r = 0.5 * sc;
    const double al = kU * r * (1.0 + 0x1p-52) + 1.7320508075688772 * kTau;
    const double be = kU * (sc + r) * (1.0 + 0x1p-52) + 1.7320508075688772 * kTau;
    const double na = r + al, nb = sc + r + be;
    const double g3 = 3.0 * kU / (1.0 - 3.0 * kU);
    const double g8 = 8.0 * kU / (1.0 - 8.0 * kU);
    return 2.0 * sc * (al + be) + (al + be) * (al + be) + g3 * (na * na + nb * nb) +
           g8 * (na + nb) * (na + nb) * (1.0 + g3) + 20.0 * kTau;
}

void guard_band_gram(double e, float *lo, float *hi) { band_from(e, err_gram, lo, hi); }

// ---- fused few-edge thresholds ---------------------------------------------
//
// The vector few-edge paths never round the chord itself: with the item's
// smallest edge as reference (threshold h_ref), they form d_ref = h_ref - c in
// one chain of roundings, and for the item's other edges d_t = RN(d_ref +
// D_t), D_t = RN32(h_t - h_ref) >= 0; the sign bit of d_t is (chord above edge
// t), and 0 <= d_t <= W_t flags the chord for the binary64 re-check.  (The
// prune pass never puts an edge at 0 in a few-edge item: every chord is at or
// above it.)
//   * difference form: d_ref = RN(-s_z^2 + RN(-s_y^2 + RN(h - s_x^2))), three
//     fused multiply-adds on the binary32 differences s (|s - d| <= D as for
//     guard_band); q = |s|^2 exactly has |q - c| <= D (2 sqrt c + D); each
//     partial result is h less a partial sum of squares, at most max(h, q) in
//     magnitude, so the three roundings add <= g3 max(h, q);
//   * Gram form (tile-centred, as guard_band_gram, r <= sqrt(c)/2): na =
//     RN(|a'|^2), bw = RN(|b'|^2) (g3 each), S = RN(h - na), T = RN(S - bw),
//     then three fused multiply-adds of 2 a'_k b'_k: five roundings on values
//     of at most max(h, (|a'| + |b'|)^2 (1 + g3));
//   * an edge that is not the reference adds the rounding of D_t (<= u h_t)
//     and of the sum (<= u |d_t| <= u max(h_t, c) to first order).
// The reference is at or below edge t, so H >= h_t >= h_ref bounds every
// threshold in the chain, and E_t(c) (the chain's bound at H plus g2 (H +
// max(H, c))) bounds |d_t - (h_t - c)|; it grows with c, and E_t'(c) < 1.
// H starts at 2 e+ and is then lowered to the threshold h_t found with it
// (a smaller H gives a smaller h_t, so H >= h_t still holds).  Then, with e+
// and e- as in band_from:
//   h_t = RU32(e+ + K E_t(e+)):  d_t < 0 means c > h_t - E_t(c), so c > e+
//        (otherwise c <= e+ and h_t - E_t(c) >= e+), hence c64 >= e;
//   W_t = RU32(h_t - e- + K E_t(e-)):  a chord with c >= e- has d_t <= h_t - c
//        + E_t(c) <= h_t - e- + E_t(e-) <= W_t, so d_t > W_t means c < e-,
//        hence c64 < e.
// An edge at 0 needs no band: h = -FLT_MAX (every d is negative: above it)
// and W = 0 (a d of +0 cannot occur there).
namespace {

double err_diff_fused(double c, double H) {
    const double r = std::sqrt(c);
    const double D = delta0() + kU * r;
    const double g3 = 3.0 * kU / (1.0 - 3.0 * kU);
    return D * (2.0 * r + D) + g3 * std::max(H, (r + D) * (r + D)) + 8.0 * kTau;
}

double err_gram_fused(double c, double H) {
    const double sc = std::sqrt(c);
    const double r = 0.5 * sc;
    const double al = kU * r * (1.0 + 0x1p-52) + 1.7320508075688772 * kTau;
    const double be = kU * (sc + r) * (1.0 + 0x1p-52) + 1.7320508075688772 * kTau;
    const double na = r + al, nb = sc + r + be;
    const double g3 = 3.0 * kU / (1.0 - 3.0 * kU);
    const double g5 = 5.0 * kU / (1.0 - 5.0 * kU);
    return 2.0 * sc * (al + be) + (al + be) * (al + be) + g3 * (na * na + nb * nb) +
           g5 * std::max(H, (na + nb) * (na + nb) * (1.0 + g3)) + 20.0 * kTau;
}

}  // namespace

void fused_bands(const std::vector<double> &e64, bool gram, std::vector<float> &h, std::vector<float> &w) {
    const size_t n = e64.size();
    h.assign(n, -std::numeric_limits<float>::max());
    w.assign(n, 0.0f);
    const double g5 = 5.0 * kV / (1.0 - 5.0 * kV);
    const double g2 = 2.0 * kU / (1.0 - 2.0 * kU);
    auto eplus = [&](double e) { return (e + 5.0 * 0x1p-1074) / (1.0 - g5) * (1.0 + 8.0 * kV); };
    auto eminus = [&](double e) { return (e - 5.0 * 0x1p-1074) / (1.0 + g5) * (1.0 - 8.0 * kV); };
    // H bounds the edge's own threshold, hence the reference's (at most two
    // edges down); thresholds come out within a few hundred ulp of e+, and the
    // loop widens H should one not fit under it
    std::vector<double> H(n);
    for (size_t k = 0; k < n; ++k) H[k] = 2.0 * eplus(e64[k]);
    for (int pass = 0; pass < 8; ++pass) {
        for (size_t k = 0; k < n; ++k) {
            const double e = e64[k];
            if (e <= 0.0) continue;
            auto E = [&](double c) {
                const double base = gram ? err_gram_fused(c, H[k]) : err_diff_fused(c, H[k]);
                return base + g2 * (H[k] + std::max(H[k], c)) + 2.0 * kTau;
            };
            const double ep = eplus(e), em = eminus(e);
            const float hk = round_up32(ep + kK * E(ep));
            h[k] = hk;
            w[k] = round_up32((static_cast<double>(hk) - em + kK * E(std::max(em, 0.0))) * (1.0 + 4.0 * kV));
        }
        // first pass: lower H to the thresholds found; later passes: done
        // once every threshold fits under its H
        bool fits = pass > 0;
        for (size_t k = 0; k < n; ++k) {
            if (h[k] > H[k]) {
                H[k] = 2.0 * h[k];
                fits = false;
            } else if (pass == 0 && e64[k] > 0.0) {
                H[k] = h[k];
            }
        }
        if (fits) return;
    }
}

namespace {

// ---- binary32 cell table ------------------------------------------------
//
// Cell key = bits of c32 clamped to [clamp_lo, clamp_hi]; cell = key >> S.
// For a cell with value range [mn, mx]: k_base = #bands wholly below (hi < mn);
// if exactly one band meets the cell, entry = (k_base, k_base+1, lo, hi);
// none: (k_base, k_base, +inf, +inf); several: (k_base, k_base, -inf, +inf),
// i.e. always re-check.  Bands are sorted (lo and hi non-decreasing in e).

void build_lut32(const std::vector<float> &lo, const std::vector<float> &hi, uint32_t row_bytes, Lut32 &out) {
    const int n = static_cast<int>(lo.size());
    const float inf = std::numeric_limits<float>::infinity();
    float lo_min = inf, hi_max = -inf;
    bool any_neg_lo = false;
    for (int k = 0; k < n; ++k) {
        if (hi[k] < 0.0f) continue;  // always below every c32
        if (lo[k] <= 0.0f) any_neg_lo = true;
        lo_min = std::min(lo_min, lo[k]);
        hi_max = std::max(hi_max, hi[k]);
    }
    if (hi_max < 0.0f) {  // every edge always passed: one cell
        lo_min = 1.0f;
        hi_max = 1.0f;
    }
    const uint32_t clo = any_neg_lo ? 0u : f2u(lo_min);
    const uint32_t chi = f2u(hi_max);
    // band cell-key intervals (lo clipped at +0)
    auto key_lo = [&](int k) { return lo[k] <= 0.0f ? 0u : f2u(lo[k]); };
    int best_s = -1, best_multi = 1 << 30;
    for (int s = 23; s >= 4; --s) {
        const uint64_t cells = static_cast<uint64_t>(chi >> s) - (clo >> s) + 1;
        if (cells > static_cast<uint64_t>(kMaxLutCells)) break;
        int multi = 0;
        int prev = -1;
        for (int k = 0; k < n; ++k) {
            if (hi[k] < 0.0f) continue;
            if (prev >= 0 && (f2u(hi[prev]) >> s) >= (key_lo(k) >> s)) ++multi;
            prev = k;
        }
        if (multi < best_multi) {
            best_multi = multi;
            best_s = s;
        }
        if (multi == 0) break;
    }
    if (best_s < 0) best_s = 23;  // cannot happen: S = 23 needs < 300 cells
    const uint32_t s = static_cast<uint32_t>(best_s);
    out.shift = s;
    out.clamp_lo = clo;
    out.clamp_hi = chi;
    const uint32_t c0 = clo >> s, c1 = chi >> s;
    out.entries.clear();
    out.multi = 0;
    for (uint32_t c = c0; c <= c1; ++c) {
        const float mn = u2f(c << s);
        const float mx = u2f(static_cast<uint32_t>(((static_cast<uint64_t>(c) + 1) << s) - 1));
        uint32_t k_base = 0;
        int n_in = 0, k_in = -1;
        for (int k = 0; k < n; ++k) {
            if (hi[k] < mn) ++k_base;
            else if (lo[k] <= mx) { ++n_in; k_in = k; }
        }
        LutEntry32 e;
        e.off_lo = k_base * row_bytes;
        if (n_in == 0) {
            e.wbits = 0u;
            e.lo = inf;
            e.hi = inf;
        } else if (n_in == 1) {
            e.lo = lo[k_in];
            e.hi = hi[k_in];
            e.wbits = f2u(e.hi - e.lo);  // binary32 subtraction, as the kernel's
        } else {
            e.wbits = 0xFFFFFFFFu;
            e.lo = -inf;
            e.hi = inf;
            ++out.multi;
        }
        out.entries.push_back(e);
    }
}

// ---- binary64 cell table ------------------------------------------------
//
// Cell key = high 32 bits of c64 clamped; cell = key >> S.  For a cell with
// value range [mn, mx]: k_base = #edges <= mn; at most one edge may lie in
// (mn, mx]; entry = (k_base, k_base+1, that edge) or (k_base, k_base, +inf).
// When no S within the size budget isolates every edge, the kernel falls back
// to a binary search over the edges for every pair.

void build_lut64(HostTable &t) {
    const int n = static_cast<int>(t.e64.size());
    double e_pos = 0.0;
    for (int k = 0; k < n; ++k)
        if (t.e64[k] > 0.0) { e_pos = t.e64[k]; break; }
    const double below = std::nextafter(e_pos, 0.0);
    const uint32_t clo = static_cast<uint32_t>(d2u(below) >> 32);
    const uint32_t chi = static_cast<uint32_t>(d2u(t.e64[n - 1]) >> 32);
    auto count_le = [&](double x) {
        return static_cast<uint32_t>(std::upper_bound(t.e64.begin(), t.e64.end(), x) - t.e64.begin());
    };
    int chosen = -1;
    for (int s = 20; s >= 0; --s) {
        const uint64_t cells = static_cast<uint64_t>(chi >> s) - (clo >> s) + 1;
        if (cells > static_cast<uint64_t>(kMaxLutCells)) break;
        bool ok = true;
        for (uint32_t c = clo >> s; c <= (chi >> s) && ok; ++c) {
            const double mn = u2d(static_cast<uint64_t>(c << s) << 32);
            const double mx = u2d((static_cast<uint64_t>((static_cast<uint64_t>(c) + 1) << s) << 32) - 1);
            if (count_le(mx) - count_le(mn) > 1) ok = false;
        }
        if (ok) { chosen = s; break; }
    }
    t.lut64.clear();
    if (chosen < 0) {
        t.search64 = true;
        t.shift64 = 0;
        t.clamp_lo64 = clo;
        t.clamp_hi64 = clo;
        return;
    }
    t.search64 = false;
    const uint32_t s = static_cast<uint32_t>(chosen);
    t.shift64 = s;
    t.clamp_lo64 = clo;
    t.clamp_hi64 = chi;
    for (uint32_t c = clo >> s; c <= (chi >> s); ++c) {
        const double mn = u2d(static_cast<uint64_t>(c << s) << 32);
        const double mx = u2d((static_cast<uint64_t>((static_cast<uint64_t>(c) + 1) << s) << 32) - 1);
        const uint32_t kb = count_le(mn), kt = count_le(mx);
        LutEntry64 e;
        e.off_lo = kb * t.row_bytes64;
        if (kt == kb) {
            e.off_hi = e.off_lo;
            e.e = std::numeric_limits<double>::infinity();
        } else {
            e.off_hi = (kb + 1) * t.row_bytes64;
            e.e = t.e64[kb];
        }
        t.lut64.push_back(e);
    }
}

}  // namespace

bool validate_edges(const double *theta_deg, int n_edges, std::string &err) {
    if (!theta_deg) {
        err = "theta_edges_deg is NULL";
        return false;
    }
    if (n_edges < 2) {
        err = "n_edges must be >= 2";
        return false;
    }
    if (n_edges > kMaxEdges) {
        err = "n_edges must be <= 1024";
        return false;
    }
    for (int k = 0; k < n_edges; ++k) {
        const double x = theta_deg[k];
        if (!std::isfinite(x) || x < 0.0 || x > 180.0) {
            err = "theta edges must be finite and in [0, 180] degrees";
            return false;
        }
        if (k > 0 && !(x > theta_deg[k - 1])) {
            err = "theta edges must be strictly increasing";
            return false;
        }
    }
    return true;
}

bool build_table(const double *theta_deg, int n_edges, HostTable &t, std::string &err, int cols32) {
    if (!validate_edges(theta_deg, n_edges, err)) return false;
    t.theta.assign(theta_deg, theta_deg + n_edges);
    t.e64.resize(n_edges);
    t.lo.resize(n_edges);
    t.hi.resize(n_edges);
    t.lo_g.resize(n_edges);
    t.hi_g.resize(n_edges);
    for (int k = 0; k < n_edges; ++k) {
        t.e64[k] = chord2_of_theta(theta_deg[k]);
        guard_band(t.e64[k], &t.lo[k], &t.hi[k]);
        guard_band_gram(t.e64[k], &t.lo_g[k], &t.hi_g[k]);
    }
    fused_bands(t.e64, false, t.fh, t.fw);
    fused_bands(t.e64, true, t.fh_g, t.fw_g);
    // widest histogram (up to the kernel's preferred width, at least `narrowest`
    // columns) that keeps the per-wave histogram, plus `extra` bytes of table,
    // within the LDS target; narrower histograms let more waves share a CU
    auto pick = [&](int widest, int narrowest, uint64_t extra) {
        for (int c = widest; c > narrowest; c >>= 1)
            if (static_cast<uint64_t>(n_edges + 3) * row_bytes_for(c) + extra <= kLdsTarget) return c;
        return narrowest;
    };
    if (cols32 != 0 && (cols32 < 4 || cols32 > 64 || (cols32 & (cols32 - 1)) != 0)) {
        err = "histogram columns must be a power of two in [4, 64]";
        return false;
    }
    t.cols64 = pick(PC_COLS64, 8, 0);
    t.row_bytes64 = row_bytes_for(t.cols64);
    if (cols32) {
        t.cols32 = cols32;
    } else {
        // the mixed kernel's cell table shares the wave's LDS with its
        // histogram (the table's size does not depend on the columns)
        build_lut32(t.lo, t.hi, row_bytes_for(PC_COLS32), t.lut32);
        t.cols32 = pick(PC_COLS32, 4, sizeof(LutEntry32) * t.lut32.entries.size());
    }
    t.row_bytes32 = row_bytes_for(t.cols32);
    build_lut32(t.lo, t.hi, t.row_bytes32, t.lut32);
    // the 8-byte form of the same cells, when every row offset fits in the
    // low bits of the rounded-up width
    t.lut32.compact.clear();
    bool fits = true;
    for (const LutEntry32 &e : t.lut32.entries) fits = fits && e.off_lo <= kCtOffMask;
    if (fits) {
        t.lut32.compact.reserve(t.lut32.entries.size());
        for (const LutEntry32 &e : t.lut32.entries) {
            const uint64_t up = (static_cast<uint64_t>(e.wbits) + kCtOffMask) & ~static_cast<uint64_t>(kCtOffMask);
            const uint32_t w = up > 0xFFFFFFFFull ? ~kCtOffMask : static_cast<uint32_t>(up);
            t.lut32.compact.push_back({f2u(e.hi), w | e.off_lo});
        }
    }
    build_lut64(t);
    return true;
}

}  // namespace pc

// ------------------------------------------------------------- bin presets
//
// The paper's three preset bin widths (Sec. 2.1: the user sets the low and
// high limits of the histogram and picks evenly spaced, natural-log or
// base-10-log bins).  In the preset's scale F (theta, ln theta, log10 theta)
// the edges are F^-1(F(lo) + k w) for k = 0 .. n-1, then hi exactly, with w
// = (F(hi) - F(lo)) / n_bins, or the given width and n = ceil((F(hi) -
// F(lo)) / width) (the last bin narrower when the range is not a whole
// number of widths).  Equal widths in ln and in log10 give the same edges
// (up to rounding): the two presets differ in the units of the width.
extern "C" int pc_bin_edges(int32_t preset, double lo_deg, double hi_deg, int32_t n_bins, double width,
                            int32_t max_edges, double *edges, int32_t *n_edges) {
    pc::clear_error();
    if (!n_edges) return pc::fail(PC_ERR_INVALID, "n_edges is NULL");
    if (preset < PC_BINS_EVEN || preset > PC_BINS_LOG10) return pc::fail(PC_ERR_INVALID, "unknown bin preset");
    if (!std::isfinite(lo_deg) || !std::isfinite(hi_deg) || !(lo_deg < hi_deg) || lo_deg < 0.0 || hi_deg > 180.0)
        return pc::fail(PC_ERR_INVALID, "need 0 <= lo < hi <= 180 degrees");
    if (preset != PC_BINS_EVEN && !(lo_deg > 0.0))
        return pc::fail(PC_ERR_INVALID, "logarithmic bins need lo > 0");
    auto F = [&](double x) { return preset == PC_BINS_EVEN ? x : preset == PC_BINS_LN ? std::log(x) : std::log10(x); };
    auto Finv = [&](double y) {
        return preset == PC_BINS_EVEN ? y : preset == PC_BINS_LN ? std::exp(y) : std::pow(10.0, y);
    };
    const double f0 = F(lo_deg), f1 = F(hi_deg), span = f1 - f0;
    double w = 0.0;
    int64_t n = 0;
    if (n_bins > 0) {
        n = n_bins;
        w = span / static_cast<double>(n);
    } else {
        if (!(width > 0.0) || !std::isfinite(width)) return pc::fail(PC_ERR_INVALID, "need n_bins > 0 or width > 0");
        const double q = span / width;
        n = static_cast<int64_t>(std::ceil(q * (1.0 - 1e-12)));
        if (n < 1) n = 1;
        if (q > 1e7) return pc::fail(PC_ERR_INVALID, "more than 1023 bins");
        w = width;
    }
    if (n + 1 > pc::kMaxEdges) return pc::fail(PC_ERR_INVALID, "more than 1023 bins");
    std::vector<double> e(static_cast<size_t>(n) + 1);
    e[0] = lo_deg;
    for (int64_t k = 1; k < n; ++k) e[static_cast<size_t>(k)] = Finv(f0 + static_cast<double>(k) * w);
    e[static_cast<size_t>(n)] = hi_deg;
    std::string err;
    if (!pc::validate_edges(e.data(), static_cast<int>(e.size()), err))
        return pc::fail(PC_ERR_INVALID, "preset gives unusable edges: " + err);
    *n_edges = static_cast<int32_t>(e.size());
    if (edges && max_edges >= static_cast<int32_t>(e.size())) memcpy(edges, e.data(), sizeof(double) * e.size());
    else if (edges) return pc::fail(PC_ERR_INVALID, "edges buffer holds fewer than n_edges values");
    return PC_OK;
}
