/*
 * pc_oracle.c -- CPU reference ("oracle") for exact angular pair counting.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg load it.  It shares no
 * code, header, table or constant generator with the GPU library.
 *
 * What it computes (paper, Sec. 2, Eq. 2 and Appendix A):
 *   DD / RR: every unordered pair i<j of one catalogue, n(n-1)/2 pairs, no
 *            self-pairs and no double counting (Sec. 2, pair counts);
 *   DR:      every (data, random) pair, n*n_r pairs (Sec. 2 and Sec. 2.1);
 *   each pair is binned by its great-circle separation theta (Appendix A).
 *
 * Readings taken where the paper is silent (each listed in the design notes):
 *   - theta is binned through the chord length: for unit vectors a, b the
 *     squared chord c = |a-b|^2 = 4 sin^2(theta/2) is monotone in theta on
 *     [0, 180] deg, so theta >= theta_k  <=>  c >= 4 sin^2(theta_k/2).  The
 *     paper's arctan form of Appendix A is read as atan2 (it is wrong for
 *     theta > 90 deg as printed); the chord form is the pinned definition.
 *   - bins are half-open [theta_k, theta_{k+1}); pairs below the first edge
 *     and at or above the last edge are kept in explicit under/overflow
 *     counters so the counts always sum to the number of pairs;
 *   - degrees are turned into sines and cosines by sincosd() below: exact
 *     reduction in degrees, then Taylor polynomials in +,-,* only, so that
 *     any IEEE-754 binary64 implementation of the same steps gets the same
 *     bits (no libm in the path);
 *   - all arithmetic is binary64, round-to-nearest, no fused multiply-add
 *     (build with -ffp-contract=off);
 *   - unit vector: x = cos(dec)cos(ra), y = cos(dec)sin(ra), z = sin(dec);
 *     chord: dx = xi-xj, ...; c = (dx*dx + dy*dy) + dz*dz, left to right;
 *     edge:  e_k = 4*(s*s), s = sin(theta_k/2) by sincosd;
 *     bin index = number of edges e_k <= c (0 = underflow, B+1 = overflow);
 *   - Landy-Szalay (Eq. 2) uses counts normalised by their pair totals:
 *     w = ((dd - 2 dr) + rr) / rr with dd = DD/(nD(nD-1)/2),
 *     dr = DR/(nD nR), rr = RR/(nR(nR-1)/2).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- sincosd */

/* pi/180 rounded to the nearest binary64 value. */
static const double DEG2RAD = 0x1.1df46a2529d39p-6;

/* n! as a double; exact for n <= 18 (18! < 2^53). */
static double factorial(int n)
{
    double f = 1.0;
    for (int k = 2; k <= n; ++k) f *= (double)k;
    return f;
}

/*
 * Sine and cosine of an angle in degrees.
 *   r = fmod(x, 360) in (-360, 360) (exact); q = nearest quarter turn
 *   (-4..4, ties away from the previous quadrant by strict compares);
 *   y = r - 90 q in [-45, 45] (exact: r and 90q are within a factor 2);
 *   t = y * (pi/180);
 *   sin t = t + t*(t^2 * P(t^2)),  P = sum_{m=1..8} (-1)^m t^{2(m-1)} / (2m+1)!
 *   cos t = 1 + t^2 * Q(t^2),      Q = sum_{m=1..9} (-1)^m t^{2(m-1)} / (2m)!
 * (Taylor series; the first omitted term is below 1e-19 for |t| <= pi/4),
 * each coefficient the binary64 value nearest 1/n!, evaluated by Horner.
 * The quarter turn is applied by the exact identities
 *   sin(y+90) = cos y, cos(y+90) = -sin y, and so on (q mod 4).
 */
void oracle_sincosd(double x, double *s_out, double *c_out)
{
    double r = fmod(x, 360.0);
    int q;
    if (r < -315.0) q = -4;
    else if (r < -225.0) q = -3;
    else if (r < -135.0) q = -2;
    else if (r < -45.0) q = -1;
    else if (r < 45.0) q = 0;
    else if (r < 135.0) q = 1;
    else if (r < 225.0) q = 2;
    else if (r < 315.0) q = 3;
    else q = 4;
    double y = r - 90.0 * (double)q;
    double t = y * DEG2RAD;
    double t2 = t * t;

    /* sine: odd terms 3, 5, ..., 17 */
    double p = 0.0;
    for (int n = 17; n >= 3; n -= 2) {
        double coef = 1.0 / factorial(n);
        if (((n - 1) / 2) % 2 == 1) coef = -coef;   /* n = 3, 7, 11, 15 negative */
        p = (n == 17) ? coef : p * t2 + coef;
    }
    double s = t + t * (t2 * p);

    /* cosine: even terms 2, 4, ..., 18 */
    double qq = 0.0;
    for (int n = 18; n >= 2; n -= 2) {
        double coef = 1.0 / factorial(n);
        if ((n / 2) % 2 == 1) coef = -coef;         /* n = 2, 6, 10, 14, 18 negative */
        qq = (n == 18) ? coef : qq * t2 + coef;
    }
    double c = 1.0 + t2 * qq;

    switch (((q % 4) + 4) % 4) {
    case 0: *s_out = s;  *c_out = c;  break;
    case 1: *s_out = c;  *c_out = -s; break;
    case 2: *s_out = -s; *c_out = -c; break;
    default: *s_out = -c; *c_out = s; break;
    }
}

/* ------------------------------------------------------------ unit vectors */

/* xyz[3*i + 0..2] = unit vector of (ra[i], dec[i]) in degrees. */
void oracle_unit_vectors(int64_t n, const double *ra, const double *dec, double *xyz)
{
    for (int64_t i = 0; i < n; ++i) {
        double sa, ca, sd, cd;
        oracle_sincosd(ra[i], &sa, &ca);
        oracle_sincosd(dec[i], &sd, &cd);
        xyz[3 * i + 0] = cd * ca;
        xyz[3 * i + 1] = cd * sa;
        xyz[3 * i + 2] = sd;
    }
}

/* e[k] = 4 sin^2(theta_k / 2): squared chord of the separation theta_k (deg). */
void oracle_chord2_edges(int32_t n_edges, const double *theta_deg, double *e)
{
    for (int32_t k = 0; k < n_edges; ++k) {
        double s, c;
        oracle_sincosd(0.5 * theta_deg[k], &s, &c);
        e[k] = 4.0 * (s * s);
    }
}

/* Number of edges e[k] <= c (edges strictly increasing). */
static int32_t bin_index(double c, int32_t n_edges, const double *e)
{
    int32_t lo = 0, hi = n_edges;           /* answer lies in [lo, hi] */
    while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (e[mid] <= c) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

static double chord2(const double *a, const double *b)
{
    double dx = a[0] - b[0];
    double dy = a[1] - b[1];
    double dz = a[2] - b[2];
    double c = dx * dx;
    c = c + dy * dy;
    c = c + dz * dz;
    return c;
}

/*
 * Pair counts from unit vectors.
 *   auto_flag = 1: pairs (i, j) of A with i < j, i in [row_begin, row_end);
 *   auto_flag = 0: pairs (i, j) in A x B, i in [row_begin, row_end).
 *   counts[0..n_edges] (n_edges + 1 entries) are overwritten:
 *   counts[idx] = number of pairs whose bin index (edges <= c) is idx.
 */
void oracle_count_xyz(int64_t nA, const double *xyzA, int64_t nB, const double *xyzB,
                      int32_t auto_flag, int32_t n_edges, const double *e,
                      int64_t row_begin, int64_t row_end, uint64_t *counts)
{
    int32_t nc = n_edges + 1;
    memset(counts, 0, sizeof(uint64_t) * (size_t)nc);
    if (row_end > nA) row_end = nA;
    if (row_begin < 0) row_begin = 0;
#pragma omp parallel
    {
        uint64_t *h = (uint64_t *)calloc((size_t)nc, sizeof(uint64_t));
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = row_begin; i < row_end; ++i) {
            const double *a = xyzA + 3 * i;
            if (auto_flag) {
                for (int64_t j = i + 1; j < nA; ++j)
                    h[bin_index(chord2(a, xyzA + 3 * j), n_edges, e)] += 1;
            } else {
                for (int64_t j = 0; j < nB; ++j)
                    h[bin_index(chord2(a, xyzB + 3 * j), n_edges, e)] += 1;
            }
        }
#pragma omp critical
        for (int32_t k = 0; k < nc; ++k) counts[k] += h[k];
        free(h);
    }
}

/* Pair counts straight from RA/Dec (degrees) and theta edges (degrees).
 * Returns 0, or -1 if memory runs out.  For auto_flag = 1, B is ignored. */
int oracle_count(int64_t nA, const double *raA, const double *decA,
                 int64_t nB, const double *raB, const double *decB,
                 int32_t auto_flag, int32_t n_edges, const double *theta_deg,
                 int64_t row_begin, int64_t row_end, uint64_t *counts)
{
    double *xa = (double *)malloc(sizeof(double) * 3 * (size_t)(nA > 0 ? nA : 1));
    double *xb = NULL;
    double *e = (double *)malloc(sizeof(double) * (size_t)n_edges);
    if (!xa || !e) { free(xa); free(e); return -1; }
    oracle_unit_vectors(nA, raA, decA, xa);
    if (!auto_flag) {
        xb = (double *)malloc(sizeof(double) * 3 * (size_t)(nB > 0 ? nB : 1));
        if (!xb) { free(xa); free(e); return -1; }
        oracle_unit_vectors(nB, raB, decB, xb);
    }
    oracle_chord2_edges(n_edges, theta_deg, e);
    oracle_count_xyz(nA, xa, nB, xb, auto_flag, n_edges, e, row_begin, row_end, counts);
    free(xa); free(xb); free(e);
    return 0;
}

/*
 * Landy-Szalay estimator (Eq. 2) on normalised counts, for n_bins bins:
 *   w[k] = ((dd - 2 dr) + rr) / rr.  rr = 0 gives NaN (no error).
 */
void oracle_wtheta(const uint64_t *DD, const uint64_t *DR, const uint64_t *RR, int32_t n_bins,
                   int64_t nD, int64_t nR, double *w)
{
    double fD = (double)nD, fR = (double)nR;
    double nDD = 0.5 * fD * (fD - 1.0);
    double nDR = fD * fR;
    double nRR = 0.5 * fR * (fR - 1.0);
    for (int32_t k = 0; k < n_bins; ++k) {
        double dd = (double)DD[k] / nDD;
        double dr = (double)DR[k] / nDR;
        double rr = (double)RR[k] / nRR;
        w[k] = ((dd - 2.0 * dr) + rr) / rr;
    }
}

/* The other usual estimators on the same normalised counts (Sec. 2 notes that
 * the choice of estimator is open): kind 1 natural dd/rr - 1, kind 2
 * Davis-Peebles dd/dr - 1, kind 3 Hamilton dd*rr/dr^2 - 1; kind 0 is
 * oracle_wtheta.  Each written from its textbook definition. */
void oracle_estimator(int32_t kind, const uint64_t *DD, const uint64_t *DR, const uint64_t *RR,
                      int32_t n_bins, int64_t nD, int64_t nR, double *w)
{
    if (kind == 0) {
        oracle_wtheta(DD, DR, RR, n_bins, nD, nR, w);
        return;
    }
    double fD = (double)nD, fR = (double)nR;
    double nDD = 0.5 * fD * (fD - 1.0);
    double nDR = fD * fR;
    double nRR = 0.5 * fR * (fR - 1.0);
    for (int32_t k = 0; k < n_bins; ++k) {
        double dd = (double)DD[k] / nDD;
        double dr = DR ? (double)DR[k] / nDR : 0.0;
        double rr = RR ? (double)RR[k] / nRR : 0.0;
        double ratio;
        if (kind == 1)
            ratio = dd / rr;
        else if (kind == 2)
            ratio = dd / dr;
        else
            ratio = (dd * rr) / (dr * dr);
        w[k] = ratio - 1.0;
    }
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the number of threads later calls use (n >= 1); a no-op without OpenMP.
 * Used to time the oracle on one core, the comparison the paper's speed-ups
 * are quoted against (Sec. 4, Table 1). */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}
