/*
 * ap_oracle.c -- CPU reference ("oracle") for aperture-mass maps.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg load it.  It shares no
 * code, header, table or constant generator with the GPU library.
 *
 * What it computes (paper, Sec. 3, Eq. 3, Eq. 4 and Eq. 5): for each
 * reconstruction point p, a sum over the galaxies i that lie inside the
 * filter radius theta_max of p:
 *   x_i      = |theta_i - p| / theta_max
 *   Q(x)     = 1 / (1 + exp(6 - 150 x) + exp(-47 + 50 x)) * tanh(x/0.15) / (x/0.15)   (Eq. 4)
 *   eps_t,i  = tangential ellipticity of galaxy i about p
 *   M_ap(p)  = (1/n_gal) * sum_i Q(x_i) eps_t,i                                     (Eq. 3)
 *   SNR(p)   = sqrt(2) * sum_i Q(x_i) eps_t,i / sqrt(sum_i Q(x_i)^2 |eps_i|^2)         (Eq. 5)
 *
 * Readings taken where the paper is silent (each listed in the design notes):
 *   - positions are flat-sky tangent-plane coordinates (x, y), in the same
 *     unit as theta_max (the paper's field is a few square degrees);
 *   - the position angle phi of galaxy i about p is measured from the +x
 *     axis, and eps_t = -(e1 cos 2phi + e2 sin 2phi), so that ellipticities
 *     aligned tangentially around p give eps_t > 0; with d = theta_i - p,
 *     cos 2phi = (dx^2 - dy^2)/|d|^2 and sin 2phi = 2 dx dy/|d|^2;
 *   - n_gal in Eq. 3 is a number density supplied by the caller;
 *   - Eq. 5 uses eps_t in the numerator and |eps|^2 = e1^2 + e2^2 in the
 *     denominator; with no galaxy in the aperture (or all |eps| = 0) the SNR
 *     is NaN;
 *   - "galaxies that contribute" are those with 0 < |d|^2 < theta_max^2,
 *     where |d|^2 = dx*dx + dy*dy in binary64, dx = x_i - x_p, dy = y_i - y_p,
 *     no fused multiply-add: the cut is a decision, so it is pinned to these
 *     exact operations.  A galaxy exactly on p has no tangential direction
 *     and is left out;
 *   - grid point (ix, iy) is (x0 + ix*dx, y0 + iy*dy) in binary64 (product
 *     then sum, no fused multiply-add), stored at index iy*nx + ix;
 *   - tanh(u)/u is 1 at u = 0.
 * All arithmetic is binary64 (libm exp, tanh, sqrt), no contraction.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

/* Eq. 4: the filter matched to an NFW halo profile, x = theta / theta_max. */
double oracle_q_nfw(double x)
{
    double logistic = 1.0 / (1.0 + exp(6.0 - 150.0 * x) + exp(-47.0 + 50.0 * x));
    double u = x / 0.15;
    double shape = (u == 0.0) ? 1.0 : tanh(u) / u;
    return logistic * shape;
}

/*
 * Aperture mass at n_pts points (px, py).  Outputs per point: map (Eq. 3),
 * snr (Eq. 5), n_in (galaxies inside the aperture) and, when sums is not
 * NULL, sums[3p..3p+2] = (sum Q eps_t, sum Q^2 |eps|^2, sum Q |eps|).
 */
void oracle_aperture_points(int64_t n, const double *gx, const double *gy, const double *e1, const double *e2,
                            int64_t n_pts, const double *px, const double *py, double theta_max, double n_gal,
                            double *map, double *snr, uint32_t *n_in, double *sums)
{
    const double r2 = theta_max * theta_max;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < n_pts; ++p) {
        double s1 = 0.0, s2 = 0.0, sa = 0.0;
        uint32_t cnt = 0;
        for (int64_t i = 0; i < n; ++i) {
            double dx = gx[i] - px[p];
            double dy = gy[i] - py[p];
            double d2 = dx * dx + dy * dy;
            if (!(d2 > 0.0 && d2 < r2)) continue;
            double q = oracle_q_nfw(sqrt(d2) / theta_max);
            double cos2 = (dx * dx - dy * dy) / d2;
            double sin2 = (2.0 * dx * dy) / d2;
            double et = -(e1[i] * cos2 + e2[i] * sin2);
            double ee = e1[i] * e1[i] + e2[i] * e2[i];
            s1 += q * et;
            s2 += (q * q) * ee;
            sa += q * sqrt(ee);
            cnt += 1;
        }
        map[p] = s1 / n_gal;
        snr[p] = (s2 > 0.0) ? (sqrt(2.0) * s1) / sqrt(s2) : NAN;
        n_in[p] = cnt;
        if (sums) {
            sums[3 * p + 0] = s1;
            sums[3 * p + 1] = s2;
            sums[3 * p + 2] = sa;
        }
    }
}

/* The same on the nx*ny grid (x0 + ix*dx, y0 + iy*dy), row-major in iy. */
int oracle_aperture_grid(int64_t n, const double *gx, const double *gy, const double *e1, const double *e2,
                         double x0, double y0, double dx, double dy, int32_t nx, int32_t ny, double theta_max,
                         double n_gal, double *map, double *snr, uint32_t *n_in, double *sums)
{
    int64_t m = (int64_t)nx * (int64_t)ny;
    double *px = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    double *py = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    if (!px || !py) {
        free(px);
        free(py);
        return 1;
    }
    for (int32_t iy = 0; iy < ny; ++iy)
        for (int32_t ix = 0; ix < nx; ++ix) {
            int64_t p = (int64_t)iy * nx + ix;
            px[p] = x0 + (double)ix * dx;
            py[p] = y0 + (double)iy * dy;
        }
    oracle_aperture_points(n, gx, gy, e1, e2, m, px, py, theta_max, n_gal, map, snr, n_in, sums);
    free(px);
    free(py);
    return 0;
}
