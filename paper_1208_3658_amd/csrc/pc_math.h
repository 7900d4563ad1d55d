// pc_math.h -- binary64 arithmetic shared by the library's host and device code.
//
// Everything here must give the same bits on the CPU (table construction) and
// on gfx950 (conversion kernel, re-check), so only IEEE-754 +, -, * and the
// exact fmod are used, with contraction disabled.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pc {

// 1/n! rounded to binary64 (n! itself is exact in binary64 for n <= 18).
constexpr double inv_factorial(int n) {
    double f = 1.0;
    for (int k = 2; k <= n; ++k) f *= static_cast<double>(k);
    return 1.0 / f;
}

// Taylor coefficients of sin t / t - 1 (in t^2) and (cos t - 1) / t^2.
constexpr double kS3 = -inv_factorial(3), kS5 = inv_factorial(5), kS7 = -inv_factorial(7),
                 kS9 = inv_factorial(9), kS11 = -inv_factorial(11), kS13 = inv_factorial(13),
                 kS15 = -inv_factorial(15), kS17 = inv_factorial(17);
constexpr double kC2 = -inv_factorial(2), kC4 = inv_factorial(4), kC6 = -inv_factorial(6),
                 kC8 = inv_factorial(8), kC10 = -inv_factorial(10), kC12 = inv_factorial(12),
                 kC14 = -inv_factorial(14), kC16 = inv_factorial(16), kC18 = -inv_factorial(18);

// pi/180, nearest binary64.
constexpr double kDeg2Rad = 0x1.1df46a2529d39p-6;

// sin and cos of x degrees.  The angle is reduced exactly in degrees to
// y in [-45, 45] plus q quarter turns, y is scaled to radians once, and the
// Taylor polynomials (exact to < 1e-19 on [-pi/4, pi/4]) are evaluated by
// Horner's rule; the quarter turns are applied by exact identities.
__host__ __device__ inline void sincosd(double x, double *s_out, double *c_out) {
#pragma clang fp contract(off)
    const double r = fmod(x, 360.0);  // exact, |r| < 360
    int q = 4;
    if (r < -315.0) q = -4;
    else if (r < -225.0) q = -3;
    else if (r < -135.0) q = -2;
    else if (r < -45.0) q = -1;
    else if (r < 45.0) q = 0;
    else if (r < 135.0) q = 1;
    else if (r < 225.0) q = 2;
    else if (r < 315.0) q = 3;
    const double y = r - 90.0 * static_cast<double>(q);  // exact (Sterbenz)
    const double t = y * kDeg2Rad;
    const double t2 = t * t;
    double p = kS17;
    p = p * t2 + kS15;
    p = p * t2 + kS13;
    p = p * t2 + kS11;
    p = p * t2 + kS9;
    p = p * t2 + kS7;
    p = p * t2 + kS5;
    p = p * t2 + kS3;
    const double s = t + t * (t2 * p);
    double k = kC18;
    k = k * t2 + kC16;
    k = k * t2 + kC14;
    k = k * t2 + kC12;
    k = k * t2 + kC10;
    k = k * t2 + kC8;
    k = k * t2 + kC6;
    k = k * t2 + kC4;
    k = k * t2 + kC2;
    const double c = 1.0 + t2 * k;
    switch (q & 3) {  // two's complement: q mod 4 for negative q too
        case 0: *s_out = s; *c_out = c; break;
        case 1: *s_out = c; *c_out = -s; break;
        case 2: *s_out = -s; *c_out = -c; break;
        default: *s_out = -c; *c_out = s; break;
    }
}

// Squared chord of an edge separation theta (degrees): 4 sin^2(theta/2).
__host__ __device__ inline double chord2_of_theta(double theta_deg) {
#pragma clang fp contract(off)
    double s, c;
    sincosd(0.5 * theta_deg, &s, &c);
    return 4.0 * (s * s);
}

}  // namespace pc
