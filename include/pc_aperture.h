/*
 * pc_aperture.h -- aperture-mass maps on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libpc.so, second workload of Bard et al., "Cosmological
 * calculations on the GPU", Sec. 3 (shear peak statistics).  Conventions as
 * in pc.h: a pc_status return code, pc_last_error() text, the caller owns
 * every buffer, and a hipStream_t `stream` (NULL = the null stream).
 *
 * For every reconstruction point p of a regular grid the call forms, over
 * the galaxies i with 0 < |theta_i - p| < theta_max:
 *   x_i    = |theta_i - p| / theta_max
 *   Q(x)   = tanh(x/0.15) / (x/0.15) / (1 + exp(6 - 150x) + exp(-47 + 50x))  (Eq. 4,
 *            the filter matched to an NFW halo; tanh(u)/u = 1 at u = 0)
 *   eps_t  = -(e1 cos 2phi + e2 sin 2phi), phi the position angle of galaxy
 *            i about p measured from +x (tangential alignment gives eps_t > 0)
 *   map    = sum Q(x_i) eps_t,i / n_gal                                    (Eq. 3)
 *   snr    = sqrt(2) sum Q(x_i) eps_t,i / sqrt(sum Q(x_i)^2 |eps_i|^2)      (Eq. 5)
 *            (NaN when the aperture holds no galaxy or all |eps| are 0)
 *   n_in   = number of galaxies in the aperture.
 * Positions are flat-sky (tangent-plane) coordinates in one unit, shared by
 * theta_max and the grid (arcmin in the paper's workload); n_gal is the
 * galaxy number density per unit area of that unit.
 *
 * Precision.  The aperture cut is a decision and gives exactly the result
 * of the binary64 definition: dx = x_i - x_p, dy = y_i - y_p and
 * |d|^2 = dx*dx + dy*dy in binary64 without fused multiply-add, grid point
 * (ix, iy) at (x0 + ix*dx_grid, y0 + iy*dy_grid) likewise, galaxy in iff
 * 0 < |d|^2 < theta_max^2 (binary64).  The library decides it from a
 * binary32 |d|^2 wherever a proven error bound allows and from the binary64
 * definition otherwise, so n_in is exact.  The filter and the tangential term
 * are evaluated in binary32 from offsets to a reference point of the point's
 * block of the grid and summed in binary32 over at most 64 galaxies, then in
 * binary64: map and snr agree with the binary64 definition to within
 * 1e-4 * sum_i Q(x_i)|eps_i| / n_gal (map) and the corresponding bound on
 * snr; the exact form of the bound is in the library's design notes.
 */
#ifndef PC_APERTURE_H
#define PC_APERTURE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* A shear catalogue of n galaxies: position (x, y) and ellipticity
 * components (e1, e2), binary64, n entries each, all finite.  e1 is the
 * component along the x axis.  0 <= n < 2^31.  on_device = 1: the four
 * pointers are device memory; 0: host memory. */
typedef struct {
    const double *x;
    const double *y;
    const double *e1;
    const double *e2;
    int64_t n;
    int32_t on_device;
    int32_t reserved;
} pc_shear_catalog;

/* Reconstruction grid: nx * ny points, point (ix, iy) at
 * (x0 + ix*dx, y0 + iy*dy), stored at index iy*nx + ix.  x0, y0 finite;
 * dx, dy finite and > 0; nx, ny >= 0 and nx*ny < 2^31. */
typedef struct {
    double x0, y0;
    double dx, dy;
    int32_t nx, ny;
} pc_grid;

/*
 * pc_aperture_mass -- aperture mass (Eq. 3), its signal-to-noise ratio
 * (Eq. 5) and the aperture occupancy on a grid (Sec. 3, GPU implementation:
 * one reconstruction point per GPU lane, galaxies far outside the filter
 * radius never visited).
 *
 *   cat        galaxies (host or device, see pc_shear_catalog)
 *   grid       reconstruction points
 *   theta_max  filter radius, finite and > 0, unit of the positions
 *   n_gal      galaxy number density, finite and > 0
 *   map        nx*ny doubles (required)
 *   snr        nx*ny doubles, or NULL
 *   n_in       nx*ny uint32, or NULL
 *   out_on_device  1: map/snr/n_in are device memory, written on `stream`;
 *                  0: host memory
 *   stream     hipStream_t or NULL
 *
 * Blocks until the outputs are written.  Errors: PC_ERR_INVALID for a NULL
 * or malformed argument, a non-finite coordinate or ellipticity (device
 * catalogues are checked on the device before any output is written), sizes
 * out of range, or a grid whose extent plus 2 theta_max reaches 1e15 units
 * along either axis; PC_ERR_NOMEM when the work space (about 80 bytes per
 * galaxy plus 4-8 bytes per cell of the search lattice, plus 20 bytes per
 * grid point for host outputs) cannot be allocated; PC_ERR_DEVICE for HIP
 * failures.  Outputs are untouched on error.
 */
int pc_aperture_mass(const pc_shear_catalog *cat, const pc_grid *grid, double theta_max, double n_gal,
                     double *map, double *snr, uint32_t *n_in, int32_t out_on_device, void *stream);

/*
 * pc_debug_last_aperture -- the calling thread's last pc_aperture_mass call:
 * time of the map kernel in ms from HIP events on the call's stream (-1 when
 * pc_debug_set_timing is off), galaxy-point pairs tested against the cut,
 * pairs inside the aperture, and the side of a search-lattice cell.  Any
 * pointer may be NULL.
 */
int pc_debug_last_aperture(double *kernel_ms, uint64_t *pairs_tested, uint64_t *pairs_in, double *cell_side);

/*
 * pc_debug_ap_filter -- the filter Q(x) of Eq. 4 as the map kernel evaluates
 * it, on the host: x = theta / theta_max in [0, 1] (host array of n doubles),
 * looked up in the kernel's table (1024 cells over [0, 1], a cubic in the
 * position inside each cell, fitted in binary64 at the cell's Chebyshev
 * points) with the kernel's binary32 steps; q (n doubles) written.  For
 * checking the table against the binary64 definition.  PC_ERR_INVALID for
 * NULL arrays with n > 0 or n < 0.
 */
int pc_debug_ap_filter(const double *x, int64_t n, double *q);

/*
 * pc_debug_ap_points_per_lane -- points = 1 or 2: the calling thread's later
 * pc_aperture_mass calls give each GPU lane points x points grid points (a
 * wave a block of 8 x 8 or 16 x 16 points); 0 restores the choice the call
 * makes itself (2 when a 16 x 16 block spans at most a quarter of theta_max
 * and the grid has at least 16 such blocks per compute unit).
 * Same results within the stated tolerance, n_in identical.  For testing both
 * kernel instances on one input.  PC_ERR_INVALID for other values.
 */
int pc_debug_ap_points_per_lane(int32_t points);

#ifdef __cplusplus
}
#endif

#endif /* PC_APERTURE_H */
