// pc_estimator.cpp -- the Landy-Szalay estimator (paper Eq. 2) and the other
// usual estimators on the same counts (Sec. 2 leaves the choice open).
//
// Eq. 2 is written with the raw counts; they are used here normalised by the
// number of pairs of each kind (DD over nD(nD-1)/2, DR over nD nR, RR over
// nR(nR-1)/2), which is the form of the estimator that is zero for unclustered
// data.  binary64, the operation order below, no fused multiply-add.
#include "pc_runtime.hpp"

namespace pc {

void landy_szalay(const uint64_t *DD, const uint64_t *DR, const uint64_t *RR, int32_t n_bins, int64_t nD,
                  int64_t nR, double *w) {
#pragma clang fp contract(off)
    const double fD = static_cast<double>(nD);
    const double fR = static_cast<double>(nR);
    const double pairs_dd = 0.5 * fD * (fD - 1.0);
    const double pairs_dr = fD * fR;
    const double pairs_rr = 0.5 * fR * (fR - 1.0);
    for (int32_t k = 0; k < n_bins; ++k) {
        const double dd = static_cast<double>(DD[k]) / pairs_dd;
        const double dr = static_cast<double>(DR[k]) / pairs_dr;
        const double rr = static_cast<double>(RR[k]) / pairs_rr;
        w[k] = ((dd - 2.0 * dr) + rr) / rr;
    }
}

void estimator(int32_t kind, const uint64_t *DD, const uint64_t *DR, const uint64_t *RR, int32_t n_bins,
               int64_t nD, int64_t nR, double *w) {
#pragma clang fp contract(off)
    if (kind == 0) {
        landy_szalay(DD, DR, RR, n_bins, nD, nR, w);
        return;
    }
    const double fD = static_cast<double>(nD);
    const double fR = static_cast<double>(nR);
    const double pairs_dd = 0.5 * fD * (fD - 1.0);
    const double pairs_dr = fD * fR;
    const double pairs_rr = 0.5 * fR * (fR - 1.0);
    for (int32_t k = 0; k < n_bins; ++k) {
        const double dd = static_cast<double>(DD[k]) / pairs_dd;
        if (kind == 1) {
            const double rr = static_cast<double>(RR[k]) / pairs_rr;
            w[k] = dd / rr - 1.0;
        } else if (kind == 2) {
            const double dr = static_cast<double>(DR[k]) / pairs_dr;
            w[k] = dd / dr - 1.0;
        } else {
            const double dr = static_cast<double>(DR[k]) / pairs_dr;
            const double rr = static_cast<double>(RR[k]) / pairs_rr;
            w[k] = (dd * rr) / (dr * dr) - 1.0;
        }
    }
}

}  // namespace pc
