// Level estimates for float thresholds on (nearly) a grid: the fit and its
// margins (host code).
#include "ecc_levels.h"

#include <algorithm>
#include <cmath>

namespace ecc {

// How far the float32 estimate fma(x, inv, c) lies on the wrong side of a
// level boundary at the thresholds.  The estimate is monotone in x (the fma
// and rounding to nearest both are), so every x <= t_l has an estimate at most
// its value at t_l, and every x > t_l one at least its value at the next float
// above t_l.  Level l's boundary sits at g0 + l: values at or below t_l must
// estimate below it, values above t_l above it.  Any margin larger than the
// largest overshoot therefore flags every estimate that rounds to a wrong
// level.  The host fmaf rounds exactly as the device's fma (both are the
// correctly rounded fused operation).
static double estimate_overshoot(const float *thr, int L, float inv, float c, double g0) {
    double m = 0.0;
    for (int l = 0; l < L; ++l) {
        const double b = g0 + l;
        const double at = std::fmaf(thr[l], inv, c);
        const double past = std::fmaf(std::nextafterf(thr[l], INFINITY), inv, c);
        m = std::max(m, std::max(at - b, b - past));
    }
    return m;
}

bool affine_levels(const float *thr, int L, AffineFit *fit) {
    if (L < 2) return false;
    const double t0 = thr[0], step = ((double)thr[L - 1] - t0) / (L - 1);
    if (!(step > 0 && std::isfinite(step) && std::isfinite(t0) && std::isfinite((double)thr[L - 1]))) return false;
    // error bound for any pass constant: eps/2 bounds the thresholds' deviation
    // from the grid (in steps) plus the rounding of the estimate: 1/step and
    // the constant are rounded once each and the fma once, which for
    // |u| <= L + 2 moves it by at most (2 (L + 2) + |t0/step|) 2^-24 (with a
    // 1 % margin)
    double dev = 0;
    for (int l = 0; l < L; ++l) dev = std::max(dev, std::fabs(thr[l] - (t0 + l * step)) / step);
    const float inv_f = (float)(1.0 / step);
    const double u0_d = -t0 * (double)inv_f;
    const double round_u = (2.0 * (L + 2.0) + std::fabs(t0 / step) + 2.0) * 1.01 * std::ldexp(1.0, -24);
    const double e_far = 2.0 * (dev + round_u) + 1e-6;
    // the first pass and the level form, from the estimates themselves; the
    // 1e-6 covers the rounding of 0.5 - eps on the device
    const double over = std::max(estimate_overshoot(thr, L, inv_f, pass_constant(u0_d, 0), kBinOff + 0.5),
                                 estimate_overshoot(thr, L, inv_f, (float)u0_d, 0.0));
    const double e = over + 1e-6;
    // the settle step takes the level within one of the estimate
    if (!(e < 0.25 && e_far < 0.25)) return false;
    fit->u0 = (float)u0_d;
    fit->u0d = u0_d;
    fit->inv_step = inv_f;
    fit->eps = (float)e;
    fit->eps_far = (float)std::max(e_far, e);
    return true;
}

}  // namespace ecc
