// Level estimates for float thresholds on (nearly) a grid (host code, no device
// calls).
//
// The level of a value x is min{l : x <= t_l} (Eq. (2)).
// When the thresholds lie close to a grid t_0 + l * step, the kernels estimate
// it from one float32 fma and settle it against the thresholds only where the
// estimate lies within eps of a level boundary.  Two forms are used:
//   level form: u = fma(x, inv_step, u0); level = floor(u) + 1, boundaries at
//     the integers l (tile, batched-volume, 4D and 3D class-count kernels);
//   bin form: y = fma(x, inv_step, c_lo) with the pass constant
//     c_lo = u0d + kBinOff + 0.5 - lo rounded once; bin = round(y), boundaries
//     at the half-integers l + kBinOff + 0.5 - lo (2D and z-marching kernels,
//     pass window starting at level lo).
#pragma once

#include <cstdint>

#include "ecc_internal.h"

namespace ecc {

struct AffineFit {
    float u0 = 0.f;        // -t_0 * inv_step, rounded to float
    double u0d = 0.0;      // the same before rounding
    float inv_step = 0.f;  // 1 / step, rounded to float
    // Margin for the level form and for the bin form of the first pass window
    // (lo = 0): every estimate farther than eps from a level boundary is the
    // exact level.  Found by evaluating the float32 estimates at every
    // threshold and at the float just above it.
    float eps = 0.f;
    // A margin that holds for the bin form of every pass constant (passes
    // whose window starts past level 0), from an error bound.
    float eps_far = 0.f;
};

// The pass constant of the bin form for the pass window starting at level lo.
inline float pass_constant(double u0d, int lo) { return (float)(u0d + kBinOff + 0.5 - lo); }

// Fits the grid to L non-decreasing thresholds; false when they are too far
// from a grid for the estimate (then the kernels search the thresholds).
bool affine_levels(const float *thr, int L, AffineFit *fit);

}  // namespace ecc
