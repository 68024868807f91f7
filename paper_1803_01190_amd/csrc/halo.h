// Fixed external field of the disk workloads: a cored isothermal sphere with
// density rho0 / (1 + r^2/rc^2) and V^2 = 4 pi G rho0 rc^2 (not part of the
// paper, whose disk is fully self-gravitating).  With s = r / rc:
//   G M(<r) / r^3 = V^2 (1 - atan(s)/s) / r^2
//   Phi(r)       = V^2 [atan(s)/s + ln(1 + s^2)/2]      (Phi(0) = V^2)
// 1 - atan(s)/s cancels for small s; below s = 1/2 it is evaluated as
// s^2 * sum_{k>=1} (-1)^{k+1} s^{2k-2} / (2k+1) (Horner, 28 terms, the
// truncation is below 1e-18 relative there).  Always float64.
#pragma once

#include <hip/hip_runtime.h>

namespace nb {

__device__ __forceinline__ double halo_series_over_s2(double s2) {
    double acc = 0.0;
#pragma unroll
    for (int k = 28; k >= 1; --k) acc = __builtin_fma(acc, s2, ((k & 1) ? 1.0 : -1.0) / (2.0 * k + 1.0));
    return acc;
}

// G M(<r) / r^3 at squared radius r2.  Not inlined: its ~60 float64
// constants would otherwise be hoisted out of the persistent kernels' item
// loops and held in registers for the whole loop.
__device__ __noinline__ double halo_g_over_r3(double r2, double v2, double rc) {
    const double r = sqrt(r2);
    const double s = r / rc;
    if (s < 0.5) return v2 / (rc * rc) * halo_series_over_s2(s * s);
    return v2 * (1.0 - atan(s) / s) / r2;
}

// g'(r) / r, with g = G M(<r) / r^3, for the halo's jerk j_h = -g v - (g'/r)(r.v) r.
// With F(s) = (1 - atan(s)/s) / s^2 (g = V^2 F / rc^2), g'/r = V^2 H(s) / rc^4
// where H(s) = F'(s)/s = 1/(s^2 (1 + s^2)) - 3/s^4 + 3 atan(s)/s^5; below
// s = 1/2 the sum sum_{m>=0} (-1)^{m+1} (2m+2)/(2m+5) s^{2m} (Horner, 28 terms).
__device__ __forceinline__ double halo_dg_over_r(double r2, double v2, double rc) {
    const double rc2 = rc * rc;
    const double s2 = r2 / rc2;
    double h;
    if (s2 < 0.25) {
        h = 0.0;
#pragma unroll
        for (int m = 27; m >= 0; --m)
            h = __builtin_fma(h, s2, ((m & 1) ? 1.0 : -1.0) * (2.0 * m + 2.0) / (2.0 * m + 5.0));
    } else {
        const double s = sqrt(s2);
        const double s4 = s2 * s2;
        h = 1.0 / (s2 * (1.0 + s2)) - 3.0 / s4 + 3.0 * atan(s) / (s4 * s);
    }
    return v2 * h / (rc2 * rc2);
}

__device__ __forceinline__ double halo_potential(double r2, double v2, double rc) {
    const double s2 = r2 / (rc * rc);
    const double s = sqrt(s2);
    const double atan_over_s = (s < 0.5) ? 1.0 - s2 * halo_series_over_s2(s2) : atan(s) / s;
    return v2 * (atan_over_s + 0.5 * log1p(s2));
}

}  // namespace nb
