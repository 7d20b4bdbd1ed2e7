// contact_model.h -- the lagged contact model of one contact in its frame
// (normal impulse of a compliant, optionally dissipative contact; regularised
// Coulomb friction with the normal impulse lagged to the substep start),
// shared by the contact solve and its reverse pass.
#pragma once
#include <hip/hip_runtime.h>

namespace mpm {

__device__ __forceinline__ double normal_impulse(double vn, double phi0, double k, double d, double h) {
    const double a = phi0 - h * vn, b = 1.0 - d * vn;
    return (a > 0.0 && b > 0.0) ? h * k * a * b : 0.0;
}

// Contact model in the contact frame (lagged model: compliant normal impulse,
// regularised Coulomb friction with the lagged normal impulse n0). Returns
// gamma = -dl/dvc and the nonzero entries of G = d2l/dvc2:
// G = [[g00, g01, 0], [g01, g11, 0], [0, 0, gnn]].
struct ContactParams {
    double phi0, mun0, k, d, eps_s, h;
};

// 1/sqrt(x) for normal x > 0: the hardware estimate refined by two Newton
// steps y <- y (3/2 - x y^2 / 2) (each step squares the relative error).
__device__ __forceinline__ double inv_sqrt(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * fma(-hx * y, y, 1.5);
    y = y * fma(-hx * y, y, 1.5);
    return y;
}

// 1/x for normal x > 0: the hardware estimate refined by two Newton steps
// r <- r + r (1 - x r) (each step squares the relative error); a short
// dependency chain where the IEEE-exact quotient is not needed.
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

// The normal impulse is active while both factors (phi0 - h vn) and
// (1 - d vn) are positive; the friction terms share one reciprocal square root.
__device__ __forceinline__ void contact_model(const ContactParams& P, const double vc[3],
                                              double gam[3], double* g00, double* g01,
                                              double* g11, double* gnn) {
    const double vn = vc[2];
    const double a = P.phi0 - P.h * vn, b = 1.0 - P.d * vn;
    if (a > 0.0 && b > 0.0) {
        gam[2] = P.h * P.k * a * b;
        *gnn = P.h * P.k * (P.h * b + P.d * a);
    } else {
        gam[2] = 0.0;
        *gnn = 0.0;
    }
    const double s2 = vc[0] * vc[0] + vc[1] * vc[1] + P.eps_s * P.eps_s;
    const double inv_s = inv_sqrt(s2);
    const double inv_s2 = inv_s * inv_s;
    const double cs = P.mun0 * inv_s;
    gam[0] = -cs * vc[0];
    gam[1] = -cs * vc[1];
    *g00 = cs * (1.0 - vc[0] * vc[0] * inv_s2);
    *g01 = -cs * vc[0] * vc[1] * inv_s2;
    *g11 = cs * (1.0 - vc[1] * vc[1] * inv_s2);
}

}  // namespace mpm
