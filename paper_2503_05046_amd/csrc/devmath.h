// devmath.h -- float32 device math of the MPM substep for gfx950: quadratic
// B-spline weights, a branch-light 3x3 SVD, the fixed-corotated and Hencky
// Kirchhoff stresses and the Drucker-Prager return map.
#pragma once
#include <hip/hip_runtime.h>

namespace mpm {

struct M3 {
    float a[9];  // row-major
};

__device__ __forceinline__ float sq(float x) { return x * x; }

// Quadratic B-spline weights along one axis for fractional offset f in
// [0.5, 1.5): nodes base, base+1, base+2 (MLS-MPM transfer, Sec. V-A).
__device__ __forceinline__ void bspline_w(float f, float w[3]) {
    w[0] = 0.5f * sq(1.5f - f);
    w[1] = 0.75f - sq(f - 1.0f);
    w[2] = 0.5f * sq(f - 0.5f);
}

// Integer stencil base and fraction of one coordinate. The base is computed
// with explicitly rounded binary32 operations (no contraction) so that it is
// bit-identical to the cell index of the sort key.
__device__ __forceinline__ int cell_base(float x, float origin, float inv_dx, float* frac) {
    float d = __fsub_rn(x, origin);
    float t = __fmul_rn(d, inv_dx);
    float u = __fsub_rn(t, 0.5f);
    float b = floorf(u);
    *frac = t - b;
    return (int)b;
}

// ---------------------------------------------------------------------------
// 3x3 SVD, F = U diag(s) V^T with det U = det V = +1, s sorted by decreasing
// magnitude, s[2] carrying the sign of det F. Method of McAdams, Selle,
// Tamstorf, Teran, Sifakis (2011): cyclic Jacobi eigen-analysis of the
// symmetric S = F^T F for V, ordering of the columns of F V by norm, then a
// Givens QR of F V for U and s.
//
// Each Jacobi rotation in the (p, q) plane is the exact one that zeroes S_pq:
// with theta = (S_qq - S_pp) / (2 S_pq), t = tan of the angle =
// sign(theta) / (|theta| + sqrt(theta^2 + 1)) (the smaller root, |t| <= 1),
// c = 1 / sqrt(1 + t^2), s = t c, the rotated matrix has S_pp - t S_pq and
// S_qq + t S_pq on the diagonal, zero at (p, q), and the third row's entries
// rotated by (c, s); only the six distinct entries of S are kept. Reciprocals
// and square roots use the hardware's single-instruction approximations
// (about one ulp): c and s stay normalised to rounding because c is the
// reciprocal square root of 1 + t^2 and s = t c, so V stays orthogonal to
// rounding whatever error the angle carries. Four cyclic sweeps.
// ---------------------------------------------------------------------------
constexpr float kSvdTiny = 5.9604645e-8f;  // 2^-24, the unit roundoff of float32
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// One Jacobi rotation of the symmetric matrix (spp, sqq, spq; spr, sqr the
// entries of the third row) and of the columns p, q of V.
template <int p, int q>
__device__ __forceinline__ void sym_jacobi(float& spp, float& sqq, float& spq, float& spr, float& sqr, float V[9]) {
    const float b = spq;
    // an off-diagonal entry below the rounding of the smaller diagonal one
    // moves no eigenvalue: no rotation (V then stays exactly orthogonal where
    // F is a rotation to rounding, e.g. F = I)
    const bool skip = !(fabsf(b) > kSvdTiny * fminf(fabsf(spp), fabsf(sqq))) || fabsf(b) < 1e-30f;
    const float theta = (sqq - spp) * fast_rcp(2.0f * (skip ? 1.0f : b));
    const float t0 = fast_rcp(fabsf(theta) + fast_sqrt(fmaf(theta, theta, 1.0f)));
    const float t = skip ? 0.0f : copysignf(t0, theta);
    const float c = skip ? 1.0f : fast_rsq(fmaf(t, t, 1.0f));
    const float s = t * c;
    spp = fmaf(-t, b, spp);
    sqq = fmaf(t, b, sqq);
    spq = 0.0f;
    const float r0 = spr, r1 = sqr;
    spr = c * r0 - s * r1;
    sqr = s * r0 + c * r1;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float vkp = V[k * 3 + p], vkq = V[k * 3 + q];
        V[k * 3 + p] = c * vkp - s * vkq;
        V[k * 3 + q] = s * vkp + c * vkq;
    }
}

__device__ __forceinline__ void swap_cols(float B[9], float V[9], int i, int j, bool negate) {
    for (int k = 0; k < 3; ++k) {
        float b = B[k * 3 + i], v = V[k * 3 + i];
        B[k * 3 + i] = B[k * 3 + j];
        V[k * 3 + i] = V[k * 3 + j];
        B[k * 3 + j] = negate ? -b : b;
        V[k * 3 + j] = negate ? -v : v;
    }
}

// Givens rotation acting on rows (i, j) of B chosen to zero B[j][col];
// accumulates Q^T = G ... so that U = Q.
__device__ __forceinline__ void givens_qr(float B[9], float U[9], int i, int j, int col) {
    float a = B[i * 3 + col], b = B[j * 3 + col];
    float r2 = a * a + b * b;
    // nothing to zero below the rounding of the pivot
    const bool skip = r2 < 1e-38f || !(fabsf(b) > kSvdTiny * fabsf(a));
    float inv = fast_rsq(skip ? 1.0f : r2);
    float c = skip ? 1.0f : a * inv, s = skip ? 0.0f : b * inv;
    for (int k = 0; k < 3; ++k) {
        float bi = B[i * 3 + k], bj = B[j * 3 + k];
        B[i * 3 + k] = c * bi + s * bj;
        B[j * 3 + k] = -s * bi + c * bj;
    }
    // U <- U G^T (columns i, j)
    for (int k = 0; k < 3; ++k) {
        float ui = U[k * 3 + i], uj = U[k * 3 + j];
        U[k * 3 + i] = c * ui + s * uj;
        U[k * 3 + j] = -s * ui + c * uj;
    }
}

__device__ inline void svd3(const float F[9], float U[9], float s[3], float V[9]) {
    // the six distinct entries of S = F^T F
    float s00 = F[0] * F[0] + F[3] * F[3] + F[6] * F[6];
    float s11 = F[1] * F[1] + F[4] * F[4] + F[7] * F[7];
    float s22 = F[2] * F[2] + F[5] * F[5] + F[8] * F[8];
    float s01 = F[0] * F[1] + F[3] * F[4] + F[6] * F[7];
    float s02 = F[0] * F[2] + F[3] * F[5] + F[6] * F[8];
    float s12 = F[1] * F[2] + F[4] * F[5] + F[7] * F[8];
#pragma unroll
    for (int k = 0; k < 9; ++k) V[k] = (k % 4 == 0) ? 1.0f : 0.0f;
#pragma unroll
    for (int sweep = 0; sweep < 4; ++sweep) {
        sym_jacobi<0, 1>(s00, s11, s01, s02, s12, V);
        sym_jacobi<0, 2>(s00, s22, s02, s01, s12, V);
        sym_jacobi<1, 2>(s11, s22, s12, s01, s02, V);
    }
    // B = F V; order columns by decreasing norm, keeping det V = +1
    float B[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            B[r * 3 + c] = F[r * 3 + 0] * V[0 * 3 + c] + F[r * 3 + 1] * V[1 * 3 + c] +
                           F[r * 3 + 2] * V[2 * 3 + c];
    float n0 = sq(B[0]) + sq(B[3]) + sq(B[6]);
    float n1 = sq(B[1]) + sq(B[4]) + sq(B[7]);
    float n2 = sq(B[2]) + sq(B[5]) + sq(B[8]);
    if (n0 < n1) { swap_cols(B, V, 0, 1, true); float t = n0; n0 = n1; n1 = t; }
    if (n0 < n2) { swap_cols(B, V, 0, 2, true); float t = n0; n0 = n2; n2 = t; }
    if (n1 < n2) { swap_cols(B, V, 1, 2, true); float t = n1; n1 = n2; n2 = t; }
    // the Jacobi rotations keep det V = +1 and each swap negates one column
    // QR of B by Givens rotations: zero B[1][0], B[2][0], B[2][1]
#pragma unroll
    for (int k = 0; k < 9; ++k) U[k] = (k % 4 == 0) ? 1.0f : 0.0f;
    givens_qr(B, U, 0, 1, 0);
    givens_qr(B, U, 0, 2, 0);
    givens_qr(B, U, 1, 2, 1);
    s[0] = B[0];
    s[1] = B[4];
    s[2] = B[8];
    // the QR leaves s[0], s[1] >= 0 for full-rank leading columns; flip a
    // negative s[1] into s[2] to keep det U = +1 with the sign on the last
    if (s[1] < 0.0f) {
        s[1] = -s[1];
        s[2] = -s[2];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            U[k * 3 + 1] = -U[k * 3 + 1];
            U[k * 3 + 2] = -U[k * 3 + 2];
        }
    }
    if (s[0] < 0.0f) {
        s[0] = -s[0];
        s[2] = -s[2];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            U[k * 3 + 0] = -U[k * 3 + 0];
            U[k * 3 + 2] = -U[k * 3 + 2];
        }
    }
}

struct Material {
    int type;      // 0 fixed-corotated, 1 Hencky + Drucker-Prager
    float mu, la;  // Lame parameters
    float alpha;   // Drucker-Prager cone coefficient sqrt(2/3) 2 sin(phi) / (3 - sin(phi))
};

// Kirchhoff stress tau = P F^T from an SVD of F.
// The rotation of F near a rotation (polar decomposition F = R S), by three
// steps of Newton's iteration R <- (R + R^-T) / 2 (R^-T = cofactor(R) / det R),
// which converges quadratically from F; returns false, leaving R unspecified,
// when R^T R is not the identity within 1e-5 after them (F far from a
// rotation: the caller takes the SVD instead).
__device__ __forceinline__ bool polar_rotation_near(const float F[9], float R[9]) {
#pragma unroll
    for (int k = 0; k < 9; ++k) R[k] = F[k];
#pragma unroll
    for (int it = 0; it < 3; ++it) {
        const float c[9] = {R[4] * R[8] - R[5] * R[7], R[5] * R[6] - R[3] * R[8], R[3] * R[7] - R[4] * R[6],
                            R[2] * R[7] - R[1] * R[8], R[0] * R[8] - R[2] * R[6], R[1] * R[6] - R[0] * R[7],
                            R[1] * R[5] - R[2] * R[4], R[2] * R[3] - R[0] * R[5], R[0] * R[4] - R[1] * R[3]};
        const float d = R[0] * c[0] + R[1] * c[1] + R[2] * c[2];
        const float h = 0.5f / d;
#pragma unroll
        for (int k = 0; k < 9; ++k) R[k] = fmaf(c[k], h, 0.5f * R[k]);
    }
    float err = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = a; b < 3; ++b) {
            const float g = R[a] * R[b] + R[3 + a] * R[3 + b] + R[6 + a] * R[6 + b] - (a == b ? 1.0f : 0.0f);
            err = fmaxf(err, fabsf(g));
        }
    return err < 1e-5f;  // false for a NaN too
}

// Hencky stress tau = U (2 mu eps + la tr(eps) I) U^T from the left singular
// vectors U and the Hencky strain eps = ln s.
__device__ __forceinline__ void hencky_tau(const Material& m, const float U[9], float e0, float e1, float e2,
                                           float tau[9]) {
    float tr = e0 + e1 + e2;
    float d0 = 2.0f * m.mu * e0 + m.la * tr, d1 = 2.0f * m.mu * e1 + m.la * tr,
          d2 = 2.0f * m.mu * e2 + m.la * tr;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = r; c < 3; ++c) {
            float v = U[r * 3 + 0] * d0 * U[c * 3 + 0] + U[r * 3 + 1] * d1 * U[c * 3 + 1] +
                      U[r * 3 + 2] * d2 * U[c * 3 + 2];
            tau[r * 3 + c] = v;
            tau[c * 3 + r] = v;
        }
}

__device__ __forceinline__ void kirchhoff_from_svd(const Material& m, const float F[9],
                                                   const float U[9], const float s[3],
                                                   const float V[9], float tau[9]) {
    if (m.type == 0) {
        // fixed-corotated: tau = 2 mu (F - R) F^T + la (J - 1) J I, R = U V^T
        float R[9];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                R[r * 3 + c] = U[r * 3 + 0] * V[c * 3 + 0] + U[r * 3 + 1] * V[c * 3 + 1] +
                               U[r * 3 + 2] * V[c * 3 + 2];
        float J = s[0] * s[1] * s[2];
        float D[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) D[k] = F[k] - R[k];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                tau[r * 3 + c] = 2.0f * m.mu *
                                 (D[r * 3 + 0] * F[c * 3 + 0] + D[r * 3 + 1] * F[c * 3 + 1] +
                                  D[r * 3 + 2] * F[c * 3 + 2]);
        float vol = m.la * (J - 1.0f) * J;
        tau[0] += vol;
        tau[4] += vol;
        tau[8] += vol;
    } else {
        // Hencky: eps = ln s
        hencky_tau(m, U, logf(fmaxf(s[0], 1e-6f)), logf(fmaxf(s[1], 1e-6f)), logf(fmaxf(s[2], 1e-6f)), tau);
    }
}

// Drucker-Prager return map in Hencky strain (zero cohesion, no hardening),
// applied to the singular values; F is rebuilt as U exp(eps) V^T, and the
// projected eps is returned (the Hencky stress's strain, without taking the
// logarithm of exp(eps) again). Returns true in tension, where eps = 0 and
// s = 1 exactly (no exponentials to take).
__device__ __forceinline__ bool dp_return_map(const Material& m, float U[9], float s[3],
                                              const float V[9], float F[9], float eps[3]) {
    float e[3] = {logf(fmaxf(s[0], 1e-6f)), logf(fmaxf(s[1], 1e-6f)), logf(fmaxf(s[2], 1e-6f))};
    float tr = e[0] + e[1] + e[2];
    const bool tension = tr >= 0.0f;
    if (tension) {
        e[0] = e[1] = e[2] = 0.0f;  // tension: cone tip
        s[0] = s[1] = s[2] = 1.0f;
    } else {
        float dv[3] = {e[0] - tr / 3.0f, e[1] - tr / 3.0f, e[2] - tr / 3.0f};
        float nd = sqrtf(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
        float dg = nd + (3.0f * m.la + 2.0f * m.mu) / (2.0f * m.mu) * tr * m.alpha;
        if (dg > 0.0f) {
            float r = dg / nd;
            e[0] -= r * dv[0];
            e[1] -= r * dv[1];
            e[2] -= r * dv[2];
        }
        s[0] = expf(e[0]);
        s[1] = expf(e[1]);
        s[2] = expf(e[2]);
    }
    eps[0] = e[0];
    eps[1] = e[1];
    eps[2] = e[2];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            F[r * 3 + c] = U[r * 3 + 0] * s[0] * V[c * 3 + 0] + U[r * 3 + 1] * s[1] * V[c * 3 + 1] +
                           U[r * 3 + 2] * s[2] * V[c * 3 + 2];
    return tension;
}

}  // namespace mpm
