// contact.hip -- contact registration and the convex contact solve of one
// substep (Sec. IV-B, IV-C, V-B; Eq. (7)-(10); Algorithm 1) on gfx950.
//
// Registration: one contact per (particle, rigid primitive) pair with the
// particle strictly inside the primitive at the substep start, against the
// pose frozen for the host step; compacted in (particle, primitive) order.
// The signed distances are evaluated in double precision.
//
// Contact-node table: the 27 stencil nodes of every contact are sorted by node
// (stable radix sort), which gives the distinct contact nodes ("slots") in
// ascending node order and, per slot, its (contact, stencil offset) pairs in
// contact order: a deterministic CSR with no atomics.
//
// Solver: one persistent cooperative kernel runs Algorithm 1 to convergence
// for every environment, each environment's problem on its own group of
// blocks, with the iterate, gradient, block Hessian, search direction,
// contact velocities and every reduction in double precision. Per iteration:
//   node pass   each slot gathers its contacts' impulses and Hessians (each
//               contact's model is re-evaluated by its 27 nodes instead of
//               being scattered, which saves a barrier and all atomics),
//               forms g = m (v - v*) - j and H, solves the 3x3 block by
//               Cholesky, and adds its share of the norms;
//   barrier     every block of the group reduces the per-block partials in
//               the same order, so all take the same stopping decision;
//   contact pass u_c = R_c^T sum w dv;
//   barrier     then the exact line search of Algorithm 1 (1-D Newton with a
//               bisection fallback) runs redundantly in every block of the
//               group over the environment's contacts with block-local
//               reductions, so it needs no further synchronisation; every
//               block obtains the same step length.
// Contact velocities are carried as v_c + alpha u_c (the contact velocity is
// linear in the grid velocity), double-buffered by iteration parity.
// One-barrier form (k_qn<true>, for a handle of one environment, launched
// first: it solves the environment when its blocks all hold their contact
// nodes in the compact form and it has at most kScatterMax contacts, and
// otherwise leaves it to k_qn<false>): the
// node pass also forms u_c = R_c^T sum w dv over its entries (a block sum in
// LDS, projected, then one device-scope FP64 atomic add per distinct contact
// and component, into one of three buffers by iteration), so after the
// barrier every block forms the line-search coefficients and phi''(0) of all
// the environment's contacts itself, and the contact pass and the second
// barrier go away. Each block carries the contact velocities it
// needs (its distinct contacts in LDS, the line search's in a scratch array of
// its own), updated with the same arithmetic from the same values, so they
// agree in every block. The order of the atomic adds varies from run to run,
// so this form is reproducible to rounding, not bit for bit.
#include "contact_model.h"
#include "mpm_internal.h"
#include "sort_util.h"

#include <algorithm>
#include <cstddef>

namespace mpm {

constexpr unsigned kFlagNoconv = 1u;
constexpr unsigned kFlagCapacity = 8u;
constexpr unsigned kFlagHang = 16u;
constexpr long long kBarrierTimeoutCycles = 5000000000ll;  // ~2 s: a healthy barrier takes microseconds
constexpr int kQnThreads = 512;
constexpr int kSlotChunk = 512;     // contact nodes whose accumulators are staged in LDS at once
static_assert(kSlotChunk <= kQnThreads, "one contact node of a chunk per thread");
constexpr int kMaxRigid = 256;

__device__ __forceinline__ int env_of_particle_c(const DevEnv* envs, int n_envs, long long p) {
    int lo = 0, hi = n_envs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (envs[mid].p_begin <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Rigid primitives (double precision)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double rigid_sdf(const DevRigid& r, const double x[3], double n[3]) {
    const double d[3] = {x[0] - r.t[0], x[1] - r.t[1], x[2] - r.t[2]};
    double p[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) p[c] = r.R[0 * 3 + c] * d[0] + r.R[1 * 3 + c] * d[1] + r.R[2 * 3 + c] * d[2];
    double nb[3];
    double s;
    if (r.shape == 0) {
        s = r.normal[0] * p[0] + r.normal[1] * p[1] + r.normal[2] * p[2] - r.offset;
        nb[0] = r.normal[0]; nb[1] = r.normal[1]; nb[2] = r.normal[2];
    } else {
        double q[3], qp[3];
        double mx = -1e300;
        int ks = 0;
        bool outside = false;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            q[a] = fabs(p[a]) - r.half[a];
            qp[a] = q[a] > 0.0 ? q[a] : 0.0;
            outside |= q[a] > 0.0;
            if (q[a] > mx) { mx = q[a]; ks = a; }
        }
        const double no = sqrt(qp[0] * qp[0] + qp[1] * qp[1] + qp[2] * qp[2]);
        s = no + (mx < 0.0 ? mx : 0.0);
        if (outside) {
#pragma unroll
            for (int a = 0; a < 3; ++a) nb[a] = qp[a] * (p[a] >= 0.0 ? 1.0 : -1.0) / no;
        } else {
            nb[0] = nb[1] = nb[2] = 0.0;
            nb[ks] = p[ks] >= 0.0 ? 1.0 : -1.0;
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) n[a] = r.R[a * 3 + 0] * nb[0] + r.R[a * 3 + 1] * nb[1] + r.R[a * 3 + 2] * nb[2];
    return s;
}

// Contact frame columns (t1, t2, n): orthonormal completion of Duff et al. 2017.
__device__ __forceinline__ void frame_of(const double n[3], double t1[3], double t2[3]) {
    const double sg = n[2] >= 0.0 ? 1.0 : -1.0;
    const double a = -1.0 / (sg + n[2]);
    const double b = n[0] * n[1] * a;
    t1[0] = 1.0 + sg * n[0] * n[0] * a; t1[1] = sg * b; t1[2] = -sg * n[0];
    t2[0] = b; t2[1] = sg + n[1] * n[1] * a; t2[2] = -n[1];
}

// Line search along v_c(alpha) = v_c + alpha u_c: the contact's terms of
// phi'(alpha) = -gamma(v_c(alpha)) . u_c and phi''(alpha) = u_c^T G u_c in
// closed form. With v_t, u_t the tangential parts,
//   s^2(alpha) = |v_t + alpha u_t|^2 + eps_s^2 = q0 + 2 p0 alpha + q2 alpha^2,
//   friction:  phi'  += mu n0 (p0 + alpha q2) / s,
//              phi'' += mu n0 / s (q2 - (p0 + alpha q2)^2 / s^2);
//   normal, while a = phi0 - h v_n(alpha) > 0 and b = 1 - d v_n(alpha) > 0:
//              phi'  -= h k u_n a b,   phi'' += h k u_n^2 (h b + d a).
struct LsCoef {
    double q0, p0, q2, mun0;  // friction
    double a0, a1, b0, b1;    // a = a0 - alpha a1, b = b0 - alpha b1
    double kn, eh, ed;        // h k u_n, h k u_n^2 h, h k u_n^2 d
};

__device__ __forceinline__ LsCoef ls_coef(const ContactParams& P, const double vc[3], const double u[3]) {
    LsCoef L;
    L.q0 = vc[0] * vc[0] + vc[1] * vc[1] + P.eps_s * P.eps_s;
    L.p0 = vc[0] * u[0] + vc[1] * u[1];
    L.q2 = u[0] * u[0] + u[1] * u[1];
    L.mun0 = P.mun0;
    L.a0 = P.phi0 - P.h * vc[2];
    L.a1 = P.h * u[2];
    L.b0 = 1.0 - P.d * vc[2];
    L.b1 = P.d * u[2];
    const double hk = P.h * P.k, hkuu = hk * u[2] * u[2];
    L.kn = hk * u[2];
    L.eh = hkuu * P.h;
    L.ed = hkuu * P.d;
    return L;
}

// Values the solver's blocks exchange inside the iteration loop (search
// directions, contact velocities and their projections u_c, line-search
// coefficients, block partial sums) are stored and loaded as device-scope
// relaxed atomics, which write through and read past the per-XCD caches. With
// each thread's stores acknowledged before its block arrives at a barrier,
// the loop's barriers then need no write-back or invalidation of the caches,
// and the data that stays fixed during the solve stays cached.
__device__ __forceinline__ double ld_x(const double* p) {
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_x(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Line-search coefficients of every contact, in chunks of 64 contacts: chunk
// c / 64 holds 11 arrays of 64 values (in the order of LsCoef's members), so a
// wave reading consecutive contacts reads consecutive words, and the array
// offsets are constants of the load instructions.
constexpr int kCoefChunk = 64;
constexpr int kCoefWords = 11;
__device__ __forceinline__ long long coef_index(long long c) {
    return (c / kCoefChunk) * (kCoefChunk * kCoefWords) + (c % kCoefChunk);
}
__device__ __forceinline__ void store_coef(double* __restrict__ buf, long long c, const LsCoef& L) {
    double* p = buf + coef_index(c);
    const double q[kCoefWords] = {L.q0, L.p0, L.q2, L.mun0, L.a0, L.a1, L.b0, L.b1, L.kn, L.eh, L.ed};
#pragma unroll
    for (int j = 0; j < kCoefWords; ++j) st_x(p + j * kCoefChunk, q[j]);
}
__device__ __forceinline__ LsCoef load_coef(const double* __restrict__ buf, long long c) {
    const double* p = buf + coef_index(c);
    LsCoef L;
    L.q0 = ld_x(p); L.p0 = ld_x(p + 64); L.q2 = ld_x(p + 128); L.mun0 = ld_x(p + 192); L.a0 = ld_x(p + 256);
    L.a1 = ld_x(p + 320); L.b0 = ld_x(p + 384); L.b1 = ld_x(p + 448); L.kn = ld_x(p + 512); L.eh = ld_x(p + 576);
    L.ed = ld_x(p + 640);
    return L;
}

// The one-barrier form's line search keeps its contacts in registers in a
// compact form: one environment's contacts share eps_s, d and h k (copied
// from the environment at registration), so only what differs per contact is
// held, and a1 = h u_n, b1 = d u_n, h k u_n are formed at each evaluation
// from the block-uniform constants (LsUni).
struct LsUni {
    double eps2, h, d, hk;
};
// A value equal in every lane of the wave, moved to scalar registers.
__device__ __forceinline__ double uniform_f64(double x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// A line-search contact held in registers for the whole solve: its contact
// velocity, the iteration's u_c, mu n0 and phi0. The zero state
// (ls_state_zero) contributes exactly zero.
struct LsState {
    double vc[3], u[3], mun0, phi0;
};
__device__ __forceinline__ LsState ls_state_zero() {
    LsState S;
#pragma unroll
    for (int a = 0; a < 3; ++a) S.vc[a] = S.u[a] = 0.0;
    S.mun0 = 0.0;
    S.phi0 = -1.0;
    return S;
}
// The iteration's coefficients of such a contact (LsCoef's q0, p0, q2, mun0,
// a0, b0 with the same roundings, and u_n).
struct LsCoefC {
    double q0, p0, q2, mun0, a0, b0, un;
};
__device__ __forceinline__ LsCoefC ls_coefc(const LsUni& E, double mun0, double phi0, const double vc[3],
                                            const double u[3]) {
    LsCoefC L;
    L.q0 = vc[0] * vc[0] + vc[1] * vc[1] + E.eps2;
    L.p0 = vc[0] * u[0] + vc[1] * u[1];
    L.q2 = u[0] * u[0] + u[1] * u[1];
    L.mun0 = mun0;
    L.a0 = phi0 - E.h * vc[2];
    L.b0 = 1.0 - E.d * vc[2];
    L.un = u[2];
    return L;
}
__device__ __forceinline__ LsCoefC ls_coefc_of(const LsState& S, const LsUni& E) {
    return ls_coefc(E, S.mun0, S.phi0, S.vc, S.u);
}

// Coefficients that contribute exactly zero (padding lanes).
__device__ __forceinline__ LsCoef ls_coef_zero() {
    LsCoef L;
    L.q0 = 1.0; L.p0 = L.q2 = L.mun0 = 0.0;
    L.a0 = -1.0; L.a1 = L.b0 = L.b1 = 0.0;
    L.kn = L.eh = L.ed = 0.0;
    return L;
}

__device__ __forceinline__ void ls_eval(const LsCoef& L, double alpha, double* d1, double* d2) {
    const double pa = fma(alpha, L.q2, L.p0);
    const double s2 = fma(alpha, pa + L.p0, L.q0);
    const double is = inv_sqrt(s2);
    const double cs = L.mun0 * is;
    const double pis = pa * is;
    double e1 = cs * pa;
    double e2 = cs * fma(-pis, pis, L.q2);
    const double a = fma(-alpha, L.a1, L.a0), b = fma(-alpha, L.b1, L.b0);
    if (a > 0.0 && b > 0.0) {
        e1 -= L.kn * a * b;
        e2 += fma(L.eh, b, L.ed * a);
    }
    *d1 = e1;
    *d2 = e2;
}

// phi''' and phi'''' of a contact's terms at alpha from its full coefficients
// (the derivatives as in ls_eval4 below), added to d[0..1].
__device__ __forceinline__ void ls_eval34(const LsCoef& L, double alpha, double (&d)[2]) {
    const double pa = fma(alpha, L.q2, L.p0);
    const double s2 = fma(alpha, pa + L.p0, L.q0);
    const double is = inv_sqrt(s2);
    const double pis = pa * is;
    const double f2 = L.mun0 * is * fma(-pis, pis, L.q2);
    double e3 = -3.0 * f2 * (pis * is);
    const double e4 = -3.0 * f2 * (is * is) * fma(-5.0 * pis, pis, L.q2);
    const double a = fma(-alpha, L.a1, L.a0), b = fma(-alpha, L.b1, L.b0);
    if (a > 0.0 && b > 0.0) e3 -= fma(L.eh, L.b1, L.ed * L.a1);
    d[0] += e3;
    d[1] += e4;
}

// phi' and phi'' of one contact's terms added to d[0..1], from either form of
// the coefficients (the full form gives ls_eval's values).
__device__ __forceinline__ void ls_eval2(const LsCoef& L, const LsUni&, double alpha, double (&d)[2]) {
    double d1, d2;
    ls_eval(L, alpha, &d1, &d2);
    d[0] += d1;
    d[1] += d2;
}
__device__ __forceinline__ void ls_eval2(const LsCoefC& L, const LsUni& E, double alpha, double (&d)[2]) {
    const double pa = fma(alpha, L.q2, L.p0);
    const double s2 = fma(alpha, pa + L.p0, L.q0);
    const double is = inv_sqrt(s2);
    const double cs = L.mun0 * is;
    const double pis = pa * is;
    double e1 = cs * pa;
    double e2 = cs * fma(-pis, pis, L.q2);
    const double a1 = E.h * L.un, b1 = E.d * L.un;
    const double a = fma(-alpha, a1, L.a0), b = fma(-alpha, b1, L.b0);
    if (a > 0.0 && b > 0.0) {
        const double kn = E.hk * L.un;
        e1 -= kn * a * b;
        e2 += kn * fma(a1, b, b1 * a);
    }
    d[0] += e1;
    d[1] += e2;
}
// The same for a compact contact with the next two derivatives, added to
// d[0..3] (phi', phi'', phi''', phi''''). Along the line s(alpha) =
// |v_t + alpha u_t|^2 + eps^2 has s'' = 2 q2 and a constant q0 q2 - p0^2, so
// the friction term's curvature e2 = mu n0 (q0 q2 - p0^2) / s^(3/2)
// differentiates to e3 = -3 e2 pa / s and e4 = -3 e2 (q2 - 5 pa^2 / s) / s;
// the active normal term is a quadratic in alpha (e3 = -2 h k u_n a1 b1,
// e4 = 0).
__device__ __forceinline__ void ls_eval4(const LsCoefC& L, const LsUni& E, double alpha, double (&d)[4]) {
    const double pa = fma(alpha, L.q2, L.p0);
    const double s2 = fma(alpha, pa + L.p0, L.q0);
    const double is = inv_sqrt(s2);
    const double cs = L.mun0 * is;
    const double pis = pa * is;
    const double f2 = cs * fma(-pis, pis, L.q2);
    double e1 = cs * pa, e2 = f2;
    double e3 = -3.0 * f2 * (pis * is);
    const double e4 = -3.0 * f2 * (is * is) * fma(-5.0 * pis, pis, L.q2);
    const double a1 = E.h * L.un, b1 = E.d * L.un, kn = E.hk * L.un;
    const double a = fma(-alpha, a1, L.a0), b = fma(-alpha, b1, L.b0);
    if (a > 0.0 && b > 0.0) {
        e1 -= kn * a * b;
        e2 += kn * fma(a1, b, b1 * a);
        e3 -= 2.0 * kn * (a1 * b1);
    }
    d[0] += e1;
    d[1] += e2;
    d[2] += e3;
    d[3] += e4;
}

// ---------------------------------------------------------------------------
// Registration
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_reg_count(const float* __restrict__ x, long long P, const DevEnv* __restrict__ envs, int n_envs,
            const DevRigid* __restrict__ rigids, unsigned* __restrict__ cmask,
            unsigned* __restrict__ blk, const DevCounters* cnt) {
    __shared__ unsigned wsum[17];
    long long beg, end;
    chunk_range(P, blockIdx.x, gridDim.x, &beg, &end);
    unsigned c = 0;
    if (!cnt->abort_step) {
        for (long long p = beg + threadIdx.x; p < end; p += blockDim.x) {
            const DevEnv& E = envs[env_of_particle_c(envs, n_envs, p)];
            const double xp[3] = {x[p], x[P + p], x[2 * P + p]};
            unsigned m = 0;
            for (int r = E.rigid_begin; r < E.rigid_end; ++r) {
                double n[3];
                if (rigid_sdf(rigids[r], xp, n) < 0.0) m |= 1u << (r - E.rigid_begin);
            }
            cmask[p] = m;
            c += __popc(m);
        }
    }
    unsigned tot;
    block_exclusive_scan_total(c, wsum, &tot);
    if (threadIdx.x == 0) blk[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(256)
k_reg_write(const float* __restrict__ x, const float* __restrict__ v, long long P,
            const DevEnv* __restrict__ envs, int n_envs, const DevRigid* __restrict__ rigids,
            const unsigned* __restrict__ cmask, const unsigned* __restrict__ blk, double h,
            long long cap, int* __restrict__ c_pid, int* __restrict__ c_rid, int* __restrict__ c_env,
            int* __restrict__ c_base, float* __restrict__ c_w, ContactRec* __restrict__ c_rec,
            ContactDyn* __restrict__ c_dyn, int substep, DevCounters* cnt) {
    __shared__ unsigned wsum[17];
    if (cnt->abort_step) return;
    long long beg, end;
    chunk_range(P, blockIdx.x, gridDim.x, &beg, &end);
    unsigned run = blk[blockIdx.x];
    for (long long base = beg; base < end; base += blockDim.x) {
        const long long p = base + threadIdx.x;
        const unsigned m = p < end ? cmask[p] : 0u;
        unsigned tot;
        const unsigned off = block_exclusive_scan_total(__popc(m), wsum, &tot);
        if (m) {
            const int e = env_of_particle_c(envs, n_envs, p);
            const DevEnv& E = envs[e];
            const float xf[3] = {x[p], x[P + p], x[2 * P + p]};
            const double xp[3] = {xf[0], xf[1], xf[2]};
            const double vp[3] = {v[p], v[P + p], v[2 * P + p]};
            // stencil of the particle (same float32 rule as P2G)
            int b[3];
            float f[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                int bi = cell_base(xf[a], E.origin[a], E.inv_dx, &f[a]);
                const int hi = E.dims[a] - 3;
                if (bi < 0 || bi > hi) { bi = bi < 0 ? 0 : hi; f[a] = fminf(fmaxf(f[a], 0.5f), 1.5f); }
                b[a] = bi;
            }
            const long long node0 = E.node_base + b[0] + (long long)E.dims[0] * (b[1] + (long long)E.dims[1] * b[2]);
            unsigned j = 0;
            for (int r = E.rigid_begin; r < E.rigid_end; ++r) {
                if (!((m >> (r - E.rigid_begin)) & 1u)) continue;
                const long long c = (long long)run + off + j++;
                if (c >= cap) continue;
                const DevRigid& R = rigids[r];
                double n[3];
                const double s = rigid_sdf(R, xp, n);
                const double rel[3] = {xp[0] - R.t[0], xp[1] - R.t[1], xp[2] - R.t[2]};
                const double vr[3] = {R.V[0] + R.w[1] * rel[2] - R.w[2] * rel[1],
                                      R.V[1] + R.w[2] * rel[0] - R.w[0] * rel[2],
                                      R.V[2] + R.w[0] * rel[1] - R.w[1] * rel[0]};
                double t1[3], t2[3];
                frame_of(n, t1, t2);
                const double phi0 = -s;
                const double vn0 = n[0] * (vp[0] - vr[0]) + n[1] * (vp[1] - vr[1]) + n[2] * (vp[2] - vr[2]);
                const double n0 = normal_impulse(vn0, phi0, E.k, E.d, h);
                ContactRec rec;
#pragma unroll
                for (int a = 0; a < 3; ++a) { rec.t1[a] = t1[a]; rec.t2[a] = t2[a]; rec.n[a] = n[a]; }
                rec.phi0 = phi0;
                rec.mun0 = R.mu * n0;
                rec.k = E.k; rec.d = E.d; rec.eps_s = E.eps_s;
                c_rec[c] = rec;
                ContactDyn& D = c_dyn[c];
                D.b[0] = -(t1[0] * vr[0] + t1[1] * vr[1] + t1[2] * vr[2]);
                D.b[1] = -(t2[0] * vr[0] + t2[1] * vr[1] + t2[2] * vr[2]);
                D.b[2] = -(n[0] * vr[0] + n[1] * vr[1] + n[2] * vr[2]);
                c_pid[c] = (int)p;
                c_rid[c] = r;
                c_env[c] = e;
                c_base[c] = (int)node0;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    float w3[3];
                    bspline_w(f[a], w3);
                    c_w[(3 * a + 0) * cap + c] = w3[0];
                    c_w[(3 * a + 1) * cap + c] = w3[1];
                    c_w[(3 * a + 2) * cap + c] = w3[2];
                }
            }
        }
        run += tot;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && (long long)cnt->n_contacts > cap) {
        atomicOr(&cnt->flags, kFlagCapacity);
        cnt->abort_substep = (unsigned)substep;
        cnt->abort_step = 1u;
    }
}

hipError_t launch_registration(const Work& w, const float* x, const float* v, double h,
                               int substep, hipStream_t s) {
    hipLaunchKernelGGL(k_reg_count, dim3(kSortBlocks), dim3(256), 0, s, x, w.P, w.envs, w.n_envs,
                       w.rigids, w.cmask, w.blk, (const DevCounters*)w.cnt);
    hipError_t e = launch_scan_blocks(w.blk, kSortBlocks, &w.cnt->n_contacts, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reg_write, dim3(kSortBlocks), dim3(256), 0, s, x, v, w.P, w.envs,
                       w.n_envs, w.rigids, w.cmask, w.blk, h, w.cap_c, w.c_pid, w.c_rid, w.c_env,
                       w.c_base, w.c_w, w.c_rec, w.c_dyn, substep, w.cnt);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Contact-node table
// ---------------------------------------------------------------------------
__device__ __forceinline__ float stencil_weight(const float* c_w, long long cap, long long c, int o) {
    const int a = o % 3, b = (o / 3) % 3, cz = o / 9;
    return c_w[(0 + a) * cap + c] * c_w[(3 + b) * cap + c] * c_w[(6 + cz) * cap + c];
}

__device__ __forceinline__ long long stencil_node(const DevEnv& E, int base, int o) {
    const int a = o % 3, b = (o / 3) % 3, cz = o / 9;
    return (long long)base + a + (long long)E.dims[0] * (b + (long long)E.dims[1] * cz);
}

__global__ void __launch_bounds__(256)
k_pairs(const DevEnv* __restrict__ envs, const int* __restrict__ c_env, const int* __restrict__ c_base,
        const float* __restrict__ c_w, long long cap, unsigned invalid_key,
        unsigned* __restrict__ pk, unsigned* __restrict__ pv, DevCounters* cnt) {
    const long long nc = cnt->abort_step ? 0 : std::min<long long>(cnt->n_contacts, cap);
    if (blockIdx.x == 0 && threadIdx.x == 0) cnt->n_pairs = (unsigned)(27 * nc);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < 27 * nc;
         i += (long long)gridDim.x * blockDim.x) {
        const long long c = i / 27;
        const int o = (int)(i % 27);
        const float w = stencil_weight(c_w, cap, c, o);
        pk[i] = w > 0.f ? (unsigned)stencil_node(envs[c_env[c]], c_base[c], o) : invalid_key;
        pv[i] = (unsigned)i;
    }
}

__global__ void __launch_bounds__(256)
k_csr_count(const unsigned* __restrict__ keys, const DevCounters* cnt, unsigned invalid_key,
            unsigned* __restrict__ blk) {
    __shared__ unsigned wsum[17];
    const long long n = cnt->n_pairs;
    long long beg, end;
    chunk_range(n, blockIdx.x, gridDim.x, &beg, &end);
    unsigned c = 0;
    for (long long i = beg + threadIdx.x; i < end; i += blockDim.x)
        c += (keys[i] != invalid_key && (i == 0 || keys[i] != keys[i - 1])) ? 1u : 0u;
    unsigned tot;
    block_exclusive_scan_total(c, wsum, &tot);
    if (threadIdx.x == 0) blk[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(256)
k_csr_write(const unsigned* __restrict__ keys, const unsigned* __restrict__ vals,
            const DevCounters* cnt, unsigned invalid_key, const unsigned* __restrict__ blk,
            long long cap, const float* __restrict__ c_w, int* __restrict__ s_node,
            int* __restrict__ s_beg, ContactStencil* __restrict__ c_st, Entry* __restrict__ e_ent) {
    __shared__ unsigned wsum[17];
    const long long n = cnt->n_pairs;
    long long beg, end;
    chunk_range(n, blockIdx.x, gridDim.x, &beg, &end);
    unsigned run = blk[blockIdx.x];
    for (long long base = beg; base < end; base += blockDim.x) {
        const long long i = base + threadIdx.x;
        const bool in = i < end;
        const unsigned key = in ? keys[i] : invalid_key;
        const bool valid = in && key != invalid_key;
        const unsigned head = (valid && (i == 0 || key != keys[i - 1])) ? 1u : 0u;
        unsigned tot;
        const unsigned off = block_exclusive_scan_total(head, wsum, &tot);
        if (in) {
            const unsigned pv = vals[i];
            const long long c = pv / 27;
            const int o = (int)(pv % 27);
            if (valid) {
                const unsigned slot = run + off + head - 1;
                if (head) {
                    s_node[slot] = (int)key;
                    s_beg[slot] = (int)i;
                }
                const float w = stencil_weight(c_w, cap, c, o);
                c_st[c].slot[o] = (int)slot;
                c_st[c].w[o] = w;
                Entry en;
                en.c = (unsigned)c;
                en.slot = (int)slot;
                en.w = w;
                en.pad = 0.f;
                e_ent[i] = en;
                if (i + 1 == n || keys[i + 1] == invalid_key) s_beg[cnt->n_slots] = (int)(i + 1);
            } else {
                c_st[c].slot[o] = -1;
                c_st[c].w[o] = 0.f;
            }
        }
        run += tot;
    }
}

// Slot state: m and v* from the grid, iterate v = v* (Algorithm 1 starts from
// the free-motion velocity).
__global__ void __launch_bounds__(256)
k_slot_init(const int* __restrict__ s_node, const float4* __restrict__ vel, const DevCounters* cnt,
            SlotRec* __restrict__ s_rec) {
    const long long ns = cnt->n_slots;
    for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < ns;
         s += (long long)gridDim.x * blockDim.x) {
        const float4 g = vel[s_node[s]];
        SlotRec r;
        r.m = g.w;
        r.v[0] = r.vstar[0] = g.x;
        r.v[1] = r.vstar[1] = g.y;
        r.v[2] = r.vstar[2] = g.z;
        r.dv[0] = r.dv[1] = r.dv[2] = 0.0;
        s_rec[s] = r;
    }
}

// First index in a[0, n) whose value is >= key (a ascending).
__device__ __forceinline__ long long lower_bound_i(const int* a, long long n, long long key) {
    long long lo = 0, hi = n;
    while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if ((long long)a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Contacts and contact nodes of every environment: contacts are numbered in
// particle order and contact nodes in global node order, and both orders
// group the environments, so each environment owns one range of each.
__global__ void __launch_bounds__(256)
k_env_ranges(const DevEnv* __restrict__ envs, int n_envs, const int* __restrict__ c_env,
             const int* __restrict__ s_node, const DevCounters* cnt, long long cap, int* __restrict__ range) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_envs) return;
    const bool aborted = cnt->abort_step != 0u;
    const long long nc = aborted ? 0 : std::min<long long>(cnt->n_contacts, cap);
    const long long ns = aborted ? 0 : (long long)cnt->n_slots;
    const DevEnv& E = envs[e];
    const long long n0 = E.node_base, n1 = n0 + (long long)E.dims[0] * E.dims[1] * E.dims[2];
    range[4 * e + 0] = (int)lower_bound_i(c_env, nc, e);
    range[4 * e + 1] = (int)lower_bound_i(c_env, nc, e + 1);
    range[4 * e + 2] = (int)lower_bound_i(s_node, ns, n0);
    range[4 * e + 3] = (int)lower_bound_i(s_node, ns, n1);
}

// Key width of the contact-node pairs (node index, or n_nodes for a
// zero-weight stencil entry).
static int pair_key_bits(const Work& w) {
    int bits = 1;
    while ((1ull << bits) <= (unsigned long long)w.n_nodes) ++bits;
    return bits;
}

hipError_t launch_contact_setup(const Work& w, hipStream_t s) {
    const unsigned invalid_key = (unsigned)w.n_nodes;
    const int bits = pair_key_bits(w);
    hipLaunchKernelGGL(k_pairs, dim3(2048), dim3(256), 0, s, w.envs, w.c_env, w.c_base, w.c_w,
                       w.cap_c, invalid_key, w.pk_a, w.pv_a, w.cnt);
    unsigned *ks, *vs;
    hipError_t e = radix_sort(w, w.pk_a, w.pv_a, w.pk_b, w.pv_b, &w.cnt->n_pairs, 0, bits, s, &ks, &vs);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_csr_count, dim3(kSortBlocks), dim3(256), 0, s, ks, (const DevCounters*)w.cnt,
                       invalid_key, w.blk);
    e = launch_scan_blocks(w.blk, kSortBlocks, &w.cnt->n_slots, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_csr_write, dim3(kSortBlocks), dim3(256), 0, s, ks, vs,
                       (const DevCounters*)w.cnt, invalid_key, w.blk, w.cap_c, w.c_w, w.s_node,
                       w.s_beg, w.c_st, w.e_ent);
    hipLaunchKernelGGL(k_slot_init, dim3(1024), dim3(256), 0, s, w.s_node, w.vel,
                       (const DevCounters*)w.cnt, w.s_rec);
    hipLaunchKernelGGL(k_env_ranges, dim3((w.n_envs + 255) / 256), dim3(256), 0, s, w.envs, w.n_envs,
                       w.c_env, w.s_node, (const DevCounters*)w.cnt, w.cap_c, w.env_range);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Shared pieces of the two solver kernels
// ---------------------------------------------------------------------------
struct QnArgs {
    const DevRigid* rigids;
    const float* x;         // particle positions at substep start (torque arms)
    long long P;
    float4* vel;
    long long cap;
    const int *c_pid, *c_rid;
    const ContactRec* c_rec;
    const ContactStencil* c_st;
    ContactDyn* c_dyn;
    double* c_coef;
    const int *s_node, *s_beg;
    const Entry* e_ent;
    SlotRec* s_rec;
    double* partial;        // per block: the node pass's sums
    double* partial_odd;    // the same for odd iterations of the one-barrier form
    double* partial2;       // [3][kQnMaxBlocks] per block: the contact pass's shares of phi''(0) - A, phi''', phi''''
    double* rigid_acc;
    int n_rigid;
    SubstepStats* stats;
    int substep;
    double h, eps_r, eps_a;
    int max_iter, ls_max_steps;
    const int2* qn_map;        // per block: (environment, rank in its group)
    const int* env_qn;         // per environment: first block and size of its group
    const int* env_range;      // per environment: contacts [c0, c1), contact nodes [s0, s1)
    const double* env_pnorm;   // per environment: sum m |v*|^2 over its active nodes
    unsigned* env_bar;         // per environment: barrier count and generation
    unsigned* env_ctr;         // per environment: loop-barrier arrival counters
    int n_envs;
    int env_stride;            // > 0: block b solves environments b, b + stride, ... alone
    int compact;               // 0: no block takes the compact node pass
    int* env_pend;             // per environment: 1 when k_qn<true> left it to k_qn<false>
    double* u_acc;             // [3 buffers][3][kQnScatterMax] per-contact sums U_c of the one-barrier form
    double* vc_blk;            // per group rank: kQnRankWords doubles (see the one-barrier set-up)
    double* ls_prm;            // [5][kQnScatterMax]: eps_s^2, mu n0, phi0, d, h k per contact (one-barrier form)
    int timers;                // 1: the first block of each environment times the solver's phases
    int slots_per_block;       // contact nodes per block that set an environment's group size
    double* ls_part;           // [2][kQnMaxBlocks][2] line-search sums of the distributed line search
    double* nt_slot;           // exact-Newton variant: per contact-node vectors
    double* nt_con;            // exact-Newton variant: per-contact terms
    DevCounters* cnt;
};

__device__ __forceinline__ ContactParams params_of(const ContactRec& R, double h) {
    ContactParams P;
    P.phi0 = R.phi0;
    P.mun0 = R.mun0;
    P.k = R.k;
    P.d = R.d;
    P.eps_s = R.eps_s;
    P.h = h;
    return P;
}

// Contact velocity at iteration k: v_c^0 from the initial gather, then
// v_c^k = v_c^{k-1} + alpha_{k-1} u_c^{k-1} (exact: v_c is linear in v). The
// iteration that computes u_c^k also stores v_c^k in buffer k&1.
__device__ __forceinline__ void contact_velocity(const ContactDyn& D, int k, double alpha_prev, double vc[3]) {
    const int src = k == 0 ? 0 : (k - 1) & 1;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        vc[a] = k == 0 ? ld_x(&D.vc[0][a]) : fma(alpha_prev, ld_x(&D.uc[src][a]), ld_x(&D.vc[src][a]));
}

// u = R_c^T U in the contact frame, with the same rounding wherever it is formed.
__device__ __forceinline__ void frame_project(const double t1[3], const double t2[3], const double n[3],
                                              const double U[3], double u[3]) {
    u[0] = fma(t1[0], U[0], fma(t1[1], U[1], t1[2] * U[2]));
    u[1] = fma(t2[0], U[0], fma(t2[1], U[1], t2[2] * U[2]));
    u[2] = fma(n[0], U[0], fma(n[1], U[1], n[2] * U[2]));
}
__device__ __forceinline__ void frame_project(const ContactRec& R, const double U[3], double u[3]) {
    frame_project(R.t1, R.t2, R.n, U, u);
}

// Sum of x over the 64 lanes of a wave, the same bits in every lane: DPP
// exchanges inside each row of 16 lanes (pairs, quads, half rows, rows; each
// step adds two equal partial sums in either order, so the lanes stay equal),
// then the rows pairwise and the halves by the permlane swaps of gfx950: the
// total is (row 0 + row 1) + (row 2 + row 3) in every lane. Every lane of the
// wave must be active.
template <int kCtrl>
__device__ __forceinline__ double dpp_move(double x) {
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, kCtrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), kCtrl, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
// x plus its value in the partner row (kHalf = false: rows 0-1 and 2-3) or
// half (true); both swap results together hold the lane's own value and the
// partner's, in an order that is the same in every lane of a pair.
template <bool kHalf>
__device__ __forceinline__ double swap_add(double x) {
    const long long b = __builtin_bit_cast(long long, x);
    const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
    const auto l = kHalf ? __builtin_amdgcn_permlane32_swap(lo, lo, false, false)
                         : __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = kHalf ? __builtin_amdgcn_permlane32_swap(hi, hi, false, false)
                         : __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    const double a = __builtin_bit_cast(double, ((long long)h[0] << 32) | (long long)l[0]);
    const double c = __builtin_bit_cast(double, ((long long)h[1] << 32) | (long long)l[1]);
    return a + c;
}
__device__ __forceinline__ double wave_sum(double x) {
    x += dpp_move<0xB1>(x);   // quad_perm [1, 0, 3, 2]
    x += dpp_move<0x4E>(x);   // quad_perm [2, 3, 0, 1]
    x += dpp_move<0x141>(x);  // row_half_mirror
    x += dpp_move<0x140>(x);  // row_mirror
    x = swap_add<false>(x);   // rows 0 + 1, rows 2 + 3
    return swap_add<true>(x); // the two halves
}

// The value x of the lane 32 (kHalf) or 16 lanes away (lane ^ 32, lane ^ 16)
// by the permlane swaps: of the two results one is the lane's own value,
// the other its partner's (told apart by comparing the bits).
template <bool kHalf>
__device__ __forceinline__ double lane_partner(double x) {
    const long long b = __builtin_bit_cast(long long, x);
    const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
    const auto l = kHalf ? __builtin_amdgcn_permlane32_swap(lo, lo, false, false)
                         : __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = kHalf ? __builtin_amdgcn_permlane32_swap(hi, hi, false, false)
                         : __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    const bool first_is_own = l[0] == lo && h[0] == hi;
    const unsigned plo = first_is_own ? l[1] : l[0], phi = first_is_own ? h[1] : h[0];
    return __builtin_bit_cast(double, ((long long)phi << 32) | (long long)plo);
}
template <int kDist>
__device__ __forceinline__ double lane_xor(double x) {
    if constexpr (kDist == 32) return lane_partner<true>(x);
    else if constexpr (kDist == 16) return lane_partner<false>(x);
    else return dpp_move<0x128>(x);  // kDist == 8: row_ror:8
}
// One halving step of a multi-value wave reduction: the lanes with bit kDist
// clear keep the first H values, the others the last H, each plus the
// partner's copy of the same value.
template <int kDist, int H, int P>
__device__ __forceinline__ void split_step(double (&w)[P]) {
    const bool up = (threadIdx.x & kDist) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const double send = up ? w[i] : w[H + i];
        const double keep = up ? w[H + i] : w[i];
        w[i] = keep + lane_xor<kDist>(send);
    }
}

// Block-wide FP64 sums of NV <= 8 values per thread over a block of NW waves,
// returned in every thread with the same bits in every thread (and in every
// block that sums the same values). In each wave the values (padded to P, a
// power of two) are first split across the lane halves, quarters and eighths
// (lane ^ 32, ^ 16, ^ 8: each exchange moves half of the remaining values),
// so that every group of 64 / P lanes ends with one value, which a butterfly
// over the group completes (each step adds two equal-rank partial sums in
// either order, so the group's lanes agree); one workgroup barrier, then each
// thread adds the wave sums in wave order. buf holds 2 x 16 x NV doubles used
// alternately, so a wave that runs ahead cannot overwrite sums another wave is
// still reading.
template <int NV, int NW = kQnThreads / 64>
__device__ __forceinline__ void block_allsum(double (&v)[NV], double* buf, unsigned& parity) {
    static_assert(NV >= 1 && NV <= 8, "up to eight values");
    constexpr int P = NV == 1 ? 1 : NV == 2 ? 2 : NV <= 4 ? 4 : 8;
    static_assert(NW * P <= 16 * NV, "wave sums fit the buffer");
    double* b = buf + (parity & 1u) * 16 * NV;
    parity ^= 1u;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double w[P];
#pragma unroll
    for (int i = 0; i < P; ++i) w[i] = i < NV ? v[i] : 0.0;
    int idx = 0;
    if constexpr (P >= 2) { split_step<32, P / 2>(w); idx += (lane & 32) ? P / 2 : 0; }
    if constexpr (P >= 4) { split_step<16, P / 4>(w); idx += (lane & 16) ? P / 4 : 0; }
    if constexpr (P >= 8) { split_step<8, 1>(w); idx += (lane & 8) ? 1 : 0; }
    double x = w[0];
    x += dpp_move<0xB1>(x);   // quad_perm [1, 0, 3, 2]
    x += dpp_move<0x4E>(x);   // quad_perm [2, 3, 0, 1]
    x += dpp_move<0x141>(x);  // row_half_mirror
    if constexpr (P <= 4) x += dpp_move<0x140>(x);  // row_mirror
    if constexpr (P <= 2) x = swap_add<false>(x);   // rows 0 + 1, rows 2 + 3
    if constexpr (P == 1) x = swap_add<true>(x);    // the two halves
    if ((lane & (64 / P - 1)) == 0 && idx < NV) b[wave * P + idx] = x;
    __syncthreads();
    // NW is the block's wave count: a constant, so all the reads issue together
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double t = 0.0;
#pragma unroll
        for (int w2 = 0; w2 < NW; ++w2) t += b[w2 * P + k];
        v[k] = t;
    }
}

// Sum over the 27 stencil nodes of a contact of w times a 3-vector of the
// node's slot record (kField: offset in doubles inside SlotRec). The loads of
// a 9-node layer are issued together; a node with no slot (zero weight) reads
// slot 0 with weight 0.
template <int kField>
__device__ __forceinline__ void stencil_sum(const QnArgs& A, long long c, double acc[3]) {
    const ContactStencil& st = A.c_st[c];
    acc[0] = acc[1] = acc[2] = 0.0;
#pragma unroll 1
    for (int g = 0; g < 3; ++g) {
        int sl[9];
        double w[9];
#pragma unroll
        for (int o = 0; o < 9; ++o) {
            const int q = st.slot[9 * g + o];
            sl[o] = q < 0 ? 0 : q;
            w[o] = q < 0 ? 0.0 : (double)st.w[9 * g + o];
        }
        double val[9][3];
#pragma unroll
        for (int o = 0; o < 9; ++o) {
            const double* r = &A.s_rec[sl[o]].m + kField;
            val[o][0] = r[0]; val[o][1] = r[1]; val[o][2] = r[2];
        }
#pragma unroll
        for (int o = 0; o < 9; ++o)
#pragma unroll
            for (int a = 0; a < 3; ++a) acc[a] += w[o] * val[o][a];
    }
}
constexpr int kSlotV = 1;   // SlotRec::v
static_assert(offsetof(SlotRec, v) == kSlotV * sizeof(double), "SlotRec layout");

// Initial contact velocity v_c^0 = R_c^T sum w v*_i + b_c.
__device__ __forceinline__ void initial_contact_velocity(const QnArgs& A, long long c) {
    double sacc[3];
    stencil_sum<kSlotV>(A, c, sacc);
    const ContactRec& rec = A.c_rec[c];
    ContactDyn& D = A.c_dyn[c];
    // device-scope stores: other blocks read v_c^0 after the solve's first barrier
    st_x(&D.vc[0][0], rec.t1[0] * sacc[0] + rec.t1[1] * sacc[1] + rec.t1[2] * sacc[2] + D.b[0]);
    st_x(&D.vc[0][1], rec.t2[0] * sacc[0] + rec.t2[1] * sacc[1] + rec.t2[2] * sacc[2] + D.b[1]);
    st_x(&D.vc[0][2], rec.n[0] * sacc[0] + rec.n[1] * sacc[1] + rec.n[2] * sacc[2] + D.b[2]);
}

// g, H -> dv by 3x3 Cholesky, and this node's share of the iteration sums.
// A contact node's mass, iterate and free-motion velocity.
struct SlotVals {
    double m, v[3], vs[3];
};

__device__ __forceinline__ SlotVals slot_vals(const SlotRec& S) {
    SlotVals o;
    o.m = S.m;
#pragma unroll
    for (int a = 0; a < 3; ++a) { o.v[a] = S.v[a]; o.vs[a] = S.vstar[a]; }
    return o;
}

// g, H -> dv = -H^{-1} g by 3x3 Cholesky (reciprocal square roots), and this
// node's share of the iteration sums.
__device__ __forceinline__ void node_solve(const SlotVals& S, const double j[3], const double Hc[6],
                                           double sums[kQnSums], double dv[3]) {
    const double m = S.m, inv_m = rcp_nr(m);
    const double H[6] = {m + Hc[0], Hc[1], Hc[2], m + Hc[3], Hc[4], m + Hc[5]};  // 00 01 02 11 12 22
    double g[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) g[a] = m * (S.v[a] - S.vs[a]) - j[a];
    const double i00 = inv_sqrt(H[0]);
    const double l10 = H[1] * i00, l20 = H[2] * i00;
    const double i11 = inv_sqrt(H[3] - l10 * l10);
    const double l21 = (H[4] - l20 * l10) * i11;
    const double i22 = inv_sqrt(H[5] - l20 * l20 - l21 * l21);
    const double y0 = -g[0] * i00;
    const double y1 = (-g[1] - l10 * y0) * i11;
    const double y2 = (-g[2] - l20 * y0 - l21 * y1) * i22;
    dv[2] = y2 * i22;
    dv[1] = (y1 - l21 * dv[2]) * i11;
    dv[0] = (y0 - l10 * dv[1] - l20 * dv[2]) * i00;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        sums[0] += g[a] * g[a] * inv_m;              // |grad~|^2
        sums[1] += j[a] * j[a] * inv_m;              // |j~|^2
        sums[2] += m * S.v[a] * S.v[a];              // contact-node part of |p~|^2
        sums[3] += m * S.vs[a] * S.vs[a];            // same nodes at v*
        sums[4] += m * dv[a] * dv[a];                // A
        sums[5] += m * dv[a] * (S.v[a] - S.vs[a]);   // B
        sums[6] += g[a] * dv[a];                     // phi'(0)
    }
}

// R gamma and the upper triangle of R G R^T of one contact at contact velocity vc.
__device__ __forceinline__ void contact_terms(const double t1[3], const double t2[3], const double n[3],
                                              const ContactParams& P, const double vc[3],
                                              double rg[3], double rgr[6]) {
    double g[3], g00, g01, g11, gnn;
    contact_model(P, vc, g, &g00, &g01, &g11, &gnn);
#pragma unroll
    for (int a = 0; a < 3; ++a) rg[a] = t1[a] * g[0] + t2[a] * g[1] + n[a] * g[2];
    int q = 0;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int cc = r; cc < 3; ++cc)
            rgr[q++] = g00 * t1[r] * t1[cc] + g01 * (t1[r] * t2[cc] + t2[r] * t1[cc]) + g11 * t2[r] * t2[cc] +
                       gnn * n[r] * n[cc];
}
__device__ __forceinline__ void contact_terms(const ContactRec& rec, double h, const double vc[3],
                                              double rg[3], double rgr[6]) {
    contact_terms(rec.t1, rec.t2, rec.n, params_of(rec, h), vc, rg, rgr);
}

// Impulse on the rigid bodies at the final iterate (minus the impulse on MPM),
// reduced per body in LDS (racc: 6 doubles per body, zeroed by the caller).
__device__ __forceinline__ void contact_impulse_at(const QnArgs& A, long long c, const double vc[3],
                                                   double* racc) {
    ContactDyn& D = A.c_dyn[c];
    const ContactRec& rec = A.c_rec[c];
    double g[3], g00, g01, g11, gnn;
    contact_model(params_of(rec, A.h), vc, g, &g00, &g01, &g11, &gnn);
    double rg[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        rg[a] = rec.t1[a] * g[0] + rec.t2[a] * g[1] + rec.n[a] * g[2];
        D.gam[a] = g[a];
    }
    const int r = A.c_rid[c];
    const long long p = A.c_pid[c];
    const DevRigid& R = A.rigids[r];
    const double arm[3] = {(double)A.x[p] - R.t[0], (double)A.x[A.P + p] - R.t[1],
                           (double)A.x[2 * A.P + p] - R.t[2]};
    const double tq[3] = {arm[1] * rg[2] - arm[2] * rg[1], arm[2] * rg[0] - arm[0] * rg[2],
                          arm[0] * rg[1] - arm[1] * rg[0]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        atomicAdd(&racc[r * 6 + a], -rg[a]);
        atomicAdd(&racc[r * 6 + 3 + a], -tq[a]);
    }
}
__device__ __forceinline__ void contact_impulse(const QnArgs& A, long long c, int k, double alpha_prev,
                                                double* racc) {
    double vc[3];
    contact_velocity(A.c_dyn[c], k, alpha_prev, vc);
    contact_impulse_at(A, c, vc, racc);
}

// The line search's first trial step from alpha = 0, given f = phi'(0) and
// f1..f3 = phi'', phi''', phi'''' there (f1 > 0): Householder's third-order
// step, written in t = f / f1, r2 = f2 / f1, r3 = f3 / f1 so that no power of
// the derivatives can leave the exponent range; Newton's step -t where its
// denominator is not positive. With f2 = f3 = 0 it is Newton's step.
__device__ __forceinline__ double ls_first_step(double f, double f1, double f2, double f3) {
    const double r = rcp_nr(f1);
    const double t = f * r, r2 = f2 * r, r3 = f3 * r;
    const double den = fma(t, fma(t, r3 * (1.0 / 6.0), -r2), 1.0);
    return den > 0.0 ? -t * fma(-0.5 * t, r2, 1.0) * rcp_nr(den) : -t;
}

// Exact line search: the root of phi'(alpha) for alpha > 0 (phi is convex
// with phi'(0) = d0 < 0). Safeguarded 1-D Newton from alpha0: while no point
// with phi' >= 0 is known the step only grows (Newton, or doubling when
// Newton does not advance); once the root is bracketed, a Newton step that
// leaves the bracket or does not halve |phi'| is replaced by bisection. Stops
// at |phi'| <= 1e-10 |d0| or a bracket narrower than 1e-12 of its upper end.
// EVAL(alpha, &phi'') returns phi'(alpha); it must be called uniformly by
// the whole block.
template <typename Eval>
__device__ double exact_line_search(Eval eval, double alpha0, double d0, int max_steps, int* n_eval) {
    double lo = 0.0, hi = 0.0, alpha = alpha0, prev = fabs(d0), dd;
    bool bracketed = false;
    for (int it = 0; it < max_steps + 80; ++it) {
        const double da = eval(alpha, &dd);
        ++*n_eval;
        if (fabs(da) <= 1e-10 * fabs(d0)) break;
        if (da < 0.0) {
            lo = alpha;
        } else {
            hi = alpha;
            bracketed = true;
        }
        if (bracketed && hi - lo <= 1e-12 * hi) break;
        double an = dd > 0.0 ? alpha - da * rcp_nr(dd) : -1.0;
        if (bracketed) {
            if (!(an > lo && an < hi) || fabs(da) > 0.5 * prev) an = 0.5 * (lo + hi);
        } else if (!(an > alpha)) {
            an = 2.0 * alpha;
        }
        prev = fabs(da);
        alpha = an;
    }
    return alpha;
}

__device__ __forceinline__ void write_stats(const QnArgs& A, int env, long long nc, long long ns, int k,
                                            int converged, int ls_total, double res, double thr,
                                            const unsigned long long tph[8], bool aborted, int kind) {
    SubstepStats st;
    st.n_contacts = (int)nc;
    st.n_slots = (int)ns;
    st.iterations = k;
    st.converged = converged;
    st.ls_rounds = ls_total;
    st.pad = kind;
    st.residual = res;
    st.threshold = thr;
    for (int q = 0; q < 8; ++q) st.t_phase[q] = tph[q];
    A.stats[(size_t)A.substep * A.n_envs + env] = st;
    if (!converged && !aborted) atomicOr(&A.cnt->flags, kFlagNoconv);
}

// ---------------------------------------------------------------------------
// Solver: one persistent cooperative kernel for every environment. Each
// environment's contact problem is independent (its own stopping test and
// line search) and is solved by a group of blocks: the group splits the
// environment's contact nodes and contacts evenly and meets at two group
// barriers per iteration; a group of one block needs workgroup barriers only.
// With more environments than co-resident blocks, every block solves
// environments b, b + stride, ... one after the other, alone.
// ---------------------------------------------------------------------------

// Barrier of the G blocks of one group (bar[0]: arrivals, bar[1]: generation).
// Returns false when a member did not arrive within the time limit (the
// kernel then stops and the step reports a device error).
__device__ __forceinline__ bool group_sync(unsigned* bar, unsigned G, unsigned* gen, unsigned* s_ok,
                                           DevCounters* cnt) {
    if (G == 1u) {
        __syncthreads();
        return true;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned target = *gen + 1u;
        bool ok = true;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned arrived = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == G - 1u) {
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&bar[1], target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const long long t0 = clock64();
            unsigned polls = 0;
            while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != target) {
                __builtin_amdgcn_s_sleep(1);
                if ((++polls & 255u) == 0u &&
                    ((__hip_atomic_load(&cnt->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kFlagHang) ||
                     clock64() - t0 > kBarrierTimeoutCycles)) {
                    atomicOr(&cnt->flags, kFlagHang);
                    ok = false;
                    break;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_ok = ok ? 1u : 0u;
    }
    __syncthreads();
    *gen += 1u;
    return *s_ok != 0u;
}

// Barrier of the iteration loop, for data exchanged through ld_x / st_x.
// Arrivals are spread over kCtrLanes counters that only grow (a block adds to
// counter rank mod kCtrLanes, each in its own cache line, so groups of up to
// kCtrLanes blocks never contend for one); the i-th barrier after the start of
// the solve completes when their sum reaches its value at the start plus i *
// G. The lanes of the first wave poll the counters together, one each. Each thread waits for its own stores
// to be acknowledged before the block arrives. Same time limit as group_sync.
__device__ __forceinline__ unsigned ctr_sum(unsigned* ctr) {
    const int lane = threadIdx.x & 63;
    int v = lane < kCtrLanes
                ? (int)__hip_atomic_load(&ctr[lane * kCtrStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                : 0;
#pragma unroll
    for (int m = 1; m < kCtrLanes; m <<= 1) v += __shfl_xor(v, m, 64);
    return (unsigned)__shfl(v, 0, 64);
}
__device__ __forceinline__ bool loop_sync(unsigned* ctr, int rank, unsigned G, unsigned* target, unsigned* s_ok,
                                          DevCounters* cnt) {
    if (G == 1u) {
        __syncthreads();
        return true;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    *target += G;
    if (threadIdx.x < 64) {
        bool ok = true;
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(&ctr[(rank % kCtrLanes) * kCtrStride], 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        const long long t0 = clock64();
        unsigned polls = 0;
        while ((int)(ctr_sum(ctr) - *target) < 0) {
            __builtin_amdgcn_s_sleep(1);
            if ((++polls & 255u) == 0u &&
                ((__hip_atomic_load(&cnt->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kFlagHang) ||
                 clock64() - t0 > kBarrierTimeoutCycles)) {
                if (threadIdx.x == 0) atomicOr(&cnt->flags, kFlagHang);
                ok = false;
                break;
            }
        }
        if (threadIdx.x == 0) *s_ok = ok ? 1u : 0u;
    }
    __syncthreads();
    return *s_ok != 0u;
}

constexpr int kEntBatch = 2;     // CSR entries per thread whose loads are issued together
constexpr int kLsPer = 3;        // contacts per thread the line search keeps in registers
constexpr int kUniqMax = kQnUniqMax;  // distinct contacts of a block's entries the compact node pass holds
constexpr int kEntMax = 2048;    // CSR entries of a block the compact node pass holds
constexpr int kHashBits = 12;
constexpr int kHash = 1 << kHashBits;  // open-addressing table that finds the distinct contacts
static_assert(kHash * sizeof(int) <= 9 * kSlotChunk * sizeof(double), "hash table lives in nacc");
static_assert(9 * kUniqMax <= 11 * kQnThreads, "contact terms live in the line-search buffer");
static_assert(kEntMax <= kHash / 2, "the hash table is at most half full");
static_assert(kUniqMax <= 65536, "block-local contact indices are 16-bit");
static_assert(kUniqMax <= kQnThreads, "at most one distinct contact per thread in the one-barrier set-up");
constexpr int kEntPer = kEntMax / kQnThreads;  // entries per thread in the compact set-up
// contacts of an environment the one-barrier form takes: each thread keeps
// kLsPer in registers and one in LDS during the line search
constexpr int kScatterMax = (kLsPer + 1) * kQnThreads;
static_assert(kScatterMax == kQnScatterMax, "scratch of the one-barrier form");
static_assert(3 * kUniqMax <= 4 * kQnThreads, "contact velocities live in the stencil cache");
static_assert(9 * kUniqMax <= 9 * kSlotChunk, "per-contact sums live in nacc");

template <bool kOne>
__global__ void __launch_bounds__(kQnThreads)
k_qn(QnArgs A) {
    __shared__ double rbuf[2 * 16 * kQnSums];
    __shared__ double tot[kQnSums];
    __shared__ double racc[kMaxRigid * 6];
    __shared__ unsigned s_ok;
    // line-search contacts beyond the registers; in the compact node pass, the
    // terms of the block's distinct contacts ([9][kUniqMax])
    __shared__ double ovf_raw[11 * kQnThreads];
    using LsC = std::conditional_t<kOne, LsCoefC, LsCoef>;  // a line-search contact's coefficients
    static_assert(sizeof(LsC) <= 11 * sizeof(double), "line-search LDS contacts");
    LsC* ls_ovf = reinterpret_cast<LsC*>(ovf_raw);
    double* u_term = ovf_raw;
    __shared__ double nacc[9][kSlotChunk];  // j (3) and R G R^T (6) of a chunk of owned slots
    __shared__ unsigned short ent_c[kEntMax];  // compact pass: block-local contact of each entry
    __shared__ float ent_w[kEntMax];           // and its stencil weight
    __shared__ int beg_l[kSlotChunk + 1];           // compact pass: first entry of each contact node
    __shared__ int u_list[kUniqMax];                // compact pass: the distinct contacts
    __shared__ unsigned scan_w[17];
    __shared__ double node_v[3][kSlotChunk];  // compact pass: the iterate of the block's contact nodes,
    __shared__ double node_mv[4][kSlotChunk]; // and their mass and free-motion velocity
    // contact pass of a block with at most T/8 contacts: each lane's stencil
    // slots and weights; in the one-barrier form, the contact velocities of
    // the block's distinct contacts ([3][kUniqMax])
    __shared__ double cst_raw[4 * kQnThreads];
    int(*cst_slot)[kQnThreads] = reinterpret_cast<int(*)[kQnThreads]>(cst_raw);
    float(*cst_w)[kQnThreads] = reinterpret_cast<float(*)[kQnThreads]>(cst_raw + 2 * kQnThreads);
    double* vcl = cst_raw;

    DevCounters* cnt = A.cnt;
    const bool aborted = cnt->abort_step != 0u;
    const int tid = threadIdx.x, T = kQnThreads;  // the launch always takes kQnThreads
    const int2 me = A.qn_map[blockIdx.x];
    unsigned rpar = 0;  // parity of the block-sum buffer
    for (int env = me.x; env < A.n_envs; env += A.env_stride > 0 ? A.env_stride : A.n_envs) {
        const int first = A.env_stride > 0 ? (int)blockIdx.x : A.env_qn[2 * env];
        // blocks launched for this environment; the group uses as many as its
        // contact nodes in this substep ask for (the launch is planned on the
        // host from an earlier substep), and the others skip it
        const unsigned G_launch = A.env_stride > 0 ? 1u : (unsigned)A.env_qn[2 * env + 1];
        const int rank = A.env_stride > 0 ? 0 : me.y;
        const bool writer = rank == 0 && tid == 0;  // writes the environment's stats
        const bool timer = writer && A.timers != 0; // and, when asked, times the phases
        unsigned long long tph[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        unsigned long long tmark = 0;
        // after the one-barrier kernel, only the environments it left
        if (!kOne && A.env_pend != nullptr && A.env_pend[env] == 0) continue;
        if (kOne && writer) A.env_pend[env] = aborted ? 0 : 1;
        if (aborted) {
            if (writer) write_stats(A, env, 0, 0, 0, 1, 0, 0.0, 0.0, tph, true, 0);
            continue;
        }
        unsigned* bar = A.env_bar + (size_t)env * kBarStride;
        unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // read before the first barrier, which no block passes before all have read it
        unsigned* ctr = A.env_ctr + (size_t)env * kCtrLanes * kCtrStride;
        unsigned ltarget = ctr_sum(ctr);
        const long long ec0 = A.env_range[4 * env], ec1 = A.env_range[4 * env + 1];
        const long long es0 = A.env_range[4 * env + 2], es1 = A.env_range[4 * env + 3];
        const long long nc = ec1 - ec0, ns = es1 - es0;
        const unsigned G = (unsigned)std::min<long long>(
            G_launch, std::max<long long>(1, (ns + A.slots_per_block - 1) / A.slots_per_block));
        if ((unsigned)rank >= G) continue;
        if (kOne && nc > kScatterMax) continue;
        // contact nodes split so that every block gets about the same number of
        // CSR entries (the node pass's work); contacts split evenly
        long long s0 = es0, s1 = es1;
        if (G > 1u) {
            const long long e_lo = A.s_beg[es0], e_n = (long long)A.s_beg[es1] - e_lo;
            s0 = rank == 0 ? es0 : es0 + lower_bound_i(A.s_beg + es0, ns, e_lo + (e_n * rank + G - 1) / G);
            s1 = rank + 1 == (int)G ? es1 : es0 + lower_bound_i(A.s_beg + es0, ns, e_lo + (e_n * (rank + 1) + G - 1) / G);
        }
        const long long cper = (nc + G - 1) / G;
        const long long c0 = ec0 + std::min<long long>(nc, cper * rank), c1 = std::min<long long>(ec1, c0 + cper);
        const double pnorm_env = A.env_pnorm[env];
        double* partial = A.partial + (size_t)first * kQnSums;
        double* partial2 = A.partial2 + first;
        // the one-barrier form alternates two buffers of block sums by iteration
        // parity: a block may post iteration k + 1's sums before another has read
        // iteration k's, but not iteration k + 2's (that needs the other's arrival
        // at the next barrier)
        double* partial_odd = A.partial_odd + (size_t)first * kQnSums;

        for (long long c = c0 + tid; c < c1; c += T) initial_contact_velocity(A, c);
        if (kOne) {
            // the line search's per-contact constants, read by every block of
            // the group after the first barrier
            for (long long c = c0 + tid; c < c1; c += T) {
                const ContactRec& R = A.c_rec[c];
                double* q = A.ls_prm + (c - ec0);
                q[0] = R.eps_s * R.eps_s;
                q[kQnScatterMax] = R.mun0;
                q[2 * kQnScatterMax] = R.phi0;
                q[3 * kQnScatterMax] = R.d;
                q[4 * kQnScatterMax] = A.h * R.k;
            }
        }

        // Compact node pass: when the block's contact nodes fit one chunk, its
        // CSR entries number at most kEntMax, and they name at most kUniqMax distinct
        // contacts, the entries stay in LDS for the whole solve (the contact as
        // a block-local index, and the weight) and each distinct contact's terms
        // are formed once per iteration instead of once per entry.
        const int E0s = A.s_beg[s0], n_ent = A.s_beg[s1] - E0s;
        bool compact = A.compact != 0 && s1 - s0 <= kSlotChunk && n_ent <= kEntMax;
        int n_u = 0;
        if (compact) {
            int* htab = reinterpret_cast<int*>(&nacc[0][0]);
            for (int q = tid; q < kHash; q += T) htab[q] = -1;
            __syncthreads();
            int pos[kEntPer];
            float ew[kEntPer];
#pragma unroll
            for (int u = 0; u < kEntPer; ++u) {
                const int e = tid + u * T;
                pos[u] = -1;
                if (e < n_ent) {
                    const Entry en = A.e_ent[E0s + e];
                    ew[u] = en.w;
                    // linear probing; the table is at most half full, so a free
                    // or matching position is always found
                    unsigned hsh = (en.c * 2654435761u) >> (32 - kHashBits);
                    for (;;) {
                        const int prev = atomicCAS(&htab[hsh], -1, (int)en.c);
                        if (prev == -1 || prev == (int)en.c) break;
                        hsh = (hsh + 1) & (kHash - 1);
                    }
                    pos[u] = (int)hsh;
                }
            }
            __syncthreads();
            // number the occupied positions in table order
            constexpr int kPer = kHash / kQnThreads;
            int occ = 0;
#pragma unroll
            for (int q = 0; q < kPer; ++q) occ += htab[tid * kPer + q] >= 0 ? 1 : 0;
            unsigned n_occ;
            int base = (int)block_exclusive_scan_total((unsigned)occ, scan_w, &n_occ);
            n_u = (int)n_occ;
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                const int h = tid * kPer + q;
                const int c = htab[h];
                if (c >= 0) {
                    if (base < kUniqMax) u_list[base] = c;
                    htab[h] = base++;
                }
            }
            __syncthreads();
            compact = n_u <= kUniqMax;
            if (compact) {
#pragma unroll
                for (int u = 0; u < kEntPer; ++u)
                    if (pos[u] >= 0) {
                        ent_c[tid + u * T] = (unsigned short)htab[pos[u]];
                        ent_w[tid + u * T] = ew[u];
                    }
                if (tid < s1 - s0) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) node_v[a][tid] = A.s_rec[s0 + tid].v[a];
                    node_mv[0][tid] = A.s_rec[s0 + tid].m;
#pragma unroll
                    for (int a = 0; a < 3; ++a) node_mv[1 + a][tid] = A.s_rec[s0 + tid].vstar[a];
                    beg_l[tid] = A.s_beg[s0 + tid] - E0s;
                }
                if (tid == 0) beg_l[s1 - s0] = n_ent;
            }
            __syncthreads();
        }
        // compact pass: nl adjacent lanes share a contact node's entries (as many
        // as the block's threads allow, up to 8)
        int lg_nl = 0;
        while (lg_nl < 3 && (s1 - s0) << (lg_nl + 1) <= T) ++lg_nl;
        const int nl = 1 << lg_nl;
        // contact pass of a block whose contacts fit one pass (eight lanes each):
        // the lanes' stencil slots and weights stay in LDS for the whole solve
        const bool ccache = c1 - c0 <= T / 8;
        if (ccache) {
            const long long c = c0 + (tid >> 3);
            const int part = tid & 7;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int o = part + 8 * j;
                const int q = (o < 27 && c < c1) ? A.c_st[c].slot[o] : -1;
                cst_slot[j][tid] = q < 0 ? 0 : q;
                cst_w[j][tid] = q < 0 ? 0.f : A.c_st[c].w[o];
            }
        }

        // the one-barrier form needs every block of the group in the compact
        // form: each block posts its flag before the first barrier and reads
        // the others' after it; the first two iterations' sums start at zero
        if (kOne) {
            if (G > 1u && tid == 0) st_x(&partial2[rank], compact ? 1.0 : 0.0);
            for (long long c = c0 + tid; c < c1; c += T)
#pragma unroll
                for (int q = 0; q < 6; ++q) st_x(&A.u_acc[q * kQnScatterMax + (c - ec0)], 0.0);
        }

        int k = 0, ls_total = 0, converged = 0;
        unsigned ls_par = 0;  // buffer parity of the distributed line search
        double alpha_prev = 1.0, res = 0.0, thr = 0.0;
        // every thread's stores above (v_c^0, cleared sums, flags) acknowledged
        // before its block arrives
        __builtin_amdgcn_s_waitcnt(0);
        bool ok = group_sync(bar, G, &gen, &s_ok, cnt);
        bool all_compact = compact;
        if (kOne && ok && G > 1u) {
            if (tid < 64) {
                double a = 0.0;
                for (unsigned b = tid; b < G; b += 64) a += ld_x(&partial2[b]);
                a = wave_sum(a);
                if (tid == 0) tot[0] = a;
            }
            __syncthreads();
            all_compact = tot[0] == (double)G;
            __syncthreads();
        }
        if (kOne && !all_compact) continue;  // left to k_qn<false>
        constexpr bool scatter = kOne;
        const bool cmp = kOne || compact;  // the compact node pass
        // The rank's scratch (rank < G <= kQnMaxGroup), in arrays of kQnThreads
        // doubles so that a wave's loads are contiguous: [kLsPer + 1][6][T]
        // v_c, u_c of the thread's line-search contacts ec0 + tid + u T, then
        // [kQnRecWords][kUniqMax] the records of the block's distinct contacts
        // (t1, t2, n, phi0, mu n0, k, d, eps_s), read only by the thread that
        // wrote them.
        static_assert(6 * (kLsPer + 1) * kQnThreads == 6 * kQnScatterMax, "rank scratch layout");
        double* vblk = A.vc_blk + (size_t)rank * kQnRankWords;
        double* crec = vblk + 6 * kQnScatterMax;
        if (scatter) {
            for (int t = tid; t < n_u; t += T) {
                const int c = u_list[t];
#pragma unroll
                for (int a = 0; a < 3; ++a) vcl[a * kUniqMax + t] = ld_x(&A.c_dyn[c].vc[0][a]);
                const ContactRec& R = A.c_rec[c];
                const double r[kQnRecWords] = {R.t1[0], R.t1[1], R.t1[2], R.t2[0], R.t2[1], R.t2[2],
                                               R.n[0],  R.n[1],  R.n[2],  R.phi0,  R.mun0,  R.k,
                                               R.d,     R.eps_s};
#pragma unroll
                for (int j = 0; j < kQnRecWords; ++j) crec[j * kUniqMax + t] = r[j];
            }
            // the line search's contacts start from v_c^0 with a zero step
            for (int u = 0; u <= kLsPer; ++u) {
                const long long c = ec0 + tid + (long long)u * T;
                if (c >= ec1) break;
                double* vb = vblk + u * 6 * kQnThreads + tid;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    vb[a * kQnThreads] = ld_x(&A.c_dyn[c].vc[0][a]);
                    vb[(3 + a) * kQnThreads] = 0.0;
                }
            }
            __syncthreads();
        }
        int buf = 0;  // the iteration's buffer of the per-contact sums (k mod 3)
        // One-barrier form: the thread's first kLsPer line-search contacts
        // (ec0 + tid + u T) live in registers for the whole solve: v_c^0 and
        // the constants loaded once, u_c^k loaded after each iteration's
        // barrier, v_c^{k+1} = v_c^k + alpha_k u_c^k formed in the update. A
        // contact past kLsPer T keeps v_c, u_c in the rank's scratch instead.
        LsState st[kLsPer];
        // the environment's eps_s^2, d and h k (equal for all its contacts), as
        // block-uniform values
        LsUni lsu{1.0, A.h, 0.0, 0.0};
        if (scatter && nc > 0) {
            lsu.eps2 = uniform_f64(A.ls_prm[0]);
            lsu.d = uniform_f64(A.ls_prm[3 * kQnScatterMax]);
            lsu.hk = uniform_f64(A.ls_prm[4 * kQnScatterMax]);
        }
#pragma unroll
        for (int u = 0; u < kLsPer; ++u) {
            st[u] = ls_state_zero();
            const long long c = ec0 + tid + (long long)u * T;
            if (scatter && c < ec1) {
                const double* q = A.ls_prm + (c - ec0);
#pragma unroll
                for (int a = 0; a < 3; ++a) st[u].vc[a] = ld_x(&A.c_dyn[c].vc[0][a]);
                st[u].mun0 = q[kQnScatterMax];
                st[u].phi0 = q[2 * kQnScatterMax];
            }
        }
        struct SetupIn {
            double uu[3], vo[3], uo[3], pr[5];
        };
        const long long clast = nc > 0 ? ec1 - 1 : ec0;
        while (ok) {
            if (timer) tmark = wall_clock64();
            // ---- node pass: CSR entries spread over the threads, FP64 LDS sums ----
            double sums[kQnSums];
#pragma unroll
            for (int q = 0; q < kQnSums; ++q) sums[q] = 0.0;
            if (cmp) {
                const int ls = tid >> lg_nl, sub = tid & (nl - 1);
                const bool mine = ls < s1 - s0;    // a lane of contact node ls
                const bool own = mine && sub == 0; // its first lane, which keeps its results
                SlotVals sv;
                sv.m = mine ? node_mv[0][ls] : 1.0;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    sv.vs[a] = mine ? node_mv[1 + a][ls] : 0.0;
                    sv.v[a] = mine ? node_v[a][ls] : 0.0;
                }
                for (int t = tid; t < n_u; t += T) {
                    const unsigned c = (unsigned)u_list[t];
                    double vc[3], rg[3], rgr[6];
                    if (scatter) {
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            vc[a] = vcl[a * kUniqMax + t];
                            nacc[3 + a][t] = 0.0;
                        }
                    } else {
                        contact_velocity(A.c_dyn[c], k, alpha_prev, vc);
                    }
                    if (scatter) {
                        // the record cached in the rank's scratch (coalesced loads)
                        double r[kQnRecWords];
#pragma unroll
                        for (int j = 0; j < kQnRecWords; ++j) r[j] = crec[j * kUniqMax + t];
                        ContactParams P;
                        P.phi0 = r[9]; P.mun0 = r[10]; P.k = r[11]; P.d = r[12]; P.eps_s = r[13]; P.h = A.h;
                        contact_terms(r, r + 3, r + 6, P, vc, rg, rgr);
                    } else {
                        contact_terms(A.c_rec[c], A.h, vc, rg, rgr);
                    }
#pragma unroll
                    for (int a = 0; a < 3; ++a) u_term[a * kUniqMax + t] = rg[a];
#pragma unroll
                    for (int q = 0; q < 6; ++q) u_term[(3 + q) * kUniqMax + t] = rgr[q];
                }
                __syncthreads();
                // the nl lanes of a contact node add every nl-th of its entries'
                // terms, then combine their sums by DPP exchanges
                double j[3] = {0.0, 0.0, 0.0}, Hc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                if (mine) {
                    const int e1 = beg_l[ls + 1];
                    for (int e = beg_l[ls] + sub; e < e1; e += nl) {
                        const int lc = ent_c[e];
                        const double w = (double)ent_w[e];
#pragma unroll
                        for (int a = 0; a < 3; ++a) j[a] = fma(w, u_term[a * kUniqMax + lc], j[a]);
                        const double w2 = w * w;
#pragma unroll
                        for (int q = 0; q < 6; ++q) Hc[q] = fma(w2, u_term[(3 + q) * kUniqMax + lc], Hc[q]);
                    }
                }
                // (DPP butterflies over the nl lanes: quad_perm [1, 0, 3, 2],
                // [2, 3, 0, 1], then the other quad of the eight by
                // row_half_mirror; each step adds two values in either order,
                // so all nl lanes hold the same bits)
                if (nl > 1) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) j[a] += dpp_move<0xB1>(j[a]);
#pragma unroll
                    for (int q = 0; q < 6; ++q) Hc[q] += dpp_move<0xB1>(Hc[q]);
                }
                if (nl > 2) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) j[a] += dpp_move<0x4E>(j[a]);
#pragma unroll
                    for (int q = 0; q < 6; ++q) Hc[q] += dpp_move<0x4E>(Hc[q]);
                }
                if (nl > 4) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) j[a] += dpp_move<0x141>(j[a]);
#pragma unroll
                    for (int q = 0; q < 6; ++q) Hc[q] += dpp_move<0x141>(Hc[q]);
                }
                if (timer) { const unsigned long long t = wall_clock64(); tph[0] += t - tmark; tmark = t; }
                // every lane of the node solves it (the same bits in each), so
                // all of them hold dv for the scatter; its first lane keeps the sums
                double dv[3] = {0.0, 0.0, 0.0};
                if (mine) {
                    double ns[kQnSums];
#pragma unroll
                    for (int q = 0; q < kQnSums; ++q) ns[q] = 0.0;
                    node_solve(sv, j, Hc, ns, dv);
                    if (own) {
#pragma unroll
                        for (int q = 0; q < kQnSums; ++q) sums[q] = ns[q];
                        if (!scatter) {
                            SlotRec& S = A.s_rec[s0 + ls];
                            st_x(&S.dv[0], dv[0]); st_x(&S.dv[1], dv[1]); st_x(&S.dv[2], dv[2]);
                        }
#pragma unroll
                        for (int a = 0; a < 3; ++a) nacc[a][ls] = dv[a];  // kept for the update
                    }
                }
                if (scatter) {
                    // U_c += w dv over the node's entries: the node's lanes add
                    // their entries into the block's per-contact sums, which then
                    // go to the buffer of this iteration; the next iteration's
                    // buffer is cleared for the block's contacts
                    const double d[3] = {dv[0], dv[1], dv[2]};
                    if (mine) {
                        const int e1 = beg_l[ls + 1];
                        for (int e = beg_l[ls] + sub; e < e1; e += nl) {
                            const int lc = ent_c[e];
                            const double w = (double)ent_w[e];
#pragma unroll
                            for (int a = 0; a < 3; ++a) atomicAdd(&nacc[3 + a][lc], w * d[a]);
                        }
                    }
                    __syncthreads();
                    double* U = A.u_acc + buf * 3 * kQnScatterMax;  // [3][kQnScatterMax]
                    for (int t = tid; t < n_u; t += T) {
                        const long long c = u_list[t];
                        const double Uw[3] = {nacc[3][t], nacc[4][t], nacc[5][t]};
                        double fr[9];
#pragma unroll
                        for (int j = 0; j < 9; ++j) fr[j] = crec[j * kUniqMax + t];
                        double uu[3];
                        frame_project(fr, fr + 3, fr + 6, Uw, uu);
#pragma unroll
                        for (int a = 0; a < 3; ++a)
                            __hip_atomic_fetch_add(&U[a * kQnScatterMax + (c - ec0)], uu[a], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                    }
                    double* Un = A.u_acc + (buf == 2 ? 0 : buf + 1) * 3 * kQnScatterMax;
                    for (long long c = c0 + tid; c < c1; c += T)
#pragma unroll
                        for (int a = 0; a < 3; ++a) st_x(&Un[a * kQnScatterMax + (c - ec0)], 0.0);
                }
            }
            for (long long sa = s0; sa < s1 && !cmp; sa += kSlotChunk) {
                const long long sb = std::min<long long>(s1, sa + kSlotChunk);
                // this thread's contact node of the chunk, loaded before the gather
                const bool own = tid < sb - sa;
                const SlotVals sv = slot_vals(A.s_rec[own ? sa + tid : sa]);
                for (int q = tid; q < 9 * kSlotChunk; q += T) (&nacc[0][0])[q] = 0.0;
                __syncthreads();
                const int E0 = A.s_beg[sa], E1 = A.s_beg[sb];
                for (int eb = E0; eb < E1; eb += T * kEntBatch) {
                    // all loads of a batch of entries first, then the model and the LDS sums
                    Entry en[kEntBatch];
#pragma unroll
                    for (int u = 0; u < kEntBatch; ++u) {
                        const int e = eb + tid + u * T;
                        en[u] = A.e_ent[e < E1 ? e : E0];
                    }
                    double vc[kEntBatch][3], fr[kEntBatch][9];
                    ContactParams P[kEntBatch];
#pragma unroll
                    for (int u = 0; u < kEntBatch; ++u) {
                        contact_velocity(A.c_dyn[en[u].c], k, alpha_prev, vc[u]);
                        const ContactRec& R = A.c_rec[en[u].c];
#pragma unroll
                        for (int a = 0; a < 3; ++a) { fr[u][a] = R.t1[a]; fr[u][3 + a] = R.t2[a]; fr[u][6 + a] = R.n[a]; }
                        P[u] = params_of(R, A.h);
                    }
#pragma unroll
                    for (int u = 0; u < kEntBatch; ++u) {
                        if (eb + tid + u * T >= E1) continue;
                        const int ls = en[u].slot - (int)sa;
                        const double w = en[u].w;
                        double rg[3], rgr[6];
                        contact_terms(fr[u], fr[u] + 3, fr[u] + 6, P[u], vc[u], rg, rgr);
#pragma unroll
                        for (int a = 0; a < 3; ++a) atomicAdd(&nacc[a][ls], w * rg[a]);
#pragma unroll
                        for (int q = 0; q < 6; ++q) atomicAdd(&nacc[3 + q][ls], w * w * rgr[q]);
                    }
                }
                __syncthreads();
                if (timer) { const unsigned long long t = wall_clock64(); tph[0] += t - tmark; tmark = t; }
                if (own) {
                    const int ls = tid;
                    const double j[3] = {nacc[0][ls], nacc[1][ls], nacc[2][ls]};
                    const double Hc[6] = {nacc[3][ls], nacc[4][ls], nacc[5][ls], nacc[6][ls], nacc[7][ls], nacc[8][ls]};
                    double dv[3];
                    node_solve(sv, j, Hc, sums, dv);
                    SlotRec& S = A.s_rec[sa + tid];
                    st_x(&S.dv[0], dv[0]); st_x(&S.dv[1], dv[1]); st_x(&S.dv[2], dv[2]);
                }
                __syncthreads();
            }
            double* part = (kOne && (k & 1)) ? partial_odd : partial;
            block_allsum<kQnSums>(sums, rbuf, rpar);
            if (G > 1u && tid == 0) {
#pragma unroll
                for (int q = 0; q < kQnSums; ++q) st_x(&part[(size_t)rank * kQnSums + q], sums[q]);
            }
            if (timer) { const unsigned long long t = wall_clock64(); tph[1] += t - tmark; tmark = t; }
            ok = loop_sync(ctr, rank, G, &ltarget, &s_ok, cnt);
            if (timer) { const unsigned long long t = wall_clock64(); tph[2] += t - tmark; tmark = t; }
            if (!ok) break;
            // group sums: wave q adds sum q of the group's blocks (the same bits in
            // every block); the loads are issued here and used after the contact
            // pass, which runs before the stopping test (its stores go to
            // parity buffers and the coefficients, which the exit does not read)
            const int wv = tid >> 6, lane = tid & 63;
            double ga = 0.0;
            if (G > 1u && wv < kQnSums) {
                // the first 64 blocks' sums without a loop, so that their loads
                // overlap the set-up's
                if ((unsigned)lane < G) ga = ld_x(&part[(size_t)lane * kQnSums + wv]);
                for (unsigned b = lane + 64; b < G; b += 64) ga += ld_x(&part[(size_t)b * kQnSums + wv]);
            }
            double curv[3] = {0.0, 0.0, 0.0};  // phi'' - A, phi''', phi'''' at alpha = 0
            LsC lc[kLsPer];
            const long long c_lds = ec0 + tid + (long long)kLsPer * T;
            const bool use_lds = (long long)kLsPer * T < nc;
            // an environment with more contacts than a block's registers and LDS
            // hold evaluates the line search distributed: each block sums its
            // own contacts, and every evaluation meets at a group barrier (one
            // barrier instead of every block streaming all coefficients)
            const bool dist = !scatter && G > 1u && nc > (long long)(kLsPer + 1) * T;
            if constexpr (scatter) {
                // ---- line-search set-up in every block, over all the environment's
                // contacts (contact ec0 + i taken by thread i mod T): u_c^k from the
                // sums (v_c^k is already in the thread's registers), the
                // closed-form coefficients, and phi''(0). Only the sums are read
                // after the barrier, every load issued before the first use:
                // indices past the environment's contacts read a valid contact
                // and their values are discarded. U is [3][kQnScatterMax] by the
                // environment's contact: a wave's loads of one component cover
                // 512 contiguous bytes.
                const double* U = A.u_acc + buf * 3 * kQnScatterMax;
                // u_c^k of the register contacts and of the block's distinct
                // contacts (at most one per thread, for their velocities' update),
                // all loads issued together
                double ul[kLsPer][3];
#pragma unroll
                for (int u = 0; u < kLsPer; ++u) {
                    const long long c = ec0 + tid + (long long)u * T;
                    const long long cc = c < ec1 ? c : clast;
#pragma unroll
                    for (int a = 0; a < 3; ++a) ul[u][a] = ld_x(&U[a * kQnScatterMax + (cc - ec0)]);
                }
                const bool has_u = tid < n_u;
                const long long cu = has_u ? (long long)u_list[tid] : clast;
                double un[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) un[a] = ld_x(&U[a * kQnScatterMax + (cu - ec0)]);
#pragma unroll
                for (int u = 0; u < kLsPer; ++u) {
                    const long long c = ec0 + tid + (long long)u * T;
                    if (c < ec1) {
#pragma unroll
                        for (int a = 0; a < 3; ++a) st[u].u[a] = ul[u][a];
                    }
                    // the coefficients, held for this iteration's line search
                    lc[u] = ls_coefc_of(st[u], lsu);
                    double z[4] = {0.0, 0.0, 0.0, 0.0};
                    ls_eval4(lc[u], lsu, 0.0, z);
#pragma unroll
                    for (int q = 0; q < 3; ++q) curv[q] += z[1 + q];
                }
                if (use_lds) {
                    // the contact past kLsPer T (uniform branch: only large sets):
                    // v_c^k = v_c^{k-1} + alpha_{k-1} u_c^{k-1} from the scratch (at
                    // k = 0 it holds v_c^0 and a zero u_c), stored with u_c^k
                    const long long c = ec0 + tid + (long long)kLsPer * T;
                    const long long cc = c < ec1 ? c : clast;
                    double* vb = vblk + kLsPer * 6 * kQnThreads + tid;
                    double uu[3], vo[3], uo[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        uu[a] = ld_x(&U[a * kQnScatterMax + (cc - ec0)]);
                        vo[a] = vb[a * kQnThreads];
                        uo[a] = vb[(3 + a) * kQnThreads];
                    }
                    const double mun0 = A.ls_prm[kQnScatterMax + (cc - ec0)];
                    const double phi0 = A.ls_prm[2 * kQnScatterMax + (cc - ec0)];
                    LsCoefC L = ls_coefc_of(ls_state_zero(), lsu);
                    if (c < ec1) {
                        double vc[3];
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            vc[a] = fma(alpha_prev, uo[a], vo[a]);
                            vb[a * kQnThreads] = vc[a];
                            vb[(3 + a) * kQnThreads] = uu[a];
                        }
                        L = ls_coefc(lsu, mun0, phi0, vc, uu);
                        double z[4] = {0.0, 0.0, 0.0, 0.0};
                        ls_eval4(L, lsu, 0.0, z);
#pragma unroll
                        for (int q = 0; q < 3; ++q) curv[q] += z[1 + q];
                    }
                    ls_ovf[tid] = L;
                }
                if (has_u) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) nacc[6 + a][tid] = un[a];
                }
            } else {
            // ---- contact pass: store v_c^k, u_c = R_c^T J dv, and u_c^T G(v_c^k) u_c
            // (this block's share of phi''(0)). Eight lanes gather one contact's
            // 27 stencil nodes and combine their sums by shuffles.
                const int part = tid & 7;
                for (long long cb = c0; cb < c1; cb += T / 8) {
                    const long long c = cb + (tid >> 3);
                    const bool valid = c < c1;
                    const long long cc = valid ? c : c0;
                    // the contact's records, loaded before the stencil gather
                    ContactDyn& D = A.c_dyn[cc];
                    const ContactRec& R = A.c_rec[cc];
                    double vc[3], fr[9];
                    contact_velocity(D, k, alpha_prev, vc);
#pragma unroll
                    for (int a = 0; a < 3; ++a) { fr[a] = R.t1[a]; fr[3 + a] = R.t2[a]; fr[6 + a] = R.n[a]; }
                    const ContactParams Pc = params_of(R, A.h);
                    const ContactStencil& st = A.c_st[cc];
                    int sl[4];
                    double w[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        if (ccache) {
                            sl[j] = cst_slot[j][tid];
                            w[j] = (double)cst_w[j][tid];
                        } else {
                            const int o = part + 8 * j;
                            const int q = (o < 27 && valid) ? st.slot[o] : -1;
                            sl[j] = q < 0 ? 0 : q;
                            w[j] = q < 0 ? 0.0 : (double)st.w[o];
                        }
                    }
                    double dvs[4][3];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const SlotRec& S = A.s_rec[sl[j]];
                        dvs[j][0] = ld_x(&S.dv[0]); dvs[j][1] = ld_x(&S.dv[1]); dvs[j][2] = ld_x(&S.dv[2]);
                    }
                    double sacc[3] = {0.0, 0.0, 0.0};
#pragma unroll
                    for (int j = 0; j < 4; ++j)
#pragma unroll
                        for (int a = 0; a < 3; ++a) sacc[a] += w[j] * dvs[j][a];
#pragma unroll
                    for (int m = 4; m >= 1; m >>= 1)
#pragma unroll
                        for (int a = 0; a < 3; ++a) sacc[a] += __shfl_xor(sacc[a], m, 64);
                    if (valid && part == 0) {
                        if (k > 0) {
#pragma unroll
                            for (int a = 0; a < 3; ++a) st_x(&D.vc[k & 1][a], vc[a]);
                        }
                        double u[3];
                        u[0] = fr[0] * sacc[0] + fr[1] * sacc[1] + fr[2] * sacc[2];
                        u[1] = fr[3] * sacc[0] + fr[4] * sacc[1] + fr[5] * sacc[2];
                        u[2] = fr[6] * sacc[0] + fr[7] * sacc[1] + fr[8] * sacc[2];
#pragma unroll
                        for (int a = 0; a < 3; ++a) st_x(&D.uc[k & 1][a], u[a]);
                        const LsCoef Lc = ls_coef(Pc, vc, u);
                        store_coef(A.c_coef, c, Lc);
                        double g[3], g00, g01, g11, gnn;
                        contact_model(Pc, vc, g, &g00, &g01, &g11, &gnn);
                        curv[0] += g00 * u[0] * u[0] + 2.0 * g01 * u[0] * u[1] + g11 * u[1] * u[1] + gnn * u[2] * u[2];
                        double z[2] = {0.0, 0.0};
                        ls_eval34(Lc, 0.0, z);
                        curv[1] += z[0];
                        curv[2] += z[1];
                    }
                }
            }
            if (G > 1u && wv < kQnSums) {
                const double a = wave_sum(ga);
                if (lane == 0) tot[wv] = a;
            }
            block_allsum<3>(curv, rbuf, rpar);  // its workgroup barrier also publishes tot
            if (G > 1u) {
#pragma unroll
                for (int q = 0; q < kQnSums; ++q) sums[q] = tot[q];
            }
            const double p2 = fmax(pnorm_env - sums[3] + sums[2], 0.0);
            res = sqrt(sums[0]);
            thr = A.eps_a + A.eps_r * fmax(sqrt(p2), sqrt(sums[1]));
            const double Aq = sums[4], Bq = sums[5], d0 = sums[6];
            if (res < thr) { converged = 1; break; }
            if (k >= A.max_iter || !(d0 < 0.0)) break;
            if (timer) { const unsigned long long t = wall_clock64(); tph[3] += t - tmark; tmark = t; }
            // ---- exact line search, redundantly in every block of the group -------
            // Contact ec0 + i is taken by thread i mod T. The closed-form
            // coefficients of the first kLsPer*T contacts stay in registers for
            // all the evaluations, the next T in LDS, and any beyond are formed
            // from memory at each evaluation.
            auto coef_of = [&](long long c) -> LsCoef { return load_coef(A.c_coef, c); };
            if constexpr (!scatter) {
                if (G > 1u && tid == 0) {
#pragma unroll
                    for (int j = 0; j < 3; ++j) st_x(&partial2[j * kQnMaxBlocks + rank], curv[j]);
                }
                ok = loop_sync(ctr, rank, G, &ltarget, &s_ok, cnt);
                if (timer) { const unsigned long long t = wall_clock64(); tph[4] += t - tmark; tmark = t; }
                if (!ok) break;
                // the coefficients the contact pass stored (coalesced loads): all
                // the environment's, or with the distributed line search the block's own
                const long long cl0 = dist ? c0 : ec0, cl1 = dist ? c1 : ec1;
#pragma unroll
                for (int u = 0; u < kLsPer; ++u) {
                    const long long c = cl0 + tid + (long long)u * T;
                    lc[u] = c < cl1 ? coef_of(c) : ls_coef_zero();
                }
                if (use_lds && !dist) ls_ovf[tid] = c_lds < ec1 ? coef_of(c_lds) : ls_coef_zero();
            }
            // phi''(0) - A, phi''' and phi'''' at 0 summed over the group (waves 0
            // to 2, in block order; the one-barrier form summed every contact in
            // the block already), then the first trial step: the third-order
            // step of phi' from alpha = 0
            double curv0 = curv[0], curv1 = curv[1], curv2 = curv[2];
            if (G > 1u && !scatter) {
                const int wv = tid >> 6, lane = tid & 63;
                if (wv < 3) {
                    double a = 0.0;
                    for (unsigned b = lane; b < G; b += 64) a += ld_x(&partial2[wv * kQnMaxBlocks + b]);
                    a = wave_sum(a);
                    if (lane == 0) tot[wv] = a;
                }
                __syncthreads();
                curv0 = tot[0];
                curv1 = tot[1];
                curv2 = tot[2];
            }
            const double alpha0 = Aq + curv0 > 0.0 ? ls_first_step(d0, Aq + curv0, curv1, curv2) : alpha_prev;
            if (timer) { const unsigned long long t = wall_clock64(); tph[5] += t - tmark; tmark = t; }
            auto eval = [&](double alpha, double* d2out) -> double {
                double acc2[2] = {0.0, 0.0};
#pragma unroll
                for (int u = 0; u < kLsPer; ++u) ls_eval2(lc[u], lsu, alpha, acc2);
                if (dist) {
                    for (long long c = c0 + tid + (long long)kLsPer * T; c < c1; c += T)
                        ls_eval2(coef_of(c), lsu, alpha, acc2);
                } else if (use_lds) {
                    // (the one-barrier form holds at most (kLsPer + 1) T contacts)
                    ls_eval2(ls_ovf[tid], lsu, alpha, acc2);
                    for (long long c = c_lds + T; c < ec1; c += T) ls_eval2(coef_of(c), lsu, alpha, acc2);
                }
                block_allsum<2>(acc2, rbuf, rpar);
                if (dist) {
                    // the group's sums, in block order in every block (two buffers by
                    // evaluation parity, as for the iteration's block sums)
                    double* pb = A.ls_part + (size_t)(ls_par & 1u) * 2 * kQnMaxBlocks;
                    ls_par ^= 1u;
                    if (tid == 0) {
                        st_x(&pb[2 * (first + rank)], acc2[0]);
                        st_x(&pb[2 * (first + rank) + 1], acc2[1]);
                    }
                    if (!loop_sync(ctr, rank, G, &ltarget, &s_ok, cnt)) {
                        ok = false;
                        return 0.0;  // stops the search; the solve then ends with the flag set
                    }
                    const int wv = tid >> 6, lane = tid & 63;
                    if (wv < 2) {
                        double a = 0.0;
                        for (unsigned b = lane; b < G; b += 64) a += ld_x(&pb[2 * (first + b) + wv]);
                        a = wave_sum(a);
                        if (lane == 0) tot[wv] = a;
                    }
                    __syncthreads();
                    acc2[0] = tot[0];
                    acc2[1] = tot[1];
                    __syncthreads();
                }
                *d2out = Aq + acc2[1];
                return fma(Aq, alpha, Bq) + acc2[0];
            };
            const double alpha = exact_line_search(eval, alpha0, d0, A.ls_max_steps, &ls_total);
            if (!ok) break;
            if (timer) { const unsigned long long t = wall_clock64(); tph[6] += t - tmark; tmark = t; }
            if (cmp) {
                // by the node's first lane, which formed its dv and reads its
                // iterate at the start of the next node pass (no barrier between)
                const int ls = tid >> lg_nl;
                if ((tid & (nl - 1)) == 0 && ls < s1 - s0) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) node_v[a][ls] = fma(alpha, nacc[a][ls], node_v[a][ls]);
                }
                if (scatter) {
                    for (int t = tid; t < n_u; t += T)
#pragma unroll
                        for (int a = 0; a < 3; ++a)
                            vcl[a * kUniqMax + t] = fma(alpha, nacc[6 + a][t], vcl[a * kUniqMax + t]);
                    // the register contacts' v_c^{k+1} (zero states stay zero)
#pragma unroll
                    for (int u = 0; u < kLsPer; ++u)
#pragma unroll
                        for (int a = 0; a < 3; ++a) st[u].vc[a] = fma(alpha, st[u].u[a], st[u].vc[a]);
                }
            } else {
                for (long long s = s0 + tid; s < s1; s += T) {
                    SlotRec& S = A.s_rec[s];
#pragma unroll
                    for (int a = 0; a < 3; ++a) S.v[a] = fma(alpha, ld_x(&S.dv[a]), S.v[a]);
                }
            }
            if (timer) { const unsigned long long t = wall_clock64(); tph[7] += t - tmark; tmark = t; }
            alpha_prev = alpha;
            ++k;
            buf = buf == 2 ? 0 : buf + 1;
        }
        // ---- outputs ----------------------------------------------------------------
        if (cmp && tid < s1 - s0) {
#pragma unroll
            for (int a = 0; a < 3; ++a) A.s_rec[s0 + tid].v[a] = node_v[a][tid];
        }
        for (long long s = s0 + tid; s < s1; s += T) {
            const SlotRec& S = A.s_rec[s];
            float4 g = A.vel[A.s_node[s]];
            g.x = (float)S.v[0]; g.y = (float)S.v[1]; g.z = (float)S.v[2];
            A.vel[A.s_node[s]] = g;
        }
        for (int q = tid; q < A.n_rigid * 6; q += T) racc[q] = 0.0;
        __syncthreads();
        if (scatter) {
            // v_c at the final iterate: in the registers of the thread's
            // line-search contacts (the last, in the scratch, where the set-up
            // of the last iteration stored it); each block takes its own
#pragma unroll
            for (int u = 0; u < kLsPer; ++u) {
                const long long c = ec0 + tid + (long long)u * T;
                if (c >= c0 && c < c1) contact_impulse_at(A, c, st[u].vc, racc);
            }
            {
                const long long c = ec0 + tid + (long long)kLsPer * T;
                if (c >= c0 && c < c1) {
                    const double* vb = vblk + kLsPer * 6 * kQnThreads + tid;
                    const double vc[3] = {vb[0], vb[kQnThreads], vb[2 * kQnThreads]};
                    contact_impulse_at(A, c, vc, racc);
                }
            }
        } else {
            for (long long c = c0 + tid; c < c1; c += T) contact_impulse(A, c, k, alpha_prev, racc);
        }
        __syncthreads();
        for (int q = tid; q < A.n_rigid * 6; q += T)
            if (racc[q] != 0.0) atomicAdd(&A.rigid_acc[q], racc[q]);
        if (writer) write_stats(A, env, nc, ns, k, converged, ls_total, res, thr, tph, false, (int)G);
        if (kOne && writer) A.env_pend[env] = 0;
        __syncthreads();  // racc and the block sums are reused by the next environment
        if (!ok) break;
    }
}

// ---------------------------------------------------------------------------
// Exact-Newton variant of the contact solve (MPM_SOLVER_NEWTON), a study of the
// block-diagonal choice of Sec. IV-C: the same objective, stopping test and
// exact line search as Algorithm 1, with the search direction taken from the
// full Hessian H^ = M + sum_c J_c^T R_c G_c R_c^T J_c (nodes coupled through
// every contact's stencil) instead of its 3x3 node blocks. H^ d = -g is solved
// by conjugate gradients preconditioned with those node blocks (the matrix
// Algorithm 1 inverts), inexactly: until the residual's preconditioned norm
// falls to eta times its start, eta = min(1/2, sqrt(|grad~| / |grad~| at the
// first iteration)) (a forcing term that tightens as the gradient falls).
// Each group of blocks splits the environment's contact nodes and contacts as
// in k_qn; values other blocks read go through ld_x / st_x and a loop barrier
// separates their writes from the reads (three per conjugate-gradient
// iteration: after the contact pass, after p.H^p, after r.z).
// Per contact node (kNtSlot doubles): the inverse of its block [0, 6) (upper
// triangle 00 01 02 11 12 22), the gradient g [6, 9), the conjugate-gradient
// solution x [9, 12) (the Newton direction), residual r [12, 15), z = P r
// [15, 18), direction p in two buffers by iteration parity [18, 21) and
// [21, 24), q = H^ p [24, 27).
// Per contact (kNtCon doubles): R gamma [0, 3) and R G R^T [3, 9) (world), G in
// the contact frame [9, 13) (g00 g01 g11 gnn), and [13, 16): R G u for the
// products, then u = R^T J x for the line search.
// ---------------------------------------------------------------------------
constexpr int kNtPi = 0, kNtG = 6, kNtX = 9, kNtR = 12, kNtZ = 15, kNtP = 18, kNtQ = 24;
constexpr int kNtRg = 0, kNtRgr = 3, kNtGc = 9, kNtW = 13;
constexpr int kNtCgMax = 5000;  // conjugate-gradient iterations per Newton step

__global__ void __launch_bounds__(kQnThreads)
k_newton(QnArgs A) {
    __shared__ double rbuf[2 * 16 * kQnSums];
    __shared__ double tot[kQnSums];
    __shared__ double racc[kMaxRigid * 6];
    __shared__ unsigned s_ok;
    __shared__ double ovf_raw[11 * kQnThreads];
    LsCoef* ls_ovf = reinterpret_cast<LsCoef*>(ovf_raw);
    DevCounters* cnt = A.cnt;
    const bool aborted = cnt->abort_step != 0u;
    const int tid = threadIdx.x, T = blockDim.x;
    const int2 me = A.qn_map[blockIdx.x];
    unsigned rpar = 0;
    for (int env = me.x; env < A.n_envs; env += A.env_stride > 0 ? A.env_stride : A.n_envs) {
        const int first = A.env_stride > 0 ? (int)blockIdx.x : A.env_qn[2 * env];
        const unsigned G_launch = A.env_stride > 0 ? 1u : (unsigned)A.env_qn[2 * env + 1];
        const int rank = A.env_stride > 0 ? 0 : me.y;
        const bool writer = rank == 0 && tid == 0;
        const unsigned long long tph[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (aborted) {
            if (writer) write_stats(A, env, 0, 0, 0, 1, 0, 0.0, 0.0, tph, true, 0);
            continue;
        }
        unsigned* bar = A.env_bar + (size_t)env * kBarStride;
        unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // read before the first group barrier, which no block passes before all
        // have read it (the loop barriers' counters only grow)
        unsigned* ctr = A.env_ctr + (size_t)env * kCtrLanes * kCtrStride;
        unsigned ltarget = ctr_sum(ctr);
        const long long ec0 = A.env_range[4 * env], ec1 = A.env_range[4 * env + 1];
        const long long es0 = A.env_range[4 * env + 2], es1 = A.env_range[4 * env + 3];
        const long long nc = ec1 - ec0, ns = es1 - es0;
        const unsigned G = (unsigned)std::min<long long>(
            G_launch, std::max<long long>(1, (ns + A.slots_per_block - 1) / A.slots_per_block));
        if ((unsigned)rank >= G) continue;
        long long s0 = es0, s1 = es1;
        if (G > 1u) {
            const long long e_lo = A.s_beg[es0], e_n = (long long)A.s_beg[es1] - e_lo;
            s0 = rank == 0 ? es0 : es0 + lower_bound_i(A.s_beg + es0, ns, e_lo + (e_n * rank + G - 1) / G);
            s1 = rank + 1 == (int)G ? es1 : es0 + lower_bound_i(A.s_beg + es0, ns, e_lo + (e_n * (rank + 1) + G - 1) / G);
        }
        const long long cper = (nc + G - 1) / G;
        const long long c0 = ec0 + std::min<long long>(nc, cper * rank), c1 = std::min<long long>(ec1, c0 + cper);
        const double pnorm_env = A.env_pnorm[env];
        double* const pbuf[2] = {A.partial + (size_t)first * kQnSums, A.partial_odd + (size_t)first * kQnSums};
        int ph = 0;
        // Block sums of v[0, nv), then (groups of several blocks) the group's
        // sums in every block, the same bits everywhere; the loop barrier in
        // between also orders every st_x before it against every ld_x after it.
        auto group_sum = [&](double (&v)[kQnSums], int nv) -> bool {
            block_allsum<kQnSums>(v, rbuf, rpar);
            double* pb = pbuf[ph];
            ph ^= 1;
            if (G > 1u && tid == 0)
                for (int q = 0; q < nv; ++q) st_x(&pb[(size_t)rank * kQnSums + q], v[q]);
            if (!loop_sync(ctr, rank, G, &ltarget, &s_ok, cnt)) return false;
            if (G > 1u) {
                const int wv = tid >> 6, lane = tid & 63;
                if (wv < nv) {
                    double a = 0.0;
                    for (unsigned b = lane; b < G; b += 64) a += ld_x(&pb[(size_t)b * kQnSums + wv]);
                    a = wave_sum(a);
                    if (lane == 0) tot[wv] = a;
                }
                __syncthreads();
                for (int q = 0; q < nv; ++q) v[q] = tot[q];
                __syncthreads();
            }
            return true;
        };
        double* const ns_base = A.nt_slot;
        double* const nc_base = A.nt_con;
        auto S = [&](long long s, int off) -> double* { return ns_base + (size_t)s * kNtSlot + off; };
        auto Cw = [&](long long c, int off) -> double* { return nc_base + (size_t)c * kNtCon + off; };

        for (long long c = c0 + tid; c < c1; c += T) initial_contact_velocity(A, c);

        int k = 0, cg_total = 0, ls_total = 0, converged = 0;
        double res = 0.0, thr = 0.0, res0 = -1.0;
        __builtin_amdgcn_s_waitcnt(0);
        bool ok = group_sync(bar, G, &gen, &s_ok, cnt);
        while (ok) {
            // (1) contact terms at v_c for the block's contacts
            for (long long c = c0 + tid; c < c1; c += T) {
                const ContactRec& R = A.c_rec[c];
                const double* vc = A.c_dyn[c].vc[0];
                double g[3], g00, g01, g11, gnn;
                contact_model(params_of(R, A.h), vc, g, &g00, &g01, &g11, &gnn);
                double rg[3], rgr[6];
#pragma unroll
                for (int a = 0; a < 3; ++a) rg[a] = R.t1[a] * g[0] + R.t2[a] * g[1] + R.n[a] * g[2];
                int q = 0;
#pragma unroll
                for (int r = 0; r < 3; ++r)
#pragma unroll
                    for (int cc = r; cc < 3; ++cc)
                        rgr[q++] = g00 * R.t1[r] * R.t1[cc] + g01 * (R.t1[r] * R.t2[cc] + R.t2[r] * R.t1[cc]) +
                                   g11 * R.t2[r] * R.t2[cc] + gnn * R.n[r] * R.n[cc];
#pragma unroll
                for (int a = 0; a < 3; ++a) st_x(Cw(c, kNtRg + a), rg[a]);
#pragma unroll
                for (int a = 0; a < 6; ++a) st_x(Cw(c, kNtRgr + a), rgr[a]);
                double* gc = Cw(c, kNtGc);
                gc[0] = g00; gc[1] = g01; gc[2] = g11; gc[3] = gnn;
            }
            double sums[kQnSums];
#pragma unroll
            for (int q = 0; q < kQnSums; ++q) sums[q] = 0.0;
            if (!(ok = group_sum(sums, 0))) break;
            // (2) node pass: gradient, node blocks and their inverses, the
            // conjugate-gradient start x = 0, r = -g, z = P r
            for (long long s = s0 + tid; s < s1; s += T) {
                const SlotRec& Sr = A.s_rec[s];
                const double m = Sr.m;
                double j[3] = {0.0, 0.0, 0.0}, Hc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                for (int e = A.s_beg[s]; e < A.s_beg[s + 1]; ++e) {
                    const Entry en = A.e_ent[e];
                    const double w = en.w;
#pragma unroll
                    for (int a = 0; a < 3; ++a) j[a] = fma(w, ld_x(Cw(en.c, kNtRg + a)), j[a]);
#pragma unroll
                    for (int a = 0; a < 6; ++a) Hc[a] = fma(w * w, ld_x(Cw(en.c, kNtRgr + a)), Hc[a]);
                }
                const double H[6] = {m + Hc[0], Hc[1], Hc[2], m + Hc[3], Hc[4], m + Hc[5]};
                const double c00 = H[3] * H[5] - H[4] * H[4], c01 = H[2] * H[4] - H[1] * H[5];
                const double c02 = H[1] * H[4] - H[2] * H[3], c11 = H[0] * H[5] - H[2] * H[2];
                const double c12 = H[1] * H[2] - H[0] * H[4], c22 = H[0] * H[3] - H[1] * H[1];
                const double id = 1.0 / (H[0] * c00 + H[1] * c01 + H[2] * c02);
                const double Pi[6] = {c00 * id, c01 * id, c02 * id, c11 * id, c12 * id, c22 * id};
                double g[3], r[3], z[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    g[a] = m * (Sr.v[a] - Sr.vstar[a]) - j[a];
                    r[a] = -g[a];
                }
                z[0] = Pi[0] * r[0] + Pi[1] * r[1] + Pi[2] * r[2];
                z[1] = Pi[1] * r[0] + Pi[3] * r[1] + Pi[4] * r[2];
                z[2] = Pi[2] * r[0] + Pi[4] * r[1] + Pi[5] * r[2];
#pragma unroll
                for (int a = 0; a < 6; ++a) S(s, kNtPi)[a] = Pi[a];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    S(s, kNtG)[a] = g[a];
                    S(s, kNtR)[a] = r[a];
                    st_x(S(s, kNtX + a), 0.0);
                    st_x(S(s, kNtZ + a), z[a]);
                    st_x(S(s, kNtP + a), 0.0);  // p of "iteration -1": the first direction is z
                    sums[0] += g[a] * g[a] / m;
                    sums[1] += j[a] * j[a] / m;
                    sums[2] += m * Sr.v[a] * Sr.v[a];
                    sums[3] += m * Sr.vstar[a] * Sr.vstar[a];
                    sums[4] += r[a] * z[a];
                }
            }
            if (!(ok = group_sum(sums, 5))) break;
            const double p2 = fmax(pnorm_env - sums[3] + sums[2], 0.0);
            res = sqrt(sums[0]);
            thr = A.eps_a + A.eps_r * fmax(sqrt(p2), sqrt(sums[1]));
            if (res < thr) { converged = 1; break; }
            if (k >= A.max_iter) break;
            if (res0 < 0.0) res0 = res;
            const double eta = fmin(0.5, sqrt(res / res0));
            const double rz0 = sums[4];
            double rz = rz0, beta = 0.0;
            // (3) preconditioned conjugate gradients on H^ x = -g
            int pb = 0;  // buffer of the previous direction
            for (int it = 0; it < kNtCgMax && rz > 0.0; ++it) {
                // contacts: R G u with u = R^T J p, p = z + beta p_prev
                for (long long c = c0 + tid; c < c1; c += T) {
                    const ContactRec& R = A.c_rec[c];
                    const ContactStencil& st = A.c_st[c];
                    double acc[3] = {0.0, 0.0, 0.0};
                    for (int o = 0; o < 27; ++o) {
                        const int sl = st.slot[o];
                        if (sl < 0) continue;
                        const double w = st.w[o];
#pragma unroll
                        for (int a = 0; a < 3; ++a)
                            acc[a] = fma(w, fma(beta, ld_x(S(sl, kNtP + 3 * pb + a)), ld_x(S(sl, kNtZ + a))), acc[a]);
                    }
                    double u[3];
                    frame_project(R, acc, u);
                    const double* gc = Cw(c, kNtGc);
                    const double y[3] = {gc[0] * u[0] + gc[1] * u[1], gc[1] * u[0] + gc[2] * u[1], gc[3] * u[2]};
#pragma unroll
                    for (int a = 0; a < 3; ++a) st_x(Cw(c, kNtW + a), R.t1[a] * y[0] + R.t2[a] * y[1] + R.n[a] * y[2]);
                }
                // the block's nodes: p = z + beta p_prev into the other buffer
                for (long long s = s0 + tid; s < s1; s += T)
#pragma unroll
                    for (int a = 0; a < 3; ++a)
                        st_x(S(s, kNtP + 3 * (pb ^ 1) + a), fma(beta, ld_x(S(s, kNtP + 3 * pb + a)), ld_x(S(s, kNtZ + a))));
#pragma unroll
                for (int q = 0; q < kQnSums; ++q) sums[q] = 0.0;
                if (!(ok = group_sum(sums, 0))) break;
                pb ^= 1;
                // q = H^ p on the block's nodes, and p.q
                for (long long s = s0 + tid; s < s1; s += T) {
                    const double m = A.s_rec[s].m;
                    double pv[3], qv[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        pv[a] = ld_x(S(s, kNtP + 3 * pb + a));
                        qv[a] = m * pv[a];
                    }
                    for (int e = A.s_beg[s]; e < A.s_beg[s + 1]; ++e) {
                        const Entry en = A.e_ent[e];
#pragma unroll
                        for (int a = 0; a < 3; ++a) qv[a] = fma((double)en.w, ld_x(Cw(en.c, kNtW + a)), qv[a]);
                    }
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        S(s, kNtQ)[a] = qv[a];
                        sums[0] += pv[a] * qv[a];
                    }
                }
                if (!(ok = group_sum(sums, 1))) break;
                const double alpha_cg = sums[0] > 0.0 ? rz / sums[0] : 0.0;
                sums[0] = 0.0;
                // x += alpha p, r -= alpha q, z = P r, and r.z
                for (long long s = s0 + tid; s < s1; s += T) {
                    const double* Pi = S(s, kNtPi);
                    double r[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        st_x(S(s, kNtX + a), fma(alpha_cg, ld_x(S(s, kNtP + 3 * pb + a)), ld_x(S(s, kNtX + a))));
                        r[a] = fma(-alpha_cg, S(s, kNtQ)[a], S(s, kNtR)[a]);
                        S(s, kNtR)[a] = r[a];
                    }
                    const double z[3] = {Pi[0] * r[0] + Pi[1] * r[1] + Pi[2] * r[2],
                                         Pi[1] * r[0] + Pi[3] * r[1] + Pi[4] * r[2],
                                         Pi[2] * r[0] + Pi[4] * r[1] + Pi[5] * r[2]};
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        st_x(S(s, kNtZ + a), z[a]);
                        sums[0] += r[a] * z[a];
                    }
                }
                if (!(ok = group_sum(sums, 1))) break;
                ++cg_total;
                beta = rz > 0.0 ? sums[0] / rz : 0.0;
                rz = sums[0];
                if (rz <= eta * eta * rz0) break;
            }
            if (!ok) break;
            // (4) exact line search along x: u_c = R^T J x, the coefficients, and
            // phi''(0); node sums A = |x|_M^2, B = x.M (v - v*), d0 = g.x
#pragma unroll
            for (int q = 0; q < kQnSums; ++q) sums[q] = 0.0;
            for (long long c = c0 + tid; c < c1; c += T) {
                const ContactRec& R = A.c_rec[c];
                const ContactStencil& st = A.c_st[c];
                double acc[3] = {0.0, 0.0, 0.0};
                for (int o = 0; o < 27; ++o) {
                    const int sl = st.slot[o];
                    if (sl < 0) continue;
                    const double w = st.w[o];
#pragma unroll
                    for (int a = 0; a < 3; ++a) acc[a] = fma(w, ld_x(S(sl, kNtX + a)), acc[a]);
                }
                double u[3];
                frame_project(R, acc, u);
#pragma unroll
                for (int a = 0; a < 3; ++a) Cw(c, kNtW)[a] = u[a];
                const double* vc = A.c_dyn[c].vc[0];
                store_coef(A.c_coef, c, ls_coef(params_of(R, A.h), vc, u));
                const double* gc = Cw(c, kNtGc);
                sums[3] += gc[0] * u[0] * u[0] + 2.0 * gc[1] * u[0] * u[1] + gc[2] * u[1] * u[1] + gc[3] * u[2] * u[2];
            }
            for (long long s = s0 + tid; s < s1; s += T) {
                const SlotRec& Sr = A.s_rec[s];
                const double* g = S(s, kNtG);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double xa = ld_x(S(s, kNtX + a));
                    sums[0] += Sr.m * xa * xa;
                    sums[1] += Sr.m * xa * (Sr.v[a] - Sr.vstar[a]);
                    sums[2] += g[a] * xa;
                }
            }
            if (!(ok = group_sum(sums, 4))) break;
            const double Aq = sums[0], Bq = sums[1], d0 = sums[2], curv0 = sums[3];
            if (!(d0 < 0.0)) break;
            const double alpha0 = Aq + curv0 > 0.0 ? -d0 / (Aq + curv0) : 1.0;
            // every block: the coefficients of all the environment's contacts
            LsCoef lc[kLsPer];
            const long long c_lds = ec0 + tid + (long long)kLsPer * T;
            const bool use_lds = (long long)kLsPer * T < nc;
#pragma unroll
            for (int u = 0; u < kLsPer; ++u) {
                const long long c = ec0 + tid + (long long)u * T;
                lc[u] = c < ec1 ? load_coef(A.c_coef, c) : ls_coef_zero();
            }
            if (use_lds) ls_ovf[tid] = c_lds < ec1 ? load_coef(A.c_coef, c_lds) : ls_coef_zero();
            auto eval = [&](double alpha, double* d2out) -> double {
                double acc2[2] = {0.0, 0.0};
#pragma unroll
                for (int u = 0; u < kLsPer; ++u) {
                    double d1, d2;
                    ls_eval(lc[u], alpha, &d1, &d2);
                    acc2[0] += d1;
                    acc2[1] += d2;
                }
                if (use_lds) {
                    double d1, d2;
                    ls_eval(ls_ovf[tid], alpha, &d1, &d2);
                    acc2[0] += d1;
                    acc2[1] += d2;
                    for (long long c = c_lds + T; c < ec1; c += T) {
                        ls_eval(load_coef(A.c_coef, c), alpha, &d1, &d2);
                        acc2[0] += d1;
                        acc2[1] += d2;
                    }
                }
                block_allsum<2>(acc2, rbuf, rpar);
                *d2out = Aq + acc2[1];
                return fma(Aq, alpha, Bq) + acc2[0];
            };
            const double alpha = exact_line_search(eval, alpha0, d0, A.ls_max_steps, &ls_total);
            // (5) update the block's nodes and contacts
            for (long long s = s0 + tid; s < s1; s += T) {
                SlotRec& Sr = A.s_rec[s];
#pragma unroll
                for (int a = 0; a < 3; ++a) Sr.v[a] = fma(alpha, ld_x(S(s, kNtX + a)), Sr.v[a]);
            }
            for (long long c = c0 + tid; c < c1; c += T) {
                double* vc = A.c_dyn[c].vc[0];
#pragma unroll
                for (int a = 0; a < 3; ++a) vc[a] = fma(alpha, Cw(c, kNtW)[a], vc[a]);
            }
            ++k;
        }
        // ---- outputs ----------------------------------------------------------------
        for (long long s = s0 + tid; s < s1; s += T) {
            const SlotRec& Sr = A.s_rec[s];
            float4 g = A.vel[A.s_node[s]];
            g.x = (float)Sr.v[0]; g.y = (float)Sr.v[1]; g.z = (float)Sr.v[2];
            A.vel[A.s_node[s]] = g;
        }
        for (int q = tid; q < A.n_rigid * 6; q += T) racc[q] = 0.0;
        __syncthreads();
        for (long long c = c0 + tid; c < c1; c += T) contact_impulse_at(A, c, A.c_dyn[c].vc[0], racc);
        __syncthreads();
        for (int q = tid; q < A.n_rigid * 6; q += T)
            if (racc[q] != 0.0) atomicAdd(&A.rigid_acc[q], racc[q]);
        if (writer) {
            write_stats(A, env, nc, ns, k, converged, ls_total, res, thr, tph, false, (int)G);
            A.stats[(size_t)A.substep * A.n_envs + env].inner_iterations = cg_total;
        }
        __syncthreads();  // racc and the block sums are reused by the next environment
        if (!ok) break;
    }
}

hipError_t launch_qn(const Work& w, const float* x, int substep, double h, double eps_r,
                     double eps_a, int max_iter, int ls_max_steps, int blocks, int env_stride,
                     int timers, int slots_per_block, hipStream_t s) {
    QnArgs A;
    A.rigids = w.rigids;
    A.x = x;
    A.P = w.P;
    A.vel = w.vel;
    A.cap = w.cap_c;
    A.c_pid = w.c_pid; A.c_rid = w.c_rid;
    A.c_rec = w.c_rec; A.c_st = w.c_st; A.c_dyn = w.c_dyn; A.c_coef = w.c_coef;
    A.compact = w.qn_compact;
    A.u_acc = w.qn_uacc;
    A.vc_blk = w.qn_vcblk;
    A.ls_prm = w.qn_lsprm;
    A.timers = timers;
    A.slots_per_block = std::max(1, slots_per_block);
    A.s_node = w.s_node; A.s_beg = w.s_beg;
    A.e_ent = w.e_ent;
    A.s_rec = w.s_rec;
    A.partial = w.partial;
    A.partial_odd = w.partial_odd;
    A.partial2 = w.partial2;
    A.rigid_acc = w.rigid_acc;
    A.n_rigid = w.n_rigid;
    A.stats = w.sstats;
    A.substep = substep;
    A.h = h; A.eps_r = eps_r; A.eps_a = eps_a;
    A.max_iter = max_iter; A.ls_max_steps = ls_max_steps;
    A.qn_map = w.qn_map;
    A.env_qn = w.env_qn;
    A.env_range = w.env_range;
    A.env_pnorm = w.env_pnorm;
    A.env_bar = w.env_bar;
    A.env_ctr = w.env_ctr;
    A.n_envs = w.n_envs;
    A.env_stride = env_stride;
    A.nt_slot = w.nt_slot;
    A.nt_con = w.nt_con;
    A.ls_part = w.qn_lspart;
    A.cnt = w.cnt;
    void* args[] = {&A};
    auto launch = [&](const void* fn) -> hipError_t {
        if (w.qn_plain_launch) {
            // blocks <= the co-resident count (qn_max_blocks), so all are resident
            // on an otherwise idle device; every barrier wait is bounded regardless
            return hipLaunchKernel(fn, dim3(blocks), dim3(kQnThreads), args, 0, s);
        }
        return hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(kQnThreads), args, 0, s);
    };
    if (w.solver == kSolverNewton) {
        A.env_pend = nullptr;
        return launch((const void*)k_newton);
    }
    if (w.qn_scatter && w.n_envs == 1) {
        // the one-barrier kernel, then the two-barrier kernel for what it left.
        // With several environments the second launch would start only after
        // the first kernel's slowest environment, so the batched form keeps the
        // two-barrier kernel for all of them.
        A.env_pend = w.qn_pend;
        const hipError_t e = launch((const void*)k_qn<true>);
        if (e != hipSuccess) return e;
    } else {
        A.env_pend = nullptr;
    }
    return launch((const void*)k_qn<false>);
}

// Blocks of k_qn that can be resident at once (the cooperative launch limit).
int qn_max_blocks() {
    int per_cu = 0;
    int per_cu1 = 0;
    int per_cu2 = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_qn<false>, kQnThreads, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu1, (const void*)k_qn<true>, kQnThreads, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu2, (const void*)k_newton, kQnThreads, 0) != hipSuccess)
        return 0;
    per_cu = std::min(per_cu, std::min(per_cu1, per_cu2));
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return per_cu * cus;
}


}  // namespace mpm
