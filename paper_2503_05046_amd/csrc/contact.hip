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
// with the iterate, gradient, block Hessian, search direction, contact
// velocities and every reduction in double precision. Per iteration:
//   node pass   each slot gathers its contacts' impulses and Hessians (each
//               contact's model is re-evaluated by its 27 nodes instead of
//               being scattered, which saves a barrier and all atomics),
//               forms g = m (v - v*) - j and H, solves the 3x3 block by
//               Cholesky, and adds its share of the norms;
//   barrier     every block reduces the per-block partials in the same order,
//               so all blocks take the same stopping decision;
//   contact pass u_c = R_c^T sum w dv, plus the line-search derivatives at a
//               batch of step lengths;
//   barrier(s)  the exact line search of Algorithm 1 is solved by rounds that
//               evaluate phi'(alpha), phi''(alpha) at kLsPoints step lengths
//               per global reduction (bracketing, then safeguarded Newton
//               clusters), instead of one sequential 1-D Newton step per
//               reduction.
// Contact velocities are carried as v_c + alpha u_c (the contact velocity is
// linear in the grid velocity), double-buffered by iteration parity.
#include "mpm_internal.h"
#include "sort_util.h"

#include <algorithm>

namespace mpm {

constexpr unsigned kFlagNoconv = 1u;
constexpr unsigned kFlagCapacity = 8u;
constexpr unsigned kFlagHang = 16u;
constexpr long long kBarrierTimeoutCycles = 5000000000ll;  // ~2 s: a healthy barrier takes microseconds
constexpr int kQnThreads = 256;
constexpr int kMaxRigid = 256;
constexpr int kPartStride = kQnSums + 4 * kLsPoints;  // node sums + 2 LS buffers (phi', phi'')

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

__device__ __forceinline__ void contact_model(const ContactParams& P, const double vc[3],
                                              double gam[3], double* g00, double* g01,
                                              double* g11, double* gnn) {
    double vbar = P.phi0 / P.h;
    if (P.d > 0.0 && 1.0 / P.d < vbar) vbar = 1.0 / P.d;
    const double vn = vc[2];
    if (vn < vbar) {
        gam[2] = P.h * P.k * (P.phi0 - P.h * vn) * (1.0 - P.d * vn);
        *gnn = P.h * P.k * (P.h * (1.0 - P.d * vn) + P.d * (P.phi0 - P.h * vn));
    } else {
        gam[2] = 0.0;
        *gnn = 0.0;
    }
    const double s2 = vc[0] * vc[0] + vc[1] * vc[1] + P.eps_s * P.eps_s;
    const double s = sqrt(s2);
    const double cs = P.mun0 / s;
    gam[0] = -cs * vc[0];
    gam[1] = -cs * vc[1];
    *g00 = cs * (1.0 - vc[0] * vc[0] / s2);
    *g01 = -cs * vc[0] * vc[1] / s2;
    *g11 = cs * (1.0 - vc[1] * vc[1] / s2);
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
            int* __restrict__ c_base, float* __restrict__ c_w, double* __restrict__ c_n,
            double* __restrict__ c_b, double* __restrict__ c_phi0, double* __restrict__ c_n0,
            double* __restrict__ c_mu, int substep, DevCounters* cnt) {
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
                c_b[0 * cap + c] = -(t1[0] * vr[0] + t1[1] * vr[1] + t1[2] * vr[2]);
                c_b[1 * cap + c] = -(t2[0] * vr[0] + t2[1] * vr[1] + t2[2] * vr[2]);
                c_b[2 * cap + c] = -(n[0] * vr[0] + n[1] * vr[1] + n[2] * vr[2]);
                const double phi0 = -s;
                const double vn0 = n[0] * (vp[0] - vr[0]) + n[1] * (vp[1] - vr[1]) + n[2] * (vp[2] - vr[2]);
                c_pid[c] = (int)p;
                c_rid[c] = r;
                c_env[c] = e;
                c_base[c] = (int)node0;
                c_phi0[c] = phi0;
                c_n0[c] = normal_impulse(vn0, phi0, E.k, E.d, h);
                c_mu[c] = R.mu;
#pragma unroll
                for (int a = 0; a < 3; ++a) c_n[a * cap + c] = n[a];
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
                       w.c_base, w.c_w, w.c_n, w.c_b, w.c_phi0, w.c_n0, w.c_mu, substep, w.cnt);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Contact-node table
// ---------------------------------------------------------------------------
__device__ __forceinline__ double stencil_weight(const float* c_w, long long cap, long long c, int o) {
    const int a = o % 3, b = (o / 3) % 3, cz = o / 9;
    return (double)c_w[(0 + a) * cap + c] * (double)c_w[(3 + b) * cap + c] * (double)c_w[(6 + cz) * cap + c];
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
        const double w = stencil_weight(c_w, cap, c, o);
        pk[i] = w > 0.0 ? (unsigned)stencil_node(envs[c_env[c]], c_base[c], o) : invalid_key;
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
            long long cap, int* __restrict__ s_node, int* __restrict__ s_beg,
            int* __restrict__ c_slot) {
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
                c_slot[o * cap + c] = (int)slot;
                if (i + 1 == n || keys[i + 1] == invalid_key) s_beg[cnt->n_slots] = (int)(i + 1);
            } else {
                c_slot[o * cap + c] = -1;
            }
        }
        run += tot;
    }
}

// Slot state: m and v* from the grid, iterate v = v* (Algorithm 1 starts from
// the free-motion velocity).
__global__ void __launch_bounds__(256)
k_slot_init(const int* __restrict__ s_node, const float4* __restrict__ vel, const DevCounters* cnt,
            long long cap_s, double* __restrict__ s_m, double* __restrict__ s_vstar,
            double* __restrict__ s_v) {
    const long long ns = cnt->n_slots;
    for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < ns;
         s += (long long)gridDim.x * blockDim.x) {
        const float4 g = vel[s_node[s]];
        s_m[s] = g.w;
        s_vstar[0 * cap_s + s] = g.x; s_vstar[1 * cap_s + s] = g.y; s_vstar[2 * cap_s + s] = g.z;
        s_v[0 * cap_s + s] = g.x; s_v[1 * cap_s + s] = g.y; s_v[2 * cap_s + s] = g.z;
    }
}

hipError_t launch_contact_setup(const Work& w, hipStream_t s) {
    const unsigned invalid_key = (unsigned)w.n_nodes;
    int bits = 1;
    while ((1ull << bits) <= (unsigned long long)w.n_nodes) ++bits;
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
                       (const DevCounters*)w.cnt, invalid_key, w.blk, w.cap_c, w.s_node, w.s_beg,
                       w.c_slot);
    hipLaunchKernelGGL(k_slot_init, dim3(1024), dim3(256), 0, s, w.s_node, w.vel,
                       (const DevCounters*)w.cnt, w.cap_s, w.s_m, w.s_vstar, w.s_v);
    // the sorted pair values are what the solver walks
    if (vs != w.pv_a) {
        e = hipMemcpyAsync(w.pv_a, vs, sizeof(unsigned) * 27 * w.cap_c, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Grid barrier for the cooperative solver (all blocks co-resident). The wait
// is bounded: on time-out every block sees the broken flag and leaves.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool grid_sync(DevCounters* cnt, unsigned nblocks, unsigned* gen,
                                          unsigned* s_ok) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned target = *gen + 1u;
        __threadfence();
        const unsigned arrived =
            __hip_atomic_fetch_add(&cnt->bar_count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        bool ok = true;
        if (arrived == nblocks - 1u) {
            __hip_atomic_store(&cnt->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&cnt->bar_gen, target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const long long t0 = clock64();
            while (__hip_atomic_load(&cnt->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != target) {
                __builtin_amdgcn_s_sleep(1);
                if ((__hip_atomic_load(&cnt->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kFlagHang) ||
                    clock64() - t0 > kBarrierTimeoutCycles) {
                    atomicOr(&cnt->flags, kFlagHang);
                    ok = false;
                    break;
                }
            }
        }
        __threadfence();
        if (__hip_atomic_load(&cnt->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kFlagHang) ok = false;
        *s_ok = ok ? 1u : 0u;
    }
    __syncthreads();
    *gen += 1u;
    return *s_ok != 0u;
}

// Block-wide FP64 sum of NV values per thread into out[NV] (thread 0 writes).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds, double* out) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
        if ((threadIdx.x & 63) == 0) lds[(threadIdx.x >> 6) * NV + k] = x;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int wv = 0; wv < (int)(blockDim.x >> 6); ++wv) s += lds[wv * NV + threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

struct QnArgs {
    const DevEnv* envs;
    const DevRigid* rigids;
    const float* x;         // particle positions at substep start (torque arms)
    long long P;
    float4* vel;
    long long cap, cap_s;
    const int *c_pid, *c_rid, *c_env, *c_slot;
    const float* c_w;
    const double *c_n, *c_b, *c_phi0, *c_n0, *c_mu;
    double *c_vc, *c_uc, *c_gam;
    const int *s_node, *s_beg;
    const unsigned* pv;     // sorted (contact * 27 + offset) per CSR entry
    double *s_v, *s_vstar, *s_dv, *s_m;
    double* partial;
    double* rigid_acc;
    int n_rigid;
    SubstepStats* stats;
    int substep;
    double h, eps_r, eps_a;
    int max_iter, ls_rounds;
    DevCounters* cnt;
};

__device__ __forceinline__ ContactParams params_of(const QnArgs& A, long long c) {
    const DevEnv& E = A.envs[A.c_env[c]];
    ContactParams P;
    P.phi0 = A.c_phi0[c];
    P.mun0 = A.c_mu[c] * A.c_n0[c];
    P.k = E.k;
    P.d = E.d;
    P.eps_s = E.eps_s;
    P.h = A.h;
    return P;
}

// Contact velocity at iteration k: v_c^0 from the initial gather, then
// v_c^k = v_c^{k-1} + alpha_{k-1} u_c^{k-1} (exact: v_c is linear in v).
__device__ __forceinline__ void contact_velocity(const QnArgs& A, long long c, int k, double alpha_prev,
                                                 double vc[3]) {
    const double* src = A.c_vc + (size_t)((k == 0 ? 0 : (k - 1) & 1)) * 3 * A.cap;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double v0 = src[a * A.cap + c];
        vc[a] = k == 0 ? v0 : fma(alpha_prev, A.c_uc[a * A.cap + c], v0);
    }
}

__device__ __forceinline__ void ls_terms(const ContactParams& P, const double vc[3], const double u[3],
                                         double alpha, double* d1, double* d2) {
    double v[3] = {fma(alpha, u[0], vc[0]), fma(alpha, u[1], vc[1]), fma(alpha, u[2], vc[2])};
    double g[3], g00, g01, g11, gnn;
    contact_model(P, v, g, &g00, &g01, &g11, &gnn);
    *d1 = -(g[0] * u[0] + g[1] * u[1] + g[2] * u[2]);
    *d2 = g00 * u[0] * u[0] + 2.0 * g01 * u[0] * u[1] + g11 * u[1] * u[1] + gnn * u[2] * u[2];
}

__global__ void __launch_bounds__(kQnThreads)
k_qn(QnArgs A) {
    __shared__ double lds[16 * 8];
    __shared__ double tot[kPartStride];
    __shared__ double ls_acc[kQnThreads / kLsPoints][kLsPoints][2];
    __shared__ double alphas[kLsPoints];
    __shared__ double racc[kMaxRigid * 6];
    __shared__ unsigned s_ok;
    __shared__ int s_done;
    __shared__ double s_alpha;

    DevCounters* cnt = A.cnt;
    const unsigned G = gridDim.x;
    unsigned gen = __hip_atomic_load(&cnt->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    const bool aborted = cnt->abort_step != 0u;
    const long long nc = aborted ? 0 : std::min<long long>(cnt->n_contacts, A.cap);
    const long long ns = aborted ? 0 : cnt->n_slots;
    const int tid = threadIdx.x;
    // block-contiguous ownership
    const long long sper = (ns + G - 1) / G, cper = (nc + G - 1) / G;
    const long long s0 = std::min<long long>(ns, sper * blockIdx.x), s1 = std::min<long long>(ns, s0 + sper);
    const long long c0 = std::min<long long>(nc, cper * blockIdx.x), c1 = std::min<long long>(nc, c0 + cper);
    const double pnorm_all = cnt->pnorm_all;

    // initial contact velocities v_c^0 = R_c^T sum w v*_i + b_c
    for (long long c = c0 + tid; c < c1; c += blockDim.x) {
        double sacc[3] = {0.0, 0.0, 0.0};
        for (int o = 0; o < 27; ++o) {
            const int sl = A.c_slot[o * A.cap + c];
            if (sl < 0) continue;
            const double w = stencil_weight(A.c_w, A.cap, c, o);
#pragma unroll
            for (int a = 0; a < 3; ++a) sacc[a] += w * A.s_v[a * A.cap_s + sl];
        }
        const double n[3] = {A.c_n[c], A.c_n[A.cap + c], A.c_n[2 * A.cap + c]};
        double t1[3], t2[3];
        frame_of(n, t1, t2);
        A.c_vc[0 * A.cap + c] = t1[0] * sacc[0] + t1[1] * sacc[1] + t1[2] * sacc[2] + A.c_b[c];
        A.c_vc[1 * A.cap + c] = t2[0] * sacc[0] + t2[1] * sacc[1] + t2[2] * sacc[2] + A.c_b[A.cap + c];
        A.c_vc[2 * A.cap + c] = n[0] * sacc[0] + n[1] * sacc[1] + n[2] * sacc[2] + A.c_b[2 * A.cap + c];
    }

    int k = 0;
    double alpha_prev = 1.0;   // alpha_{k-1}; also the centre of the first line-search round
    double res = 0.0, thr = 0.0;
    int converged = 0;
    bool ok = grid_sync(cnt, G, &gen, &s_ok);
    if (nc == 0) converged = 1;
    while (ok && nc > 0) {
        // ---- node pass -----------------------------------------------------
        double sums[kQnSums];
#pragma unroll
        for (int q = 0; q < kQnSums; ++q) sums[q] = 0.0;
        for (long long s = s0 + tid; s < s1; s += blockDim.x) {
            const double m = A.s_m[s];
            double v[3], vs[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                v[a] = A.s_v[a * A.cap_s + s];
                vs[a] = A.s_vstar[a * A.cap_s + s];
            }
            double j[3] = {0.0, 0.0, 0.0};
            double H[6] = {m, 0.0, 0.0, m, 0.0, m};  // 00 01 02 11 12 22
            const int e0 = A.s_beg[s], e1 = A.s_beg[s + 1];
            for (int e = e0; e < e1; ++e) {
                const unsigned pv = A.pv[e];
                const long long c = pv / 27;
                const int o = (int)(pv % 27);
                const double w = stencil_weight(A.c_w, A.cap, c, o);
                double vc[3];
                contact_velocity(A, c, k, alpha_prev, vc);
                const ContactParams P = params_of(A, c);
                double g[3], g00, g01, g11, gnn;
                contact_model(P, vc, g, &g00, &g01, &g11, &gnn);
                const double n[3] = {A.c_n[c], A.c_n[A.cap + c], A.c_n[2 * A.cap + c]};
                double t1[3], t2[3];
                frame_of(n, t1, t2);
                // R gamma and R G R^T with R = [t1 t2 n]
#pragma unroll
                for (int a = 0; a < 3; ++a) j[a] += w * (t1[a] * g[0] + t2[a] * g[1] + n[a] * g[2]);
                const double ww = w * w;
                int q = 0;
#pragma unroll
                for (int r = 0; r < 3; ++r)
#pragma unroll
                    for (int cc = r; cc < 3; ++cc) {
                        const double val = g00 * t1[r] * t1[cc] + g01 * (t1[r] * t2[cc] + t2[r] * t1[cc]) +
                                           g11 * t2[r] * t2[cc] + gnn * n[r] * n[cc];
                        H[q++] += ww * val;
                    }
            }
            double g[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) g[a] = m * (v[a] - vs[a]) - j[a];
            // dv = -H^-1 g by Cholesky
            const double l00 = sqrt(H[0]);
            const double l10 = H[1] / l00, l20 = H[2] / l00;
            const double l11 = sqrt(H[3] - l10 * l10);
            const double l21 = (H[4] - l20 * l10) / l11;
            const double l22 = sqrt(H[5] - l20 * l20 - l21 * l21);
            const double y0 = -g[0] / l00;
            const double y1 = (-g[1] - l10 * y0) / l11;
            const double y2 = (-g[2] - l20 * y0 - l21 * y1) / l22;
            double dv[3];
            dv[2] = y2 / l22;
            dv[1] = (y1 - l21 * dv[2]) / l11;
            dv[0] = (y0 - l10 * dv[1] - l20 * dv[2]) / l00;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                A.s_dv[a * A.cap_s + s] = dv[a];
                sums[0] += g[a] * g[a] / m;            // |grad~|^2
                sums[1] += j[a] * j[a] / m;            // |j~|^2
                sums[2] += m * v[a] * v[a];            // contact-node part of |p~|^2
                sums[3] += m * vs[a] * vs[a];          // same nodes at v*
                sums[4] += m * dv[a] * dv[a];          // A
                sums[5] += m * dv[a] * (v[a] - vs[a]); // B
                sums[6] += g[a] * dv[a];               // phi'(0)
            }
        }
        block_sum<kQnSums>(sums, lds, A.partial + (size_t)blockIdx.x * kPartStride);
        ok = grid_sync(cnt, G, &gen, &s_ok);
        if (!ok) break;
        if (tid < kQnSums) {
            double acc = 0.0;
            for (unsigned b = 0; b < G; ++b) acc += A.partial[(size_t)b * kPartStride + tid];
            tot[tid] = acc;
        }
        __syncthreads();
        const double grad2 = tot[0], j2 = tot[1];
        const double p2 = fmax(pnorm_all - tot[3] + tot[2], 0.0);
        res = sqrt(grad2);
        const double pn = sqrt(p2), jn = sqrt(j2);
        thr = A.eps_a + A.eps_r * fmax(pn, jn);
        const double Aq = tot[4], Bq = tot[5], d0 = tot[6];
        if (res < thr) { converged = 1; break; }
        if (k >= A.max_iter || !(d0 < 0.0)) break;

        // ---- contact pass: u_c = R_c^T sum w dv_i; store v_c^k ------------
        for (long long c = c0 + tid; c < c1; c += blockDim.x) {
            double vc[3];
            contact_velocity(A, c, k, alpha_prev, vc);
            if (k > 0) {
#pragma unroll
                for (int a = 0; a < 3; ++a) A.c_vc[(size_t)(k & 1) * 3 * A.cap + a * A.cap + c] = vc[a];
            }
            double sacc[3] = {0.0, 0.0, 0.0};
            for (int o = 0; o < 27; ++o) {
                const int sl = A.c_slot[o * A.cap + c];
                if (sl < 0) continue;
                const double w = stencil_weight(A.c_w, A.cap, c, o);
#pragma unroll
                for (int a = 0; a < 3; ++a) sacc[a] += w * A.s_dv[a * A.cap_s + sl];
            }
            const double n[3] = {A.c_n[c], A.c_n[A.cap + c], A.c_n[2 * A.cap + c]};
            double t1[3], t2[3];
            frame_of(n, t1, t2);
            A.c_uc[0 * A.cap + c] = t1[0] * sacc[0] + t1[1] * sacc[1] + t1[2] * sacc[2];
            A.c_uc[1 * A.cap + c] = t2[0] * sacc[0] + t2[1] * sacc[1] + t2[2] * sacc[2];
            A.c_uc[2 * A.cap + c] = n[0] * sacc[0] + n[1] * sacc[1] + n[2] * sacc[2];
        }
        __syncthreads();  // this block's u_c are read by its own threads below

        // ---- exact line search by rounds of kLsPoints evaluations ----------
        // bracket [lo, hi] with phi'(lo) < 0 <= phi'(hi); lo starts at 0.
        double lo = 0.0, dlo = d0, hi = 0.0, dhi = 0.0, ddhi = 0.0, ddlo = -1.0;
        bool have_hi = false;
        double alpha = alpha_prev;
        double centre = alpha_prev;
        double best = 0.0, dbest = d0, newton_step = 0.0;
        for (int round = 0; round < A.ls_rounds; ++round) {
            if (tid == 0) {
                for (int jj = 0; jj < kLsPoints; ++jj) {
                    double a;
                    if (!have_hi) {
                        // geometric sweep around the centre (first round: the last step length)
                        a = centre * exp2((double)(jj - kLsPoints / 2) / 4.0);
                    } else {
                        // a cluster of half-width r/2 at the safeguarded Newton
                        // estimate, r = length of the Newton correction
                        const double wdt = hi - lo;
                        double r = fabs(newton_step);
                        if (!(r > 0.0) || r > wdt) r = wdt;
                        a = centre + 0.5 * r * ((double)jj - 0.5 * (kLsPoints - 1)) / (0.5 * (kLsPoints - 1));
                        const double eps = 1e-3 * wdt / kLsPoints;
                        a = fmin(fmax(a, lo + eps), hi - eps);
                    }
                    alphas[jj] = a;
                }
            }
            __syncthreads();
            // partial phi', phi'' of this block's contacts at every point
            {
                const int jj = tid % kLsPoints, lane_c = tid / kLsPoints;
                const double a = alphas[jj];
                double d1s = 0.0, d2s = 0.0;
                for (long long c = c0 + lane_c; c < c1; c += kQnThreads / kLsPoints) {
                    double vc[3];
                    const double* src = A.c_vc + (size_t)(k == 0 ? 0 : (k & 1)) * 3 * A.cap;
#pragma unroll
                    for (int q = 0; q < 3; ++q) vc[q] = src[q * A.cap + c];
                    const double u[3] = {A.c_uc[c], A.c_uc[A.cap + c], A.c_uc[2 * A.cap + c]};
                    double d1, d2;
                    ls_terms(params_of(A, c), vc, u, a, &d1, &d2);
                    d1s += d1;
                    d2s += d2;
                }
                ls_acc[lane_c][jj][0] = d1s;
                ls_acc[lane_c][jj][1] = d2s;
            }
            __syncthreads();
            double* part = A.partial + (size_t)blockIdx.x * kPartStride + kQnSums + (round & 1) * 2 * kLsPoints;
            if (tid < 2 * kLsPoints) {
                const int jj = tid >> 1, q = tid & 1;
                double s = 0.0;
                for (int l = 0; l < kQnThreads / kLsPoints; ++l) s += ls_acc[l][jj][q];
                part[tid] = s;
            }
            ok = grid_sync(cnt, G, &gen, &s_ok);
            if (!ok) break;
            if (tid < 2 * kLsPoints) {
                double s = 0.0;
                for (unsigned b = 0; b < G; ++b)
                    s += A.partial[(size_t)b * kPartStride + kQnSums + (round & 1) * 2 * kLsPoints + tid];
                tot[kQnSums + tid] = s;
            }
            __syncthreads();
            if (tid == 0) {
                int done = 0;
                for (int jj = 0; jj < kLsPoints; ++jj) {
                    const double a = alphas[jj];
                    const double d1 = Aq * a + Bq + tot[kQnSums + 2 * jj];
                    const double d2 = Aq + tot[kQnSums + 2 * jj + 1];
                    if (fabs(d1) < fabs(dbest)) { best = a; dbest = d1; }
                    if (d1 < 0.0) {
                        if (a > lo) { lo = a; dlo = d1; ddlo = d2; }
                    } else if (!have_hi || a < hi) {
                        hi = a; dhi = d1; ddhi = d2; have_hi = true;
                    }
                }
                if (have_hi && lo >= hi) { lo = 0.0; dlo = d0; ddlo = -1.0; }  // cannot happen for convex phi
                if (fabs(dbest) <= 1e-10 * fabs(d0) || (have_hi && hi - lo <= 1e-12 * hi)) done = 1;
                if (!have_hi) {
                    centre = alphas[kLsPoints - 1] * 16.0;  // keep expanding
                } else {
                    // Newton from the better bracket end, safeguarded to (lo, hi)
                    double est;
                    if (fabs(dhi) < fabs(dlo) || ddlo < 0.0) { est = hi - dhi / ddhi; newton_step = dhi / ddhi; }
                    else { est = lo - dlo / ddlo; newton_step = dlo / ddlo; }
                    if (!(est > lo && est < hi)) { est = 0.5 * (lo + hi); newton_step = hi - lo; }
                    centre = est;
                }
                alpha = (done || !have_hi) ? best : centre;
                s_done = done;
                s_alpha = alpha;
            }
            __syncthreads();
            alpha = s_alpha;
            if (s_done) break;
        }
        if (!ok) break;
        // ---- v <- v + alpha dv ---------------------------------------------
        for (long long s = s0 + tid; s < s1; s += blockDim.x) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
                A.s_v[a * A.cap_s + s] = fma(alpha, A.s_dv[a * A.cap_s + s], A.s_v[a * A.cap_s + s]);
        }
        alpha_prev = alpha;
        ++k;
    }

    // ---- outputs: grid velocity, impulses at the final iterate, stats ------
    for (long long s = s0 + tid; s < s1; s += blockDim.x) {
        float4 g = A.vel[A.s_node[s]];
        g.x = (float)A.s_v[s];
        g.y = (float)A.s_v[A.cap_s + s];
        g.z = (float)A.s_v[2 * A.cap_s + s];
        A.vel[A.s_node[s]] = g;
    }
    for (int q = tid; q < A.n_rigid * 6; q += blockDim.x) racc[q] = 0.0;
    __syncthreads();
    for (long long c = c0 + tid; c < c1; c += blockDim.x) {
        double vc[3];
        contact_velocity(A, c, k, alpha_prev, vc);
        double g[3], g00, g01, g11, gnn;
        contact_model(params_of(A, c), vc, g, &g00, &g01, &g11, &gnn);
        const double n[3] = {A.c_n[c], A.c_n[A.cap + c], A.c_n[2 * A.cap + c]};
        double t1[3], t2[3];
        frame_of(n, t1, t2);
        double rg[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            rg[a] = t1[a] * g[0] + t2[a] * g[1] + n[a] * g[2];
            A.c_gam[a * A.cap + c] = g[a];
        }
        const int r = A.c_rid[c];
        const long long p = A.c_pid[c];
        const DevRigid& R = A.rigids[r];
        const double arm[3] = {(double)A.x[p] - R.t[0], (double)A.x[A.P + p] - R.t[1],
                               (double)A.x[2 * A.P + p] - R.t[2]};
        const double tq[3] = {arm[1] * rg[2] - arm[2] * rg[1], arm[2] * rg[0] - arm[0] * rg[2],
                              arm[0] * rg[1] - arm[1] * rg[0]};
        // impulse on the rigid body is minus the impulse on MPM
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            atomicAdd(&racc[r * 6 + a], -rg[a]);
            atomicAdd(&racc[r * 6 + 3 + a], -tq[a]);
        }
    }
    __syncthreads();
    for (int q = tid; q < A.n_rigid * 6; q += blockDim.x)
        if (racc[q] != 0.0) atomicAdd(&A.rigid_acc[q], racc[q]);
    if (blockIdx.x == 0 && tid == 0) {
        SubstepStats st;
        st.n_contacts = (int)nc;
        st.n_slots = (int)ns;
        st.iterations = k;
        st.converged = converged;
        st.residual = res;
        st.threshold = thr;
        A.stats[A.substep] = st;
        if (!converged && !aborted) atomicOr(&cnt->flags, kFlagNoconv);
    }
}

hipError_t launch_qn(const Work& w, const float* x, int substep, double h, double eps_r,
                       double eps_a, int max_iter, int ls_rounds, hipStream_t s) {
    QnArgs A;
    A.envs = w.envs;
    A.rigids = w.rigids;
    A.x = x;
    A.P = w.P;
    A.vel = w.vel;
    A.cap = w.cap_c;
    A.cap_s = w.cap_s;
    A.c_pid = w.c_pid; A.c_rid = w.c_rid; A.c_env = w.c_env; A.c_slot = w.c_slot;
    A.c_w = w.c_w;
    A.c_n = w.c_n; A.c_b = w.c_b; A.c_phi0 = w.c_phi0; A.c_n0 = w.c_n0; A.c_mu = w.c_mu;
    A.c_vc = w.c_vc; A.c_uc = w.c_uc; A.c_gam = w.c_gam;
    A.s_node = w.s_node; A.s_beg = w.s_beg;
    A.pv = w.pv_a;
    A.s_v = w.s_v; A.s_vstar = w.s_vstar; A.s_dv = w.s_dv; A.s_m = w.s_m;
    A.partial = w.partial;
    A.rigid_acc = w.rigid_acc;
    A.n_rigid = w.n_rigid;
    A.stats = w.sstats;
    A.substep = substep;
    A.h = h; A.eps_r = eps_r; A.eps_a = eps_a;
    A.max_iter = max_iter; A.ls_rounds = ls_rounds;
    A.cnt = w.cnt;
    void* args[] = {&A};
    return hipLaunchCooperativeKernel((const void*)k_qn, dim3(w.qn_blocks), dim3(kQnThreads), args, 0, s);
}

int qn_max_blocks() {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_qn, kQnThreads, 0) != hipSuccess)
        return 0;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return per_cu * cus;
}

}  // namespace mpm
