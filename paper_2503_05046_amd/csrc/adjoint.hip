// adjoint.hip -- reverse-mode derivative of the free-motion part of the
// substep (Eq. (6): P2G, grid update, G2P with the fixed-corotated stress)
// and of the host step's particle gather, for the backward form.
//
// The state carried between substeps is (x, v, F, Q) with the fused matrix
// Q = m_p C - h V0 (4/dx^2) tau(F) (MLS-MPM). One substep is
//   P2G      m_i = sum_p w_ip m_p,  p_i = sum_p w_ip (m_p v_p + Q_p (x_i - x_p))
//   grid     v*_i = p_i / m_i + h g (outward components in the boundary band
//            set to zero)
//   G2P      v'_p = sum_i w_ip v_i,  C'_p = D sum_i w_ip v_i (x_i - x_p)^T,
//            F'_p = (I + h C'_p) F_p,  x'_p = x_p + h v'_p,
//            Q'_p = m_p C'_p - h V0 D tau(F'_p)
// with quadratic B-spline weights w_ip = N((x_i - x_p)/dx) and D = 4/dx^2.
// The adjoint runs these steps backwards; the weights depend on x_p through
// their fractions f = (x_p - origin)/dx - base, with dw/dx = (dw/df)/dx and
// d(x_i - x_p)/dx_p = -I. The derivative of tau uses the SVD F = U S V^T:
// the rotation R = U V^T varies as dR = U W V^T with
// W_ij = (M_ij - M_ji) / (s_i + s_j), M = U^T dF V.
//
// Particle adjoints live in component-major float32 arrays like the state;
// node adjoints are scattered with float atomics into a float4 grid array.
// The Lame-parameter adjoints are reduced per environment in FP64.
#include "mpm_internal.h"

namespace mpm {

namespace {

__device__ __forceinline__ int env_of_particle_a(const DevEnv* envs, int n_envs, long long p) {
    int lo = 0, hi = n_envs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (envs[mid].p_begin <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int env_of_node(const DevEnv* envs, int n_envs, long long n) {
    int lo = 0, hi = n_envs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (envs[mid].node_base <= n) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Stencil of a particle as in the forward transfers (same float32 rule),
// with the weight derivatives dw/df per axis.
struct Stencil {
    int b[3];
    float w[3][3], dw[3][3], d[3][3];  // per axis: weight, dweight/df, (a - f) dx
};

__device__ __forceinline__ void stencil_of(const DevEnv& E, const float x[3], Stencil& S) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float f;
        int bi = cell_base(x[a], E.origin[a], E.inv_dx, &f);
        const int hi = E.dims[a] - 3;
        if (bi < 0 || bi > hi) {
            bi = bi < 0 ? 0 : hi;
            f = fminf(fmaxf(f, 0.5f), 1.5f);
        }
        S.b[a] = bi;
        bspline_w(f, S.w[a]);
        S.dw[a][0] = -(1.5f - f);
        S.dw[a][1] = -2.0f * (f - 1.0f);
        S.dw[a][2] = f - 0.5f;
#pragma unroll
        for (int o = 0; o < 3; ++o) S.d[a][o] = ((float)o - f) * E.dx;
    }
}

__device__ __forceinline__ long long node_of(const DevEnv& E, int i, int j, int k) {
    return E.node_base + (long long)i + (long long)E.dims[0] * ((long long)j + (long long)E.dims[1] * k);
}

// Adjoint of tau(F) = 2 mu (F - R) F^T + la (J - 1) J I: given Tb = dL/dtau,
// adds dL/dF to Fb and returns dL/dmu, dL/dla.
__device__ __forceinline__ void tau_adjoint(const Material& m, const float F[9], const float Tb[9], float Fb[9],
                                            float* mub, float* lab) {
    float U[9], s[3], V[9];
    svd3(F, U, s, V);
    float R[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            R[r * 3 + c] = U[r * 3 + 0] * V[c * 3 + 0] + U[r * 3 + 1] * V[c * 3 + 1] + U[r * 3 + 2] * V[c * 3 + 2];
    const float J = s[0] * s[1] * s[2];
    // A = Tb F, G = Tb^T (F - R)
    float A[9], G[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float a = 0.f, g = 0.f;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                a += Tb[r * 3 + q] * F[q * 3 + c];
                g += Tb[q * 3 + r] * (F[q * 3 + c] - R[q * 3 + c]);
            }
            A[r * 3 + c] = a;
            G[r * 3 + c] = g;
        }
    // B = U^T A V; K_ij = (B_ij - B_ji) / (s_i + s_j); dR-term = U K V^T
    float B[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            float acc = 0.f;
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) acc += U[r * 3 + i] * A[r * 3 + c] * V[c * 3 + j];
            B[i * 3 + j] = acc;
        }
    float K[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            K[i * 3 + j] = i == j ? 0.f : (B[i * 3 + j] - B[j * 3 + i]) / fmaxf(s[i] + s[j], 1e-6f);
    const float trT = Tb[0] + Tb[4] + Tb[8];
    const float cs[3] = {s[1] * s[2], s[0] * s[2], s[0] * s[1]};  // cof F = U diag(cs) V^T
    const float vol = m.la * (2.0f * J - 1.0f) * trT;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float uk = 0.f, cof = 0.f;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                cof += U[r * 3 + i] * cs[i] * V[c * 3 + i];
#pragma unroll
                for (int j = 0; j < 3; ++j) uk += U[r * 3 + i] * K[i * 3 + j] * V[c * 3 + j];
            }
            Fb[r * 3 + c] += 2.0f * m.mu * (A[r * 3 + c] + G[r * 3 + c] - uk) + vol * cof;
        }
    // dL/dmu = <Tb, 2 (F - R) F^T>, dL/dla = (J - 1) J tr(Tb)
    float mb = 0.f;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float t = 0.f;
#pragma unroll
            for (int q = 0; q < 3; ++q) t += (F[r * 3 + q] - R[r * 3 + q]) * F[c * 3 + q];
            mb += Tb[r * 3 + c] * 2.0f * t;
        }
    *mub = mb;
    *lab = (J - 1.0f) * J * trT;
}

// Per-environment FP64 sums of two values: a wave whose lanes share one
// environment adds them with shuffles first.
__device__ __forceinline__ void add_env_pair(double* acc, int env, double a, double b) {
    const int env0 = __shfl(env, 0, 64);
    const bool uniform = __all(env == env0);
    if (uniform) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            a += __shfl_down(a, o, 64);
            b += __shfl_down(b, o, 64);
        }
        if ((threadIdx.x & 63) == 0 && (a != 0.0 || b != 0.0)) {
            atomicAdd(&acc[2 * env0], a);
            atomicAdd(&acc[2 * env0 + 1], b);
        }
    } else if (a != 0.0 || b != 0.0) {
        atomicAdd(&acc[2 * env], a);
        atomicAdd(&acc[2 * env + 1], b);
    }
}

}  // namespace

// Adjoint of G2P for one substep. In: the tape's x, F at the substep start
// and grid velocities after the contact solve; the adjoints of x', v', F' and
// of Q' (next substep) or C' (last substep of a host step). Out: ax = the part
// of dL/dx from G2P, aF = dL/dF, node adjoints dL/dv_i added into gbar.
__global__ void __launch_bounds__(256)
k_g2p_adj(long long P, const DevEnv* __restrict__ envs, int n_envs, float h, const float* __restrict__ x,
          const float* __restrict__ F, const float4* __restrict__ vel, float* __restrict__ ax,
          const float* __restrict__ av, float* __restrict__ aF, const float* __restrict__ aQ,
          const float* __restrict__ aC, float4* __restrict__ gbar, double* __restrict__ lame) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = p < P;
    const long long q = live ? p : 0;
    const int env = env_of_particle_a(envs, n_envs, q);
    const DevEnv& E = envs[env];
    const float xp[3] = {x[q], x[P + q], x[2 * P + q]};
    float Fp[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Fp[k] = F[k * P + q];
    Stencil S;
    stencil_of(E, xp, S);
    // forward quantities: v', C', F'
    float vi[27][3];
    float vp[3] = {0.f, 0.f, 0.f}, Cp[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int bb = 0; bb < 3; ++bb)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int o = (c * 3 + bb) * 3 + a;
                const float4 g = vel[node_of(E, S.b[0] + a, S.b[1] + bb, S.b[2] + c)];
                vi[o][0] = g.x; vi[o][1] = g.y; vi[o][2] = g.z;
                const float w = S.w[0][a] * S.w[1][bb] * S.w[2][c];
                const float d[3] = {S.d[0][a], S.d[1][bb], S.d[2][c]};
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    vp[r] += w * vi[o][r];
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) Cp[r * 3 + cc] += w * vi[o][r] * d[cc];
                }
            }
#pragma unroll
    for (int k = 0; k < 9; ++k) Cp[k] *= E.D;
    float Fn[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            Fn[r * 3 + c] = Fp[r * 3 + c] + h * (Cp[r * 3 + 0] * Fp[0 * 3 + c] + Cp[r * 3 + 1] * Fp[1 * 3 + c] +
                                                 Cp[r * 3 + 2] * Fp[2 * 3 + c]);
    // incoming adjoints
    float xb[3], vb[3], Fnb[9], Cb[9];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        xb[a] = ax[a * P + q];
        vb[a] = av[a * P + q] + h * xb[a];  // x' = x + h v'
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        Fnb[k] = aF[k * P + q];
        Cb[k] = aC ? aC[k * P + q] : 0.f;
    }
    float mub = 0.f, lab = 0.f;
    if (aQ) {
        // Q' = m_p C' - h V0 D tau(F')
        float Qb[9], Tb[9];
        const float c = h * E.V0 * E.D;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            Qb[k] = aQ[k * P + q];
            Cb[k] += E.m_p * Qb[k];
            Tb[k] = -c * Qb[k];
        }
        tau_adjoint(E.mat, Fn, Tb, Fnb, &mub, &lab);
    }
    // F' = (I + h C') F
    float Fb[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float acc = Fnb[r * 3 + c];
#pragma unroll
            for (int k = 0; k < 3; ++k) acc += h * Cp[k * 3 + r] * Fnb[k * 3 + c];
            Fb[r * 3 + c] = acc;
        }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float acc = 0.f;
#pragma unroll
            for (int k = 0; k < 3; ++k) acc += Fnb[r * 3 + k] * Fp[c * 3 + k];
            Cb[r * 3 + c] += h * acc;
        }
    // v' and C' from the node velocities
    float xo[3] = {xb[0], xb[1], xb[2]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float t = 0.f;
#pragma unroll
        for (int r = 0; r < 3; ++r) t += Cb[r * 3 + a] * vp[r];
        xo[a] -= E.D * t;  // d(x_i - x_p)/dx_p = -I
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int bb = 0; bb < 3; ++bb)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int o = (c * 3 + bb) * 3 + a;
                const float d[3] = {S.d[0][a], S.d[1][bb], S.d[2][c]};
                // s = vb . v_i + D v_i^T Cb d
                float gvi[3];
                float sdot = 0.f;
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const float cd = Cb[r * 3 + 0] * d[0] + Cb[r * 3 + 1] * d[1] + Cb[r * 3 + 2] * d[2];
                    gvi[r] = vb[r] + E.D * cd;
                    sdot += vi[o][r] * gvi[r];
                }
                const float w = S.w[0][a] * S.w[1][bb] * S.w[2][c];
                const float gw[3] = {S.dw[0][a] * S.w[1][bb] * S.w[2][c] * E.inv_dx,
                                     S.w[0][a] * S.dw[1][bb] * S.w[2][c] * E.inv_dx,
                                     S.w[0][a] * S.w[1][bb] * S.dw[2][c] * E.inv_dx};
#pragma unroll
                for (int r = 0; r < 3; ++r) xo[r] += gw[r] * sdot;
                if (live) {
                    float* g = reinterpret_cast<float*>(&gbar[node_of(E, S.b[0] + a, S.b[1] + bb, S.b[2] + c)]);
#pragma unroll
                    for (int r = 0; r < 3; ++r) atomicAdd(g + r, w * gvi[r]);
                }
            }
    if (live) {
#pragma unroll
        for (int a = 0; a < 3; ++a) ax[a * P + p] = xo[a];
#pragma unroll
        for (int k = 0; k < 9; ++k) aF[k * P + p] = Fb[k];
    }
    add_env_pair(lame, env, live ? (double)mub : 0.0, live ? (double)lab : 0.0);
}

// Adjoint of the grid update, in place on gbar: dL/dv*_i -> (dL/dp_i, dL/dm_i)
// at nodes with mass; components zeroed by the boundary band pass nothing.
__global__ void __launch_bounds__(256)
k_grid_adj(long long n_nodes, const DevEnv* __restrict__ envs, int n_envs, float h,
           const float4* __restrict__ vstar, float4* __restrict__ gbar) {
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_nodes) return;
    const float4 g = gbar[n];
    if (g.x == 0.f && g.y == 0.f && g.z == 0.f) return;
    const float4 vs = vstar[n];
    if (!(vs.w > 0.f)) {
        gbar[n] = make_float4(0.f, 0.f, 0.f, 0.f);
        return;
    }
    const DevEnv& E = envs[env_of_node(envs, n_envs, n)];
    const long long l = n - E.node_base;
    const int idx[3] = {(int)(l % E.dims[0]), (int)((l / E.dims[0]) % E.dims[1]), (int)(l / ((long long)E.dims[0] * E.dims[1]))};
    float gb[3] = {g.x, g.y, g.z};
    const float vv[3] = {vs.x, vs.y, vs.z};
    float mb = 0.f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool band = idx[a] < 3 || idx[a] >= E.dims[a] - 3;
        if (band && vv[a] == 0.f) gb[a] = 0.f;  // clamped to zero: no dependence
        mb -= gb[a] * (vv[a] - h * E.gravity[a]);
    }
    const float inv_m = 1.0f / vs.w;
    gbar[n] = make_float4(gb[0] * inv_m, gb[1] * inv_m, gb[2] * inv_m, mb * inv_m);
}

// Adjoint of P2G: from (dL/dp_i, dL/dm_i) in gbar to dL/dv_p, dL/dQ_p and the
// P2G part of dL/dx_p (added to ax).
__global__ void __launch_bounds__(256)
k_p2g_adj(long long P, const DevEnv* __restrict__ envs, int n_envs, const float* __restrict__ x,
          const float* __restrict__ v, const float* __restrict__ Q, const float4* __restrict__ gbar,
          float* __restrict__ ax, float* __restrict__ av, float* __restrict__ aQ) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const DevEnv& E = envs[env_of_particle_a(envs, n_envs, p)];
    const float xp[3] = {x[p], x[P + p], x[2 * P + p]};
    const float mv[3] = {E.m_p * v[p], E.m_p * v[P + p], E.m_p * v[2 * P + p]};
    float Qm[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Qm[k] = Q[k * P + p];
    Stencil S;
    stencil_of(E, xp, S);
    float sp[3] = {0.f, 0.f, 0.f}, sq[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float xo[3] = {ax[p], ax[P + p], ax[2 * P + p]};
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int bb = 0; bb < 3; ++bb)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const float4 g = gbar[node_of(E, S.b[0] + a, S.b[1] + bb, S.b[2] + c)];
                const float pb[3] = {g.x, g.y, g.z};
                const float w = S.w[0][a] * S.w[1][bb] * S.w[2][c];
                const float d[3] = {S.d[0][a], S.d[1][bb], S.d[2][c]};
                // contribution value: m_p m_i-adjoint + pb . (m_p v + Q d)
                float val = E.m_p * g.w;
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    val += pb[r] * (mv[r] + Qm[r * 3 + 0] * d[0] + Qm[r * 3 + 1] * d[1] + Qm[r * 3 + 2] * d[2]);
                    sp[r] += w * pb[r];
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) sq[r * 3 + cc] += w * pb[r] * d[cc];
                }
                const float gw[3] = {S.dw[0][a] * S.w[1][bb] * S.w[2][c] * E.inv_dx,
                                     S.w[0][a] * S.dw[1][bb] * S.w[2][c] * E.inv_dx,
                                     S.w[0][a] * S.w[1][bb] * S.dw[2][c] * E.inv_dx};
#pragma unroll
                for (int r = 0; r < 3; ++r) xo[r] += gw[r] * val;
            }
    // d(x_i - x_p)/dx_p = -I: - Q^T sum w pb
#pragma unroll
    for (int a = 0; a < 3; ++a) xo[a] -= Qm[0 * 3 + a] * sp[0] + Qm[1 * 3 + a] * sp[1] + Qm[2 * 3 + a] * sp[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        ax[a * P + p] = xo[a];
        av[a * P + p] = E.m_p * sp[a];
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) aQ[k * P + p] = sq[k];
}

// Adjoint of the host step's gather Q = m_p C - h V0 D tau(F), (x, v, F, C) in
// sorted order <- caller order: scatters (dL/dx, dL/dv, dL/dF, dL/dC) back to
// the order before the sort.
__global__ void __launch_bounds__(256)
k_permute_adj(long long P, const DevEnv* __restrict__ envs, int n_envs, float h, const unsigned* __restrict__ idx,
              const float* __restrict__ F, const float* __restrict__ ax, const float* __restrict__ av,
              const float* __restrict__ aF, const float* __restrict__ aQ, float* __restrict__ ox,
              float* __restrict__ ov, float* __restrict__ oF, float* __restrict__ oC, double* __restrict__ lame) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = i < P;
    const long long q = live ? i : 0;
    const int env = env_of_particle_a(envs, n_envs, q);
    const DevEnv& E = envs[env];
    float Fp[9], Qb[9], Fb[9], Tb[9];
    const float c = h * E.V0 * E.D;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        Fp[k] = F[k * P + q];
        Qb[k] = aQ[k * P + q];
        Fb[k] = aF[k * P + q];
        Tb[k] = -c * Qb[k];
    }
    float mub, lab;
    tau_adjoint(E.mat, Fp, Tb, Fb, &mub, &lab);
    if (live) {
        const long long s = idx[i];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            ox[a * P + s] = ax[a * P + i];
            ov[a * P + s] = av[a * P + i];
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            oF[k * P + s] = Fb[k];
            oC[k * P + s] = E.m_p * Qb[k];
        }
    }
    add_env_pair(lame, env, live ? (double)mub : 0.0, live ? (double)lab : 0.0);
}

hipError_t launch_g2p_adj(const Work& w, const TapeStep& t, float h, float* ax, const float* av, float* aF,
                          const float* aQ, const float* aC, float4* gbar, double* lame, hipStream_t s) {
    const unsigned blocks = (unsigned)((w.P + 255) / 256);
    hipLaunchKernelGGL(k_g2p_adj, dim3(blocks), dim3(256), 0, s, w.P, w.envs, w.n_envs, h, t.x, t.F, t.vel, ax,
                       av, aF, aQ, aC, gbar, lame);
    return hipGetLastError();
}

hipError_t launch_grid_adj(const Work& w, const TapeStep& t, float h, float4* gbar, hipStream_t s) {
    const unsigned blocks = (unsigned)((w.n_nodes + 255) / 256);
    hipLaunchKernelGGL(k_grid_adj, dim3(blocks), dim3(256), 0, s, w.n_nodes, w.envs, w.n_envs, h, t.vstar, gbar);
    return hipGetLastError();
}

hipError_t launch_p2g_adj(const Work& w, const TapeStep& t, const float4* gbar, float* ax, float* av, float* aQ,
                          hipStream_t s) {
    const unsigned blocks = (unsigned)((w.P + 255) / 256);
    hipLaunchKernelGGL(k_p2g_adj, dim3(blocks), dim3(256), 0, s, w.P, w.envs, w.n_envs, t.x, t.v, t.Q, gbar, ax,
                       av, aQ);
    return hipGetLastError();
}

hipError_t launch_permute_adj(const Work& w, const TapeStep& t, float h, const unsigned* idx, const float* ax,
                              const float* av, const float* aF, const float* aQ, float* ox, float* ov, float* oF,
                              float* oC, double* lame, hipStream_t s) {
    const unsigned blocks = (unsigned)((w.P + 255) / 256);
    hipLaunchKernelGGL(k_permute_adj, dim3(blocks), dim3(256), 0, s, w.P, w.envs, w.n_envs, h, idx, t.F, ax, av,
                       aF, aQ, ox, ov, oF, oC, lame);
    return hipGetLastError();
}

}  // namespace mpm
