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
//
// Contact solve (Eq. (8)): at the optimum M (v - v*) + sum_c J_c^T R_c dl_c = 0
// with v_c = R_c^T J_c v + b_c. Differentiating, an adjoint vb on the contact
// nodes becomes vb* = M lam with H lam = vb, H = M + sum_c J_c^T R_c G_c R_c^T J_c
// the full Hessian (solved by preconditioned conjugate gradients in FP64 with
// the 3x3 node blocks of H as preconditioner). With y_c = R_c^T J_c lam:
//   bias          bb_c   = -G_c y_c
//   penetration   phib_c = -y_c . d(dl_c)/dphi0
//   friction      mun0b  = -y_c . d(dl_c)/d(mu n0)
//   weights       wb_ic  = -(R_c G_c y_c) . v_i + lam_i . (R_c gamma_c)
// and through registration: phi0 = -sdf(x_p), n0 = gamma_n(n . (v_p - v_r)),
// b_c = -R_c^T v_r with v_r = V + w x (x_p - t) the rigid velocity at x_p. The
// normal of a half-space or of the inside of a box does not vary with x_p,
// so the frame R_c carries no adjoint to the particle.
#include "contact_model.h"
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

// Adjoint of the Hencky update of the Drucker-Prager material. From the trial
// F_t = U diag(sig) V^T the forward forms s, the return map in Hencky strain
// (eps = ln sig projected onto the cone; at its tip when tr eps >= 0) when
// plastic, else s = sig, and writes F_out = U diag(s) V^T and
// tau = U diag(t) U^T with t = 2 mu ln s + la tr(ln s). Given Fob = dL/dF_out
// and Tb = dL/dtau, adds dL/dF_t to Ftb and returns dL/dmu and dL/dla. Both
// outputs are isotropic functions of F_t: a perturbation dP = U^T dF_t V
// changes their diagonals (in the frames U, V and U, U) through the Jacobians
// of s and t with respect to sig, and their off-diagonal entries through
// divided differences of s and t times the symmetric and skew parts of dP;
// where two singular values coincide the divided differences take their
// limits from the Jacobians. Evaluated in FP64 from the forward's own FP32 SVD.
__device__ void hencky_dp_adjoint(const Material& m, bool plastic, const float Ft[9], const float Fob[9],
                                  const float Tb[9], float Ftb[9], float* mub, float* lab) {
    float Uf[9], sf[3], Vf[9];
    svd3(Ft, Uf, sf, Vf);
    double U[9], V[9], sig[3], e[3];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        U[k] = Uf[k];
        V[k] = Vf[k];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        sig[i] = fmax((double)sf[i], 1e-6);
        e[i] = log(sig[i]);
    }
    const double mu = m.mu, la = m.la, tr = e[0] + e[1] + e[2];
    // eps_p(eps), its Jacobian Jp (row i, column k: d eps_p,i / d eps_k), and
    // d eps_p / d kappa, kappa = (3 la + 2 mu) alpha / (2 mu) (the cone)
    double ep[3] = {e[0], e[1], e[2]}, Jp[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, dkap[3] = {0, 0, 0};
    if (plastic) {
        if (tr >= 0.0) {
#pragma unroll
            for (int i = 0; i < 3; ++i) ep[i] = 0.0;
#pragma unroll
            for (int k = 0; k < 9; ++k) Jp[k] = 0.0;
        } else {
            const double dv[3] = {e[0] - tr / 3.0, e[1] - tr / 3.0, e[2] - tr / 3.0};
            const double nd = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
            const double kap = (3.0 * la + 2.0 * mu) / (2.0 * mu) * (double)m.alpha;
            if (nd > 0.0 && nd + kap * tr > 0.0) {
                // eps_p = (tr/3) 1 - kappa tr n, n = dev(eps) / |dev(eps)|
                const double n[3] = {dv[0] / nd, dv[1] / nd, dv[2] / nd};
                const double g = kap * tr / nd;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    ep[i] = tr / 3.0 - kap * tr * n[i];
                    dkap[i] = -tr * n[i];
#pragma unroll
                    for (int k = 0; k < 3; ++k)
                        Jp[i * 3 + k] = 1.0 / 3.0 - kap * n[i] - g * ((i == k ? 1.0 : 0.0) - n[i] * n[k] - 1.0 / 3.0);
                }
            }
        }
    }
    const double trp = ep[0] + ep[1] + ep[2];
    double sv[3], tv[3], Js[9], Jt[9];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        sv[i] = exp(ep[i]);
        tv[i] = 2.0 * mu * ep[i] + la * trp;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double colsum = Jp[0 * 3 + k] + Jp[1 * 3 + k] + Jp[2 * 3 + k];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            Js[i * 3 + k] = sv[i] * Jp[i * 3 + k] / sig[k];
            Jt[i * 3 + k] = (2.0 * mu * Jp[i * 3 + k] + la * colsum) / sig[k];
        }
    }
    // the adjoints in the frames: Ab = U^T Fob V, Bb = U^T sym(Tb) U
    double Ab[9], Bb[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double a = 0.0, b = 0.0;
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    a += U[r * 3 + i] * (double)Fob[r * 3 + c] * V[c * 3 + j];
                    b += U[r * 3 + i] * 0.5 * ((double)Tb[r * 3 + c] + (double)Tb[c * 3 + r]) * U[c * 3 + j];
                }
            Ab[i * 3 + j] = a;
            Bb[i * 3 + j] = b;
        }
    double Pb[9];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) acc += Ab[i * 4] * Js[i * 3 + k] + Bb[i * 4] * Jt[i * 3 + k];
        Pb[k * 4] = acc;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i + 1; j < 3; ++j) {
            const double gap = sig[j] - sig[i], sum = sig[i] + sig[j];
            const bool close = fabs(gap) <= 1e-6 * sum;
            const double a = close ? Js[i * 3 + i] - Js[i * 3 + j] : (sv[j] - sv[i]) / gap;
            const double b = (sv[i] + sv[j]) / sum;
            const double c = close ? Jt[i * 3 + i] - Jt[i * 3 + j] : (tv[j] - tv[i]) / gap;
            const double d = (tv[j] - tv[i]) / sum;
            const double symA = 0.5 * (Ab[i * 3 + j] + Ab[j * 3 + i]), skwA = 0.5 * (Ab[i * 3 + j] - Ab[j * 3 + i]);
            const double bs = Bb[i * 3 + j] + Bb[j * 3 + i];
            Pb[i * 3 + j] = a * symA + b * skwA + 0.5 * bs * (c + d);
            Pb[j * 3 + i] = a * symA - b * skwA + 0.5 * bs * (c - d);
        }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) acc += U[r * 3 + i] * Pb[i * 3 + j] * V[c * 3 + j];
            Ftb[r * 3 + c] += (float)acc;
        }
    // the Lame parameters: directly in t, and through kappa on the cone
    const double dkap_dmu = -3.0 * la * (double)m.alpha / (2.0 * mu * mu);
    const double dkap_dla = 3.0 * (double)m.alpha / (2.0 * mu);
    double mb = 0.0, lb = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double dep_mu = dkap[i] * dkap_dmu, dep_la = dkap[i] * dkap_dla;
        mb += Ab[i * 4] * sv[i] * dep_mu + Bb[i * 4] * (2.0 * ep[i] + 2.0 * mu * dep_mu);
        lb += Ab[i * 4] * sv[i] * dep_la + Bb[i * 4] * (trp + 2.0 * mu * dep_la);
    }
    *mub = (float)mb;
    *lab = (float)lb;
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
    float Tb[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (aQ) {
        // Q' = m_p C' - h V0 D tau(F')
        const float c = h * E.V0 * E.D;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const float Qb = aQ[k * P + q];
            Cb[k] += E.m_p * Qb;
            Tb[k] = -c * Qb;
        }
    }
    if (E.mat.type == 1) {
        // sand: F' and tau both come from the return map of the trial F
        float Ftb[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        hencky_dp_adjoint(E.mat, true, Fn, Fnb, Tb, Ftb, &mub, &lab);
#pragma unroll
        for (int k = 0; k < 9; ++k) Fnb[k] = Ftb[k];
    } else if (aQ) {
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
// at nodes with mass (plus the direct dL/dm_i already in the fourth
// component); components zeroed by the boundary band pass nothing.
__global__ void __launch_bounds__(256)
k_grid_adj(long long n_nodes, const DevEnv* __restrict__ envs, int n_envs, float h,
           const float4* __restrict__ vstar, float4* __restrict__ gbar) {
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_nodes) return;
    const float4 g = gbar[n];  // dL/dv* (xyz) and a direct dL/dm from the contact solve (w)
    if (g.x == 0.f && g.y == 0.f && g.z == 0.f && g.w == 0.f) return;
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
    gbar[n] = make_float4(gb[0] * inv_m, gb[1] * inv_m, gb[2] * inv_m, mb * inv_m + g.w);
}

// Adjoint of P2G: from (dL/dp_i, dL/dm_i) in gbar to dL/dv_p, dL/dQ_p and the
// P2G part of dL/dx_p (added to ax).
__global__ void __launch_bounds__(256)
k_p2g_adj(long long P, const DevEnv* __restrict__ envs, int n_envs, const float* __restrict__ x,
          const float* __restrict__ v, const float* __restrict__ Q, const float4* __restrict__ gbar,
          const float* __restrict__ cx, const float* __restrict__ cv, float* __restrict__ ax,
          float* __restrict__ av, float* __restrict__ aQ) {
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
        ax[a * P + p] = xo[a] + (cx ? cx[a * P + p] : 0.f);
        av[a * P + p] = E.m_p * sp[a] + (cv ? cv[a * P + p] : 0.f);
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
    if (E.mat.type == 1) {
        // the Hencky stress of the stored (already projected) F
        const float zero[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        hencky_dp_adjoint(E.mat, false, Fp, zero, Tb, Fb, &mub, &lab);
    } else {
        tau_adjoint(E.mat, Fp, Tb, Fb, &mub, &lab);
    }
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

// ---------------------------------------------------------------------------
// Contact solve in reverse
// ---------------------------------------------------------------------------
__device__ __forceinline__ ContactParams params_a(const ContactRec& R, double h) {
    ContactParams P;
    P.phi0 = R.phi0; P.mun0 = R.mun0; P.k = R.k; P.d = R.d; P.eps_s = R.eps_s; P.h = h;
    return P;
}

// world vector w -> contact frame, and back
__device__ __forceinline__ void to_frame(const ContactRec& R, const double w[3], double c[3]) {
    c[0] = R.t1[0] * w[0] + R.t1[1] * w[1] + R.t1[2] * w[2];
    c[1] = R.t2[0] * w[0] + R.t2[1] * w[1] + R.t2[2] * w[2];
    c[2] = R.n[0] * w[0] + R.n[1] * w[1] + R.n[2] * w[2];
}
__device__ __forceinline__ void from_frame(const ContactRec& R, const double c[3], double w[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) w[a] = R.t1[a] * c[0] + R.t2[a] * c[1] + R.n[a] * c[2];
}
__device__ __forceinline__ void cross3(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ __forceinline__ void apply_G(double g00, double g01, double g11, double gnn, const double u[3], double o[3]) {
    o[0] = g00 * u[0] + g01 * u[1];
    o[1] = g01 * u[0] + g11 * u[1];
    o[2] = gnn * u[2];
}

// v_c at the optimum from the recorded node velocities (slot nodes of the grid
// after the solve), kept in ContactDyn::vc[0].
__global__ void __launch_bounds__(256)
k_cadj_vc(const DevCounters* cnt, long long cap, const ContactRec* __restrict__ rec,
          const ContactStencil* __restrict__ st, const int* __restrict__ s_node, const float4* __restrict__ vel,
          ContactDyn* __restrict__ dyn) {
    const long long nc = std::min<long long>(cnt->n_contacts, cap);
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (long long)gridDim.x * blockDim.x) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int o = 0; o < 27; ++o) {
            const int sl = st[c].slot[o];
            if (sl < 0) continue;
            const float4 g = vel[s_node[sl]];
            const double w = st[c].w[o];
            acc[0] += w * g.x; acc[1] += w * g.y; acc[2] += w * g.z;
        }
        double vc[3];
        to_frame(rec[c], acc, vc);
        ContactDyn& D = dyn[c];
#pragma unroll
        for (int a = 0; a < 3; ++a) D.vc[0][a] = vc[a] + D.b[a];
    }
}

// Per contact node: the inverse of its 3x3 block m I + sum w^2 R G R^T
// (symmetric, 6 entries), the right-hand side vb (from the node adjoints), and
// the CG start lam = 0, r = vb, z = P r, p = z; sums r.z and r.r.
__global__ void __launch_bounds__(256)
k_cadj_start(const DevCounters* cnt, double h, const ContactRec* __restrict__ rec, const ContactDyn* __restrict__ dyn,
             const int* __restrict__ s_node, const int* __restrict__ s_beg, const Entry* __restrict__ ent,
             const SlotRec* __restrict__ srec, const float4* __restrict__ gbar, double* __restrict__ pinv,
             double3* __restrict__ lam, double3* __restrict__ r, double3* __restrict__ z, double3* __restrict__ p,
             double* __restrict__ sc) {
    const long long ns = cnt->n_slots;
    double rz = 0.0, rr = 0.0;
    for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < ns; s += (long long)gridDim.x * blockDim.x) {
        const double m = srec[s].m;
        double H[6] = {m, 0.0, 0.0, m, 0.0, m};  // 00 01 02 11 12 22
        for (int e = s_beg[s]; e < s_beg[s + 1]; ++e) {
            const Entry en = ent[e];
            const ContactRec& R = rec[en.c];
            double gam[3], g00, g01, g11, gnn;
            contact_model(params_a(R, h), dyn[en.c].vc[0], gam, &g00, &g01, &g11, &gnn);
            const double ww = (double)en.w * en.w;
            const double* t1 = R.t1; const double* t2 = R.t2; const double* n = R.n;
            int q = 0;
            for (int a = 0; a < 3; ++a)
                for (int b = a; b < 3; ++b)
                    H[q++] += ww * (g00 * t1[a] * t1[b] + g01 * (t1[a] * t2[b] + t2[a] * t1[b]) + g11 * t2[a] * t2[b] +
                                    gnn * n[a] * n[b]);
        }
        // inverse by cofactors (H is SPD)
        const double c00 = H[3] * H[5] - H[4] * H[4], c01 = H[2] * H[4] - H[1] * H[5], c02 = H[1] * H[4] - H[2] * H[3];
        const double c11 = H[0] * H[5] - H[2] * H[2], c12 = H[1] * H[2] - H[0] * H[4], c22 = H[0] * H[3] - H[1] * H[1];
        const double det = H[0] * c00 + H[1] * c01 + H[2] * c02;
        const double id = 1.0 / det;
        double* Pi = pinv + 6 * s;
        Pi[0] = c00 * id; Pi[1] = c01 * id; Pi[2] = c02 * id; Pi[3] = c11 * id; Pi[4] = c12 * id; Pi[5] = c22 * id;
        const float4 g = gbar[s_node[s]];
        const double rv[3] = {g.x, g.y, g.z};
        const double zv[3] = {Pi[0] * rv[0] + Pi[1] * rv[1] + Pi[2] * rv[2], Pi[1] * rv[0] + Pi[3] * rv[1] + Pi[4] * rv[2],
                              Pi[2] * rv[0] + Pi[4] * rv[1] + Pi[5] * rv[2]};
        lam[s] = make_double3(0.0, 0.0, 0.0);
        r[s] = make_double3(rv[0], rv[1], rv[2]);
        z[s] = make_double3(zv[0], zv[1], zv[2]);
        p[s] = make_double3(zv[0], zv[1], zv[2]);
        rz += rv[0] * zv[0] + rv[1] * zv[1] + rv[2] * zv[2];
        rr += rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        rz += __shfl_down(rz, o, 64);
        rr += __shfl_down(rr, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&sc[0], rz);
        atomicAdd(&sc[5], rr);  // |r0|^2
    }
}

// q_c = R G R^T J_c p (world frame)
__global__ void __launch_bounds__(256)
k_cg_q(const DevCounters* cnt, long long cap, double h, const ContactRec* __restrict__ rec,
       const ContactDyn* __restrict__ dyn, const ContactStencil* __restrict__ st, const double3* __restrict__ p,
       double3* __restrict__ q) {
    const long long nc = std::min<long long>(cnt->n_contacts, cap);
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (long long)gridDim.x * blockDim.x) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int o = 0; o < 27; ++o) {
            const int sl = st[c].slot[o];
            if (sl < 0) continue;
            const double w = st[c].w[o];
            const double3 pv = p[sl];
            acc[0] += w * pv.x; acc[1] += w * pv.y; acc[2] += w * pv.z;
        }
        const ContactRec& R = rec[c];
        double u[3], gu[3], out[3], gam[3], g00, g01, g11, gnn;
        to_frame(R, acc, u);
        contact_model(params_a(R, h), dyn[c].vc[0], gam, &g00, &g01, &g11, &gnn);
        apply_G(g00, g01, g11, gnn, u, gu);
        from_frame(R, gu, out);
        q[c] = make_double3(out[0], out[1], out[2]);
    }
}

// Hp_s = m p_s + sum_e w_e q_c(e); sums p.Hp into sc[2]
__global__ void __launch_bounds__(256)
k_cg_hp(const DevCounters* cnt, const int* __restrict__ s_beg, const Entry* __restrict__ ent,
        const SlotRec* __restrict__ srec, const double3* __restrict__ p, const double3* __restrict__ q,
        double3* __restrict__ hp, double* __restrict__ sc) {
    const long long ns = cnt->n_slots;
    double php = 0.0;
    for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < ns; s += (long long)gridDim.x * blockDim.x) {
        const double m = srec[s].m;
        const double3 pv = p[s];
        double a[3] = {m * pv.x, m * pv.y, m * pv.z};
        for (int e = s_beg[s]; e < s_beg[s + 1]; ++e) {
            const Entry en = ent[e];
            const double3 qv = q[en.c];
            a[0] += en.w * qv.x; a[1] += en.w * qv.y; a[2] += en.w * qv.z;
        }
        hp[s] = make_double3(a[0], a[1], a[2]);
        php += pv.x * a[0] + pv.y * a[1] + pv.z * a[2];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) php += __shfl_down(php, o, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(&sc[2], php);
}

// alpha = rz / pHp; lam += alpha p; r -= alpha Hp; z = P r; sums r.z (sc[1]) and r.r (sc[3])
__global__ void __launch_bounds__(256)
k_cg_update(const DevCounters* cnt, const double* __restrict__ pinv, const double3* __restrict__ p,
            const double3* __restrict__ hp, double3* __restrict__ lam, double3* __restrict__ r,
            double3* __restrict__ z, double* __restrict__ sc) {
    const long long ns = cnt->n_slots;
    const double alpha = sc[2] > 0.0 ? sc[0] / sc[2] : 0.0;
    double rz = 0.0, rr = 0.0;
    for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < ns; s += (long long)gridDim.x * blockDim.x) {
        const double3 pv = p[s], hv = hp[s];
        double3 l = lam[s], rv = r[s];
        l.x += alpha * pv.x; l.y += alpha * pv.y; l.z += alpha * pv.z;
        rv.x -= alpha * hv.x; rv.y -= alpha * hv.y; rv.z -= alpha * hv.z;
        lam[s] = l;
        r[s] = rv;
        const double* Pi = pinv + 6 * s;
        const double3 zv = make_double3(Pi[0] * rv.x + Pi[1] * rv.y + Pi[2] * rv.z,
                                        Pi[1] * rv.x + Pi[3] * rv.y + Pi[4] * rv.z,
                                        Pi[2] * rv.x + Pi[4] * rv.y + Pi[5] * rv.z);
        z[s] = zv;
        rz += rv.x * zv.x + rv.y * zv.y + rv.z * zv.z;
        rr += rv.x * rv.x + rv.y * rv.y + rv.z * rv.z;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        rz += __shfl_down(rz, o, 64);
        rr += __shfl_down(rr, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&sc[1], rz);
        atomicAdd(&sc[3], rr);
    }
}

// p = z + beta p with beta = rz_new / rz
__global__ void __launch_bounds__(256)
k_cg_dir(const DevCounters* cnt, const double3* __restrict__ z, double3* __restrict__ p, const double* __restrict__ sc) {
    const long long ns = cnt->n_slots;
    const double beta = sc[0] > 0.0 ? sc[1] / sc[0] : 0.0;
    for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < ns; s += (long long)gridDim.x * blockDim.x) {
        const double3 zv = z[s];
        double3 pv = p[s];
        pv.x = zv.x + beta * pv.x; pv.y = zv.y + beta * pv.y; pv.z = zv.z + beta * pv.z;
        p[s] = pv;
    }
}

// scalars for the next iteration: sc[4] = last |r|^2, rz = rz_new, the sums cleared
__global__ void k_cg_next(double* sc) {
    sc[4] = sc[3];
    sc[0] = sc[1];
    sc[1] = 0.0;
    sc[2] = 0.0;
    sc[3] = 0.0;
}

// Per contact: the adjoints of the contact's parameters, chained through
// registration to the particle (x, v at the substep start: into cx, cv) and
// to the rigid body (into rg, 12 doubles per body: V, t, w through the
// velocity V + w x (x - t), and a small rotation th of the pose about t,
// R -> (I + [th]x) R).
__global__ void __launch_bounds__(256)
k_cadj_params(const DevCounters* cnt, long long cap, long long P, double h, const DevEnv* __restrict__ envs,
              const DevRigid* __restrict__ rigids, const ContactRec* __restrict__ rec,
              const ContactDyn* __restrict__ dyn, const ContactStencil* __restrict__ st,
              const int* __restrict__ c_pid, const int* __restrict__ c_rid, const int* __restrict__ c_env,
              const int* __restrict__ s_node, const float4* __restrict__ vel, const double3* __restrict__ lam,
              const float* __restrict__ x, const float* __restrict__ v, float* __restrict__ cx,
              float* __restrict__ cv, double* __restrict__ rg) {
    const long long nc = std::min<long long>(cnt->n_contacts, cap);
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (long long)gridDim.x * blockDim.x) {
        const ContactRec& R = rec[c];
        const double* vcf = dyn[c].vc[0];
        double ly[3] = {0.0, 0.0, 0.0};
        for (int o = 0; o < 27; ++o) {
            const int sl = st[c].slot[o];
            if (sl < 0) continue;
            const double w = st[c].w[o];
            const double3 l = lam[sl];
            ly[0] += w * l.x; ly[1] += w * l.y; ly[2] += w * l.z;
        }
        double y[3];
        to_frame(R, ly, y);
        const ContactParams Pm = params_a(R, h);
        double gam[3], g00, g01, g11, gnn;
        contact_model(Pm, vcf, gam, &g00, &g01, &g11, &gnn);
        double Gy[3];
        apply_G(g00, g01, g11, gnn, y, Gy);
        // parameters of the contact
        double bb[3] = {-Gy[0], -Gy[1], -Gy[2]};
        const double an = Pm.phi0 - h * vcf[2], bn = 1.0 - Pm.d * vcf[2];
        double phib = (an > 0.0 && bn > 0.0) ? h * Pm.k * bn * y[2] : 0.0;
        const double s2 = vcf[0] * vcf[0] + vcf[1] * vcf[1] + Pm.eps_s * Pm.eps_s;
        const double mun0b = -(y[0] * vcf[0] + y[1] * vcf[1]) * inv_sqrt(s2);
        // weights of the stencil
        const long long p = c_pid[c];
        const DevEnv& E = envs[c_env[c]];
        const DevRigid& B = rigids[c_rid[c]];
        const float xf[3] = {x[p], x[P + p], x[2 * P + p]};
        Stencil S;
        stencil_of(E, xf, S);
        double RGy[3], Rg[3];
        from_frame(R, Gy, RGy);
        from_frame(R, gam, Rg);
        double xb[3] = {0.0, 0.0, 0.0}, vb[3] = {0.0, 0.0, 0.0};
        for (int o = 0; o < 27; ++o) {
            const int sl = st[c].slot[o];
            if (sl < 0) continue;
            const float4 g = vel[s_node[sl]];
            const double3 l = lam[sl];
            const double wb = -(RGy[0] * g.x + RGy[1] * g.y + RGy[2] * g.z) + (l.x * Rg[0] + l.y * Rg[1] + l.z * Rg[2]);
            const int a = o % 3, bq = (o / 3) % 3, cz = o / 9;
            xb[0] += wb * (double)(S.dw[0][a] * S.w[1][bq] * S.w[2][cz] * E.inv_dx);
            xb[1] += wb * (double)(S.w[0][a] * S.dw[1][bq] * S.w[2][cz] * E.inv_dx);
            xb[2] += wb * (double)(S.w[0][a] * S.w[1][bq] * S.dw[2][cz] * E.inv_dx);
        }
        // registration: n0 = gamma_n(n . (v_p - v_r)), lagged
        const double xp[3] = {xf[0], xf[1], xf[2]};
        const double rel[3] = {xp[0] - B.t[0], xp[1] - B.t[1], xp[2] - B.t[2]};
        const double vr[3] = {B.V[0] + B.w[1] * rel[2] - B.w[2] * rel[1], B.V[1] + B.w[2] * rel[0] - B.w[0] * rel[2],
                              B.V[2] + B.w[0] * rel[1] - B.w[1] * rel[0]};
        const double vp[3] = {v[p], v[P + p], v[2 * P + p]};
        const double vn0 = R.n[0] * (vp[0] - vr[0]) + R.n[1] * (vp[1] - vr[1]) + R.n[2] * (vp[2] - vr[2]);
        const double a0 = Pm.phi0 - h * vn0, b0 = 1.0 - Pm.d * vn0;
        double vrb[3];
        {
            double rbb[3];
            from_frame(R, bb, rbb);  // b = -R^T v_r
            vrb[0] = -rbb[0]; vrb[1] = -rbb[1]; vrb[2] = -rbb[2];
        }
        double vn0b = 0.0;
        if (a0 > 0.0 && b0 > 0.0) {
            const double n0b = B.mu * mun0b;
            phib += n0b * h * Pm.k * b0;
            vn0b = n0b * h * Pm.k * (-h * b0 - Pm.d * a0);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                vb[q] += vn0b * R.n[q];
                vrb[q] -= vn0b * R.n[q];
            }
        }
        // phi0 = -sdf(x_p; pose): d/dx = -n, d/dt = n
        // v_r = V + w x (x_p - t): d/dx = [w]x, d/dt = -[w]x
        const double wx[3] = {vrb[1] * B.w[2] - vrb[2] * B.w[1], vrb[2] * B.w[0] - vrb[0] * B.w[2],
                              vrb[0] * B.w[1] - vrb[1] * B.w[0]};  // vrb x w
#pragma unroll
        for (int q = 0; q < 3; ++q) xb[q] += -phib * R.n[q] + wx[q];
        // w: d(w x rel) = dw x rel, so dL/dw = rel x vrb
        double wb[3];
        cross3(rel, vrb, wb);
        // a rotation th of the pose about t: phi0 changes by th . (rel x n);
        // the normal turns with the body (dn = th x n), and so does the
        // contact frame (the model is isotropic about n, so any completion of
        // the turned normal gives the same impulse); in the solve's optimality
        // condition the term J^T R grad l(R^T (J v - v_r)) then changes by
        // J^T (-th x R gamma - R G R^T (th x u)), u = R v_c, and -lam^T of
        // that is th . (R gamma x J lam + u x R G y)
        double thb[3], tq[3], u[3];
        cross3(rel, R.n, thb);
#pragma unroll
        for (int q = 0; q < 3; ++q) thb[q] *= phib;
        const double dvp[3] = {vp[0] - vr[0], vp[1] - vr[1], vp[2] - vr[2]};
        cross3(R.n, dvp, tq);
#pragma unroll
        for (int q = 0; q < 3; ++q) thb[q] += vn0b * tq[q];
        cross3(Rg, ly, tq);
#pragma unroll
        for (int q = 0; q < 3; ++q) thb[q] += tq[q];
        from_frame(R, vcf, u);
        cross3(u, RGy, tq);
#pragma unroll
        for (int q = 0; q < 3; ++q) thb[q] += tq[q];
        const int rid = c_rid[c];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            atomicAdd(&cx[q * P + p], (float)xb[q]);
            atomicAdd(&cv[q * P + p], (float)vb[q]);
            atomicAdd(&rg[kRigidGradStride * rid + q], vrb[q]);
            atomicAdd(&rg[kRigidGradStride * rid + 3 + q], phib * R.n[q] - wx[q]);
            atomicAdd(&rg[kRigidGradStride * rid + 6 + q], wb[q]);
            atomicAdd(&rg[kRigidGradStride * rid + 9 + q], thb[q]);
        }
    }
}

// Contact nodes: the node adjoint becomes the adjoint of v*, m lam, and the
// solve's own dependence on the node mass (M (v - v*) in its optimality
// condition) gives dL/dm = -lam . (v - v*), kept in the fourth component for
// the grid update's reverse pass.
__global__ void __launch_bounds__(256)
k_cadj_vstar(const DevCounters* cnt, const int* __restrict__ s_node, const SlotRec* __restrict__ srec,
             const double3* __restrict__ lam, const float4* __restrict__ vel, const float4* __restrict__ vstar,
             float4* __restrict__ gbar) {
    const long long ns = cnt->n_slots;
    for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < ns; s += (long long)gridDim.x * blockDim.x) {
        const double m = srec[s].m;
        const double3 l = lam[s];
        const long long n = s_node[s];
        const float4 v = vel[n], vs = vstar[n];
        const double mb = -(l.x * ((double)v.x - vs.x) + l.y * ((double)v.y - vs.y) + l.z * ((double)v.z - vs.z));
        gbar[n] = make_float4((float)(m * l.x), (float)(m * l.y), (float)(m * l.z), (float)mb);
    }
}

hipError_t launch_cadj_start(const Work& w, double h, const float4* vel, hipStream_t s) {
    const DevCounters* cnt = w.cnt;
    hipLaunchKernelGGL(k_cadj_vc, dim3(256), dim3(256), 0, s, cnt, w.cap_c, w.c_rec, w.c_st, w.s_node, vel, w.c_dyn);
    double3* V = reinterpret_cast<double3*>(w.cg_vec);
    const size_t S = w.cap_s;
    hipLaunchKernelGGL(k_cadj_start, dim3(256), dim3(256), 0, s, cnt, h, w.c_rec, w.c_dyn, w.s_node, w.s_beg,
                       w.e_ent, w.s_rec, w.gbar, w.cg_pinv, V, V + S, V + 2 * S, V + 3 * S, w.cg_sc);
    return hipGetLastError();
}

hipError_t launch_cg_iteration(const Work& w, double h, hipStream_t s) {
    const DevCounters* cnt = w.cnt;
    double3* V = reinterpret_cast<double3*>(w.cg_vec);
    const size_t S = w.cap_s;
    double3 *lam = V, *r = V + S, *z = V + 2 * S, *p = V + 3 * S, *hp = V + 4 * S;
    hipLaunchKernelGGL(k_cg_q, dim3(256), dim3(256), 0, s, cnt, w.cap_c, h, w.c_rec, w.c_dyn, w.c_st, p,
                       reinterpret_cast<double3*>(w.cg_q));
    hipLaunchKernelGGL(k_cg_hp, dim3(256), dim3(256), 0, s, cnt, w.s_beg, w.e_ent, w.s_rec, p,
                       reinterpret_cast<const double3*>(w.cg_q), hp, w.cg_sc);
    hipLaunchKernelGGL(k_cg_update, dim3(256), dim3(256), 0, s, cnt, w.cg_pinv, p, hp, lam, r, z, w.cg_sc);
    hipLaunchKernelGGL(k_cg_dir, dim3(256), dim3(256), 0, s, cnt, z, p, w.cg_sc);
    hipLaunchKernelGGL(k_cg_next, dim3(1), dim3(1), 0, s, w.cg_sc);
    return hipGetLastError();
}

hipError_t launch_cadj_finish(const Work& w, double h, const TapeStep& t, const float4* vel, float* cx, float* cv,
                              double* rg, hipStream_t s) {
    const DevCounters* cnt = w.cnt;
    const double3* lam = reinterpret_cast<const double3*>(w.cg_vec);
    hipLaunchKernelGGL(k_cadj_params, dim3(256), dim3(256), 0, s, cnt, w.cap_c, w.P, h, w.envs, w.rigids, w.c_rec,
                       w.c_dyn, w.c_st, w.c_pid, w.c_rid, w.c_env, w.s_node, vel, lam, t.x, t.v, cx, cv, rg);
    hipLaunchKernelGGL(k_cadj_vstar, dim3(256), dim3(256), 0, s, cnt, w.s_node, w.s_rec, lam, vel, t.vstar, w.gbar);
    return hipGetLastError();
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

hipError_t launch_p2g_adj(const Work& w, const TapeStep& t, const float4* gbar, const float* cx, const float* cv,
                          float* ax, float* av, float* aQ, hipStream_t s) {
    const unsigned blocks = (unsigned)((w.P + 255) / 256);
    hipLaunchKernelGGL(k_p2g_adj, dim3(blocks), dim3(256), 0, s, w.P, w.envs, w.n_envs, t.x, t.v, t.Q, gbar, cx, cv,
                       ax, av, aQ);
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
