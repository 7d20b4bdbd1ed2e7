/*
 * oracle_mpm.c -- FP64 CPU oracle of one MPM substep coupled to rigid bodies
 * (arXiv 2503.05046). TEST INFRASTRUCTURE: loaded only by the test suite, the
 * smoke check and the benchmark's CPU-baseline leg; never by the product path.
 * Shares no code with the GPU library.
 *
 * Build: gcc -O2 -ffp-contract=off -shared -fPIC oracle_mpm.c -lm
 * (no fused multiply-add, no fast-math: the float32 cell-key routine must be
 * plain IEEE binary32 arithmetic, and every double step is rounded as written).
 *
 * Readings of points the paper leaves open (each is marked READING below):
 *  R1  lagged contact model (Sec. IV-B defers to Castro et al. 2023): compliant
 *      normal impulse h*k*(phi0 - h*vn)_+ * (1 - d*vn)_+ and regularised
 *      Coulomb friction with the normal impulse n0 lagged at the particle's
 *      substep-start velocity.
 *  R2  Algorithm 1 starts from the free-motion velocity v* (the grid is rebuilt
 *      every substep; strong convexity makes the optimum independent of it).
 *  R3  returned impulse on MPM is gamma = -dl_c/dv_c (Sec. IV-B; the sign in
 *      the return line of Algorithm 1 is read as a typo).
 *  R4  scaled norms of the stopping test use D = M^-1/2: |grad~|^2 =
 *      sum |g_i|^2/m_i, |p~|^2 = sum m_i |v_i|^2 over all active nodes,
 *      |j~|^2 = sum |j_i|^2/m_i.
 *  R5  line search: safeguarded 1-D Newton on phi'(alpha) with bisection
 *      fallback inside a bracket found by doubling from alpha = 1.
 *  R6  "diagonal terms" of the Hessian = the 3x3 diagonal blocks (Sec. IV-C).
 *  R7  contacts registered for sdf(x_p) < 0 at substep start against the pose
 *      frozen at the start of the host step; bias b = -R_c^T v_rigid(x_p)
 *      evaluated at the current particle position.
 *  R8  free-motion forces at the current substep state (standard explicit MPM,
 *      Sec. V-A), MLS-MPM = APIC transfer with D^-1 = 4/dx^2 and the stress
 *      folded into the affine term.
 *  R9  elastic model: fixed-corotated; granular model: Hencky elasticity with a
 *      Drucker-Prager return map, zero cohesion, no hardening.
 *  R10 boundary: slip/separate in a 3-node band at every grid face, applied to
 *      the free-motion velocity before the contact solve.
 */
#include "oracle_mpm.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* 3x3 helpers, row-major                                              */
/* ------------------------------------------------------------------ */
static void mat_mul(const double A[9], const double B[9], double Cm[9]) {
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[r * 3 + k] * B[k * 3 + c];
            Cm[r * 3 + c] = s;
        }
}
static void mat_mul_bt(const double A[9], const double B[9], double Cm[9]) { /* A B^T */
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[r * 3 + k] * B[c * 3 + k];
            Cm[r * 3 + c] = s;
        }
}
static void mat_vec(const double A[9], const double x[3], double y[3]) {
    for (int r = 0; r < 3; ++r) y[r] = A[r * 3] * x[0] + A[r * 3 + 1] * x[1] + A[r * 3 + 2] * x[2];
}
static void mat_tvec(const double A[9], const double x[3], double y[3]) { /* A^T x */
    for (int c = 0; c < 3; ++c) y[c] = A[c] * x[0] + A[3 + c] * x[1] + A[6 + c] * x[2];
}
static double mat_det(const double A[9]) {
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}
static void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* ------------------------------------------------------------------ */
/* Quadratic B-spline stencil (MLS-MPM, Sec. IV-B / V-A)               */
/* ------------------------------------------------------------------ */
void oracle_stencil(const oracle_env* env, const double xp[3], int base[3], double w[27],
                    double dpos[81]) {
    double wa[3][3], fa[3];
    for (int a = 0; a < 3; ++a) {
        double t = (xp[a] - env->origin[a]) / env->dx;
        double b = floor(t - 0.5);
        double f = t - b; /* in [0.5, 1.5) */
        base[a] = (int)b;
        fa[a] = f;
        wa[a][0] = 0.5 * (1.5 - f) * (1.5 - f);
        wa[a][1] = 0.75 - (f - 1.0) * (f - 1.0);
        wa[a][2] = 0.5 * (f - 0.5) * (f - 0.5);
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c) {
                int o = (a * 3 + b) * 3 + c;
                w[o] = wa[0][a] * wa[1][b] * wa[2][c];
                dpos[3 * o + 0] = ((double)a - fa[0]) * env->dx;
                dpos[3 * o + 1] = ((double)b - fa[1]) * env->dx;
                dpos[3 * o + 2] = ((double)c - fa[2]) * env->dx;
            }
}

static long node_index(const oracle_env* env, int i, int j, int k) {
    return (long)i + (long)env->nx * ((long)j + (long)env->ny * (long)k);
}

static void stencil_nodes(const oracle_env* env, const int base[3], long nodes[27]) {
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c)
                nodes[(a * 3 + b) * 3 + c] = node_index(env, base[0] + a, base[1] + b, base[2] + c);
}

static int base_in_domain(const oracle_env* env, const int base[3]) {
    const int n[3] = {env->nx, env->ny, env->nz};
    for (int a = 0; a < 3; ++a)
        if (base[a] < 0 || base[a] > n[a] - 3) return 0;
    return 1;
}

/* ------------------------------------------------------------------ */
/* Cell keys in IEEE binary32 and the stable cell-major order          */
/* ------------------------------------------------------------------ */
void oracle_cell_keys_f32(int P, const float* xs, const float origin[3], float inv_dx, int nx,
                          int ny, int nz, unsigned int* keys) {
    const int n[3] = {nx, ny, nz};
    const unsigned tiles[3] = {(unsigned)(nx + 3) / 4u, (unsigned)(ny + 3) / 4u, (unsigned)(nz + 3) / 4u};
    for (int p = 0; p < P; ++p) {
        int b[3];
        for (int a = 0; a < 3; ++a) {
            float d = xs[(long)a * P + p] - origin[a];
            float t = d * inv_dx;
            float u = t - 0.5f;
            int bi = (int)floorf(u);
            if (bi < 0) bi = 0;
            if (bi > n[a] - 3) bi = n[a] - 3;
            b[a] = bi;
        }
        unsigned tile = ((unsigned)b[0] >> 2) +
                        tiles[0] * (((unsigned)b[1] >> 2) + tiles[1] * ((unsigned)b[2] >> 2));
        unsigned cell = ((unsigned)b[0] & 3u) | (((unsigned)b[1] & 3u) << 2) | (((unsigned)b[2] & 3u) << 4);
        keys[p] = (tile << 6) | cell;
    }
}

static const unsigned int* g_sort_keys;
static int cmp_key_index(const void* pa, const void* pb) {
    int a = *(const int*)pa, b = *(const int*)pb;
    unsigned ka = g_sort_keys[a], kb = g_sort_keys[b];
    if (ka != kb) return ka < kb ? -1 : 1;
    return a < b ? -1 : (a > b ? 1 : 0);
}
void oracle_stable_order(int P, const unsigned int* keys, int* perm) {
    for (int i = 0; i < P; ++i) perm[i] = i;
    g_sort_keys = keys;
    qsort(perm, (size_t)P, sizeof(int), cmp_key_index);
    g_sort_keys = NULL;
}

/* ------------------------------------------------------------------ */
/* 3x3 SVD by one-sided (Hestenes) Jacobi, iterated to convergence     */
/* F = U diag(S) V^T with det U = det V = +1, S sorted by decreasing   */
/* magnitude, the last one carrying the sign of det F.                 */
/* ------------------------------------------------------------------ */
void oracle_svd3(const double F[9], double U[9], double S[3], double V[9]) {
    double B[9], Vm[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    memcpy(B, F, sizeof(B));
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int pair = 0; pair < 3; ++pair) {
            int p = pair == 2 ? 1 : 0, q = pair == 0 ? 1 : 2;
            double al = 0, be = 0, ga = 0;
            for (int r = 0; r < 3; ++r) {
                al += B[r * 3 + p] * B[r * 3 + p];
                be += B[r * 3 + q] * B[r * 3 + q];
                ga += B[r * 3 + p] * B[r * 3 + q];
            }
            if (ga == 0.0) continue;
            double rel = fabs(ga) / sqrt(al * be);
            if (rel > off) off = rel;
            if (rel < 1e-17) continue;
            double zeta = (be - al) / (2.0 * ga);
            double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
            for (int r = 0; r < 3; ++r) {
                double bp = B[r * 3 + p], bq = B[r * 3 + q];
                B[r * 3 + p] = c * bp - s * bq;
                B[r * 3 + q] = s * bp + c * bq;
                double vp = Vm[r * 3 + p], vq = Vm[r * 3 + q];
                Vm[r * 3 + p] = c * vp - s * vq;
                Vm[r * 3 + q] = s * vp + c * vq;
            }
        }
        if (off < 1e-16) break;
    }
    /* column norms, sort decreasing */
    double nrm[3];
    int order[3] = {0, 1, 2};
    for (int k = 0; k < 3; ++k)
        nrm[k] = sqrt(B[k] * B[k] + B[3 + k] * B[3 + k] + B[6 + k] * B[6 + k]);
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2 - i; ++j)
            if (nrm[order[j]] < nrm[order[j + 1]]) {
                int tmp = order[j];
                order[j] = order[j + 1];
                order[j + 1] = tmp;
            }
    double Bs[9], Vs[9];
    for (int k = 0; k < 3; ++k)
        for (int r = 0; r < 3; ++r) {
            Bs[r * 3 + k] = B[r * 3 + order[k]];
            Vs[r * 3 + k] = Vm[r * 3 + order[k]];
        }
    if (mat_det(Vs) < 0) {
        for (int r = 0; r < 3; ++r) {
            Vs[r * 3 + 2] = -Vs[r * 3 + 2];
            Bs[r * 3 + 2] = -Bs[r * 3 + 2];
        }
    }
    double b0[3] = {Bs[0], Bs[3], Bs[6]}, b1[3] = {Bs[1], Bs[4], Bs[7]}, b2[3] = {Bs[2], Bs[5], Bs[8]};
    double u0[3], u1[3], u2[3];
    double n0 = sqrt(dot3(b0, b0));
    if (n0 > 1e-300) {
        for (int r = 0; r < 3; ++r) u0[r] = b0[r] / n0;
    } else {
        u0[0] = 1; u0[1] = 0; u0[2] = 0;
    }
    double pr = dot3(u0, b1);
    double tmp[3] = {b1[0] - pr * u0[0], b1[1] - pr * u0[1], b1[2] - pr * u0[2]};
    double n1 = sqrt(dot3(tmp, tmp));
    if (n1 > 1e-300 * (n0 + 1.0)) {
        for (int r = 0; r < 3; ++r) u1[r] = tmp[r] / n1;
    } else { /* any unit vector orthogonal to u0 */
        int ax = fabs(u0[0]) < fabs(u0[1]) ? (fabs(u0[0]) < fabs(u0[2]) ? 0 : 2) : (fabs(u0[1]) < fabs(u0[2]) ? 1 : 2);
        double e[3] = {0, 0, 0};
        e[ax] = 1;
        double pe = dot3(e, u0);
        for (int r = 0; r < 3; ++r) tmp[r] = e[r] - pe * u0[r];
        double ne = sqrt(dot3(tmp, tmp));
        for (int r = 0; r < 3; ++r) u1[r] = tmp[r] / ne;
    }
    cross3(u0, u1, u2);
    S[0] = dot3(u0, b0);
    S[1] = dot3(u1, b1);
    S[2] = dot3(u2, b2);
    for (int r = 0; r < 3; ++r) {
        U[r * 3 + 0] = u0[r];
        U[r * 3 + 1] = u1[r];
        U[r * 3 + 2] = u2[r];
    }
    memcpy(V, Vs, sizeof(Vs));
}

/* ------------------------------------------------------------------ */
/* Constitutive models (READING R9)                                    */
/* ------------------------------------------------------------------ */
static void lame(const oracle_env* env, double* mu, double* la) {
    *mu = env->E / (2.0 * (1.0 + env->nu));
    *la = env->E * env->nu / ((1.0 + env->nu) * (1.0 - 2.0 * env->nu));
}

void oracle_kirchhoff(const oracle_env* env, const double F[9], double tau[9]) {
    double mu, la;
    lame(env, &mu, &la);
    double U[9], S[3], V[9];
    oracle_svd3(F, U, S, V);
    if (env->material == OR_FIXED_COROTATED) {
        /* tau = 2 mu (F - R) F^T + la (J - 1) J I, R = U V^T */
        double R[9], FmR[9], A[9];
        mat_mul_bt(U, V, R);
        for (int i = 0; i < 9; ++i) FmR[i] = F[i] - R[i];
        mat_mul_bt(FmR, F, A);
        double J = S[0] * S[1] * S[2];
        for (int i = 0; i < 9; ++i) tau[i] = 2.0 * mu * A[i];
        for (int i = 0; i < 3; ++i) tau[i * 4] += la * (J - 1.0) * J;
    } else {
        /* Hencky: tau = U (2 mu eps + la tr(eps) I) U^T, eps = ln sigma */
        double eps[3], tr = 0.0;
        for (int k = 0; k < 3; ++k) {
            eps[k] = log(S[k] > 1e-6 ? S[k] : 1e-6);
            tr += eps[k];
        }
        double D[3];
        for (int k = 0; k < 3; ++k) D[k] = 2.0 * mu * eps[k] + la * tr;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double s = 0.0;
                for (int k = 0; k < 3; ++k) s += U[r * 3 + k] * D[k] * U[c * 3 + k];
                tau[r * 3 + c] = s;
            }
    }
}

int oracle_dp_project(const oracle_env* env, double F[9]) {
    double mu, la;
    lame(env, &mu, &la);
    double sphi = sin(env->friction_angle * M_PI / 180.0);
    double alpha = sqrt(2.0 / 3.0) * 2.0 * sphi / (3.0 - sphi);
    double U[9], S[3], V[9];
    oracle_svd3(F, U, S, V);
    double eps[3], tr = 0.0;
    for (int k = 0; k < 3; ++k) {
        eps[k] = log(S[k] > 1e-6 ? S[k] : 1e-6);
        tr += eps[k];
    }
    int projected = 0;
    if (tr >= 0.0) { /* tension: project to the cone tip */
        eps[0] = eps[1] = eps[2] = 0.0;
        projected = 1;
    } else {
        double dev[3], nd = 0.0;
        for (int k = 0; k < 3; ++k) {
            dev[k] = eps[k] - tr / 3.0;
            nd += dev[k] * dev[k];
        }
        nd = sqrt(nd);
        double dgamma = nd + (3.0 * la + 2.0 * mu) / (2.0 * mu) * tr * alpha;
        if (dgamma > 0.0) {
            for (int k = 0; k < 3; ++k) eps[k] -= dgamma * dev[k] / nd;
            projected = 1;
        }
    }
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += U[r * 3 + k] * exp(eps[k]) * V[c * 3 + k];
            F[r * 3 + c] = s;
        }
    return projected;
}

/* ------------------------------------------------------------------ */
/* Contact model (READING R1)                                          */
/* ------------------------------------------------------------------ */
double oracle_normal_impulse(double vn, double phi0, double k, double d, double h) {
    double a = phi0 - h * vn, b = 1.0 - d * vn;
    if (a <= 0.0 || b <= 0.0) return 0.0;
    return h * k * a * b;
}

/* Phi(s) = phi0 s - (h + d phi0) s^2 / 2 + h d s^3 / 3, so that
 * h k (Phi(vbar) - Phi(vn)) integrates the normal impulse from vn to vbar. */
static double normal_antideriv(double s, double phi0, double d, double h) {
    return phi0 * s - 0.5 * (h + d * phi0) * s * s + h * d * s * s * s / 3.0;
}

double oracle_contact_model(const double vc[3], double phi0, double n0, double mu, double k,
                            double d, double eps_s, double h, double gamma[3], double G[9]) {
    for (int i = 0; i < 9; ++i) G[i] = 0.0;
    double ell = 0.0;
    /* normal part */
    double vn = vc[2];
    double vbar = phi0 / h;
    if (d > 0.0 && 1.0 / d < vbar) vbar = 1.0 / d;
    if (vn < vbar) {
        gamma[2] = h * k * (phi0 - h * vn) * (1.0 - d * vn);
        ell += h * k * (normal_antideriv(vbar, phi0, d, h) - normal_antideriv(vn, phi0, d, h));
        G[8] = h * k * (h * (1.0 - d * vn) + d * (phi0 - h * vn));
    } else {
        gamma[2] = 0.0;
    }
    /* regularised Coulomb friction with lagged normal impulse n0 */
    double s = sqrt(vc[0] * vc[0] + vc[1] * vc[1] + eps_s * eps_s);
    double c = mu * n0;
    ell += c * (s - eps_s);
    gamma[0] = -c * vc[0] / s;
    gamma[1] = -c * vc[1] / s;
    double cs = c / s;
    G[0] = cs * (1.0 - vc[0] * vc[0] / (s * s));
    G[1] = G[3] = -cs * vc[0] * vc[1] / (s * s);
    G[4] = cs * (1.0 - vc[1] * vc[1] / (s * s));
    return ell;
}

/* ------------------------------------------------------------------ */
/* Rigid primitives and contact frames                                 */
/* ------------------------------------------------------------------ */
double oracle_sdf(const oracle_rigid* r, const double x[3], double n[3]) {
    double d[3] = {x[0] - r->t[0], x[1] - r->t[1], x[2] - r->t[2]};
    double p[3], nb[3];
    mat_tvec(r->R, d, p);
    double s;
    if (r->shape == OR_HALF_SPACE) {
        s = dot3(r->normal, p) - r->offset;
        nb[0] = r->normal[0];
        nb[1] = r->normal[1];
        nb[2] = r->normal[2];
    } else {
        double q[3], qp[3], mx = -INFINITY;
        int kstar = 0, outside = 0;
        for (int a = 0; a < 3; ++a) {
            q[a] = fabs(p[a]) - r->half[a];
            qp[a] = q[a] > 0.0 ? q[a] : 0.0;
            if (q[a] > 0.0) outside = 1;
            if (q[a] > mx) {
                mx = q[a];
                kstar = a;
            }
        }
        double no = sqrt(dot3(qp, qp));
        s = no + (mx < 0.0 ? mx : 0.0);
        if (outside) {
            for (int a = 0; a < 3; ++a) nb[a] = qp[a] * (p[a] >= 0.0 ? 1.0 : -1.0) / no;
        } else {
            nb[0] = nb[1] = nb[2] = 0.0;
            nb[kstar] = p[kstar] >= 0.0 ? 1.0 : -1.0;
        }
    }
    mat_vec(r->R, nb, n);
    return s;
}

void oracle_contact_frame(int basis, const double n[3], double Rc[9]) {
    double t1[3], t2[3];
    if (basis == 0) { /* Duff, Burgess, Christensen, Hery, Kensler, Liani, Villemin 2017 */
        double sg = n[2] >= 0.0 ? 1.0 : -1.0;
        double a = -1.0 / (sg + n[2]);
        double b = n[0] * n[1] * a;
        t1[0] = 1.0 + sg * n[0] * n[0] * a;
        t1[1] = sg * b;
        t1[2] = -sg * n[0];
        t2[0] = b;
        t2[1] = sg + n[1] * n[1] * a;
        t2[2] = -n[1];
    } else { /* project the least-aligned axis onto the tangent plane */
        int ax = 0;
        for (int a = 1; a < 3; ++a)
            if (fabs(n[a]) < fabs(n[ax])) ax = a;
        double e[3] = {0, 0, 0};
        e[ax] = 1.0;
        double pe = dot3(e, n);
        for (int r = 0; r < 3; ++r) t1[r] = e[r] - pe * n[r];
        double nt = sqrt(dot3(t1, t1));
        for (int r = 0; r < 3; ++r) t1[r] /= nt;
        cross3(n, t1, t2);
    }
    for (int r = 0; r < 3; ++r) {
        Rc[r * 3 + 0] = t1[r];
        Rc[r * 3 + 1] = t2[r];
        Rc[r * 3 + 2] = n[r];
    }
}

void oracle_advance_pose(oracle_rigid* r, double dt) {
    for (int a = 0; a < 3; ++a) r->t[a] += dt * r->V[a];
    double wn = sqrt(dot3(r->w, r->w));
    double th = wn * dt;
    if (th == 0.0) return;
    double kx = r->w[0] / wn, ky = r->w[1] / wn, kz = r->w[2] / wn;
    double K[9] = {0, -kz, ky, kz, 0, -kx, -ky, kx, 0};
    double K2[9], Rot[9], Rn[9];
    mat_mul(K, K, K2);
    for (int i = 0; i < 9; ++i) Rot[i] = sin(th) * K[i] + (1.0 - cos(th)) * K2[i];
    Rot[0] += 1.0;
    Rot[4] += 1.0;
    Rot[8] += 1.0;
    mat_mul(Rot, r->R, Rn);
    memcpy(r->R, Rn, sizeof(Rn));
}

/* ------------------------------------------------------------------ */
/* Algorithm 1: quasi-Newton with block-diagonal Hessian and exact     */
/* line search (Sec. IV-C, V-B; READINGS R2-R6)                        */
/* ------------------------------------------------------------------ */
typedef struct {
    const oracle_env* env;
    int n_c;
    const double *phi0, *n0, *mu;
    const double *vc, *uc;
    double A, B;
} ls_problem;

/* phi'(alpha) and phi''(alpha) of phi(alpha) = l_p(v + alpha dv) */
static double ls_deriv(const ls_problem* L, double alpha, double* d2) {
    const oracle_env* e = L->env;
    double d1 = L->A * alpha + L->B;
    double dd = L->A;
    for (int c = 0; c < L->n_c; ++c) {
        double v[3], g[3], G[9], Gu[3];
        for (int a = 0; a < 3; ++a) v[a] = L->vc[3 * c + a] + alpha * L->uc[3 * c + a];
        oracle_contact_model(v, L->phi0[c], L->n0[c], L->mu[c], e->k, e->d, e->eps_s, e->h, g, G);
        const double* u = &L->uc[3 * c];
        d1 -= dot3(g, u);
        mat_vec(G, u, Gu);
        dd += dot3(u, Gu);
    }
    *d2 = dd;
    return d1;
}

static double line_search(const ls_problem* L, double d0, int max_steps, int* steps) {
    /* bracket [lo, hi] with phi'(lo) < 0 <= phi'(hi) */
    double lo = 0.0, hi = 1.0, dd;
    double dh = ls_deriv(L, hi, &dd);
    ++*steps;
    for (int n = 0; dh < 0.0 && n < 60; ++n) {
        lo = hi;
        hi *= 2.0;
        dh = ls_deriv(L, hi, &dd);
        ++*steps;
    }
    if (dh < 0.0) return hi;
    double a = hi, da = dh, dda = dd, prev = INFINITY;
    for (int it = 0; it < max_steps; ++it) {
        if (fabs(da) <= 1e-10 * fabs(d0)) break;
        if (da < 0.0) lo = a; else hi = a;
        if (hi - lo <= 1e-12 * hi) break;
        double an = a - da / dda;
        if (!(an > lo && an < hi) || fabs(da) > 0.5 * prev) an = 0.5 * (lo + hi);
        prev = fabs(da);
        a = an;
        da = ls_deriv(L, a, &dda);
        ++*steps;
    }
    return a;
}

static void chol3_solve(const double H[9], const double rhs[3], double x[3]) {
    double l00 = sqrt(H[0]);
    double l10 = H[3] / l00, l20 = H[6] / l00;
    double l11 = sqrt(H[4] - l10 * l10);
    double l21 = (H[7] - l20 * l10) / l11;
    double l22 = sqrt(H[8] - l20 * l20 - l21 * l21);
    double y0 = rhs[0] / l00;
    double y1 = (rhs[1] - l10 * y0) / l11;
    double y2 = (rhs[2] - l20 * y0 - l21 * y1) / l22;
    x[2] = y2 / l22;
    x[1] = (y1 - l21 * x[2]) / l11;
    x[0] = (y0 - l10 * x[1] - l20 * x[2]) / l00;
}

/* Algorithm 1 over n nodes; p2_rest is the part of |p~|^2 = sum m |v|^2 that
 * comes from active nodes outside the problem (nodes no contact stencil
 * touches, whose iterate stays at v* exactly: their gradient is zero at v*,
 * so their Newton direction is zero; reading R3). */
static int qn_solve_core(const oracle_env* env, int n, const double* m, const double* vstar, int nc,
                         const int* nodes, const double* w, const double* Rc, const double* b,
                         const double* phi0, const double* n0, const double* mu, double* v,
                         double* gamma_out, oracle_substep_stats* st, double* lp_hist,
                         double p2_rest) {
    double* vc = (double*)malloc(sizeof(double) * 3 * (size_t)(nc > 0 ? nc : 1));
    double* uc = (double*)malloc(sizeof(double) * 3 * (size_t)(nc > 0 ? nc : 1));
    double* gam = (double*)malloc(sizeof(double) * 3 * (size_t)(nc > 0 ? nc : 1));
    double* Gc = (double*)malloc(sizeof(double) * 9 * (size_t)(nc > 0 ? nc : 1));
    double* j = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    double* g = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    double* H = (double*)malloc(sizeof(double) * 9 * (size_t)(n > 0 ? n : 1));
    double* dv = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    int iter = 0, ls_steps = 0, converged = 0, status = OR_OK;
    double res = 0.0, thr = 0.0, pn = 0.0, jn = 0.0;
    for (;;) {
        /* contact velocities v_c = R_c^T (sum_i w_ic v_i) + b_c and the model */
        double lc = 0.0;
        for (int c = 0; c < nc; ++c) {
            double s[3] = {0, 0, 0};
            for (int o = 0; o < 27; ++o) {
                const double* vi = &v[3 * (size_t)nodes[27 * c + o]];
                for (int a = 0; a < 3; ++a) s[a] += w[27 * c + o] * vi[a];
            }
            mat_tvec(&Rc[9 * c], s, &vc[3 * c]);
            for (int a = 0; a < 3; ++a) vc[3 * c + a] += b[3 * c + a];
            lc += oracle_contact_model(&vc[3 * c], phi0[c], n0[c], mu[c], env->k, env->d,
                                       env->eps_s, env->h, &gam[3 * c], &Gc[9 * c]);
        }
        if (lp_hist) {
            double lm = 0.0;
            for (int i = 0; i < n; ++i)
                for (int a = 0; a < 3; ++a) {
                    double dvv = v[3 * i + a] - vstar[3 * i + a];
                    lm += 0.5 * m[i] * dvv * dvv;
                }
            lp_hist[iter] = lm + lc;
        }
        /* j_i = sum_c w_ic R_c gamma_c (Eq. (9) with gamma = -dl_c/dv_c) */
        memset(j, 0, sizeof(double) * 3 * (size_t)n);
        for (int c = 0; c < nc; ++c) {
            double rg[3];
            mat_vec(&Rc[9 * c], &gam[3 * c], rg);
            for (int o = 0; o < 27; ++o) {
                double* ji = &j[3 * (size_t)nodes[27 * c + o]];
                for (int a = 0; a < 3; ++a) ji[a] += w[27 * c + o] * rg[a];
            }
        }
        double grad2 = 0.0, p2 = p2_rest, j2 = 0.0;
        for (int i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) {
                double gi = m[i] * (v[3 * i + a] - vstar[3 * i + a]) - j[3 * i + a];
                g[3 * i + a] = gi;
                grad2 += gi * gi / m[i];
                p2 += m[i] * v[3 * i + a] * v[3 * i + a];
                j2 += j[3 * i + a] * j[3 * i + a] / m[i];
            }
        res = sqrt(grad2);
        pn = sqrt(p2);
        jn = sqrt(j2);
        thr = env->eps_a + env->eps_r * (pn > jn ? pn : jn);
        if (res < thr) {
            converged = 1;
            break;
        }
        if (iter >= env->max_iter) {
            status = OR_NOCONV;
            break;
        }
        /* block-diagonal Hessian H_i = m_i I + sum_c w_ic^2 R_c G_c R_c^T (Eq. (10)) */
        for (int i = 0; i < n; ++i) {
            for (int q = 0; q < 9; ++q) H[9 * i + q] = 0.0;
            H[9 * i + 0] = H[9 * i + 4] = H[9 * i + 8] = m[i];
        }
        for (int c = 0; c < nc; ++c) {
            double RG[9], RGRt[9];
            mat_mul(&Rc[9 * c], &Gc[9 * c], RG);
            mat_mul_bt(RG, &Rc[9 * c], RGRt);
            for (int o = 0; o < 27; ++o) {
                double ww = w[27 * c + o] * w[27 * c + o];
                double* Hi = &H[9 * (size_t)nodes[27 * c + o]];
                for (int q = 0; q < 9; ++q) Hi[q] += ww * RGRt[q];
            }
        }
        /* Newton direction dv_i = -H_i^-1 g_i by 3x3 Cholesky */
        for (int i = 0; i < n; ++i) {
            double rhs[3] = {-g[3 * i], -g[3 * i + 1], -g[3 * i + 2]};
            chol3_solve(&H[9 * i], rhs, &dv[3 * i]);
        }
        /* exact line search on alpha */
        double A = 0.0, B = 0.0, d0 = 0.0;
        for (int i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) {
                A += m[i] * dv[3 * i + a] * dv[3 * i + a];
                B += m[i] * dv[3 * i + a] * (v[3 * i + a] - vstar[3 * i + a]);
                d0 += g[3 * i + a] * dv[3 * i + a];
            }
        for (int c = 0; c < nc; ++c) {
            double s[3] = {0, 0, 0};
            for (int o = 0; o < 27; ++o) {
                const double* di = &dv[3 * (size_t)nodes[27 * c + o]];
                for (int a = 0; a < 3; ++a) s[a] += w[27 * c + o] * di[a];
            }
            mat_tvec(&Rc[9 * c], s, &uc[3 * c]);
        }
        if (!(d0 < 0.0)) { /* no descent left at this precision */
            status = OR_NOCONV;
            break;
        }
        ls_problem L = {env, nc, phi0, n0, mu, vc, uc, A, B};
        double alpha = line_search(&L, d0, env->ls_max_iter, &ls_steps);
        for (int i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) v[3 * i + a] += alpha * dv[3 * i + a];
        ++iter;
    }
    if (gamma_out) memcpy(gamma_out, gam, sizeof(double) * 3 * (size_t)nc);
    if (st) {
        st->iterations = iter;
        st->ls_steps = ls_steps;
        st->converged = converged;
        st->residual = res;
        st->threshold = thr;
        st->p_norm = pn;
        st->j_norm = jn;
    }
    free(vc); free(uc); free(gam); free(Gc); free(j); free(g); free(H); free(dv);
    return status;
}

int oracle_qn_solve(const oracle_env* env, int n, const double* m, const double* vstar, int nc,
                    const int* nodes, const double* w, const double* Rc, const double* b,
                    const double* phi0, const double* n0, const double* mu, double* v,
                    double* gamma_out, oracle_substep_stats* st, double* lp_hist) {
    return qn_solve_core(env, n, m, vstar, nc, nodes, w, Rc, b, phi0, n0, mu, v, gamma_out, st, lp_hist, 0.0);
}

/* ------------------------------------------------------------------ */
/* One substep                                                         */
/* ------------------------------------------------------------------ */
typedef struct {
    long n_nodes;
    double *m, *mom, *vgrid;   /* dense grid: mass, momentum, velocity */
    int n_act;
    long* act;                 /* active node list (m > 0), ascending */
    int* act_of;               /* dense -> active index, -1 if inactive */
    int nc, cap;
    int *cp, *cr;              /* contact particle and rigid */
    int* cnodes;               /* 27 active-node indices per contact */
    double *cw, *cR, *cb, *cphi, *cn0, *cmu;
} frame_t;

static void frame_free(frame_t* f) {
    free(f->m); free(f->mom); free(f->vgrid); free(f->act); free(f->act_of);
    free(f->cp); free(f->cr); free(f->cnodes); free(f->cw); free(f->cR); free(f->cb);
    free(f->cphi); free(f->cn0); free(f->cmu);
}

static void contact_push(frame_t* f) {
    if (f->nc < f->cap) return;
    f->cap = f->cap ? 2 * f->cap : 256;
    f->cp = (int*)realloc(f->cp, sizeof(int) * f->cap);
    f->cr = (int*)realloc(f->cr, sizeof(int) * f->cap);
    f->cnodes = (int*)realloc(f->cnodes, sizeof(int) * 27 * f->cap);
    f->cw = (double*)realloc(f->cw, sizeof(double) * 27 * f->cap);
    f->cR = (double*)realloc(f->cR, sizeof(double) * 9 * f->cap);
    f->cb = (double*)realloc(f->cb, sizeof(double) * 3 * f->cap);
    f->cphi = (double*)realloc(f->cphi, sizeof(double) * f->cap);
    f->cn0 = (double*)realloc(f->cn0, sizeof(double) * f->cap);
    f->cmu = (double*)realloc(f->cmu, sizeof(double) * f->cap);
}

/* P2G, grid update and contact registration: everything before Algorithm 1. */
static int build_frame(const oracle_env* env, const oracle_rigid* rigid, int n_rigid, int P,
                       const double* x, const double* v, const double* F, const double* C,
                       frame_t* fr) {
    memset(fr, 0, sizeof(*fr));
    const double D = 4.0 / (env->dx * env->dx);
    fr->n_nodes = (long)env->nx * env->ny * env->nz;
    /* domain check before touching anything */
    for (int p = 0; p < P; ++p) {
        double xp[3] = {x[p], x[(long)P + p], x[2L * P + p]};
        int base[3];
        double w[27], dpos[81];
        oracle_stencil(env, xp, base, w, dpos);
        if (!base_in_domain(env, base)) return OR_DOMAIN;
    }
    fr->m = (double*)calloc((size_t)fr->n_nodes, sizeof(double));
    fr->mom = (double*)calloc(3 * (size_t)fr->n_nodes, sizeof(double));
    fr->vgrid = (double*)calloc(3 * (size_t)fr->n_nodes, sizeof(double));
    /* P2G with the stress folded into the affine term (Eq. (6), READING R8):
     * Q_p = m_p C_p - h V0 (4/dx^2) tau_p,
     * m_i += w m_p,  p_i += w (m_p v_p + Q_p (x_i - x_p)). */
    for (int p = 0; p < P; ++p) {
        double xp[3], vp[3], Fp[9], Cp[9], tau[9], Q[9];
        for (int a = 0; a < 3; ++a) {
            xp[a] = x[(long)a * P + p];
            vp[a] = v[(long)a * P + p];
        }
        for (int q = 0; q < 9; ++q) {
            Fp[q] = F[(long)q * P + p];
            Cp[q] = C[(long)q * P + p];
        }
        oracle_kirchhoff(env, Fp, tau);
        for (int q = 0; q < 9; ++q) Q[q] = env->m_p * Cp[q] - env->h * env->V0 * D * tau[q];
        int base[3];
        long nodes[27];
        double w[27], dpos[81];
        oracle_stencil(env, xp, base, w, dpos);
        stencil_nodes(env, base, nodes);
        for (int o = 0; o < 27; ++o) {
            double qd[3];
            mat_vec(Q, &dpos[3 * o], qd);
            fr->m[nodes[o]] += w[o] * env->m_p;
            for (int a = 0; a < 3; ++a) fr->mom[3 * nodes[o] + a] += w[o] * (env->m_p * vp[a] + qd[a]);
        }
    }
    /* grid update: v* = p/m + h g, then the boundary band (READING R10) */
    fr->act_of = (int*)malloc(sizeof(int) * (size_t)fr->n_nodes);
    int n_act = 0;
    for (long i = 0; i < fr->n_nodes; ++i) {
        fr->act_of[i] = -1;
        if (fr->m[i] > 0.0) ++n_act;
    }
    fr->act = (long*)malloc(sizeof(long) * (size_t)(n_act > 0 ? n_act : 1));
    fr->n_act = 0;
    const int nn[3] = {env->nx, env->ny, env->nz};
    for (long i = 0; i < fr->n_nodes; ++i) {
        if (!(fr->m[i] > 0.0)) continue;
        fr->act_of[i] = fr->n_act;
        fr->act[fr->n_act++] = i;
        int idx[3] = {(int)(i % env->nx), (int)((i / env->nx) % env->ny), (int)(i / ((long)env->nx * env->ny))};
        for (int a = 0; a < 3; ++a) {
            double vs = fr->mom[3 * i + a] / fr->m[i] + env->h * env->gravity[a];
            if (idx[a] < 3 && vs < 0.0) vs = 0.0;
            if (idx[a] >= nn[a] - 3 && vs > 0.0) vs = 0.0;
            fr->vgrid[3 * i + a] = vs;
        }
    }
    /* contact registration (Sec. V-B, READING R7): one contact per
     * (particle, geometry) pair with the particle strictly inside */
    for (int p = 0; p < P; ++p) {
        double xp[3], vp[3];
        for (int a = 0; a < 3; ++a) {
            xp[a] = x[(long)a * P + p];
            vp[a] = v[(long)a * P + p];
        }
        for (int r = 0; r < n_rigid; ++r) {
            double nrm[3];
            double s = oracle_sdf(&rigid[r], xp, nrm);
            if (!(s < 0.0)) continue;
            contact_push(fr);
            int c = fr->nc++;
            fr->cp[c] = p;
            fr->cr[c] = r;
            double* Rc = &fr->cR[9 * c];
            oracle_contact_frame(env->basis, nrm, Rc);
            double rel[3] = {xp[0] - rigid[r].t[0], xp[1] - rigid[r].t[1], xp[2] - rigid[r].t[2]};
            double vr[3];
            cross3(rigid[r].w, rel, vr);
            for (int a = 0; a < 3; ++a) vr[a] += rigid[r].V[a];
            double bc[3];
            mat_tvec(Rc, vr, bc);
            for (int a = 0; a < 3; ++a) fr->cb[3 * c + a] = -bc[a];
            double phi0 = -s;
            fr->cphi[c] = phi0;
            double vn0 = nrm[0] * (vp[0] - vr[0]) + nrm[1] * (vp[1] - vr[1]) + nrm[2] * (vp[2] - vr[2]);
            fr->cn0[c] = oracle_normal_impulse(vn0, phi0, env->k, env->d, env->h);
            fr->cmu[c] = rigid[r].mu;
            int base[3];
            long nodes[27];
            double dpos[81];
            oracle_stencil(env, xp, base, &fr->cw[27 * c], dpos);
            stencil_nodes(env, base, nodes);
            for (int o = 0; o < 27; ++o) fr->cnodes[27 * c + o] = fr->act_of[nodes[o]];
        }
    }
    /* a zero-weight stencil node may have m = 0: give it a harmless slot by
     * pointing it at any active node with weight 0 (weights are exactly 0) */
    for (int c = 0; c < fr->nc; ++c)
        for (int o = 0; o < 27; ++o)
            if (fr->cnodes[27 * c + o] < 0) {
                fr->cnodes[27 * c + o] = 0;
                fr->cw[27 * c + o] = 0.0;
            }
    return OR_OK;
}

int oracle_substep(const oracle_env* env, const oracle_rigid* rigid, int n_rigid, int P,
                   double* x, double* v, double* F, double* C, double* impulse,
                   oracle_substep_stats* st, double* lp_hist) {
    if (env->h <= 0.0 || env->dx <= 0.0 || env->nu >= 0.5 || env->nu <= -1.0 || env->E <= 0.0)
        return OR_EINVAL;
    frame_t fr;
    int rc = build_frame(env, rigid, n_rigid, P, x, v, F, C, &fr);
    if (rc != OR_OK) {
        frame_free(&fr);
        return rc;
    }
    const double D = 4.0 / (env->dx * env->dx);
    /* Algorithm 1 (READING R3: it starts from v = v*). An active node that no
     * contact stencil touches (weight > 0) has j = 0 and g = m (v - v*) = 0 at
     * v*, so its Newton direction is zero and it keeps v = v* exactly: unless
     * env->solve_all_nodes is set, the iteration runs over the touched nodes
     * only and the others' share of |p~|^2 = sum m |v*|^2 enters as a constant
     * (the same norms and iterates; only the order of that sum differs). */
    const int n_act = fr.n_act;
    int* sub_of = (int*)malloc(sizeof(int) * (size_t)(n_act > 0 ? n_act : 1));
    int n = 0;
    for (int i = 0; i < n_act; ++i) sub_of[i] = env->solve_all_nodes ? i : -1;
    if (env->solve_all_nodes) {
        n = n_act;
    } else {
        for (int c = 0; c < fr.nc; ++c)
            for (int o = 0; o < 27; ++o)
                if (fr.cw[27 * c + o] > 0.0) sub_of[fr.cnodes[27 * c + o]] = -2;  /* touched */
        for (int i = 0; i < n_act; ++i)  /* numbered in node order */
            if (sub_of[i] == -2) sub_of[i] = n++;
    }
    int* act_node = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));  /* problem node -> active node */
    double p2_rest = 0.0;
    for (int i = 0; i < n_act; ++i) {
        if (sub_of[i] >= 0) {
            act_node[sub_of[i]] = i;
        } else {
            for (int a = 0; a < 3; ++a) p2_rest += fr.m[fr.act[i]] * fr.vgrid[3 * fr.act[i] + a] * fr.vgrid[3 * fr.act[i] + a];
        }
    }
    int* cnodes = (int*)malloc(sizeof(int) * 27 * (size_t)(fr.nc > 0 ? fr.nc : 1));
    for (int c = 0; c < fr.nc; ++c)
        for (int o = 0; o < 27; ++o) {
            /* a zero-weight stencil entry may name a node outside the problem:
             * point it at problem node 0 (its weight is exactly 0) */
            const int q = sub_of[fr.cnodes[27 * c + o]];
            cnodes[27 * c + o] = (fr.cw[27 * c + o] > 0.0 || q >= 0) ? q : 0;
        }
    double* m = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* vs = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    double* vv = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) {
        const long node = fr.act[act_node[i]];
        m[i] = fr.m[node];
        for (int a = 0; a < 3; ++a) vs[3 * i + a] = vv[3 * i + a] = fr.vgrid[3 * node + a];
    }
    double* gam = (double*)malloc(sizeof(double) * 3 * (size_t)(fr.nc > 0 ? fr.nc : 1));
    oracle_substep_stats local;
    memset(&local, 0, sizeof(local));
    int qs = qn_solve_core(env, n, m, vs, fr.nc, cnodes, fr.cw, fr.cR, fr.cb, fr.cphi,
                           fr.cn0, fr.cmu, vv, gam, &local, lp_hist, p2_rest);
    local.n_contacts = fr.nc;
    local.n_active_nodes = n_act;
    {
        char* touched = (char*)calloc((size_t)(n_act > 0 ? n_act : 1), 1);
        int cnt = 0;
        for (int c = 0; c < fr.nc; ++c)
            for (int o = 0; o < 27; ++o)
                if (fr.cw[27 * c + o] > 0.0 && !touched[fr.cnodes[27 * c + o]]) {
                    touched[fr.cnodes[27 * c + o]] = 1;
                    ++cnt;
                }
        local.n_contact_nodes = cnt;
        free(touched);
    }
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) fr.vgrid[3 * fr.act[act_node[i]] + a] = vv[3 * i + a];
    free(sub_of);
    free(act_node);
    free(cnodes);
    /* impulses on the rigid bodies: minus the impulse on MPM, Eq. (3) */
    if (impulse) {
        for (int c = 0; c < fr.nc; ++c) {
            int r = fr.cr[c], p = fr.cp[c];
            double rg[3], arm[3], tq[3];
            mat_vec(&fr.cR[9 * c], &gam[3 * c], rg);
            for (int a = 0; a < 3; ++a) arm[a] = x[(long)a * P + p] - rigid[r].t[a];
            cross3(arm, rg, tq);
            for (int a = 0; a < 3; ++a) {
                impulse[6 * r + a] -= rg[a];
                impulse[6 * r + 3 + a] -= tq[a];
            }
        }
    }
    /* G2P: v_p = sum w v_i, C_p = (4/dx^2) sum w v_i (x_i - x_p)^T,
     * F <- (I + h C_p) F, x <- x + h v_p, then the return map for sand */
    int bad = 0;
    for (int p = 0; p < P; ++p) {
        double xp[3], Fp[9];
        for (int a = 0; a < 3; ++a) xp[a] = x[(long)a * P + p];
        for (int q = 0; q < 9; ++q) Fp[q] = F[(long)q * P + p];
        int base[3];
        long nodes[27];
        double w[27], dpos[81];
        oracle_stencil(env, xp, base, w, dpos);
        stencil_nodes(env, base, nodes);
        double vp[3] = {0, 0, 0}, Cp[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int o = 0; o < 27; ++o) {
            const double* vi = &fr.vgrid[3 * nodes[o]];
            for (int a = 0; a < 3; ++a) {
                vp[a] += w[o] * vi[a];
                for (int bb = 0; bb < 3; ++bb) Cp[a * 3 + bb] += D * w[o] * vi[a] * dpos[3 * o + bb];
            }
        }
        double Af[9], Fn[9];
        for (int q = 0; q < 9; ++q) Af[q] = env->h * Cp[q];
        Af[0] += 1.0;
        Af[4] += 1.0;
        Af[8] += 1.0;
        mat_mul(Af, Fp, Fn);
        if (env->material == OR_DRUCKER_PRAGER) oracle_dp_project(env, Fn);
        for (int a = 0; a < 3; ++a) {
            x[(long)a * P + p] = xp[a] + env->h * vp[a];
            v[(long)a * P + p] = vp[a];
            if (!isfinite(vp[a])) bad = 1;
        }
        for (int q = 0; q < 9; ++q) {
            F[(long)q * P + p] = Fn[q];
            C[(long)q * P + p] = Cp[q];
            if (!isfinite(Fn[q])) bad = 1;
        }
    }
    if (st) *st = local;
    free(m); free(vs); free(vv); free(gam);
    frame_free(&fr);
    if (bad) return OR_NAN;
    return qs;
}

void oracle_integrate_dynamic(oracle_rigid* r, const double imp[6], const double g[3], double dt) {
    for (int a = 0; a < 3; ++a) r->V[a] += imp[a] / r->mass + dt * (g[a] + r->force[a] / r->mass);
    /* world inertia I_w = R diag(I) R^T and its inverse R diag(1/I) R^T */
    double Iw[9], Iinv[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s1 = 0.0, s2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                s1 += r->R[i * 3 + k] * r->inertia[k] * r->R[j * 3 + k];
                s2 += r->R[i * 3 + k] / r->inertia[k] * r->R[j * 3 + k];
            }
            Iw[i * 3 + j] = s1;
            Iinv[i * 3 + j] = s2;
        }
    double Lw[3], rhs[3];
    for (int i = 0; i < 3; ++i) Lw[i] = Iw[i * 3 + 0] * r->w[0] + Iw[i * 3 + 1] * r->w[1] + Iw[i * 3 + 2] * r->w[2];
    const double gyro[3] = {r->w[1] * Lw[2] - r->w[2] * Lw[1], r->w[2] * Lw[0] - r->w[0] * Lw[2],
                            r->w[0] * Lw[1] - r->w[1] * Lw[0]};
    for (int a = 0; a < 3; ++a) rhs[a] = imp[3 + a] + dt * (r->torque[a] - gyro[a]);
    for (int i = 0; i < 3; ++i)
        r->w[i] += Iinv[i * 3 + 0] * rhs[0] + Iinv[i * 3 + 1] * rhs[1] + Iinv[i * 3 + 2] * rhs[2];
    oracle_advance_pose(r, dt);
}

int oracle_host_step(const oracle_env* env, oracle_rigid* rigid, int n_rigid, int P, double* x,
                     double* v, double* F, double* C, double* impulse, oracle_substep_stats* st) {
    double* imp = impulse ? impulse : (double*)calloc(6 * (size_t)(n_rigid > 0 ? n_rigid : 1), sizeof(double));
    if (!imp) return OR_EINVAL;
    memset(imp, 0, sizeof(double) * 6 * (size_t)n_rigid);
    int worst = OR_OK;
    for (int k = 0; k < env->N; ++k) {
        int rc = oracle_substep(env, rigid, n_rigid, P, x, v, F, C, imp, st ? &st[k] : NULL, NULL);
        if (rc == OR_NOCONV) worst = OR_NOCONV;
        else if (rc != OR_OK) {
            if (!impulse) free(imp);
            return rc;
        }
    }
    /* the rigid side of the split, with the pose frozen until here */
    for (int r = 0; r < n_rigid; ++r) {
        if (rigid[r].motion == OR_KINEMATIC) oracle_advance_pose(&rigid[r], env->N * env->h);
        else if (rigid[r].motion == OR_DYNAMIC)
            oracle_integrate_dynamic(&rigid[r], imp + 6 * r, env->gravity, env->N * env->h);
    }
    if (!impulse) free(imp);
    return worst;
}

int oracle_contact_problem(const oracle_env* env, const oracle_rigid* rigid, int n_rigid, int P,
                           const double* x, const double* v, const double* F, const double* C,
                           int max_nodes, int max_c, int* n_nodes_out, double* m, double* vstar,
                           int* nodes, double* w, double* Rc, double* b, double* phi0, double* n0,
                           double* mu) {
    frame_t fr;
    int rc = build_frame(env, rigid, n_rigid, P, x, v, F, C, &fr);
    if (rc != OR_OK) {
        frame_free(&fr);
        return -1;
    }
    if (fr.n_act > max_nodes || fr.nc > max_c) {
        frame_free(&fr);
        return -2;
    }
    *n_nodes_out = fr.n_act;
    for (int i = 0; i < fr.n_act; ++i) {
        m[i] = fr.m[fr.act[i]];
        for (int a = 0; a < 3; ++a) vstar[3 * i + a] = fr.vgrid[3 * fr.act[i] + a];
    }
    memcpy(nodes, fr.cnodes, sizeof(int) * 27 * (size_t)fr.nc);
    memcpy(w, fr.cw, sizeof(double) * 27 * (size_t)fr.nc);
    memcpy(Rc, fr.cR, sizeof(double) * 9 * (size_t)fr.nc);
    memcpy(b, fr.cb, sizeof(double) * 3 * (size_t)fr.nc);
    memcpy(phi0, fr.cphi, sizeof(double) * (size_t)fr.nc);
    memcpy(n0, fr.cn0, sizeof(double) * (size_t)fr.nc);
    memcpy(mu, fr.cmu, sizeof(double) * (size_t)fr.nc);
    int nc = fr.nc;
    frame_free(&fr);
    return nc;
}
