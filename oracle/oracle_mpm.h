/*
 * oracle_mpm.h -- FP64 CPU oracle of one MPM substep coupled to rigid bodies
 * (Yu, Du, Zong, Castro, Jiang, Han: "A Convex Formulation of Material Points
 * and Rigid Bodies with GPU-Accelerated Async-Coupling for Interactive
 * Simulation", arXiv 2503.05046).
 *
 * TEST INFRASTRUCTURE. This library exists to check the GPU library. Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it; the product path never does. It shares no source, header, table or
 * helper with the GPU library: this header is its own, and the two meet only
 * through the seeded input generators.
 *
 * Everything is plain single-threaded C in double precision, written so that
 * each step can be read against the paper:
 *   - asynchronous split, Eq. (3)-(4): the rigid pose and twist are frozen for
 *     a host step of N substeps and the MPM->rigid impulses are summed;
 *   - free motion, Eq. (6): explicit MLS-MPM with quadratic B-splines;
 *   - contact, Eq. (7)-(8): the convex problem solved by Algorithm 1 with the
 *     3x3 block-diagonal Hessian of Sec. IV-C and the gradient and Hessian of
 *     Eq. (9)-(10), Sec. V-B;
 *   - G2P with fixed-corotated elasticity or Hencky elasticity with a
 *     Drucker-Prager return map (granular media, Sec. II-A).
 * Readings of points the paper leaves open are listed where they are used.
 *
 * Array conventions: particle arrays are component-major (x[3][P], F[9][P],
 * row-major 3x3 per particle), grid nodes are (i, j, k) with i fastest, node
 * (i, j, k) sits at origin + (i, j, k) * dx, and the grid has nx*ny*nz nodes.
 */
#ifndef ORACLE_MPM_H
#define ORACLE_MPM_H

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_OK = 0, OR_NOCONV = 1, OR_DOMAIN = 2, OR_NAN = 3, OR_EINVAL = 4 };
enum { OR_FIXED_COROTATED = 0, OR_DRUCKER_PRAGER = 1 };
enum { OR_HALF_SPACE = 0, OR_BOX = 1 };
enum { OR_STATIC = 0, OR_KINEMATIC = 1, OR_DYNAMIC = 2 };

typedef struct {
    int nx, ny, nz;            /* grid nodes per axis */
    double dx;                 /* grid spacing [m] */
    double origin[3];          /* world position of node (0,0,0) */
    double gravity[3];         /* [m/s^2] */
    int material;              /* OR_FIXED_COROTATED or OR_DRUCKER_PRAGER */
    double E, nu;              /* Young's modulus [Pa], Poisson ratio */
    double m_p, V0;            /* particle mass [kg] and rest volume [m^3] */
    double friction_angle;     /* Drucker-Prager friction angle [deg] */
    double k, d, eps_s;        /* contact stiffness [N/m], dissipation [s/m],
                                  friction regularisation [m/s] */
    double h;                  /* substep size [s] = host step / N */
    int N;                     /* substeps per host step */
    double eps_r, eps_a;       /* Algorithm 1 stopping tolerances */
    int max_iter;              /* Algorithm 1 iteration cap */
    int ls_max_iter;           /* line-search step cap */
    int basis;                 /* tangent completion: 0 Duff et al. 2017, 1 axis-based */
    int solve_all_nodes;       /* 1: Algorithm 1 iterates over every active node; 0: over the
                                  nodes a contact stencil touches (the others keep v = v*) */
} oracle_env;

typedef struct {
    int shape;                 /* OR_HALF_SPACE or OR_BOX */
    double normal[3];          /* half-space: outward unit normal, body frame */
    double offset;             /* half-space: sdf = n.(p) - offset, p in body frame */
    double half[3];            /* box: half extents, body frame */
    double mu;                 /* Coulomb friction coefficient */
    int motion;                /* OR_STATIC, OR_KINEMATIC or OR_DYNAMIC */
    double R[9];               /* body-to-world rotation, row-major */
    double t[3];               /* body origin in world */
    double V[3];               /* linear velocity of the body origin */
    double w[3];               /* angular velocity */
    /* OR_DYNAMIC (a box whose body origin is its centre of mass): */
    double mass;               /* > 0 */
    double inertia[3];         /* principal moments about the body axes, > 0 */
    double force[3];           /* constant external force (world), besides gravity */
    double torque[3];          /* constant external torque about the origin (world) */
} oracle_rigid;

typedef struct {
    int n_contacts;            /* registered contact points this substep */
    int iterations;            /* Algorithm 1 iterations (Newton directions) */
    int ls_steps;              /* total line-search evaluations */
    int converged;             /* stopping test met */
    double residual;           /* final scaled gradient norm */
    double threshold;          /* eps_a + eps_r * max(|p~|, |j~|) at exit */
    double p_norm, j_norm;     /* |p~| and |j~| at exit */
    int n_active_nodes;        /* nodes with m > 0 */
    int n_contact_nodes;       /* nodes touched by a contact stencil */
} oracle_substep_stats;

/* ---- whole steps ----------------------------------------------------- */

/* Advance one substep (Eq. (5)) in place. x, v, F, C: FP64 particle state,
 * component-major with P particles. impulse (6*n_rigid, may be NULL) receives
 * +sum of the impulse and torque about the body origin that MPM applies to
 * each rigid body in this substep (accumulated, not overwritten). Rigid poses
 * are not advanced here. lp_hist (may be NULL, max_iter+1 entries) receives
 * the contact objective after each iteration. Returns OR_* status. */
int oracle_substep(const oracle_env* env, const oracle_rigid* rigid, int n_rigid,
                   int P, double* x, double* v, double* F, double* C,
                   double* impulse, oracle_substep_stats* st, double* lp_hist);

/* One host step of the asynchronous split (Eq. (3)-(4)): N substeps with the
 * rigid pose and twist frozen, impulses summed into impulse[6*n_rigid]
 * (overwritten), then kinematic bodies are advanced by N*h. st receives N
 * entries (may be NULL). */
int oracle_host_step(const oracle_env* env, oracle_rigid* rigid, int n_rigid,
                     int P, double* x, double* v, double* F, double* C,
                     double* impulse, oracle_substep_stats* st);

/* ---- pieces exposed for the pins ------------------------------------- */

/* Quadratic B-spline stencil of one particle: base node, 27 weights and
 * offsets x_i - x_p (row o = (a*3+b)*3+c for offsets (a,b,c) along x,y,z). */
void oracle_stencil(const oracle_env* env, const double xp[3], int base[3],
                    double w[27], double dpos[81]);

/* Sort key of the cell-major particle order: the integer cell index computed
 * in IEEE binary32 exactly as the GPU does (no fused multiply-add), packed as
 * (tile, cell-in-tile) with 4x4x4-cell tiles. xs: float32 positions [3][P]. */
void oracle_cell_keys_f32(int P, const float* xs, const float origin[3],
                          float inv_dx, int nx, int ny, int nz,
                          unsigned int* keys);
/* Stable order of keys (ties broken by index). */
void oracle_stable_order(int P, const unsigned int* keys, int* perm);

void oracle_svd3(const double F[9], double U[9], double S[3], double V[9]);
/* Kirchhoff stress tau = P F^T of the material at deformation F. */
void oracle_kirchhoff(const oracle_env* env, const double F[9], double tau[9]);
/* Drucker-Prager return map of F (in place); returns 1 if projected. */
int oracle_dp_project(const oracle_env* env, double F[9]);

/* Contact potential l_c of one contact point at contact-frame velocity vc
 * (t1, t2, n). Writes gamma = -dl/dvc (impulse on MPM, contact frame) and
 * G = d2l/dvc2 (row-major 3x3). phi0: penetration at substep start, n0:
 * lagged normal impulse. */
double oracle_contact_model(const double vc[3], double phi0, double n0, double mu,
                            double k, double d, double eps_s, double h,
                            double gamma[3], double G[9]);
/* Normal impulse of the compliant model at normal velocity vn. */
double oracle_normal_impulse(double vn, double phi0, double k, double d, double h);

/* Signed distance and outward world normal of a rigid primitive. */
double oracle_sdf(const oracle_rigid* r, const double x[3], double n[3]);
/* Contact frame [t1 t2 n] (columns) for unit normal n. */
void oracle_contact_frame(int basis, const double n[3], double Rc[9]);

/* Algorithm 1 on an explicit problem: n_nodes nodes with masses m and free
 * velocities vstar[3*n], n_c contacts each with 27 node indices and weights,
 * frame Rc[9], bias b[3], phi0, n0, mu. v_io holds the initial guess on entry
 * and the result on exit; gamma_out[3*n_c] receives the contact-frame
 * impulses at the result. */
int oracle_qn_solve(const oracle_env* env, int n_nodes, const double* m,
                    const double* vstar, int n_c, const int* nodes,
                    const double* w, const double* Rc, const double* b,
                    const double* phi0, const double* n0, const double* mu,
                    double* v_io, double* gamma_out, oracle_substep_stats* st,
                    double* lp_hist);

/* Debug view of one substep's contact problem, for the dense brute-force pin:
 * runs P2G, grid update and registration, then copies the problem restricted
 * to its contact nodes. Capacities: max_nodes, max_c. Returns the number of
 * contacts (negative on overflow or error); *n_nodes_out receives the node
 * count. Node arrays: m, vstar[3]; contact arrays as in oracle_qn_solve with
 * node indices local to the returned node list. */
int oracle_contact_problem(const oracle_env* env, const oracle_rigid* rigid, int n_rigid,
                           int P, const double* x, const double* v, const double* F,
                           const double* C, int max_nodes, int max_c,
                           int* n_nodes_out, double* m, double* vstar,
                           int* nodes, double* w, double* Rc, double* b,
                           double* phi0, double* n0, double* mu);

/* Advance a kinematic pose by dt with the frozen twist (Rodrigues). */
void oracle_advance_pose(oracle_rigid* r, double dt);

/* The rigid side of the split for a free body (Eq. (3) with the body's mass
 * matrix and Coriolis term), one host step of length dt, semi-implicit:
 *   m (V' - V) = I_lin + dt (m g + f),
 *   I_w (w' - w) = I_ang + dt (tau - w x I_w w),   I_w = R diag(inertia) R^T,
 * with (I_lin, I_ang) = imp, the impulse and its moment about the origin that
 * the MPM side exerted on the body over the step; then the pose advances with
 * the new twist (oracle_advance_pose). */
void oracle_integrate_dynamic(oracle_rigid* r, const double imp[6], const double g[3], double dt);

#ifdef __cplusplus
}
#endif
#endif
