/*
 * mpm.h -- C ABI of the MI355X library for one MPM substep coupled to rigid
 * bodies (Yu, Du, Zong, Castro, Jiang, Han, "A Convex Formulation of Material
 * Points and Rigid Bodies with GPU-Accelerated Async-Coupling for Interactive
 * Simulation", arXiv 2503.05046).
 *
 * What one call of mpm_step computes (the asynchronous split of Sec. IV-A,
 * Eq. (3)-(4)): a host step of N substeps of size h. The rigid pose and twist
 * are frozen for the host step; each substep (Eq. (5)) is
 *   1. free motion, Eq. (6): MLS-MPM particle-to-grid transfer with quadratic
 *      B-splines and the Kirchhoff stress folded into the affine term, then
 *      v* = p/m + h g on the grid (Sec. V-A);
 *   2. contact registration: one contact per (particle, rigid primitive) pair
 *      with the particle strictly inside the primitive (Sec. V-B);
 *   3. the convex contact problem, Eq. (7)-(8), solved by Algorithm 1: the
 *      quasi-Newton iteration with the 3x3 block-diagonal Hessian of Sec. IV-C,
 *      gradient and Hessian of Eq. (9)-(10), exact line search, stopping test
 *      |grad~| < eps_a + eps_r max(|p~|, |j~|);
 *   4. grid-to-particle transfer updating v, C (APIC affine matrix), F and x,
 *      with the Drucker-Prager return map for granular material.
 * The impulses the substeps apply to each rigid body are summed over the host
 * step (Eq. (3)) and returned to the caller, who integrates the rigid bodies.
 *
 * Conventions: SI units, float32 state, component-major particle arrays
 * (x[3][P], v[3][P], F[9][P], C[9][P], 3x3 row-major per particle). Grid node
 * (i, j, k) of an environment sits at origin + (i, j, k) * dx; a particle's
 * stencil base floor((x - origin)/dx - 1/2) must stay in [0, dims - 3].
 * All device pointers are HIP device memory of the calling process; every
 * call is asynchronous on the handle's stream except where stated.
 *
 * Errors: no call aborts and no exception crosses the ABI. Each returns an
 * mpm_status; mpm_last_error() returns a thread-local description of the
 * last failure on the calling thread.
 */
#ifndef MPM_H
#define MPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MPM_OK = 0,
    MPM_ENOCONV = 1,  /* warning: a contact solve hit max_iter; state advanced with its last iterate */
    MPM_EDOMAIN = 2,  /* a particle stencil left the grid; its base was clamped */
    MPM_ENAN = 3,     /* non-finite particle state produced */
    MPM_EINVAL = 4,   /* invalid argument; nothing was launched */
    MPM_ENOMEM = 5,   /* workspace too small, or contact capacity exceeded during a step */
    MPM_EDEVICE = 6   /* HIP runtime error; see mpm_last_error() */
} mpm_status;

enum { MPM_FIXED_COROTATED = 0, MPM_DRUCKER_PRAGER = 1 };
enum { MPM_HALF_SPACE = 0, MPM_BOX = 1 };
enum { MPM_STATIC = 0, MPM_KINEMATIC = 1, MPM_DYNAMIC = 2 };

/* Step flags (mpm_step_stats.flags) */
enum {
    MPM_FLAG_NOCONV = 1,
    MPM_FLAG_DOMAIN = 2,
    MPM_FLAG_NAN = 4,
    MPM_FLAG_CAPACITY = 8
};

/* One simulation environment: its own grid, material and particle range.
 * Environments never interact. */
typedef struct {
    int32_t dims[3];       /* grid nodes per axis, each >= 4 */
    float dx;              /* grid spacing [m], > 0 */
    float origin[3];       /* world position of node (0,0,0) */
    float gravity[3];      /* [m/s^2] */
    int32_t material;      /* MPM_FIXED_COROTATED or MPM_DRUCKER_PRAGER */
    float E;               /* Young's modulus [Pa], > 0 */
    float nu;              /* Poisson ratio, in (-1, 0.5) */
    float m_p;             /* particle mass [kg], > 0 */
    float V0;              /* particle rest volume [m^3], > 0 */
    float friction_angle;  /* Drucker-Prager friction angle [deg], in [0, 90) */
    double k;              /* contact stiffness [N/m], > 0 */
    double d;              /* Hunt-Crossley dissipation [s/m], >= 0 */
    double eps_s;          /* friction regularisation [m/s], > 0 */
    int64_t p_begin;       /* first particle of this environment */
    int64_t p_end;         /* one past its last particle */
} mpm_env_desc;

typedef struct {
    uint32_t struct_size;      /* sizeof(mpm_desc) */
    int32_t n_envs;            /* >= 1 */
    const mpm_env_desc* envs;  /* host array [n_envs], copied; particle ranges must tile [0, n_particles) in order */
    double h;                  /* substep size [s] = host step / N, > 0 */
    int32_t N;                 /* substeps per host step, >= 1 */
    double eps_r, eps_a;       /* Algorithm 1 tolerances, >= 0 */
    int32_t max_iter;          /* Algorithm 1 iteration cap, >= 1 */
    int32_t ls_max_steps;      /* line-search Newton/bisection steps, >= 0 (0 = default 100) */
    int64_t n_particles;       /* P >= 1 */
    /* Caller-owned device arrays, borrowed for the life of the handle. The
     * library reorders particles by grid cell once per host step (a stable
     * sort, Sec. V-A); pid (may be NULL) is permuted alongside so the caller
     * can track identity. */
    float* x;                  /* [3][P] */
    float* v;                  /* [3][P] */
    float* F;                  /* [9][P] */
    float* C;                  /* [9][P] */
    int32_t* pid;              /* [P] or NULL */
    int64_t max_contacts;      /* contact capacity per substep (0 = n_particles) */
    void* workspace;           /* device memory of workspace_bytes, caller-owned, 256-byte aligned */
    size_t workspace_bytes;
    void* stream;              /* hipStream_t the handle launches on (NULL = default stream) */
    int32_t tape_substeps;     /* substeps the differentiation tape can hold (0 = no tape); a
                                  multiple of N. The workspace grows by about
                                  tape_substeps x (96 P + 32 grid nodes) bytes. */
    int32_t solver_slots_per_block; /* contact nodes per block of the contact solver, which
                                  sets each environment's group of blocks (0 = 128; the
                                  autotuner of the Python package picks it per scene) */
    int32_t solver;            /* MPM_SOLVER_QN (0): Algorithm 1, the block-diagonal quasi-Newton
                                  iteration of Sec. IV-C. MPM_SOLVER_NEWTON (1): a study variant of
                                  the same solve (same objective, stopping test and exact line
                                  search) whose search direction solves the full Hessian system by
                                  conjugate gradients preconditioned with the node blocks
                                  Algorithm 1 inverts; for comparison only. The workspace grows by
                                  224 bytes per contact node and 128 per contact. */
} mpm_desc;

enum { MPM_SOLVER_QN = 0, MPM_SOLVER_NEWTON = 1 };

/* Rigid primitive (body frame) with its initial pose and twist. */
typedef struct {
    int32_t shape;             /* MPM_HALF_SPACE or MPM_BOX */
    double normal[3];          /* half-space: unit outward normal (body frame) */
    double offset;             /* half-space: sdf(p) = normal . p - offset */
    double half[3];            /* box: half extents, each > 0 */
    double mu;                 /* Coulomb friction coefficient, >= 0 */
    int32_t motion;            /* MPM_STATIC, MPM_KINEMATIC or MPM_DYNAMIC */
    double R[9];               /* body-to-world rotation, row-major */
    double t[3];               /* body origin in world */
    double V[3];               /* linear velocity of the body origin */
    double w[3];               /* angular velocity (world) */
    /* MPM_DYNAMIC (boxes only; the body origin is the centre of mass). After
     * each host step (the pose frozen during it, Sec. V-B) the library
     * integrates the free body on the host, in FP64, from the impulse and
     * moment the MPM side exerted on it over the step (Eq. (3) with the body's
     * mass matrix and Coriolis term, semi-implicit):
     *   m (V' - V) = I_lin + N h (m g + force),
     *   I_w (w' - w) = I_ang + N h (torque - w x I_w w),  I_w = R diag(inertia) R^T,
     * then t' = t + N h V' and R' = Rot(N h w') R. g is the environment's
     * gravity. Ignored for other motions. */
    double mass;               /* > 0 */
    double inertia[3];         /* principal moments about the body axes, each > 0 */
    double force[3];           /* constant external force (world), besides gravity */
    double torque[3];          /* constant external torque about the body origin (world) */
} mpm_rigid_desc;

/* Pose and twist of one rigid body, frozen for a host step. */
typedef struct {
    double R[9];
    double t[3];
    double V[3];
    double w[3];
} mpm_rigid_state;

/* Impulse and torque (about the body origin t, world frame) that MPM applied
 * to one rigid body, summed over the N substeps of a host step; this is minus
 * the impulse the body applied to the material (Eq. (3)). */
typedef struct {
    double impulse[3];
    double torque[3];
} mpm_rigid_impulse;

/* Statistics of one host step. Per-substep arrays are caller-owned host
 * arrays of N entries and may be NULL. */
typedef struct {
    int32_t flags;             /* MPM_FLAG_* */
    int32_t max_iterations;    /* over the substeps */
    int64_t total_iterations;
    int32_t max_contacts;
    int32_t* iterations;       /* [N] Algorithm 1 iterations per substep */
    int32_t* contacts;         /* [N] registered contact points */
    int32_t* contact_nodes;    /* [N] grid nodes touched by a contact stencil */
    double* residual;          /* [N] final |grad~| */
    double* threshold;         /* [N] eps_a + eps_r max(|p~|, |j~|) at exit */
    int64_t total_inner_iterations; /* MPM_SOLVER_NEWTON: conjugate-gradient iterations of the
                                  longest solve of each substep, summed (0 for MPM_SOLVER_QN) */
} mpm_step_stats;

/* Kernel classes timed by mpm_profile. */
enum {
    MPM_K_SORT = 0,      /* cell keys, radix sort, gather, tile list (once per host step) */
    MPM_K_P2G = 1,       /* particle-to-grid scatter */
    MPM_K_GRID = 2,      /* grid update */
    MPM_K_REGISTER = 3,  /* contact registration */
    MPM_K_SETUP = 4,     /* contact-node table */
    MPM_K_SOLVE = 5,     /* Algorithm 1 */
    MPM_K_G2P = 6,       /* grid-to-particle gather and constitutive update */
    MPM_K_COUNT = 7
};

/* Accumulated device time per kernel class, measured with HIP events recorded
 * on the handle's stream around each launch group. */
typedef struct {
    double ms[MPM_K_COUNT];
    int64_t launches[MPM_K_COUNT];
    int64_t solver_iterations;    /* Algorithm 1 iterations over the timed steps */
    int64_t solver_ls_rounds;     /* line-search evaluations (each a pass over the contacts) */
    int64_t solver_contact_iters; /* sum over iterations of registered contacts */
    int64_t solver_node_iters;    /* sum over iterations of contact nodes */
    int64_t solver_contact_rounds;/* sum over line-search evaluations of registered contacts */
    double solver_phase_us[8];    /* solver time of the first block of the longest-solving environment:
                                     node-pass gather, node solve and sums, barrier, contact pass,
                                     barrier, line-search set-up, line-search evaluations, update */
} mpm_profile_data;

typedef struct mpm_handle mpm_handle;

/* Bytes of device workspace mpm_create needs for this description (the
 * caller allocates it). Host only; nothing is launched. */
mpm_status mpm_workspace_size(const mpm_desc* desc, size_t* bytes);

/* Validate the description, lay out the workspace and upload the environment
 * tables on desc->stream. The handle keeps the borrowed pointers. */
mpm_status mpm_create(const mpm_desc* desc, mpm_handle** out);

/* Add a rigid primitive to environment env (Sec. V-B registers contacts
 * against every primitive of the particle's environment). The descriptor is
 * copied. *id receives the body's index in the impulse and state arrays
 * (dense, in order of addition over the whole handle). */
mpm_status mpm_add_rigid_sdf(mpm_handle* h, int32_t env, const mpm_rigid_desc* r, int32_t* id);

/* Advance one host step of N substeps in place. in: host array of the frozen
 * pose and twist of every rigid body for this step, or NULL to use the
 * library's own state (after each step, kinematic bodies advance with their
 * twist, and dynamic bodies are integrated from the step's impulses, see
 * mpm_rigid_desc; with in given, dynamic bodies start from it). out: host array, one entry per rigid body (may be NULL). st may be
 * NULL. Synchronises the handle's stream once, to read impulses and stats.
 * Returns MPM_OK, a warning (MPM_ENOCONV), or an error (MPM_EDOMAIN, MPM_ENAN,
 * MPM_ENOMEM when the contact capacity overflowed: the step stops at that
 * substep with a consistent state). Not thread-safe per handle. */
mpm_status mpm_step(mpm_handle* h, const mpm_rigid_state* in, mpm_rigid_impulse* out,
                    mpm_step_stats* st);

/* Advance n_steps host steps as one replay of a HIP graph that holds all of
 * them (for the batched form, where many small environments make each solve
 * short and the ~16 launches per substep a visible cost): the sort and N
 * substeps of every host step, n_steps times, become one graph launch. Rigid
 * bodies follow the library's own state, as with in = NULL in mpm_step:
 * static bodies stay put, kinematic bodies advance with their twist after
 * every host step (on the device inside the graph; the host state then takes
 * the device's values). The graph is recorded on the first call and again
 * when n_steps, the number of rigid bodies or the solver's block plan
 * changes; the solver's groups are planned per replay from the latest host
 * step (the kernel sizes each group from the current substep). It runs on a
 * stream of the handle's own, after the work already queued on desc->stream,
 * and the call returns when the replay is done. out (may be NULL): impulses
 * on the rigid bodies summed over the n_steps host steps. st (may be NULL):
 * statistics of the last host step. A host step that stops (capacity
 * overflow, non-finite state, a particle outside the grid) leaves the host
 * steps after it in the replay without effect, and its error is returned as
 * in mpm_step. MPM_EINVAL while the differentiation tape records or event
 * timing is on, for n_steps < 1, or when the handle has a dynamic body (its
 * integration needs each host step's impulses on the host). */
mpm_status mpm_step_graph(mpm_handle* h, int32_t n_steps, mpm_rigid_impulse* out, mpm_step_stats* st);

/* Profiling: enable (1) or disable (0) event timing of the kernel classes
 * for the following steps; 2 also times the solver's phases (solver_phase_us),
 * whose clock reads sit on the solver's critical path and lengthen it, so
 * timings taken with 2 are for the breakdown only. out (may be NULL) receives
 * what was accumulated since the previous call, and the accumulators are
 * reset. Host only. */
mpm_status mpm_profile(mpm_handle* h, int32_t enable, mpm_profile_data* out);

/* Current pose and twist of rigid body id (host). */
mpm_status mpm_get_rigid_state(const mpm_handle* h, int32_t id, mpm_rigid_state* s);

/* Set the pose and twist of rigid body id to s advanced by host_steps >= 0
 * host steps of the library's kinematic rule (per host step t += N h V and
 * R <- Rot(N h w) R, as after each mpm_step with in = NULL; only kinematic
 * bodies advance). s is the body's reference state: the reverse pass reports
 * dV_kinematic and dw_kinematic with respect to its twist, through the host
 * steps between it and the recording as well (see mpm_rigid_grad). A pose
 * passed to mpm_step as `in` becomes the reference instead. Host only;
 * MPM_EINVAL for a bad id, host_steps < 0 or an invalid pose. */
mpm_status mpm_set_rigid_state(mpm_handle* h, int32_t id, const mpm_rigid_state* s, int32_t host_steps);

/* Release the handle (not the borrowed memory). Safe on NULL. */
void mpm_destroy(mpm_handle* h);

/* ---- Differentiation (reverse mode through recorded host steps) ----------
 * With desc->tape_substeps > 0, every mpm_step after mpm_tape_reset(h, 1) records
 * what the reverse pass needs (the state at each substep start, the grid
 * before and after the contact solve, the sort permutation of each host
 * step) until the tape is full; mpm_step returns MPM_ENOMEM, with nothing
 * advanced, when a host step would not fit. mpm_step_backward then maps the
 * adjoint of the state after the recorded steps to the adjoint of the state
 * before them, and returns the adjoints of the Lame parameters as adjoints of
 * each environment's E and nu (with k, V0 and rho held fixed) and of each
 * rigid body's twist (V, w) and pose. It covers the substep of Eq. (5)-(8): P2G,
 * grid update, the contact solve (implicit differentiation at its optimum:
 * the full Hessian system by preconditioned conjugate gradients), contact
 * registration (penetration, lagged normal impulse and bias of every
 * contact) and G2P with either material: the fixed-corotated stress, or the
 * Drucker-Prager return map of the trial Hencky strain (tip, cone and
 * elastic branches, Sec. II-A) with the Hencky stress. At a branch boundary
 * the branch the forward took is differentiated. The set of registered
 * contacts is held fixed. MPM_EINVAL for a handle with a dynamic body, whose
 * dynamics the reverse pass does not differentiate. */

/* Adjoints of one environment's material parameters. */
typedef struct {
    double dE;
    double dnu;
} mpm_env_grad;

/* Adjoints of one rigid body's motion (zero for static bodies). */
typedef struct {
    double dV[3];            /* through the velocity V used in every recorded host step */
    double dt[3];            /* through the position t, as a common shift of every recorded pose */
    double dV_kinematic[3];  /* dV plus the library's own kinematic update of t (t advances
                                by N h V after each host step), i.e. the full derivative with
                                respect to the velocity of the body's reference state (the last
                                mpm_set_rigid_state, else the first recorded pose) when the
                                host steps since it ran with in = NULL */
    double dw[3];            /* through the angular velocity w in the velocity field
                                V + w x (x - t) of every recorded host step */
    double dR[3];            /* through a small rotation (world rotation vector, about t) of
                                the first recorded pose, later poses following it by the
                                kinematic advance (R turns by N h w after each host step) */
    double dw_kinematic[3];  /* dw plus the kinematic advance's dependence of the poses on w,
                                from the reference state as for dV_kinematic */
} mpm_rigid_grad;

/* Empty the tape; with record = 1 the following mpm_step calls record, with
 * record = 0 they do not. Host only. */
mpm_status mpm_tape_reset(mpm_handle* h, int32_t record);

/* Reverse pass over the recorded host steps, on the handle's stream (the call
 * synchronises it once at the end). gx [3][P], gv [3][P], gF [9][P], gC [9][P]:
 * device arrays, on entry dL/d(x, v, F, C) of the state after the last recorded
 * step, in the particle order the state has then; on return dL/d(x, v, F, C) of
 * the state before the first recorded step, in the particle order it had then
 * (the pid array permuted by the steps maps between the two). env_grads: host
 * array of n_envs entries, rigid_grads: host array of one entry per rigid body
 * in id order (either may be NULL), overwritten. The tape is kept, so the
 * call may be repeated with other adjoints. MPM_ENOCONV if a conjugate-gradient
 * solve stopped at its iteration cap (relative residual target 1e-7). */
mpm_status mpm_step_backward(mpm_handle* h, float* gx, float* gv, float* gF, float* gC,
                             mpm_env_grad* env_grads, mpm_rigid_grad* rigid_grads);

/* ---- One host step that allocates nothing ---------------------------------
 * For callers that cannot allocate device or pinned memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc. Same
 * host step as mpm_create + mpm_add_rigid_sdf (n_rigid times) + mpm_step(in =
 * NULL) + mpm_destroy on a fresh handle, without a handle: the particle state
 * of desc (x, v, F, C, and pid when not NULL) is advanced by N substeps in place
 * and reordered by cell as mpm_step does; the rigid bodies are frozen at the
 * given poses and twists for the step and are not advanced afterwards (no state
 * is kept: the caller integrates them). The workspace is an array of
 * MPM_STATIC_SCRATCH_BYTES in device memory that the library defines: every GPU
 * it runs on holds one until the process ends, and every call on that GPU
 * shares it and overwrites what the previous call left there. The library
 * calls no allocating routine (no hipMalloc, hipHostMalloc, hipFree, no stream
 * or event creation); host staging is in fixed static arrays.
 *   desc: as for mpm_create, except desc->workspace must be NULL and
 *     workspace_bytes 0, tape_substeps 0, n_envs <= MPM_STATIC_MAX_ENVS,
 *     N <= MPM_STATIC_MAX_SUBSTEPS; the stream must belong to the current
 *     device.
 *   rigids, rigid_env: host arrays of n_rigid descriptors and their environment
 *     indices (0 <= n_rigid <= 256, at most 32 per environment, ordered by
 *     environment, validated as in mpm_add_rigid_sdf).
 *   out (may be NULL): impulses on the bodies, in the given order; st: as in mpm_step.
 * Returns as mpm_step, plus MPM_ENOMEM (nothing launched) when the scene's
 * workspace (mpm_workspace_size) exceeds MPM_STATIC_SCRATCH_BYTES. Calls on
 * one GPU share its array, so two calls whose device work overlapped would
 * race on it; the library prevents that within a process by serialising the
 * calls on the host (one lock over all devices) and returning from each only
 * after its stream has finished the step. Not usable while the caller's stream
 * is being captured (the call synchronises it). */
#define MPM_STATIC_SCRATCH_BYTES (64u * 1024u * 1024u)
#define MPM_STATIC_MAX_ENVS 8
#define MPM_STATIC_MAX_SUBSTEPS 64
mpm_status mpm_step_static(const mpm_desc* desc, const mpm_rigid_desc* rigids, const int32_t* rigid_env,
                           int32_t n_rigid, mpm_rigid_impulse* out, mpm_step_stats* st);

/* Thread-local description of the last error on the calling thread. */
const char* mpm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
