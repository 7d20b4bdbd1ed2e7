// mpm_internal.h -- device tables, workspace layout and kernel entry points
// shared by the host orchestrator and the HIP kernels of libmpm.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "devmath.h"

namespace mpm {

constexpr int kTile = 4;              // cells per tile edge (4x4x4 = 64 cells)
constexpr int kBlockNodes = 8;        // LDS node block edge: tile + 2 stencil + 1 drift each side
constexpr int kMaxRigidPerEnv = 32;   // contact mask width
constexpr int kQnSums = 8;            // per-iteration scalar sums of the node pass
constexpr int kSortBlocks = 512;      // blocks of the chunked scan / radix passes
constexpr int kSortThreads = 256;

struct DevEnv {
    int dims[3];
    int ntile[3];
    int tile_base;          // first global tile id of this environment
    int rigid_begin, rigid_end;
    long long node_base;    // first global node of this environment
    long long p_begin, p_end;
    float dx, inv_dx, D;    // D = 4 / dx^2
    float origin[3];
    float gravity[3];
    Material mat;
    float m_p, V0;
    double k, d, eps_s;
};

struct DevRigid {
    int shape;
    int env;
    double normal[3];
    double offset;
    double half[3];
    double mu;
    double R[9];
    double t[3];
    double V[3];
    double w[3];
};

// Per-substep device statistics.
struct SubstepStats {
    int n_contacts;
    int n_slots;
    int iterations;
    int converged;
    int ls_rounds;
    int pad;
    int inner_iterations;  // exact-Newton variant: conjugate-gradient iterations
    int pad2;
    double residual;
    double threshold;
    unsigned long long t_phase[8];  // solver wall-clock ticks: node gather, node solve, barrier, contact pass,
                                    // barrier, line-search set-up, line-search evaluations, update
};

// Contact solver data as compact records, so that a gather of one contact or
// one contact node touches one or two cache lines.
struct alignas(128) ContactRec {
    double t1[3], t2[3];  // tangent axes of the contact frame R_c = [t1 t2 n] (world)
    double n[3];          // world normal
    double phi0;          // penetration at substep start
    double mun0;          // mu times the lagged normal impulse
    double k, d, eps_s;
};

struct alignas(16) ContactStencil {
    int slot[27];    // contact-node slot of each stencil node, -1 for a zero weight
    float w[27];     // stencil weights
};

struct alignas(128) ContactDyn {
    double vc[2][3];  // contact velocity, double-buffered by iteration parity
    double uc[2][3];  // R_c^T J dv, double-buffered by iteration parity
    double gam[3];    // impulse on MPM at exit (contact frame)
    double b[3];      // bias velocity -R_c^T v_rigid(x_p)
};

struct alignas(16) SlotRec {
    double m;
    double v[3];      // iterate
    double vstar[3];  // free-motion velocity
    double dv[3];     // search direction
};

struct Entry {
    unsigned c;      // contact
    int slot;        // contact node
    float w;         // stencil weight
    float pad;
};

// Device scalars that live in the workspace.
struct DevCounters {
    unsigned n_ptiles;       // non-empty particle tiles after the sort
    unsigned n_active;       // active node tiles this substep
    unsigned n_contacts;     // registered contacts this substep (may exceed capacity)
    unsigned n_pairs;        // contact-node pairs
    unsigned n_slots;        // distinct contact nodes
    unsigned flags;          // MPM_FLAG_* bits
    unsigned abort_step;     // set when the step must stop (capacity overflow)
    unsigned abort_substep;  // substep at which the step stopped
    unsigned n_ntiles;       // node tiles adjacent to a particle tile (this host step)
    unsigned pad[7];
};

constexpr int kBarStride = 16;     // unsigned words between the barrier counters of two environments
constexpr int kCtrLanes = 64;      // loop-barrier arrival counters per environment (block rank mod 64)
constexpr int kCtrStride = 32;     // unsigned words between two of them (separate 128-byte lines)
constexpr int kMaxRigidTape = 256;  // rigid bodies per handle (the tape keeps each host step's table)
// adjoints per rigid body and recorded host step: V, t, w (through the
// velocity field), a small rotation of the pose about t
constexpr int kRigidGradStride = 12;
// contacts of one environment the solver's one-barrier form takes
constexpr int kQnScatterMax = 2048;
// distinct contacts of one block's contact nodes in the compact node pass
constexpr int kQnUniqMax = 512;
// per distinct contact of a block of the one-barrier form: its frame (t1, t2,
// n) and model parameters (phi0, mu n0, k, d, eps_s), kept in the rank's scratch
constexpr int kQnRecWords = 14;
// doubles of one group rank's scratch: v_c and u_c of the line search's
// contacts, then the distinct contacts' records
constexpr int kQnRankWords = 6 * kQnScatterMax + kQnRecWords * kQnUniqMax;

// Pointers into the caller's workspace.
struct Work {
    // particle sort
    unsigned *key_a, *key_b, *idx_a, *idx_b;
    float *xs, *vs, *Fs;     // gathered state for the first substep of a host step
    float* Q;                // fused affine/stress matrix [9][P]
    int* pids;               // gathered particle ids
    unsigned* cmask;         // contact bitmask per particle
    // tiles
    unsigned* tile_flag;     // [T_all] node-tile activation flags
    unsigned* active_tiles;  // [T_all]
    unsigned* ptile_id;      // [T_all] particle tiles (global tile id)
    unsigned* ptile_beg;     // [T_all + 1]
    int* ptile_of;           // [T_all] particle-tile index of a tile, -1 if it holds no particles
    unsigned* ntile_list;    // [T_all] node tiles within one tile of a particle tile
    unsigned* ntile_mark;    // [T_all] 1 for tiles in ntile_list
    float4* blkbuf;          // [T_all][512] per-tile P2G node blocks (m, p)
    const unsigned* keys_sorted;  // sorted cell keys of the current host step
    // grid (dense, all envs)
    float4* acc;             // (m, px, py, pz)
    float4* vel;             // (vx, vy, vz, m)
    // contacts (capacity cap_c)
    int *c_pid, *c_rid, *c_env, *c_base;
    float* c_w;              // [9][cap] per-axis stencil weights (pair generation)
    ContactRec* c_rec;       // [cap] per-substep contact data
    ContactStencil* c_st;    // [cap] slots and weights of the 27 stencil nodes
    ContactDyn* c_dyn;       // [cap] solver state
    double* c_coef;          // line-search coefficients of each contact, chunks of 64 contacts x 11 (contact pass)
    // contact-node pairs (capacity 27 cap_c)
    unsigned *pk_a, *pk_b, *pv_a, *pv_b;
    Entry* e_ent;            // [27 cap] (contact, slot, weight) in slot order
    // contact-node slots (capacity cap_s)
    int *s_node, *s_beg;     // s_beg has cap_s + 1 entries
    SlotRec* s_rec;          // [cap_s]
    // scratch
    unsigned* blk;           // [kSortBlocks * 256 + 2 * kSortBlocks] histograms / block sums
    double* partial;         // [solver blocks][kQnSums]
    double* partial_odd;     // [solver blocks][kQnSums] odd iterations of the one-barrier form
    double* partial2;        // [3][solver blocks]
    double* rigid_acc;       // [n_rigid][6] FP64 impulse accumulators
    SubstepStats* sstats;    // [N][n_envs]
    // per-environment contact solve
    double* env_pnorm;       // [n_envs] sum m |v*|^2 over the env's active nodes (FP64)
    int* env_range;          // [n_envs][4] contacts [c0, c1) and contact nodes [s0, s1)
    int2* qn_map;            // [solver blocks] (env, rank in the env's block group)
    int* env_qn;             // [n_envs][2] first block and block count of the env's group
    unsigned* env_bar;       // [n_envs][kBarStride] barrier arrival count and generation
    unsigned* env_ctr;       // [n_envs][kCtrLanes][kCtrStride] arrival counters of the solver's loop barriers
    // differentiation tape and reverse-pass buffers (tape_cap substeps; empty when 0)
    float* tape_p;           // [tape_cap][24][P] x, v, F, Q at each substep start
    float4* tape_g;          // [tape_cap][2][n_nodes] grid after the update and after the solve
    unsigned* tape_idx;      // [tape_cap / N][P] sort permutation of each host step
    float* adj;              // [2][24][P] particle adjoints, two orders
    float4* gbar;            // [n_nodes] node adjoints
    double* lame;            // [n_envs][2] adjoints of mu and lambda
    DevRigid* tape_rig;      // [tape_cap / N][kMaxRigidTape] rigid table of each recorded host step
    DevEnv* tape_env;        // [tape_cap / N][n_envs] environment table of each recorded host step
    double* cg_vec;          // [5][cap_s][3] conjugate gradients: lam, r, z, p, Hp
    double* cg_pinv;         // [cap_s][6] inverse node blocks
    double* cg_q;            // [cap_c][3]
    double* cg_sc;           // [8] scalars
    float* cxv;              // [6][P] particle adjoints from the contact solve (x, v)
    double* rgrad;           // [tape_cap / N][n_rigid][kRigidGradStride] rigid adjoints per host step
    int tape_cap;
    DevCounters* cnt;
    DevEnv* envs;
    DevRigid* rigids;
    // sizes
    long long P;
    long long n_nodes;
    int n_tiles;
    int n_envs;
    int n_rigid;
    long long cap_c, cap_s;
    int qn_blocks;           // co-resident solver blocks (capacity of partial and qn_map)
    int qn_compact;          // 1: blocks that fit take the compact node pass (0 only to test the other)
    int qn_scatter;          // 1: environments that fit take the solver's one-barrier form
    int qn_plain_launch;     // 1: launch the solver with hipLaunchKernel instead of the cooperative API
                             //    (the grid is still sized to the co-resident block count)
    double* qn_uacc;         // [3][3][kQnScatterMax] per-contact sums of the one-barrier form
    double* qn_vcblk;        // [kQnMaxGroup][kQnRankWords] per rank of the group: contact velocities, records
    double* qn_lsprm;        // [5][kQnScatterMax] per-contact line-search constants of the one-barrier form
    int* qn_pend;            // [n_envs] environments the one-barrier solver kernel left to the other
    int solver;              // MPM_SOLVER_QN or MPM_SOLVER_NEWTON
    int sort_policy;         // kSortTiles, kSortTruncated or kSortNone
    int transfer_blocks;     // blocks of the tiled P2G and G2P launches (each takes particle tiles in turn)
    int p2g_walks;           // walks per (component, cell) of the tiled P2G: 1 or 2
    int p2g_walks_fixed;     // nonzero: p2g_walks was set at creation and is not adapted
    double* nt_slot;         // exact-Newton variant: [cap_s][kNtSlot] per contact-node vectors
    double* nt_con;          // exact-Newton variant: [cap_c][kNtCon] per-contact terms
    double* qn_lspart;       // [2][kQnMaxBlocks][2] per-block line-search sums of the distributed line search
};

// The exact-Newton variant (the value of MPM_SOLVER_NEWTON) and its per-node and
// per-contact words (see k_newton).
constexpr int kSolverNewton = 1;
// Sort policies: full keys once per host step with the LDS-tiled transfers
// (the default), or the ablation arms: keys truncated to their top
// kTruncBits bits once per host step, or no reordering; both arms use the
// plain scatter and gather.
constexpr int kSortTiles = 0, kSortTruncated = 1, kSortNone = 2;
constexpr int kTruncBits = 10;
constexpr int kNtSlot = 28;
constexpr int kNtCon = 16;

// One recorded substep of the differentiation tape.
struct TapeStep {
    const float *x, *v, *F, *Q;  // state at the substep start, [3|9][P], in its host step's sorted order
    const float4* vstar;         // grid after the update (v*, m)
    const float4* vel;           // grid after the contact solve (v, m)
};

// ---- kernel launchers (return hipError_t of the launch) -------------------
hipError_t launch_keys(const Work& w, const float* x, int shift, hipStream_t s);
hipError_t launch_p2g_plain(const Work& w, const float* x, const float* v, hipStream_t s);
hipError_t launch_g2p_plain(const Work& w, const float* x_in, const float* F_in, float* x_out, float* v_out,
                            float* F_out, float* C_out, const int* pid_in, int* pid_out, double h, hipStream_t s);
hipError_t launch_no_tiles(const Work& w, hipStream_t s);
hipError_t radix_sort(const Work& w, unsigned* keys, unsigned* vals, unsigned* keys_tmp,
                      unsigned* vals_tmp, const unsigned* count_dev, long long count_host,
                      int bits, hipStream_t s, unsigned** keys_out, unsigned** vals_out);
hipError_t launch_permute(const Work& w, const unsigned* idx, const float* x, const float* v,
                          const float* F, const float* C, const int* pid, double h,
                          hipStream_t s);
hipError_t launch_recover_C(const Work& w, const float* F, float* C, double h, hipStream_t s);
hipError_t launch_scan_blocks(unsigned* data, int n_items, unsigned* total, hipStream_t s);
hipError_t launch_tile_list(const Work& w, const unsigned* sorted_keys, hipStream_t s);
hipError_t launch_tile_maps(const Work& w, hipStream_t s, bool clear_old);
hipError_t launch_p2g(const Work& w, const float* x, const float* v, hipStream_t s);
void p2g_adapt(Work& w, unsigned n_ptiles);  // the tiled P2G's walks for the next host step
hipError_t launch_grid_update(const Work& w, double h, hipStream_t s);
hipError_t launch_registration(const Work& w, const float* x, const float* v, double h,
                               int substep, hipStream_t s);
hipError_t launch_contact_setup(const Work& w, hipStream_t s);
hipError_t launch_qn(const Work& w, const float* x, int substep, double h, double eps_r,
                     double eps_a, int max_iter, int ls_max_steps, int blocks, int env_stride,
                     int timers, int slots_per_block, hipStream_t s);
int qn_max_blocks();
constexpr int kQnMaxGroup = 128;  // blocks of one environment's group (partials staged in LDS)
constexpr int kQnMaxBlocks = 1024;  // solver blocks a launch may have (capacity of the per-block buffers)
hipError_t launch_g2p(const Work& w, const float* x_in, const float* F_in, float* x_out,
                      float* v_out, float* F_out, float* C_out, const int* pid_in,
                      int* pid_out, double h, hipStream_t s);
hipError_t launch_clear_step(const Work& w, int N, bool stats_only, hipStream_t s);
// reverse mode (adjoint.hip)
hipError_t launch_g2p_adj(const Work& w, const TapeStep& t, float h, float* ax, const float* av, float* aF,
                          const float* aQ, const float* aC, float4* gbar, double* lame, hipStream_t s);
hipError_t launch_grid_adj(const Work& w, const TapeStep& t, float h, float4* gbar, hipStream_t s);
hipError_t launch_p2g_adj(const Work& w, const TapeStep& t, const float4* gbar, const float* cx, const float* cv,
                          float* ax, float* av, float* aQ, hipStream_t s);
hipError_t launch_cadj_start(const Work& w, double h, const float4* vel, hipStream_t s);
hipError_t launch_cg_iteration(const Work& w, double h, hipStream_t s);
hipError_t launch_cadj_finish(const Work& w, double h, const TapeStep& t, const float4* vel, float* cx, float* cv,
                              double* rg, hipStream_t s);
hipError_t launch_permute_adj(const Work& w, const TapeStep& t, float h, const unsigned* idx, const float* ax,
                              const float* av, const float* aF, const float* aQ, float* ox, float* ov, float* oF,
                              float* oC, double* lame, hipStream_t s);
hipError_t launch_clear_substep(const Work& w, hipStream_t s);

}  // namespace mpm
