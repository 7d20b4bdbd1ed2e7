// api.hip -- host side of libmpm: argument validation, workspace layout, the
// rigid-body table and the host-step loop of the asynchronous split
// (Sec. IV-A, Eq. (3)-(4)): N substeps with the rigid state frozen, impulses
// summed, then the kinematic bodies advanced on the host.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mpm.h"
#include "mpm_internal.h"

using namespace mpm;

static_assert(kSolverNewton == MPM_SOLVER_NEWTON, "solver ids of the ABI and the kernels");

namespace {

thread_local std::string g_err;

mpm_status fail(mpm_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(MPM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
    } while (0)

constexpr int kMaxRigidTotal = 256;
constexpr int kMaxQnBlocks = kQnMaxBlocks;
constexpr int kQnItemsPerBlock = 128;  // contact nodes per solver block
constexpr int kTransferBlocks = 4096;  // default blocks of the tiled P2G and G2P launches
constexpr size_t kAlign = 256;

struct Layout {
    size_t off = 0;
    char* base = nullptr;
    template <typename T>
    T* take(size_t count) {
        off = (off + kAlign - 1) & ~(kAlign - 1);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += sizeof(T) * (count > 0 ? count : 1);
        return p;
    }
};

struct Sizes {
    long long P = 0, n_nodes = 0, cap_c = 0, cap_s = 0;
    int n_tiles = 0, n_envs = 0, N = 1, tape_cap = 0, solver = 0;
};

mpm_status validate(const mpm_desc* d, Sizes* sz) {
    if (!d) return fail(MPM_EINVAL, "desc is NULL");
    if (d->struct_size != sizeof(mpm_desc))
        return fail(MPM_EINVAL, "desc->struct_size %u != %zu", d->struct_size, sizeof(mpm_desc));
    if (d->n_envs < 1 || !d->envs) return fail(MPM_EINVAL, "need at least one environment");
    if (!(d->h > 0.0) || !isfinite(d->h)) return fail(MPM_EINVAL, "h must be > 0");
    if (d->N < 1) return fail(MPM_EINVAL, "N must be >= 1");
    if (!(d->eps_r >= 0.0) || !(d->eps_a >= 0.0)) return fail(MPM_EINVAL, "tolerances must be >= 0");
    if (d->max_iter < 1) return fail(MPM_EINVAL, "max_iter must be >= 1");
    if (d->ls_max_steps < 0) return fail(MPM_EINVAL, "ls_max_steps must be >= 0");
    if (d->solver_slots_per_block < 0) return fail(MPM_EINVAL, "solver_slots_per_block must be >= 0");
    if (d->solver != MPM_SOLVER_QN && d->solver != MPM_SOLVER_NEWTON) return fail(MPM_EINVAL, "unknown solver %d", d->solver);
    if (d->n_particles < 1 || d->n_particles > (1ll << 31) - 1)
        return fail(MPM_EINVAL, "n_particles out of range");
    long long expect = 0, nodes = 0;
    long long tiles = 0;
    for (int e = 0; e < d->n_envs; ++e) {
        const mpm_env_desc& E = d->envs[e];
        if (E.p_begin != expect || E.p_end < E.p_begin)
            return fail(MPM_EINVAL, "env %d particle range does not continue the previous one", e);
        expect = E.p_end;
        for (int a = 0; a < 3; ++a)
            if (E.dims[a] < 4) return fail(MPM_EINVAL, "env %d dims must be >= 4", e);
        if (!(E.dx > 0.f)) return fail(MPM_EINVAL, "env %d dx must be > 0", e);
        if (E.material != MPM_FIXED_COROTATED && E.material != MPM_DRUCKER_PRAGER)
            return fail(MPM_EINVAL, "env %d unknown material", e);
        if (!(E.E > 0.f) || !(E.nu > -1.f && E.nu < 0.5f))
            return fail(MPM_EINVAL, "env %d needs E > 0 and -1 < nu < 0.5", e);
        if (!(E.m_p > 0.f) || !(E.V0 > 0.f)) return fail(MPM_EINVAL, "env %d needs m_p, V0 > 0", e);
        if (!(E.friction_angle >= 0.f && E.friction_angle < 90.f))
            return fail(MPM_EINVAL, "env %d friction angle out of range", e);
        if (!(E.k > 0.0) || !(E.d >= 0.0) || !(E.eps_s > 0.0))
            return fail(MPM_EINVAL, "env %d needs k > 0, d >= 0, eps_s > 0", e);
        nodes += (long long)E.dims[0] * E.dims[1] * E.dims[2];
        tiles += (long long)((E.dims[0] + 3) / 4) * ((E.dims[1] + 3) / 4) * ((E.dims[2] + 3) / 4);
    }
    if (expect != d->n_particles) return fail(MPM_EINVAL, "environments must cover all particles");
    if (tiles >= (1ll << 26)) return fail(MPM_EINVAL, "too many grid tiles for 32-bit keys");
    if (nodes >= (1ll << 31) - 1) return fail(MPM_EINVAL, "too many grid nodes");
    if (d->max_contacts < 0) return fail(MPM_EINVAL, "max_contacts must be >= 0");
    if (d->tape_substeps < 0 || d->tape_substeps % d->N != 0)
        return fail(MPM_EINVAL, "tape_substeps must be a non-negative multiple of N");
    sz->P = d->n_particles;
    sz->n_nodes = nodes;
    sz->n_tiles = (int)tiles;
    sz->n_envs = d->n_envs;
    sz->N = d->N;
    sz->cap_c = d->max_contacts > 0 ? d->max_contacts : d->n_particles;
    sz->cap_s = std::min<long long>(27 * sz->cap_c, nodes);
    sz->tape_cap = d->tape_substeps;
    sz->solver = d->solver;
    return MPM_OK;
}

size_t layout(const Sizes& z, char* base, Work* w) {
    Layout L;
    L.base = base;
    const long long P = z.P;
    w->key_a = L.take<unsigned>(P);
    w->key_b = L.take<unsigned>(P);
    w->idx_a = L.take<unsigned>(P);
    w->idx_b = L.take<unsigned>(P);
    w->xs = L.take<float>(3 * P);
    w->vs = L.take<float>(3 * P);
    w->Fs = L.take<float>(9 * P);
    w->Q = L.take<float>(9 * P);
    w->pids = L.take<int>(P);
    w->cmask = L.take<unsigned>(P);
    w->tile_flag = L.take<unsigned>(z.n_tiles);
    w->active_tiles = L.take<unsigned>(z.n_tiles);
    w->ptile_id = L.take<unsigned>(z.n_tiles);
    w->ptile_beg = L.take<unsigned>(z.n_tiles + 1);
    w->ptile_of = L.take<int>(z.n_tiles);
    w->ntile_list = L.take<unsigned>(z.n_tiles);
    w->ntile_mark = L.take<unsigned>(z.n_tiles);
    w->blkbuf = L.take<float4>((size_t)z.n_tiles * 512);
    w->acc = L.take<float4>(z.n_nodes);
    w->vel = L.take<float4>(z.n_nodes);
    const long long C = z.cap_c;
    w->c_pid = L.take<int>(C);
    w->c_rid = L.take<int>(C);
    w->c_env = L.take<int>(C);
    w->c_base = L.take<int>(C);
    w->c_w = L.take<float>(9 * C);
    w->c_rec = L.take<ContactRec>(C);
    w->c_st = L.take<ContactStencil>(C);
    w->c_dyn = L.take<ContactDyn>(C);
    w->c_coef = L.take<double>(11 * ((C + 63) / 64) * 64);
    // the solver's one-barrier form runs for handles of one environment only
    w->qn_uacc = z.n_envs == 1 ? L.take<double>((size_t)9 * kQnScatterMax) : nullptr;
    w->qn_vcblk = z.n_envs == 1 ? L.take<double>((size_t)kQnMaxGroup * kQnRankWords) : nullptr;
    w->qn_lsprm = z.n_envs == 1 ? L.take<double>((size_t)5 * kQnScatterMax) : nullptr;
    w->qn_pend = L.take<int>(z.n_envs);
    // the exact-Newton variant's vectors, only when it is asked for
    w->nt_slot = z.solver == MPM_SOLVER_NEWTON ? L.take<double>((size_t)kNtSlot * z.cap_s) : nullptr;
    w->nt_con = z.solver == MPM_SOLVER_NEWTON ? L.take<double>((size_t)kNtCon * z.cap_c) : nullptr;
    w->solver = z.solver;
    w->pk_a = L.take<unsigned>(27 * C);
    w->pk_b = L.take<unsigned>(27 * C);
    w->pv_a = L.take<unsigned>(27 * C);
    w->pv_b = L.take<unsigned>(27 * C);
    w->e_ent = L.take<Entry>(27 * C);
    const long long S = z.cap_s;
    w->s_node = L.take<int>(S);
    w->s_beg = L.take<int>(S + 1);
    w->s_rec = L.take<SlotRec>(S);
    w->blk = L.take<unsigned>(256 * kSortBlocks + 2 * kSortBlocks);
    w->partial = L.take<double>((size_t)kMaxQnBlocks * kQnSums);
    w->partial_odd = L.take<double>((size_t)kMaxQnBlocks * kQnSums);
    w->partial2 = L.take<double>(3 * kMaxQnBlocks);
    w->qn_lspart = L.take<double>((size_t)4 * kMaxQnBlocks);
    w->rigid_acc = L.take<double>(6 * kMaxRigidTotal);
    w->sstats = L.take<SubstepStats>((size_t)z.N * z.n_envs);
    w->env_pnorm = L.take<double>(z.n_envs);
    w->env_range = L.take<int>(4 * (size_t)z.n_envs);
    w->qn_map = L.take<int2>(kMaxQnBlocks);
    w->env_qn = L.take<int>(2 * (size_t)z.n_envs);
    w->env_bar = L.take<unsigned>((size_t)kBarStride * z.n_envs);
    w->env_ctr = L.take<unsigned>((size_t)kCtrLanes * kCtrStride * z.n_envs);
    const long long T = z.tape_cap;
    w->tape_p = T ? L.take<float>((size_t)T * 24 * P) : nullptr;
    w->tape_g = T ? L.take<float4>((size_t)T * 2 * z.n_nodes) : nullptr;
    w->tape_idx = T ? L.take<unsigned>((size_t)(T / z.N) * P) : nullptr;
    w->adj = T ? L.take<float>((size_t)2 * 24 * P) : nullptr;
    w->gbar = T ? L.take<float4>(z.n_nodes) : nullptr;
    w->lame = T ? L.take<double>(2 * (size_t)z.n_envs) : nullptr;
    w->tape_rig = T ? L.take<DevRigid>((size_t)(T / z.N) * kMaxRigidTape) : nullptr;
    w->tape_env = T ? L.take<DevEnv>((size_t)(T / z.N) * z.n_envs) : nullptr;
    w->cg_vec = T ? L.take<double>((size_t)5 * 3 * z.cap_s) : nullptr;
    w->cg_pinv = T ? L.take<double>((size_t)6 * z.cap_s) : nullptr;
    w->cg_q = T ? L.take<double>((size_t)3 * z.cap_c) : nullptr;
    w->cg_sc = T ? L.take<double>(8) : nullptr;
    w->cxv = T ? L.take<float>((size_t)6 * P) : nullptr;
    w->rgrad = T ? L.take<double>((size_t)(T / z.N) * kMaxRigidTape * kRigidGradStride) : nullptr;
    w->tape_cap = (int)T;
    w->cnt = L.take<DevCounters>(1);
    w->envs = L.take<DevEnv>(z.n_envs);
    w->rigids = L.take<DevRigid>(kMaxRigidTotal);
    w->P = z.P;
    w->n_nodes = z.n_nodes;
    w->n_tiles = z.n_tiles;
    w->n_envs = z.n_envs;
    w->cap_c = z.cap_c;
    w->cap_s = z.cap_s;
    return L.off + kAlign;
}

// What a workspace must hold before its first host step: empty grid
// accumulators and tile maps, zero counters and solver barriers, and the
// environment table (queued on s).
hipError_t init_workspace(const Work& W, const DevEnv* denv, hipStream_t s) {
    hipError_t e = hipMemsetAsync(W.acc, 0, sizeof(float4) * W.n_nodes, s);
    if (e == hipSuccess) e = hipMemsetAsync(W.vel, 0, sizeof(float4) * W.n_nodes, s);
    if (e == hipSuccess) e = hipMemsetAsync(W.tile_flag, 0, sizeof(unsigned) * W.n_tiles, s);
    if (e == hipSuccess) e = hipMemsetAsync(W.ntile_mark, 0, sizeof(unsigned) * W.n_tiles, s);
    if (e == hipSuccess) e = hipMemsetAsync(W.ptile_of, 0xFF, sizeof(int) * W.n_tiles, s);
    if (e == hipSuccess) e = hipMemsetAsync(W.cnt, 0, sizeof(DevCounters), s);
    if (e == hipSuccess) e = hipMemsetAsync(W.env_bar, 0, sizeof(unsigned) * kBarStride * W.n_envs, s);
    if (e == hipSuccess)
        e = hipMemsetAsync(W.env_ctr, 0, sizeof(unsigned) * kCtrLanes * kCtrStride * W.n_envs, s);
    if (e == hipSuccess) e = hipMemcpyAsync(W.envs, denv, sizeof(DevEnv) * W.n_envs, hipMemcpyHostToDevice, s);
    return e;
}

// Solver options of a handle: contact nodes per block (the description's, else
// the default), and the environment overrides used by sweeps and tests:
// MPM_SOLVER_SLOTS_PER_BLOCK overrides the block size, MPM_SOLVER_MAX_BLOCKS
// caps the blocks (below it, environments share blocks), MPM_SOLVER_COMPACT=0
// sends every block through the general node pass, MPM_SOLVER_SCATTER=0 keeps
// every environment on the two-barrier form, MPM_SOLVER_LAUNCH=plain launches
// the solver without the cooperative API (profiler runs; the grid never
// exceeds the co-resident blocks); MPM_SORT_POLICY=truncated (keys cut to
// their top kTruncBits bits) or none (no reordering) selects an arm of the
// sort ablation, with the plain scatter and gather.
void solver_options(const mpm_desc* desc, Work* w, int* slots_per_block, int* qn_cap) {
    const char* spb = getenv("MPM_SOLVER_SLOTS_PER_BLOCK");
    *slots_per_block = spb ? std::max(1, atoi(spb))
                           : (desc->solver_slots_per_block > 0 ? desc->solver_slots_per_block : kQnItemsPerBlock);
    const char* mb = getenv("MPM_SOLVER_MAX_BLOCKS");
    if (mb && atoi(mb) > 0) *qn_cap = std::min(*qn_cap, atoi(mb));
    const char* cp = getenv("MPM_SOLVER_COMPACT");
    w->qn_compact = (cp && atoi(cp) == 0) ? 0 : 1;
    const char* sc = getenv("MPM_SOLVER_SCATTER");
    w->qn_scatter = (sc && atoi(sc) == 0) ? 0 : 1;
    const char* ln = getenv("MPM_SOLVER_LAUNCH");
    w->qn_plain_launch = (ln && strcmp(ln, "plain") == 0) ? 1 : 0;
    // MPM_TRANSFER_BLOCKS: blocks of the tiled P2G and G2P launches
    const char* tb = getenv("MPM_TRANSFER_BLOCKS");
    w->transfer_blocks = (tb && atoi(tb) > 0) ? atoi(tb) : kTransferBlocks;
    // MPM_P2G_WALKS=1 or 2 fixes the tiled P2G's walks per (component, cell);
    // otherwise they follow the particle density (p2g_adapt)
    const char* pw = getenv("MPM_P2G_WALKS");
    const int pwv = pw ? atoi(pw) : 0;
    w->p2g_walks_fixed = (pwv == 1 || pwv == 2) ? 1 : 0;
    w->p2g_walks = pwv == 2 ? 2 : 1;
    // MPM_SORT_POLICY=truncated or none selects an arm of the sort ablation
    const char* sp = getenv("MPM_SORT_POLICY");
    w->sort_policy = !sp ? kSortTiles
                         : strcmp(sp, "truncated") == 0 ? kSortTruncated : strcmp(sp, "none") == 0 ? kSortNone : kSortTiles;
}

// Device table of the environments (tile and node bases in order, Lame
// parameters, the Drucker-Prager slope); returns the sort key width in bits.
int make_dev_envs(const mpm_env_desc* envs, int n_envs, DevEnv* out) {
    int tiles = 0;
    long long nodes = 0;
    for (int e = 0; e < n_envs; ++e) {
        const mpm_env_desc& E = envs[e];
        DevEnv& D = out[e];
        memset(&D, 0, sizeof(D));
        for (int a = 0; a < 3; ++a) {
            D.dims[a] = E.dims[a];
            D.ntile[a] = (E.dims[a] + 3) / 4;
            D.origin[a] = E.origin[a];
            D.gravity[a] = E.gravity[a];
        }
        D.tile_base = tiles;
        D.node_base = nodes;
        tiles += D.ntile[0] * D.ntile[1] * D.ntile[2];
        nodes += (long long)E.dims[0] * E.dims[1] * E.dims[2];
        D.p_begin = E.p_begin;
        D.p_end = E.p_end;
        D.dx = E.dx;
        D.inv_dx = 1.0f / E.dx;
        D.D = 4.0f / (E.dx * E.dx);
        D.mat.type = E.material;
        D.mat.mu = (float)(E.E / (2.0 * (1.0 + E.nu)));
        D.mat.la = (float)(E.E * E.nu / ((1.0 + E.nu) * (1.0 - 2.0 * E.nu)));
        const double sphi = sin(E.friction_angle * M_PI / 180.0);
        D.mat.alpha = (float)(sqrt(2.0 / 3.0) * 2.0 * sphi / (3.0 - sphi));
        D.m_p = E.m_p;
        D.V0 = E.V0;
        D.k = E.k;
        D.d = E.d;
        D.eps_s = E.eps_s;
        D.rigid_begin = D.rigid_end = 0;
    }
    int bits = 1;
    while ((1ll << bits) < (long long)tiles) ++bits;
    return bits + 6;
}

// Shape, motion, friction and pose of a rigid descriptor.
mpm_status check_rigid(const mpm_rigid_desc* r) {
    if (r->shape != MPM_HALF_SPACE && r->shape != MPM_BOX) return fail(MPM_EINVAL, "unknown shape");
    if (r->motion != MPM_STATIC && r->motion != MPM_KINEMATIC && r->motion != MPM_DYNAMIC)
        return fail(MPM_EINVAL, "unknown motion");
    if (r->motion == MPM_DYNAMIC) {
        if (r->shape != MPM_BOX) return fail(MPM_EINVAL, "dynamic bodies are boxes");
        if (!(r->mass > 0.0) || !isfinite(r->mass)) return fail(MPM_EINVAL, "a dynamic body needs mass > 0");
        for (int a = 0; a < 3; ++a) {
            if (!(r->inertia[a] > 0.0) || !isfinite(r->inertia[a]))
                return fail(MPM_EINVAL, "a dynamic body needs principal moments > 0");
            if (!isfinite(r->force[a]) || !isfinite(r->torque[a]))
                return fail(MPM_EINVAL, "external force and torque must be finite");
        }
    }
    if (!(r->mu >= 0.0) || !isfinite(r->mu)) return fail(MPM_EINVAL, "mu must be >= 0");
    if (r->shape == MPM_BOX && !(r->half[0] > 0 && r->half[1] > 0 && r->half[2] > 0))
        return fail(MPM_EINVAL, "degenerate box");
    if (r->shape == MPM_HALF_SPACE) {
        const double nn = r->normal[0] * r->normal[0] + r->normal[1] * r->normal[1] + r->normal[2] * r->normal[2];
        if (!(fabs(nn - 1.0) < 1e-9)) return fail(MPM_EINVAL, "half-space normal must be unit");
    }
    double RtR[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0;
            for (int q = 0; q < 3; ++q) s += r->R[q * 3 + a] * r->R[q * 3 + b];
            RtR[a * 3 + b] = s;
        }
    for (int i = 0; i < 9; ++i)
        if (fabs(RtR[i] - (i % 4 == 0 ? 1.0 : 0.0)) > 1e-9) return fail(MPM_EINVAL, "R must be a rotation");
    return MPM_OK;
}

struct HostRigid {
    mpm_rigid_desc desc;  // shape, pose and twist (pose/twist updated as the step advances)
    int env;
    int kin_steps = 0;    // kinematic host steps the pose has advanced from its reference state
                          // (the last mpm_set_rigid_state, or a pose given to mpm_step)
    int rec_steps = 0;    // the same at the start of the recording
};

__host__ __device__ void rodrigues_advance(double R[9], const double w[3], double dt) {
    const double wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    const double th = wn * dt;
    if (th == 0.0) return;
    const double k[3] = {w[0] / wn, w[1] / wn, w[2] / wn};
    const double K[9] = {0, -k[2], k[1], k[2], 0, -k[0], -k[1], k[0], 0};
    double K2[9], Rot[9], Rn[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double s = 0;
            for (int q = 0; q < 3; ++q) s += K[r * 3 + q] * K[q * 3 + c];
            K2[r * 3 + c] = s;
        }
    for (int i = 0; i < 9; ++i) Rot[i] = sin(th) * K[i] + (1.0 - cos(th)) * K2[i] + (i % 4 == 0 ? 1.0 : 0.0);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double s = 0;
            for (int q = 0; q < 3; ++q) s += Rot[r * 3 + q] * R[q * 3 + c];
            Rn[r * 3 + c] = s;
        }
    for (int i = 0; i < 9; ++i) R[i] = Rn[i];
}

// For the rotation vector phi (angle |phi| about phi / |phi|): o = Rot(phi)^T v,
// and o = J(phi)^T v with J(phi) = I + (1 - cos t)/t^2 [phi]x + (t - sin t)/t^3
// [phi]x^2, t = |phi|, the left Jacobian of the rotation map (series below
// t = 1e-4).
void rotate_transposed(const double phi[3], const double v[3], double o[3]) {
    const double t = sqrt(phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2]);
    if (t == 0.0) {
        for (int a = 0; a < 3; ++a) o[a] = v[a];
        return;
    }
    const double k[3] = {phi[0] / t, phi[1] / t, phi[2] / t};
    const double kv[3] = {k[1] * v[2] - k[2] * v[1], k[2] * v[0] - k[0] * v[2], k[0] * v[1] - k[1] * v[0]};
    const double kkv[3] = {k[1] * kv[2] - k[2] * kv[1], k[2] * kv[0] - k[0] * kv[2], k[0] * kv[1] - k[1] * kv[0]};
    for (int a = 0; a < 3; ++a) o[a] = v[a] - sin(t) * kv[a] + (1.0 - cos(t)) * kkv[a];
}
void left_jacobian_transposed(const double phi[3], const double v[3], double o[3]) {
    const double t2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2], t = sqrt(t2);
    const double a = t < 1e-4 ? 0.5 - t2 / 24.0 : (1.0 - cos(t)) / t2;
    const double b = t < 1e-4 ? 1.0 / 6.0 - t2 / 120.0 : (t - sin(t)) / (t2 * t);
    const double pv[3] = {phi[1] * v[2] - phi[2] * v[1], phi[2] * v[0] - phi[0] * v[2], phi[0] * v[1] - phi[1] * v[0]};
    const double ppv[3] = {phi[1] * pv[2] - phi[2] * pv[1], phi[2] * pv[0] - phi[0] * pv[2],
                           phi[0] * pv[1] - phi[1] * pv[0]};
    for (int q = 0; q < 3; ++q) o[q] = v[q] - a * pv[q] + b * ppv[q];
}

// A free body over one host step of length dt (the rigid side of the split,
// Eq. (3) with the body's mass matrix and Coriolis term, semi-implicit): the
// impulse imp[0..2] and its moment imp[3..5] about the body origin, which the
// MPM side exerted on the body during the step, plus gravity and the constant
// external wrench over dt, give the new twist,
//   V' = V + imp/m + dt (g + f/m),   w' = w + I_w^-1 (imp_ang + dt (tau - w x I_w w)),
// with I_w = R diag(I) R^T; the pose then advances with it (in the caller).
void integrate_free_body(mpm_rigid_desc& d, const double imp[6], const float g[3], double dt) {
    for (int a = 0; a < 3; ++a) d.V[a] = d.V[a] + imp[a] / d.mass + dt * ((double)g[a] + d.force[a] / d.mass);
    double Iw[9], Ii[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double a = 0.0, b = 0.0;
            for (int k = 0; k < 3; ++k) {
                a += d.R[i * 3 + k] * d.inertia[k] * d.R[j * 3 + k];
                b += d.R[i * 3 + k] * d.R[j * 3 + k] / d.inertia[k];
            }
            Iw[i * 3 + j] = a;
            Ii[i * 3 + j] = b;
        }
    double L[3];
    for (int i = 0; i < 3; ++i) L[i] = Iw[i * 3] * d.w[0] + Iw[i * 3 + 1] * d.w[1] + Iw[i * 3 + 2] * d.w[2];
    const double wxL[3] = {d.w[1] * L[2] - d.w[2] * L[1], d.w[2] * L[0] - d.w[0] * L[2], d.w[0] * L[1] - d.w[1] * L[0]};
    double m[3];
    for (int a = 0; a < 3; ++a) m[a] = imp[3 + a] + dt * (d.torque[a] - wxL[a]);
    double dw[3];
    for (int i = 0; i < 3; ++i) dw[i] = Ii[i * 3] * m[0] + Ii[i * 3 + 1] * m[1] + Ii[i * 3 + 2] * m[2];
    for (int a = 0; a < 3; ++a) d.w[a] += dw[a];
}

// The kinematic advance of the rigid table on the device (graph path): the
// same rule as the host's; static bodies carry a zero twist.
__global__ void k_advance_kinematic(DevRigid* r, int n, double dt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    DevRigid& q = r[i];
    for (int a = 0; a < 3; ++a) q.t[a] += dt * q.V[a];
    rodrigues_advance(q.R, q.w, dt);
}

hipError_t launch_advance_kinematic(DevRigid* r, int n, double dt, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_advance_kinematic, dim3((n + 63) / 64), dim3(64), 0, s, r, n, dt);
    return hipGetLastError();
}

}  // namespace

struct mpm_handle {
    mpm_desc d;
    std::vector<mpm_env_desc> envs;
    std::vector<DevEnv> denv;
    std::vector<HostRigid> rigids;  // in order of addition (user ids)
    Work w;
    hipStream_t stream;
    int key_bits;
    int qn_cap;          // co-resident blocks the cooperative solver may use
    double wall_khz;     // device wall-clock rate
    int slots_per_block; // contact nodes per solver block
    std::vector<int> env_slots;  // per environment: most contact nodes in a substep of the last step
    // differentiation tape
    bool tape_on = false;  // recording since mpm_tape_reset
    int tape_len = 0;      // substeps recorded
    std::vector<int> tape_ncon;  // contacts of each recorded substep (all environments)
    // pinned host staging
    DevRigid* h_rigids;
    double* h_racc;
    SubstepStats* h_stats;  // [N][n_envs]
    DevCounters* h_cnt;
    int2* h_qn_map;         // solver plan staging
    int* h_env_qn;
    // profiling
    bool prof = false;
    bool prof_phases = false;  // solver phase timers (they lengthen the solve)
    std::vector<hipEvent_t> events;   // pairs (start, stop)
    std::vector<int> ev_class;        // kernel class of each pair
    mpm_profile_data acc;
    // graph path: a stream of its own (capture needs one that is not the null
    // stream), ordered after the handle's stream by an event
    hipStream_t gstream = nullptr;
    hipEvent_t gevent = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int graph_steps = 0, graph_qn_blocks = 0, graph_stride = 0, graph_nr = -1, graph_walks = 0;
};

namespace {
// Event pair around a launch group when profiling is on.
struct ProfScope {
    mpm_handle* h;
    int pair;
    ProfScope(mpm_handle* hh, int cls, int& next) : h(hh), pair(-1) {
        if (!h || !h->prof) return;
        pair = next++;
        if ((int)h->ev_class.size() <= pair) {
            hipEvent_t a, b;
            if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) { pair = -1; --next; return; }
            h->events.push_back(a);
            h->events.push_back(b);
            h->ev_class.push_back(cls);
        }
        h->ev_class[pair] = cls;
        (void)hipEventRecord(h->events[2 * pair], h->stream);
    }
    ~ProfScope() {
        if (pair >= 0) (void)hipEventRecord(h->events[2 * pair + 1], h->stream);
    }
};
// Environment with the most solver iterations in one substep's stats.
int longest_solve(const SubstepStats* q, int n_envs) {
    int best = 0;
    for (int e = 1; e < n_envs; ++e)
        if (q[e].iterations > q[best].iterations) best = e;
    return best;
}

// Solver plan for one host step: a group of blocks per environment, sized by
// the environment's contact nodes in the previous step (at least one block,
// at most kQnMaxGroup, all groups co-resident). With more environments than
// co-resident blocks every block takes environments in turn. Fills the
// staging tables qn_map and env_qn (g: scratch of n_envs entries); returns the
// number of blocks.
int plan_groups(int n_envs, const int* env_slots, int slots_per_block, int cap, int* g, int2* qn_map,
                int* env_qn, int* env_stride) {
    if (n_envs > cap) {
        for (int b = 0; b < cap; ++b) qn_map[b] = make_int2(b, 0);
        for (int e = 0; e < n_envs; ++e) {
            env_qn[2 * e] = e % cap;
            env_qn[2 * e + 1] = 1;
        }
        *env_stride = cap;
        return cap;
    }
    int total = 0;
    for (int e = 0; e < n_envs; ++e) {
        g[e] = std::max(1, std::min(kQnMaxGroup, (env_slots[e] + slots_per_block - 1) / slots_per_block));
        total += g[e];
    }
    while (total > cap) {  // shrink the largest groups until all fit
        int big = 0;
        for (int e = 1; e < n_envs; ++e)
            if (g[e] > g[big]) big = e;
        --g[big];
        --total;
    }
    // The counts come from an earlier substep; the kernel sizes each group from
    // the current one and leaves surplus blocks idle. Spare co-resident blocks
    // go to the groups as headroom, one at a time, smallest group first, so an
    // environment whose contact grows (or starts) is not held to a stale size.
    for (bool grew = true; grew && total < cap;) {
        grew = false;
        int small = -1;
        for (int e = 0; e < n_envs; ++e)
            if (g[e] < kQnMaxGroup && (small < 0 || g[e] < g[small])) small = e;
        if (small >= 0) {
            ++g[small];
            ++total;
            grew = true;
        }
    }
    int b = 0;
    for (int e = 0; e < n_envs; ++e) {
        env_qn[2 * e] = b;
        env_qn[2 * e + 1] = g[e];
        for (int r = 0; r < g[e]; ++r) qn_map[b++] = make_int2(e, r);
    }
    *env_stride = 0;
    return total;
}

int plan_solver(mpm_handle* h, int* env_stride) {
    const int n_envs = (int)h->envs.size();
    std::vector<int> g(n_envs);
    return plan_groups(n_envs, h->env_slots.data(), h->slots_per_block, h->qn_cap, g.data(), h->h_qn_map,
                       h->h_env_qn, env_stride);
}

// Device entry k of the rigid table from a descriptor in environment env
// (static bodies carry a zero twist); extends the environment's range, so the
// entries of one environment must be placed consecutively.
void place_dev_rigid(const mpm_rigid_desc& d, int env, int k, DevRigid* R, DevEnv* denv) {
    R->shape = d.shape;
    R->env = env;
    memcpy(R->normal, d.normal, sizeof(R->normal));
    R->offset = d.offset;
    memcpy(R->half, d.half, sizeof(R->half));
    R->mu = d.mu;
    memcpy(R->R, d.R, sizeof(R->R));
    memcpy(R->t, d.t, sizeof(R->t));
    if (d.motion == MPM_STATIC) {
        memset(R->V, 0, sizeof(R->V));
        memset(R->w, 0, sizeof(R->w));
    } else {
        memcpy(R->V, d.V, sizeof(R->V));
        memcpy(R->w, d.w, sizeof(R->w));
    }
    DevEnv& D = denv[env];
    if (D.rigid_end == D.rigid_begin) D.rigid_begin = D.rigid_end = k;
    D.rigid_end = k + 1;
}

// Device-order rigid table (h_rigids) and each environment's rigid range from
// the host state, grouped by environment (stable) so that each environment
// owns a range; order[k] is the user id of device entry k.
void build_rigid_table(mpm_handle* h, std::vector<int>& order) {
    const int nr = (int)h->rigids.size();
    order.resize(nr);
    for (int i = 0; i < nr; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return h->rigids[a].env < h->rigids[b].env; });
    for (DevEnv& D : h->denv) D.rigid_begin = D.rigid_end = 0;
    for (int k = 0; k < nr; ++k) {
        const HostRigid& q = h->rigids[order[k]];
        place_dev_rigid(q.desc, q.env, k, h->h_rigids + k, h->denv.data());
    }
    h->w.n_rigid = nr;
}

// What one host step's device work needs besides the workspace: the
// description, the sort key width, the solver's group sizing, the tape
// position when recording, and the handle whose event timing is on (NULL for
// none).
struct StepCtx {
    Work* w;
    const mpm_desc* d;
    int key_bits;
    int slots_per_block;
    bool rec;
    int tape_len;
    mpm_handle* prof;
    bool phases;
};

StepCtx step_ctx(mpm_handle* h) {
    StepCtx c;
    c.w = &h->w;
    c.d = &h->d;
    c.key_bits = h->key_bits;
    c.slots_per_block = h->slots_per_block;
    c.rec = h->tape_on;
    c.tape_len = h->tape_len;
    c.prof = h;
    c.phases = h->prof_phases;
    return c;
}

// Device work of one host step on the handle's stream (the tables are already
// uploaded). Inside a graph the step clears only its statistics (the replay
// clears flags and impulse sums once), records neither tape nor events, and
// ends by advancing the kinematic bodies on the device.
mpm_status enqueue_host_step(const StepCtx& c, int qn_blocks, int env_stride, bool graph, int& npair,
                             hipStream_t s) {
    Work& W = *c.w;
    const mpm_desc& d = *c.d;
    const int N = d.N;
    const int ls_steps = d.ls_max_steps > 0 ? d.ls_max_steps : 100;
    const int n_envs = W.n_envs;
    const int nr = W.n_rigid;
    const bool rec = !graph && c.rec;
    mpm_handle* h = c.prof;
    HIP_TRY(launch_clear_step(W, N, graph, s));
    {
        // once per host step: cell keys, stable sort, gather, tile list (Sec. V-A)
        ProfScope ps(h, MPM_K_SORT, npair);
        const bool trunc = W.sort_policy == kSortTruncated;
        const int shift = trunc ? std::max(0, c.key_bits - kTruncBits) : 0;
        HIP_TRY(launch_keys(W, d.x, shift, s));
        unsigned *keys_sorted = W.key_a, *idx_sorted = W.idx_a;  // unsorted: the identity order
        if (W.sort_policy != kSortNone)
            HIP_TRY(radix_sort(W, W.key_a, W.idx_a, W.key_b, W.idx_b, nullptr, W.P, c.key_bits - shift, s,
                               &keys_sorted, &idx_sorted));
        HIP_TRY(launch_permute(W, idx_sorted, d.x, d.v, d.F, d.C, d.pid, d.h, s));
        if (rec) {
            const size_t j = (size_t)(c.tape_len / N);
            HIP_TRY(hipMemcpyAsync(W.tape_idx + j * W.P, idx_sorted, sizeof(unsigned) * W.P,
                                   hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipMemcpyAsync(W.tape_rig + j * kMaxRigidTape, W.rigids, sizeof(DevRigid) * std::max(nr, 1),
                                   hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipMemcpyAsync(W.tape_env + j * n_envs, W.envs, sizeof(DevEnv) * n_envs,
                                   hipMemcpyDeviceToDevice, s));
        }
        if (W.sort_policy == kSortTiles) {
            HIP_TRY(launch_tile_maps(W, s, true));   // forget the previous step's tiles
            HIP_TRY(launch_tile_list(W, keys_sorted, s));
            HIP_TRY(launch_tile_maps(W, s, false));
        } else {
            HIP_TRY(launch_no_tiles(W, s));
        }
        W.keys_sorted = keys_sorted;
    }
    for (int k = 0; k < N; ++k) {
        const bool first = k == 0, last = k == N - 1;
        const float* x_in = first ? W.xs : d.x;
        const float* v_in = first ? W.vs : d.v;
        const float* F_in = first ? W.Fs : d.F;
        HIP_TRY(launch_clear_substep(W, s));
        float* tp = rec ? W.tape_p + (size_t)(c.tape_len + k) * 24 * W.P : nullptr;
        float4* tg = rec ? W.tape_g + (size_t)(c.tape_len + k) * 2 * W.n_nodes : nullptr;
        if (rec) {
            const size_t P = W.P;
            HIP_TRY(hipMemcpyAsync(tp, x_in, sizeof(float) * 3 * P, hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipMemcpyAsync(tp + 3 * P, v_in, sizeof(float) * 3 * P, hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipMemcpyAsync(tp + 6 * P, F_in, sizeof(float) * 9 * P, hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipMemcpyAsync(tp + 15 * P, W.Q, sizeof(float) * 9 * P, hipMemcpyDeviceToDevice, s));
        }
        {
            ProfScope ps(h, MPM_K_P2G, npair);
            if (W.sort_policy == kSortTiles)
                HIP_TRY(launch_p2g(W, x_in, v_in, s));
            else
                HIP_TRY(launch_p2g_plain(W, x_in, v_in, s));
        }
        {
            ProfScope ps(h, MPM_K_GRID, npair);
            HIP_TRY(launch_grid_update(W, d.h, s));
        }
        if (rec) HIP_TRY(hipMemcpyAsync(tg, W.vel, sizeof(float4) * W.n_nodes, hipMemcpyDeviceToDevice, s));
        {
            ProfScope ps(h, MPM_K_REGISTER, npair);
            HIP_TRY(launch_registration(W, x_in, v_in, d.h, k, s));
        }
        {
            ProfScope ps(h, MPM_K_SETUP, npair);
            HIP_TRY(launch_contact_setup(W, s));
        }
        {
            ProfScope ps(h, MPM_K_SOLVE, npair);
            HIP_TRY(launch_qn(W, x_in, k, d.h, d.eps_r, d.eps_a, d.max_iter, ls_steps, qn_blocks,
                              env_stride, c.phases ? 1 : 0, c.slots_per_block, s));
        }
        if (rec)
            HIP_TRY(hipMemcpyAsync(tg + W.n_nodes, W.vel, sizeof(float4) * W.n_nodes, hipMemcpyDeviceToDevice, s));
        {
            ProfScope ps(h, MPM_K_G2P, npair);
            if (W.sort_policy == kSortTiles)
                HIP_TRY(launch_g2p(W, x_in, F_in, d.x, d.v, d.F, last ? d.C : nullptr,
                                   (first && d.pid) ? W.pids : nullptr, (first && d.pid) ? d.pid : nullptr, d.h, s));
            else
                HIP_TRY(launch_g2p_plain(W, x_in, F_in, d.x, d.v, d.F, last ? d.C : nullptr,
                                         (first && d.pid) ? W.pids : nullptr, (first && d.pid) ? d.pid : nullptr, d.h,
                                         s));
        }
    }
    if (graph) HIP_TRY(launch_advance_kinematic(W.rigids, nr, N * d.h, s));
    return MPM_OK;
}

// The caller's statistics of a host step from the per-substep, per-environment
// records (over the environments: the longest solve, all contacts, the worst
// residual relative to its threshold).
void fill_step_stats(const SubstepStats* stats, int N, int n_envs, unsigned flags, mpm_step_stats* st) {
    if (!st) return;
    st->flags = (int32_t)(flags & 0xF);
    st->max_iterations = 0;
    st->total_iterations = 0;
    st->max_contacts = 0;
    st->total_inner_iterations = 0;
    for (int k = 0; k < N; ++k) {
        const SubstepStats* q = stats + (size_t)k * n_envs;
        const SubstepStats& lead = q[longest_solve(q, n_envs)];
        int contacts = 0, nodes = 0, worst = 0;
        for (int e = 0; e < n_envs; ++e) {
            contacts += q[e].n_contacts;
            nodes += q[e].n_slots;
            if (q[e].threshold > 0.0 &&
                (q[worst].threshold <= 0.0 || q[e].residual * q[worst].threshold > q[worst].residual * q[e].threshold))
                worst = e;
        }
        st->max_iterations = std::max(st->max_iterations, lead.iterations);
        st->total_iterations += lead.iterations;
        st->total_inner_iterations += lead.inner_iterations;
        st->max_contacts = std::max(st->max_contacts, contacts);
        if (st->iterations) st->iterations[k] = lead.iterations;
        if (st->contacts) st->contacts[k] = contacts;
        if (st->contact_nodes) st->contact_nodes[k] = nodes;
        if (st->residual) st->residual[k] = q[worst].residual;
        if (st->threshold) st->threshold[k] = q[worst].threshold;
    }
}

// Status of a host step from its device flags.
mpm_status step_status(unsigned flags, long long cap_c, unsigned n_contacts) {
    if (flags & 16u) return fail(MPM_EDEVICE, "contact solver barrier timed out");
    if (flags & MPM_FLAG_CAPACITY)
        return fail(MPM_ENOMEM, "contact capacity %lld exceeded (%u contacts)", cap_c, n_contacts);
    if (flags & MPM_FLAG_NAN) return fail(MPM_ENAN, "non-finite particle state");
    if (flags & MPM_FLAG_DOMAIN) return fail(MPM_EDOMAIN, "a particle stencil left the grid");
    if (flags & MPM_FLAG_NOCONV) return fail(MPM_ENOCONV, "contact solve hit max_iter");
    return MPM_OK;
}

// After the stream has synchronised (counters, statistics and impulses copied
// to the host): tape bookkeeping, profile sums, outputs in user order, the
// statistics, the next step's solver plan, and the status of the host step(s).
mpm_status finish_host_steps(mpm_handle* h, const std::vector<int>& order, int npair, bool rec,
                             mpm_rigid_impulse* out, mpm_step_stats* st) {
    Work& W = h->w;
    hipStream_t s = h->stream;
    const mpm_desc& d = h->d;
    const int N = d.N;
    const int n_envs = (int)h->envs.size();
    const int nr = W.n_rigid;
    const unsigned flags = h->h_cnt->flags;
    if (rec) {
        h->tape_len += N;
        for (int k = 0; k < N; ++k) {
            int nc = 0;
            for (int e = 0; e < n_envs; ++e) nc += h->h_stats[(size_t)k * n_envs + e].n_contacts;
            h->tape_ncon.push_back(nc);
        }
    }
    if (h->prof) {
        for (int q = 0; q < npair; ++q) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, h->events[2 * q], h->events[2 * q + 1]));
            h->acc.ms[h->ev_class[q]] += ms;
            h->acc.launches[h->ev_class[q]] += 1;
        }
        for (int k = 0; k < N; ++k) {
            const SubstepStats* q = h->h_stats + (size_t)k * n_envs;
            const SubstepStats& lead = q[longest_solve(q, n_envs)];
            h->acc.solver_iterations += lead.iterations;
            h->acc.solver_ls_rounds += lead.ls_rounds;
            for (int e = 0; e < n_envs; ++e) {
                h->acc.solver_contact_iters += (int64_t)q[e].iterations * q[e].n_contacts;
                h->acc.solver_node_iters += (int64_t)q[e].iterations * q[e].n_slots;
                h->acc.solver_contact_rounds += (int64_t)q[e].ls_rounds * q[e].n_contacts;
            }
            for (int ph = 0; ph < 8; ++ph) h->acc.solver_phase_us[ph] += 1e3 * (double)lead.t_phase[ph] / h->wall_khz;
        }
    }
    if (h->h_cnt->abort_step && h->h_cnt->abort_substep > 0) {
        // the step stopped early: the caller's C lags the state; rebuild it from Q
        HIP_TRY(launch_recover_C(W, d.F, d.C, d.h, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    // outputs in user order
    if (out) {
        for (int k = 0; k < nr; ++k) {
            mpm_rigid_impulse& o = out[order[k]];
            for (int a = 0; a < 3; ++a) {
                o.impulse[a] = h->h_racc[6 * k + a];
                o.torque[a] = h->h_racc[6 * k + 3 + a];
            }
        }
    }
    fill_step_stats(h->h_stats, N, n_envs, flags, st);
    // size the next step's solver groups from this step's problems
    for (int e = 0; e < n_envs; ++e) {
        int most = 0;
        for (int k = 0; k < N; ++k) most = std::max(most, h->h_stats[(size_t)k * n_envs + e].n_slots);
        h->env_slots[e] = most;
    }
    return step_status(flags, W.cap_c, h->h_cnt->n_contacts);
}


}  // namespace

extern "C" {

const char* mpm_last_error(void) { return g_err.c_str(); }

mpm_status mpm_workspace_size(const mpm_desc* desc, size_t* bytes) {
    if (!bytes) return fail(MPM_EINVAL, "bytes is NULL");
    Sizes z;
    mpm_status st = validate(desc, &z);
    if (st != MPM_OK) return st;
    Work w;
    *bytes = layout(z, nullptr, &w);
    return MPM_OK;
}

mpm_status mpm_create(const mpm_desc* desc, mpm_handle** out) {
    if (!out) return fail(MPM_EINVAL, "out is NULL");
    *out = nullptr;
    Sizes z;
    mpm_status st = validate(desc, &z);
    if (st != MPM_OK) return st;
    if (!desc->x || !desc->v || !desc->F || !desc->C) return fail(MPM_EINVAL, "state pointers must be non-NULL");
    if (!desc->workspace) return fail(MPM_EINVAL, "workspace is NULL");
    if (((uintptr_t)desc->workspace) % kAlign) return fail(MPM_EINVAL, "workspace must be 256-byte aligned");
    Work w;
    const size_t need = layout(z, nullptr, &w);
    if (desc->workspace_bytes < need)
        return fail(MPM_ENOMEM, "workspace has %zu bytes, needs %zu", desc->workspace_bytes, need);
    const int qn_cap = qn_max_blocks();
    if (qn_cap < 1) return fail(MPM_EDEVICE, "cannot size the cooperative solver launch");

    mpm_handle* h = new mpm_handle();
    h->d = *desc;
    h->envs.assign(desc->envs, desc->envs + desc->n_envs);
    h->d.envs = nullptr;
    h->stream = (hipStream_t)desc->stream;
    layout(z, (char*)desc->workspace, &h->w);
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) {
        delete h;
        return fail(MPM_EDEVICE, "cannot query the device");
    }
    h->w.qn_blocks = std::max(1, std::min(qn_cap, kMaxQnBlocks));
    h->qn_cap = h->w.qn_blocks;
    h->env_slots.assign(desc->n_envs, 0);
    {
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) khz = 100000;
        h->wall_khz = khz;
    }
    solver_options(desc, &h->w, &h->slots_per_block, &h->qn_cap);
    if (h->w.sort_policy != kSortTiles && desc->tape_substeps > 0) {
        delete h;
        return fail(MPM_EINVAL, "the sort-policy arms run without the differentiation tape");
    }
    h->w.n_rigid = 0;
    h->denv.resize(desc->n_envs);
    h->key_bits = make_dev_envs(desc->envs, desc->n_envs, h->denv.data());
    if (hipHostMalloc((void**)&h->h_rigids, sizeof(DevRigid) * kMaxRigidTotal) != hipSuccess ||
        hipHostMalloc((void**)&h->h_racc, sizeof(double) * 6 * kMaxRigidTotal) != hipSuccess ||
        hipHostMalloc((void**)&h->h_stats, sizeof(SubstepStats) * desc->N * desc->n_envs) != hipSuccess ||
        hipHostMalloc((void**)&h->h_cnt, sizeof(DevCounters)) != hipSuccess ||
        hipHostMalloc((void**)&h->h_qn_map, sizeof(int2) * kMaxQnBlocks) != hipSuccess ||
        hipHostMalloc((void**)&h->h_env_qn, sizeof(int) * 2 * desc->n_envs) != hipSuccess) {
        mpm_destroy(h);
        return fail(MPM_EDEVICE, "hipHostMalloc failed");
    }
    hipStream_t s = h->stream;
    const Work& W = h->w;
    hipError_t e = init_workspace(W, h->denv.data(), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        mpm_destroy(h);
        return fail(MPM_EDEVICE, "workspace initialisation failed: %s", hipGetErrorString(e));
    }
    *out = h;
    return MPM_OK;
}

mpm_status mpm_add_rigid_sdf(mpm_handle* h, int32_t env, const mpm_rigid_desc* r, int32_t* id) {
    if (!h || !r) return fail(MPM_EINVAL, "handle or descriptor is NULL");
    if (env < 0 || env >= (int)h->envs.size()) return fail(MPM_EINVAL, "env %d out of range", env);
    if ((int)h->rigids.size() >= kMaxRigidTotal) return fail(MPM_EINVAL, "at most %d rigid bodies", kMaxRigidTotal);
    int in_env = 0;
    for (const HostRigid& q : h->rigids) in_env += q.env == env;
    if (in_env >= kMaxRigidPerEnv) return fail(MPM_EINVAL, "at most %d rigid bodies per environment", kMaxRigidPerEnv);
    const mpm_status rs = check_rigid(r);
    if (rs != MPM_OK) return rs;
    HostRigid q;
    q.desc = *r;
    q.env = env;
    h->rigids.push_back(q);
    if (id) *id = (int32_t)h->rigids.size() - 1;
    return MPM_OK;
}

mpm_status mpm_set_rigid_state(mpm_handle* h, int32_t id, const mpm_rigid_state* s, int32_t host_steps) {
    if (!h || !s) return fail(MPM_EINVAL, "handle or state is NULL");
    if (id < 0 || id >= (int)h->rigids.size()) return fail(MPM_EINVAL, "rigid id %d out of range", id);
    if (host_steps < 0) return fail(MPM_EINVAL, "host_steps must be >= 0");
    HostRigid& q = h->rigids[id];
    mpm_rigid_desc d = q.desc;
    memcpy(d.R, s->R, sizeof(d.R));
    memcpy(d.t, s->t, sizeof(d.t));
    memcpy(d.V, s->V, sizeof(d.V));
    memcpy(d.w, s->w, sizeof(d.w));
    const mpm_status rs = check_rigid(&d);
    if (rs != MPM_OK) return rs;
    if (host_steps > 0 && d.motion == MPM_KINEMATIC) {
        // the library's kinematic rule, host step by host step
        const double dT = h->d.N * h->d.h;
        for (int j = 0; j < host_steps; ++j) {
            for (int a = 0; a < 3; ++a) d.t[a] += dT * d.V[a];
            rodrigues_advance(d.R, d.w, dT);
        }
    }
    q.desc = d;
    q.kin_steps = d.motion == MPM_KINEMATIC ? host_steps : 0;
    return MPM_OK;
}

mpm_status mpm_get_rigid_state(const mpm_handle* h, int32_t id, mpm_rigid_state* s) {
    if (!h || !s) return fail(MPM_EINVAL, "handle or output is NULL");
    if (id < 0 || id >= (int)h->rigids.size()) return fail(MPM_EINVAL, "rigid id %d out of range", id);
    const mpm_rigid_desc& d = h->rigids[id].desc;
    memcpy(s->R, d.R, sizeof(s->R));
    memcpy(s->t, d.t, sizeof(s->t));
    memcpy(s->V, d.V, sizeof(s->V));
    memcpy(s->w, d.w, sizeof(s->w));
    return MPM_OK;
}

mpm_status mpm_step(mpm_handle* h, const mpm_rigid_state* in, mpm_rigid_impulse* out, mpm_step_stats* st) {
    if (!h) return fail(MPM_EINVAL, "handle is NULL");
    const bool rec = h->tape_on;
    if (rec && h->tape_len + h->d.N > h->w.tape_cap)
        return fail(MPM_ENOMEM, "the differentiation tape is full (%d substeps)", h->w.tape_cap);
    const int nr = (int)h->rigids.size();
    // frozen rigid state for this host step
    if (in) {
        for (int i = 0; i < nr; ++i) {
            mpm_rigid_desc& d = h->rigids[i].desc;
            memcpy(d.R, in[i].R, sizeof(d.R));
            memcpy(d.t, in[i].t, sizeof(d.t));
            memcpy(d.V, in[i].V, sizeof(d.V));
            memcpy(d.w, in[i].w, sizeof(d.w));
            h->rigids[i].kin_steps = 0;
        }
    }
    // the first host step of a recording: where the poses stand on their path
    if (rec && h->tape_len == 0)
        for (HostRigid& q : h->rigids) q.rec_steps = q.kin_steps;
    std::vector<int> order;
    build_rigid_table(h, order);
    Work& W = h->w;
    hipStream_t s = h->stream;
    const int N = h->d.N;
    const int n_envs = (int)h->envs.size();
    int env_stride = 0;
    const int qn_blocks = plan_solver(h, &env_stride);
    HIP_TRY(hipMemcpyAsync(W.rigids, h->h_rigids, sizeof(DevRigid) * std::max(nr, 1), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(W.envs, h->denv.data(), sizeof(DevEnv) * h->denv.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(W.qn_map, h->h_qn_map, sizeof(int2) * qn_blocks, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(W.env_qn, h->h_env_qn, sizeof(int) * 2 * n_envs, hipMemcpyHostToDevice, s));
    int npair = 0;
    const mpm_status es = enqueue_host_step(step_ctx(h), qn_blocks, env_stride, false, npair, s);
    if (es != MPM_OK) return es;
    HIP_TRY(hipMemcpyAsync(h->h_cnt, W.cnt, sizeof(DevCounters), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h->h_stats, W.sstats, sizeof(SubstepStats) * N * n_envs, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h->h_racc, W.rigid_acc, sizeof(double) * 6 * std::max(nr, 1), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    p2g_adapt(W, h->h_cnt->n_ptiles);
    const mpm_desc& d = h->d;
    // host side of the split: advance kinematic bodies with their twist, and
    // integrate dynamic bodies from this step's impulses (device order k)
    for (int k = 0; k < nr; ++k) {
        HostRigid& q = h->rigids[order[k]];
        const double dt = N * d.h;
        if (q.desc.motion == MPM_DYNAMIC) integrate_free_body(q.desc, h->h_racc + 6 * k, h->envs[q.env].gravity, dt);
        if (q.desc.motion == MPM_STATIC) continue;
        for (int a = 0; a < 3; ++a) q.desc.t[a] += dt * q.desc.V[a];
        rodrigues_advance(q.desc.R, q.desc.w, dt);
        ++q.kin_steps;
    }
    return finish_host_steps(h, order, npair, rec, out, st);
}

mpm_status mpm_step_graph(mpm_handle* h, int32_t n_steps, mpm_rigid_impulse* out, mpm_step_stats* st) {
    if (!h) return fail(MPM_EINVAL, "handle is NULL");
    if (n_steps < 1) return fail(MPM_EINVAL, "n_steps must be at least 1 (got %d)", (int)n_steps);
    if (h->tape_on) return fail(MPM_EINVAL, "the graph path does not record the differentiation tape");
    if (h->prof) return fail(MPM_EINVAL, "the graph path does not run while mpm_profile timing is on");
    for (const HostRigid& q : h->rigids)
        if (q.desc.motion == MPM_DYNAMIC)
            return fail(MPM_EINVAL, "the graph path advances kinematic bodies only (a dynamic body needs each "
                                    "step's impulses on the host)");
    if (!h->gstream) {
        HIP_TRY(hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&h->gevent, hipEventDisableTiming));
    }
    std::vector<int> order;
    build_rigid_table(h, order);
    Work& W = h->w;
    hipStream_t s = h->gstream;
    const int N = h->d.N;
    const int n_envs = (int)h->envs.size();
    const int nr = W.n_rigid;
    int env_stride = 0;
    const int qn_blocks = plan_solver(h, &env_stride);
    if (h->graph_exec && (h->graph_steps != n_steps || h->graph_qn_blocks != qn_blocks ||
                          h->graph_stride != env_stride || h->graph_nr != nr ||
                          h->graph_walks != W.p2g_walks)) {
        HIP_TRY(hipGraphExecDestroy(h->graph_exec));
        HIP_TRY(hipGraphDestroy(h->graph));
        h->graph_exec = nullptr;
        h->graph = nullptr;
    }
    // after everything already queued on the handle's stream
    HIP_TRY(hipEventRecord(h->gevent, h->stream));
    HIP_TRY(hipStreamWaitEvent(s, h->gevent, 0));
    HIP_TRY(hipMemcpyAsync(W.rigids, h->h_rigids, sizeof(DevRigid) * std::max(nr, 1), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(W.envs, h->denv.data(), sizeof(DevEnv) * h->denv.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(W.qn_map, h->h_qn_map, sizeof(int2) * qn_blocks, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(W.env_qn, h->h_env_qn, sizeof(int) * 2 * n_envs, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_clear_step(W, N, false, s));  // once per replay: flags, abort state, impulse sums
    if (!h->graph_exec) {
        HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        mpm_status cs = MPM_OK;
        int npair = 0;
        const StepCtx ctx = step_ctx(h);
        for (int j = 0; j < n_steps && cs == MPM_OK; ++j) cs = enqueue_host_step(ctx, qn_blocks, env_stride, true, npair, s);
        hipGraph_t g = nullptr;
        const hipError_t ee = hipStreamEndCapture(s, &g);
        if (cs != MPM_OK) {
            if (g) (void)hipGraphDestroy(g);
            return cs;
        }
        if (ee != hipSuccess) return fail(MPM_EDEVICE, "graph capture failed: %s", hipGetErrorString(ee));
        hipGraphExec_t ge = nullptr;
        const hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
            (void)hipGraphDestroy(g);
            return fail(MPM_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(ie));
        }
        h->graph = g;
        h->graph_exec = ge;
        h->graph_steps = n_steps;
        h->graph_qn_blocks = qn_blocks;
        h->graph_stride = env_stride;
        h->graph_walks = W.p2g_walks;
        h->graph_nr = nr;
    }
    HIP_TRY(hipGraphLaunch(h->graph_exec, s));
    HIP_TRY(hipMemcpyAsync(h->h_cnt, W.cnt, sizeof(DevCounters), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h->h_stats, W.sstats, sizeof(SubstepStats) * N * n_envs, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h->h_racc, W.rigid_acc, sizeof(double) * 6 * std::max(nr, 1), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h->h_rigids, W.rigids, sizeof(DevRigid) * std::max(nr, 1), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    p2g_adapt(W, h->h_cnt->n_ptiles);  // a change records the graph again at the next call
    // the host's rigid state takes the device's kinematic advance
    for (int k = 0; k < nr; ++k) {
        HostRigid& q = h->rigids[order[k]];
        if (q.desc.motion != MPM_KINEMATIC) continue;
        memcpy(q.desc.R, h->h_rigids[k].R, sizeof(q.desc.R));
        memcpy(q.desc.t, h->h_rigids[k].t, sizeof(q.desc.t));
        q.kin_steps += n_steps;
    }
    return finish_host_steps(h, order, 0, false, out, st);
}

mpm_status mpm_tape_reset(mpm_handle* h, int32_t record) {
    if (!h) return fail(MPM_EINVAL, "handle is NULL");
    if (h->w.tape_cap <= 0) return fail(MPM_EINVAL, "the handle was created without a tape (tape_substeps = 0)");
    h->tape_on = record != 0;
    h->tape_len = 0;
    h->tape_ncon.clear();
    return MPM_OK;
}

mpm_status mpm_step_backward(mpm_handle* h, float* gx, float* gv, float* gF, float* gC, mpm_env_grad* env_grads,
                             mpm_rigid_grad* rigid_grads) {
    if (!h) return fail(MPM_EINVAL, "handle is NULL");
    if (!gx || !gv || !gF || !gC) return fail(MPM_EINVAL, "adjoint arrays must be non-NULL");
    if (h->tape_len <= 0) return fail(MPM_EINVAL, "nothing recorded: call mpm_tape_reset, then mpm_step");
    for (const HostRigid& q : h->rigids)
        if (q.desc.motion == MPM_DYNAMIC)
            return fail(MPM_EINVAL, "the reverse pass covers static and kinematic bodies only");
    Work& W = h->w;
    hipStream_t s = h->stream;
    const int N = h->d.N, n_envs = (int)h->envs.size(), nr = (int)h->rigids.size();
    const int n_host = h->tape_len / N;
    const size_t P = W.P;
    const double hd = h->d.h;
    const float hf = (float)hd;
    constexpr int kCgCheck = 16;        // CG iterations between convergence checks
    constexpr int kCgMax = 200000;      // iteration cap per solve
    constexpr double kCgTol = 1e-7;     // relative residual target
    bool cg_capped = false;
    // two particle-adjoint buffers (x 3, v 3, F 9, C or Q 9 per particle)
    float* bufs[2] = {W.adj, W.adj + 24 * P};
    float* A = bufs[0];
    HIP_TRY(hipMemcpyAsync(A, gx, sizeof(float) * 3 * P, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(A + 3 * P, gv, sizeof(float) * 3 * P, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(A + 6 * P, gF, sizeof(float) * 9 * P, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(A + 15 * P, gC, sizeof(float) * 9 * P, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemsetAsync(W.lame, 0, sizeof(double) * 2 * n_envs, s));
    HIP_TRY(hipMemsetAsync(W.rgrad, 0, sizeof(double) * kRigidGradStride * kMaxRigidTape * n_host, s));
    HIP_TRY(launch_clear_step(W, N, false, s));
    W.n_rigid = nr;
    int cur = 0;
    for (int j = n_host - 1; j >= 0; --j) {
        A = bufs[cur];
        float *ax = A, *av = A + 3 * P, *aF = A + 6 * P, *aCQ = A + 15 * P;
        // the host step's rigid and environment tables, for re-running registration
        HIP_TRY(hipMemcpyAsync(W.rigids, W.tape_rig + (size_t)j * kMaxRigidTape, sizeof(DevRigid) * std::max(nr, 1),
                               hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(W.envs, W.tape_env + (size_t)j * n_envs, sizeof(DevEnv) * n_envs,
                               hipMemcpyDeviceToDevice, s));
        for (int k = N - 1; k >= 0; --k) {
            const int r = j * N + k;
            const float* tp = W.tape_p + (size_t)r * 24 * P;
            const float4* tg = W.tape_g + (size_t)r * 2 * W.n_nodes;
            const TapeStep t = {tp, tp + 3 * P, tp + 6 * P, tp + 15 * P, tg, tg + W.n_nodes};
            const bool contact = h->tape_ncon[r] > 0;
            if (contact) {
                // registration and the contact-node table of this substep, again
                HIP_TRY(launch_clear_substep(W, s));
                HIP_TRY(launch_registration(W, t.x, t.v, hd, k, s));
                Work Wv = W;
                Wv.vel = const_cast<float4*>(t.vstar);
                HIP_TRY(launch_contact_setup(Wv, s));
            }
            HIP_TRY(hipMemsetAsync(W.gbar, 0, sizeof(float4) * W.n_nodes, s));
            // the host step's last substep produces C; the others produce Q
            HIP_TRY(launch_g2p_adj(W, t, hf, ax, av, aF, k == N - 1 ? nullptr : aCQ, k == N - 1 ? aCQ : nullptr,
                                   W.gbar, W.lame, s));
            float *cx = nullptr, *cv = nullptr;
            if (contact) {
                HIP_TRY(hipMemsetAsync(W.cg_sc, 0, sizeof(double) * 8, s));
                HIP_TRY(launch_cadj_start(W, hd, t.vel, s));
                double sc[8];
                int it = 0;
                for (;;) {
                    HIP_TRY(hipMemcpyAsync(sc, W.cg_sc, sizeof(sc), hipMemcpyDeviceToHost, s));
                    HIP_TRY(hipStreamSynchronize(s));
                    const double r0 = sc[5], rr = it == 0 ? r0 : sc[4];
                    if (!(rr > kCgTol * kCgTol * r0)) break;
                    if (it >= kCgMax) { cg_capped = true; break; }
                    for (int q = 0; q < kCgCheck; ++q) HIP_TRY(launch_cg_iteration(W, hd, s));
                    it += kCgCheck;
                }
                cx = W.cxv;
                cv = W.cxv + 3 * P;
                HIP_TRY(hipMemsetAsync(W.cxv, 0, sizeof(float) * 6 * P, s));
                HIP_TRY(launch_cadj_finish(W, hd, t, t.vel, cx, cv, W.rgrad + (size_t)j * kMaxRigidTape * kRigidGradStride, s));
            }
            HIP_TRY(launch_grid_adj(W, t, hf, W.gbar, s));
            HIP_TRY(launch_p2g_adj(W, t, W.gbar, cx, cv, ax, av, aCQ, s));
        }
        // the host step's gather (Q from F and C, then the sort) in reverse
        const float* tp0 = W.tape_p + (size_t)(j * N) * 24 * P;
        const TapeStep t0 = {tp0, tp0 + 3 * P, tp0 + 6 * P, tp0 + 15 * P, nullptr, nullptr};
        float* B = bufs[1 - cur];
        HIP_TRY(launch_permute_adj(W, t0, hf, W.tape_idx + (size_t)j * P, ax, av, aF, aCQ, B, B + 3 * P, B + 6 * P,
                                   B + 15 * P, W.lame, s));
        cur = 1 - cur;
    }
    A = bufs[cur];
    HIP_TRY(hipMemcpyAsync(gx, A, sizeof(float) * 3 * P, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(gv, A + 3 * P, sizeof(float) * 3 * P, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(gF, A + 6 * P, sizeof(float) * 9 * P, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(gC, A + 15 * P, sizeof(float) * 9 * P, hipMemcpyDeviceToDevice, s));
    std::vector<double> lame(2 * n_envs), rg((size_t)kRigidGradStride * kMaxRigidTape * n_host);
    const int nr1 = std::max(nr, 1);
    std::vector<DevRigid> trig((size_t)n_host * nr1);
    HIP_TRY(hipMemcpyAsync(lame.data(), W.lame, sizeof(double) * 2 * n_envs, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(rg.data(), W.rgrad, sizeof(double) * rg.size(), hipMemcpyDeviceToHost, s));
    if (rigid_grads)
        for (int j = 0; j < n_host; ++j)
            HIP_TRY(hipMemcpyAsync(trig.data() + (size_t)j * nr1, W.tape_rig + (size_t)j * kMaxRigidTape,
                                   sizeof(DevRigid) * nr1, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (env_grads) {
        for (int e = 0; e < n_envs; ++e) {
            // mu = E / (2 (1 + nu)), la = E nu / ((1 + nu)(1 - 2 nu)), both from double E, nu
            const double E = h->envs[e].E, nu = h->envs[e].nu;
            const double mub = lame[2 * e], lab = lame[2 * e + 1];
            const double a = 1.0 + nu, b = 1.0 - 2.0 * nu;
            env_grads[e].dE = mub / (2.0 * a) + lab * nu / (a * b);
            env_grads[e].dnu = -mub * E / (2.0 * a * a) + lab * E * (1.0 + 2.0 * nu * nu) / (a * a * b * b);
        }
    }
    if (rigid_grads) {
        // device order groups the bodies by environment (stable), as in mpm_step
        std::vector<int> order(nr);
        for (int i = 0; i < nr; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return h->rigids[a].env < h->rigids[b].env; });
        const double dT = N * hd;
        for (int k = 0; k < nr; ++k) {
            mpm_rigid_grad& g = rigid_grads[order[k]];
            memset(&g, 0, sizeof(g));
            if (h->rigids[order[k]].desc.motion == MPM_STATIC) continue;
            const int j0 = h->rigids[order[k]].rec_steps;
            for (int j = 0; j < n_host; ++j) {
                const double* q = rg.data() + ((size_t)j * kMaxRigidTape + k) * kRigidGradStride;
                // pose j of the window is Rot(j dT w) applied to the first; a
                // rotation d of the first turns pose j by Rot(j dT w) d, and
                // dw turns it by j dT J(j dT w) dw (J: the left Jacobian of
                // the rotation map)
                double phi[3], rt[3], jt[3];
                for (int a = 0; a < 3; ++a) phi[a] = j * dT * trig[(size_t)j * nr1 + k].w[a];
                rotate_transposed(phi, q + 9, rt);
                left_jacobian_transposed(phi, q + 9, jt);
                for (int a = 0; a < 3; ++a) {
                    g.dV[a] += q[a];
                    g.dt[a] += q[3 + a];
                    g.dV_kinematic[a] += q[a] + j * dT * q[3 + a];
                    g.dw[a] += q[6 + a];
                    g.dR[a] += rt[a];
                    g.dw_kinematic[a] += q[6 + a] + j * dT * jt[a];
                }
            }
            if (j0 > 0) {
                // the first recorded pose is the reference state advanced by j0
                // kinematic host steps: t = t_ref + j0 dT V and R = Rot(j0 dT w) R_ref,
                // so V also moves every recorded position by j0 dT, and a change dw
                // turns the first pose by b J(b w) dw, b = j0 dT
                const double b = j0 * dT;
                double phi[3], jt[3];
                for (int a = 0; a < 3; ++a) phi[a] = b * trig[k].w[a];
                left_jacobian_transposed(phi, g.dR, jt);
                for (int a = 0; a < 3; ++a) {
                    g.dV_kinematic[a] += b * g.dt[a];
                    g.dw_kinematic[a] += b * jt[a];
                }
            }
        }
    }
    if (cg_capped) return fail(MPM_ENOCONV, "a contact adjoint solve hit its iteration cap");
    return MPM_OK;
}

mpm_status mpm_profile(mpm_handle* h, int32_t enable, mpm_profile_data* out) {
    if (!h) return fail(MPM_EINVAL, "handle is NULL");
    if (out) *out = h->acc;
    memset(&h->acc, 0, sizeof(h->acc));
    h->prof = enable != 0;
    h->prof_phases = enable >= 2;
    return MPM_OK;
}

// ---- One host step without a handle and without allocation ----------------
// The workspace is this file-scope device array: every GPU the library runs on
// holds its own copy until the process ends. Host code never passes the
// array's name to a kernel or copy (on the host it is only a stand-in for the
// symbol): the first call on a device looks up the device's address with
// hipGetSymbolAddress, with that device current, and every later use goes
// through that address.
}  // extern "C"

namespace {
constexpr size_t kStaticScratchBytes = (size_t)MPM_STATIC_SCRATCH_BYTES;
constexpr int kStaticMaxEnvs = MPM_STATIC_MAX_ENVS;
constexpr int kStaticMaxN = MPM_STATIC_MAX_SUBSTEPS;
constexpr int kStaticMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
struct StaticDevice {
    void* ptr = nullptr;  // device address of scratch on this device
    int qn_cap = 0;       // co-resident solver blocks
};
StaticDevice g_static_dev[kStaticMaxDevices];
// host staging of the calls (pageable, fixed size); calls are serialised
struct StaticHost {
    DevEnv env[kStaticMaxEnvs];
    DevRigid rig[kMaxRigidTotal];
    DevCounters cnt;
    SubstepStats stats[kStaticMaxN * kStaticMaxEnvs];
    double racc[6 * kMaxRigidTotal];
    int2 qn_map[kMaxQnBlocks];
    int env_qn[2 * kStaticMaxEnvs];
    int env_slots[kStaticMaxEnvs];
    int groups[kStaticMaxEnvs];
};
StaticHost g_static_host;
std::mutex g_static_mutex;

// The device's scratch address and solver capacity, looked up on the first
// call on the device (with it current).
mpm_status static_device(StaticDevice** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kStaticMaxDevices) return fail(MPM_EDEVICE, "device %d beyond the static table", dev);
    StaticDevice& S = g_static_dev[dev];
    if (!S.ptr) {
        void* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr || ((uintptr_t)ptr) % kAlign) return fail(MPM_EDEVICE, "static scratch address is not usable");
        const int cap = qn_max_blocks();
        if (cap < 1) return fail(MPM_EDEVICE, "cannot size the cooperative solver launch");
        S.qn_cap = std::min(cap, kMaxQnBlocks);
        S.ptr = ptr;
    }
    *out = &S;
    return MPM_OK;
}

mpm_status step_static_locked(const mpm_desc* desc, const mpm_rigid_desc* rigids, const int32_t* rigid_env,
                              int32_t n_rigid, mpm_rigid_impulse* out, mpm_step_stats* st) {
    Sizes z;
    mpm_status vs = validate(desc, &z);
    if (vs != MPM_OK) return vs;
    if (!desc->x || !desc->v || !desc->F || !desc->C) return fail(MPM_EINVAL, "state pointers must be non-NULL");
    if (desc->workspace || desc->workspace_bytes) return fail(MPM_EINVAL, "the static step takes no workspace");
    if (desc->tape_substeps) return fail(MPM_EINVAL, "the static step records no tape");
    if (desc->n_envs > kStaticMaxEnvs) return fail(MPM_EINVAL, "at most %d environments", kStaticMaxEnvs);
    if (desc->N > kStaticMaxN) return fail(MPM_EINVAL, "at most %d substeps per host step", kStaticMaxN);
    if (n_rigid < 0 || n_rigid > kMaxRigidTotal) return fail(MPM_EINVAL, "0 to %d rigid bodies", kMaxRigidTotal);
    if (n_rigid > 0 && (!rigids || !rigid_env)) return fail(MPM_EINVAL, "rigid arrays are NULL");
    int per_env = 0;
    for (int i = 0; i < n_rigid; ++i) {
        if (rigid_env[i] < 0 || rigid_env[i] >= desc->n_envs) return fail(MPM_EINVAL, "rigid %d: env out of range", i);
        if (i > 0 && rigid_env[i] < rigid_env[i - 1])
            return fail(MPM_EINVAL, "rigid bodies must be ordered by environment");
        per_env = (i > 0 && rigid_env[i] == rigid_env[i - 1]) ? per_env + 1 : 1;
        if (per_env > kMaxRigidPerEnv) return fail(MPM_EINVAL, "at most %d rigid bodies per environment", kMaxRigidPerEnv);
        const mpm_status rs = check_rigid(&rigids[i]);
        if (rs != MPM_OK) return rs;
    }
    Work W;
    const size_t need = layout(z, nullptr, &W);
    if (need > kStaticScratchBytes)
        return fail(MPM_ENOMEM, "the step needs %zu bytes of workspace, the static array holds %zu", need,
                    kStaticScratchBytes);
    StaticDevice* S = nullptr;
    const mpm_status ds = static_device(&S);
    if (ds != MPM_OK) return ds;
    layout(z, (char*)S->ptr, &W);
    W.qn_blocks = S->qn_cap;
    int spb = 0, cap = S->qn_cap;
    solver_options(desc, &W, &spb, &cap);
    StaticHost& H = g_static_host;
    const int n_envs = desc->n_envs, N = desc->N;
    StepCtx c;
    c.w = &W;
    c.d = desc;
    c.key_bits = make_dev_envs(desc->envs, n_envs, H.env);
    c.slots_per_block = spb;
    c.rec = false;
    c.tape_len = 0;
    c.prof = nullptr;
    c.phases = false;
    for (int i = 0; i < n_rigid; ++i) place_dev_rigid(rigids[i], rigid_env[i], i, H.rig + i, H.env);
    W.n_rigid = n_rigid;
    for (int e = 0; e < n_envs; ++e) H.env_slots[e] = 0;  // no earlier step: groups from headroom alone
    int env_stride = 0;
    const int qn_blocks = plan_groups(n_envs, H.env_slots, spb, cap, H.groups, H.qn_map, H.env_qn, &env_stride);
    hipStream_t s = (hipStream_t)desc->stream;
    // everything a previous call left in the array is stale
    HIP_TRY(init_workspace(W, H.env, s));
    HIP_TRY(hipMemcpyAsync(W.rigids, H.rig, sizeof(DevRigid) * std::max(n_rigid, 1), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(W.qn_map, H.qn_map, sizeof(int2) * qn_blocks, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(W.env_qn, H.env_qn, sizeof(int) * 2 * n_envs, hipMemcpyHostToDevice, s));
    int npair = 0;
    mpm_status es = enqueue_host_step(c, qn_blocks, env_stride, false, npair, s);
    if (es == MPM_OK) {
        const hipError_t e1 = hipMemcpyAsync(&H.cnt, W.cnt, sizeof(DevCounters), hipMemcpyDeviceToHost, s);
        const hipError_t e2 = hipMemcpyAsync(H.stats, W.sstats, sizeof(SubstepStats) * N * n_envs,
                                             hipMemcpyDeviceToHost, s);
        const hipError_t e3 = hipMemcpyAsync(H.racc, W.rigid_acc, sizeof(double) * 6 * std::max(n_rigid, 1),
                                             hipMemcpyDeviceToHost, s);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
            es = fail(MPM_EDEVICE, "copying the step's results failed");
    }
    // the call returns only after its device work: the next call reuses the array
    const hipError_t se = hipStreamSynchronize(s);
    if (es != MPM_OK) return es;
    if (se != hipSuccess) return fail(MPM_EDEVICE, "hipStreamSynchronize failed: %s", hipGetErrorString(se));
    const unsigned flags = H.cnt.flags;
    if (H.cnt.abort_step && H.cnt.abort_substep > 0) {
        // the step stopped early: the caller's C lags the state; rebuild it from Q
        HIP_TRY(launch_recover_C(W, desc->F, desc->C, desc->h, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    if (out) {
        for (int k = 0; k < n_rigid; ++k)
            for (int a = 0; a < 3; ++a) {
                out[k].impulse[a] = H.racc[6 * k + a];
                out[k].torque[a] = H.racc[6 * k + 3 + a];
            }
    }
    fill_step_stats(H.stats, N, n_envs, flags, st);
    return step_status(flags, W.cap_c, H.cnt.n_contacts);
}
}  // namespace

extern "C" {

mpm_status mpm_step_static(const mpm_desc* desc, const mpm_rigid_desc* rigids, const int32_t* rigid_env,
                           int32_t n_rigid, mpm_rigid_impulse* out, mpm_step_stats* st) {
    std::lock_guard<std::mutex> lock(g_static_mutex);
    return step_static_locked(desc, rigids, rigid_env, n_rigid, out, st);
}

void mpm_destroy(mpm_handle* h) {
    if (!h) return;
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    if (h->gevent) (void)hipEventDestroy(h->gevent);
    if (h->gstream) (void)hipStreamDestroy(h->gstream);
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
    if (h->h_rigids) (void)hipHostFree(h->h_rigids);
    if (h->h_racc) (void)hipHostFree(h->h_racc);
    if (h->h_stats) (void)hipHostFree(h->h_stats);
    if (h->h_cnt) (void)hipHostFree(h->h_cnt);
    if (h->h_qn_map) (void)hipHostFree(h->h_qn_map);
    if (h->h_env_qn) (void)hipHostFree(h->h_env_qn);
    delete h;
}

}  // extern "C"
