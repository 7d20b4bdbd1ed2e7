// transfer.hip -- free-motion part of the substep (Eq. (6), Sec. V-A) on
// gfx950: cell keys, the gathered first-substep state, the particle tile
// list, the LDS-tiled P2G scatter, the grid update and the LDS-staged G2P
// gather with the constitutive update.
//
// Data layout: particle arrays are component-major float32 (coalesced per
// component); the grid is dense per environment, node-major, with float4
// accumulators (m, p) and velocities (v, m). Particles are sorted by
// (environment, 4x4x4-cell tile, cell) once per host step; each block then
// owns one tile and accumulates its particles into an 8x8x8-node LDS block
// (the tile, its 2-node stencil reach and one cell of drift on every side),
// so atomics stay in LDS and only one flush per touched node reaches memory.
#include "mpm_internal.h"
#include "sort_util.h"

#include <algorithm>

namespace mpm {

constexpr unsigned kFlagDomain = 2u;
constexpr unsigned kFlagNan = 4u;
constexpr int kBN = kBlockNodes;            // 8
constexpr int kBN3 = kBN * kBN * kBN;       // 512

__device__ __forceinline__ int env_of_particle(const DevEnv* envs, int n_envs, long long p) {
    int lo = 0, hi = n_envs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (envs[mid].p_begin <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int env_of_tile(const DevEnv* envs, int n_envs, int t) {
    int lo = 0, hi = n_envs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (envs[mid].tile_base <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Stencil base per axis, clamped to the grid (flagging the clamp).
__device__ __forceinline__ void stencil_base(const DevEnv& E, const float x[3], int b[3],
                                             float f[3], bool* clamped) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int bi = cell_base(x[a], E.origin[a], E.inv_dx, &f[a]);
        int hi = E.dims[a] - 3;
        if (bi < 0 || bi > hi) {
            *clamped = true;
            bi = bi < 0 ? 0 : hi;
            f[a] = fminf(fmaxf(f[a], 0.5f), 1.5f);
        }
        b[a] = bi;
    }
}

// ---------------------------------------------------------------------------
// Cell keys: (global tile << 6) | cell-in-tile
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_keys(const float* __restrict__ x, long long P, const DevEnv* __restrict__ envs, int n_envs,
       unsigned* __restrict__ keys, unsigned* __restrict__ idx, int shift, DevCounters* cnt) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const DevEnv& E = envs[env_of_particle(envs, n_envs, i)];
    float xp[3] = {x[i], x[P + i], x[2 * P + i]};
    int b[3];
    float f[3];
    bool clamped = false;
    stencil_base(E, xp, b, f, &clamped);
    if (clamped) atomicOr(&cnt->flags, kFlagDomain);
    unsigned tile = (unsigned)E.tile_base + (unsigned)(b[0] >> 2) +
                    (unsigned)E.ntile[0] * ((unsigned)(b[1] >> 2) + (unsigned)E.ntile[1] * (unsigned)(b[2] >> 2));
    unsigned cell = (unsigned)(b[0] & 3) | ((unsigned)(b[1] & 3) << 2) | ((unsigned)(b[2] & 3) << 4);
    keys[i] = ((tile << 6) | cell) >> shift;
    idx[i] = (unsigned)i;
}

hipError_t launch_keys(const Work& w, const float* x, int shift, hipStream_t s) {
    const unsigned blocks = (unsigned)((w.P + 255) / 256);
    hipLaunchKernelGGL(k_keys, dim3(blocks), dim3(256), 0, s, x, w.P, w.envs, w.n_envs, w.key_a,
                       w.idx_a, shift, w.cnt);
    return hipGetLastError();
}

// Q = m_p C - h V0 (4/dx^2) tau(F): the affine momentum with the stress folded
// in (MLS-MPM), consumed by the next P2G.
__device__ __forceinline__ void fused_Q(const DevEnv& E, double h, const float F[9],
                                        const float C[9], float Q[9]) {
    float U[9], sv[3], V[9], tau[9];
    svd3(F, U, sv, V);
    kirchhoff_from_svd(E.mat, F, U, sv, V, tau);
    const float c = (float)h * E.V0 * E.D;
#pragma unroll
    for (int k = 0; k < 9; ++k) Q[k] = E.m_p * C[k] - c * tau[k];
}

// Gather the caller's state into sorted order for the first substep.
__global__ void __launch_bounds__(256)
k_permute(const unsigned* __restrict__ idx, long long P, const DevEnv* __restrict__ envs,
          int n_envs, double h, const float* __restrict__ x, const float* __restrict__ v,
          const float* __restrict__ F, const float* __restrict__ C, const int* __restrict__ pid,
          float* __restrict__ xs, float* __restrict__ vs, float* __restrict__ Fs,
          float* __restrict__ Q, int* __restrict__ pids) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const long long s = idx[i];
    const DevEnv& E = envs[env_of_particle(envs, n_envs, i)];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        xs[a * P + i] = x[a * P + s];
        vs[a * P + i] = v[a * P + s];
    }
    float Fp[9], Cp[9], Qp[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        Fp[k] = F[k * P + s];
        Cp[k] = C[k * P + s];
    }
    fused_Q(E, h, Fp, Cp, Qp);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        Fs[k * P + i] = Fp[k];
        Q[k * P + i] = Qp[k];
    }
    if (pid) pids[i] = pid[s];
}

hipError_t launch_permute(const Work& w, const unsigned* idx, const float* x, const float* v,
                            const float* F, const float* C, const int* pid, double h,
                            hipStream_t s) {
    const unsigned blocks = (unsigned)((w.P + 255) / 256);
    hipLaunchKernelGGL(k_permute, dim3(blocks), dim3(256), 0, s, idx, w.P, w.envs, w.n_envs, h, x,
                       v, F, C, pid, w.xs, w.vs, w.Fs, w.Q, w.pids);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Particle tile list from the sorted keys
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_tile_count(const unsigned* __restrict__ keys, long long P, unsigned* __restrict__ blk) {
    __shared__ unsigned wsum[17];
    long long beg, end;
    chunk_range(P, blockIdx.x, gridDim.x, &beg, &end);
    unsigned c = 0;
    for (long long i = beg + threadIdx.x; i < end; i += blockDim.x)
        c += (i == 0 || (keys[i] >> 6) != (keys[i - 1] >> 6)) ? 1u : 0u;
    unsigned tot;
    block_exclusive_scan_total(c, wsum, &tot);
    if (threadIdx.x == 0) blk[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(256)
k_tile_write(const unsigned* __restrict__ keys, long long P, const unsigned* __restrict__ blk,
             unsigned* __restrict__ tid_out, unsigned* __restrict__ beg_out, const DevCounters* cnt) {
    __shared__ unsigned wsum[17];
    long long beg, end;
    chunk_range(P, blockIdx.x, gridDim.x, &beg, &end);
    unsigned run = blk[blockIdx.x];
    for (long long base = beg; base < end; base += blockDim.x) {
        long long i = base + threadIdx.x;
        unsigned head = (i < end && (i == 0 || (keys[i] >> 6) != (keys[i - 1] >> 6))) ? 1u : 0u;
        unsigned tot;
        unsigned off = block_exclusive_scan_total(head, wsum, &tot);
        if (head) {
            tid_out[run + off] = keys[i] >> 6;
            beg_out[run + off] = (unsigned)i;
        }
        run += tot;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) beg_out[cnt->n_ptiles] = (unsigned)P;
}

hipError_t launch_tile_list(const Work& w, const unsigned* sorted_keys, hipStream_t s) {
    hipLaunchKernelGGL(k_tile_count, dim3(kSortBlocks), dim3(256), 0, s, sorted_keys, w.P, w.blk);
    hipError_t e = launch_scan_blocks(w.blk, kSortBlocks, &w.cnt->n_ptiles, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tile_write, dim3(kSortBlocks), dim3(256), 0, s, sorted_keys, w.P, w.blk,
                       w.ptile_id, w.ptile_beg, (const DevCounters*)w.cnt);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Node-tile activation (the grid update visits only touched node tiles)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void activate_tile(unsigned t, unsigned* tile_flag,
                                              unsigned* active, DevCounters* cnt) {
    if (atomicCAS(&tile_flag[t], 0u, 1u) == 0u) {
        unsigned k = atomicAdd(&cnt->n_active, 1u);
        active[k] = t;
    }
}

__device__ __forceinline__ unsigned node_tile(const DevEnv& E, int i, int j, int k) {
    return (unsigned)E.tile_base + (unsigned)(i >> 2) +
           (unsigned)E.ntile[0] * ((unsigned)(j >> 2) + (unsigned)E.ntile[1] * (unsigned)(k >> 2));
}

__device__ __forceinline__ long long node_index(const DevEnv& E, int i, int j, int k) {
    return E.node_base + (long long)i + (long long)E.dims[0] * ((long long)j + (long long)E.dims[1] * k);
}

__device__ __forceinline__ void tile_coords(const DevEnv& E, unsigned gt, int* tx, int* ty, int* tz) {
    int lt = (int)gt - E.tile_base;
    *tx = lt % E.ntile[0];
    *ty = (lt / E.ntile[0]) % E.ntile[1];
    *tz = lt / (E.ntile[0] * E.ntile[1]);
}

// ---------------------------------------------------------------------------
// Tile maps, once per host step: the particle-tile index of every tile and
// the node tiles within one tile of a particle tile (the only node tiles a
// particle's stencil can reach unless it drifts more than a cell).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_tile_maps_clear(const unsigned* __restrict__ ptile_id, const unsigned* __restrict__ ntile_list,
                  int* __restrict__ ptile_of, unsigned* __restrict__ ntile_mark, const DevCounters* cnt) {
    const unsigned np = cnt->n_ptiles, nn = cnt->n_ntiles;
    for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < np || i < nn; i += gridDim.x * blockDim.x) {
        if (i < np) ptile_of[ptile_id[i]] = -1;
        if (i < nn) ntile_mark[ntile_list[i]] = 0u;
    }
}

__global__ void k_reset_ntiles(DevCounters* cnt) { cnt->n_ntiles = 0u; }

__global__ void __launch_bounds__(256)
k_tile_maps_build(const unsigned* __restrict__ ptile_id, const DevEnv* __restrict__ envs, int n_envs,
                  int* __restrict__ ptile_of, unsigned* __restrict__ ntile_list,
                  unsigned* __restrict__ ntile_mark, DevCounters* cnt) {
    const unsigned np = cnt->n_ptiles;
    for (unsigned q = blockIdx.x * blockDim.x + threadIdx.x; q < 27u * np; q += gridDim.x * blockDim.x) {
        const unsigned t = q / 27u, o = q % 27u;
        const unsigned gt = ptile_id[t];
        if (o == 13u) ptile_of[gt] = (int)t;
        const DevEnv& E = envs[env_of_tile(envs, n_envs, (int)gt)];
        int tx, ty, tz;
        tile_coords(E, gt, &tx, &ty, &tz);
        const int nx = tx + (int)(o % 3u) - 1, ny = ty + (int)((o / 3u) % 3u) - 1, nz = tz + (int)(o / 9u) - 1;
        if (nx < 0 || ny < 0 || nz < 0 || nx >= E.ntile[0] || ny >= E.ntile[1] || nz >= E.ntile[2]) continue;
        const unsigned T = (unsigned)E.tile_base + (unsigned)nx + (unsigned)E.ntile[0] * ((unsigned)ny + (unsigned)E.ntile[1] * (unsigned)nz);
        if (atomicCAS(&ntile_mark[T], 0u, 1u) == 0u) ntile_list[atomicAdd(&cnt->n_ntiles, 1u)] = T;
    }
}

hipError_t launch_tile_maps(const Work& w, hipStream_t s, bool clear_old) {
    if (clear_old) {
        hipLaunchKernelGGL(k_tile_maps_clear, dim3(512), dim3(256), 0, s, w.ptile_id, w.ntile_list,
                           w.ptile_of, w.ntile_mark, (const DevCounters*)w.cnt);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_reset_ntiles, dim3(1), dim3(1), 0, s, w.cnt);
    hipLaunchKernelGGL(k_tile_maps_build, dim3(1024), dim3(256), 0, s, w.ptile_id, w.envs, w.n_envs,
                       w.ptile_of, w.ntile_list, w.ntile_mark, w.cnt);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// P2G: m_i += w m_p, p_i += w (m_p v_p + Q_p (x_i - x_p))  (Eq. (6), Sec. V-A)
// ---------------------------------------------------------------------------
// P2G, one particle tile per block: 256 threads, thread (q, cell) with
// component q = tid / 64 (mass, then the three momentum components) and cell
// = tid % 64 of the 4x4x4 tile.
//  1. The cell ranges of the tile come from the sort-time keys (sorted, so a
//     cell's particles are contiguous): the first and last particle of each
//     run of equal keys write its bounds; no counting or scan.
//  2. Each thread walks its cell's particles, loading the next particle while
//     it computes the current one, and sums its component of the
//     contributions of those whose stencil base is still the cell in 27
//     registers (the particles of a cell share one stencil). A particle whose
//     base has drifted since the sort into another cell of the tile is listed
//     for that cell, whose threads then walk it too (2b), so it needs no
//     atomics; one that left the tile is only queued: (particle, component)
//     goes to a list in LDS, so no wave issues scattered atomics for the few
//     lanes that meet one.
//  3. Each wave reduces its 64 cells' sums to the 216 nodes they reach
//     (DPP exchanges along x and y, a staging pass in LDS along z) and adds
//     each node once into the tile's 8x8x8-node LDS block, without atomics
//     (LDS float atomics, one per cell and stencil node, took about 40 % of
//     the kernel's time).
//  4. All threads take the queued entries, one (particle, component) each,
//     and add them into the LDS block, or, for a stencil outside the block, to
//     the global accumulator (activating the node tiles it touches). A list
//     that overflows leaves the rest to the walking thread, inline.
//  5. The block is stored without atomics to the tile's slot of the block
//     buffer; the grid update sums the overlapping blocks of every node.
// (Staging the tile's particles in LDS before the walks, tried, was slower:
// 189 against 162 us at 1M particles, and 1005 against 574 us at 4M.)
constexpr int kDriftMax = 1024;  // queued (particle, component) entries per tile
constexpr int kDinCap = 16;      // particles that drifted into a cell of the tile, listed per cell
constexpr int kPreCap = 1024;    // particles of a tile whose stencil base P2G forms once, in its first pass

// Component q of one particle's contribution to the 27 nodes of its stencil
// (m_p, or m_p v_q + Q_q . (x_i - x_p)), added to the LDS block when the stencil
// lies inside it, else to the global accumulator.
__device__ __forceinline__ void p2g_scatter_one(const DevEnv& E, const float* __restrict__ x,
                                                const float* __restrict__ v, const float* __restrict__ Q,
                                                long long P, long long p, int q, int ox, int oy, int oz,
                                                float (*sm)[kBN3], float4* __restrict__ acc,
                                                unsigned* __restrict__ tile_flag, unsigned* __restrict__ active,
                                                DevCounters* cnt, bool* clamped) {
    const float xp[3] = {x[p], x[P + p], x[2 * P + p]};
    int b[3];
    float f[3];
    stencil_base(E, xp, b, f, clamped);
    float wx[3], wy[3], wz[3];
    bspline_w(f[0], wx);
    bspline_w(f[1], wy);
    bspline_w(f[2], wz);
    const float dx = E.dx;
    float base_val = E.m_p, qr0 = 0.f, qr1 = 0.f, qr2 = 0.f;
    if (q > 0) {
        base_val = E.m_p * v[(q - 1) * P + p];
        qr0 = Q[(3 * (q - 1) + 0) * P + p];
        qr1 = Q[(3 * (q - 1) + 1) * P + p];
        qr2 = Q[(3 * (q - 1) + 2) * P + p];
    }
    const int lx = b[0] - ox, ly = b[1] - oy, lz = b[2] - oz;
    const bool local = lx >= 0 && lx <= kBN - 3 && ly >= 0 && ly <= kBN - 3 && lz >= 0 && lz <= kBN - 3;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int bb = 0; bb < 3; ++bb)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const float w = wx[a] * wy[bb] * wz[c];
                const float val = w * (base_val + qr0 * (((float)a - f[0]) * dx) +
                                       qr1 * (((float)bb - f[1]) * dx) + qr2 * (((float)c - f[2]) * dx));
                if (local) {
                    atomicAdd(&sm[q][((lz + c) * kBN + (ly + bb)) * kBN + (lx + a)], val);
                } else {
                    float* g = reinterpret_cast<float*>(&acc[node_index(E, b[0] + a, b[1] + bb, b[2] + c)]);
                    atomicAdd(g + q, val);
                }
            }
    if (!local && q == 0) {
        // the drifted particle's nodes span up to 2x2x2 node tiles
        for (int c = 0; c < 2; ++c)
            for (int bb = 0; bb < 2; ++bb)
                for (int a = 0; a < 2; ++a)
                    activate_tile(node_tile(E, b[0] + 2 * a, b[1] + 2 * bb, b[2] + 2 * c), tile_flag, active, cnt);
    }
}

// A float from another lane of the wave by DPP (kCtrl: the DPP control);
// lanes whose source lies outside their row read 0.
template <int kCtrl>
__device__ __forceinline__ float dpp_f(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), kCtrl, 0xF, 0xF, false));
}
constexpr int kQuadUp1 = 0x90;   // quad_perm [0, 0, 1, 2]: lane i of a quad reads lane i - 1 (lane 0 itself)
constexpr int kQuadUp2 = 0x40;   // quad_perm [0, 0, 0, 1]: lane i reads lane i - 2 (lanes 0, 1 lane 0)
constexpr int kRowUp4 = 0x114;   // row_shr:4
constexpr int kRowUp8 = 0x118;   // row_shr:8
constexpr int kSpan = kTile + 2; // nodes a tile's cell stencils reach along an axis

// Sum of the cells' stencil sums of one wave (lane = cell x + 4 y + 16 z of
// the tile, sum[(c * 3 + b) * 3 + a] its weight on node cell + (a, b, c)) into
// the LDS block, without atomics: the three axes are reduced in turn, x inside
// each quad of lanes and y inside each row by DPP, which leaves in lane (x, y,
// z) slot (i, j, c) the sum over x and y for node (x + i, y + j) at z offset c
// (slots i > 0 valid in lanes x = 3 only, j > 0 in y = 3 only); z goes through
// the wave's staging area (plain stores, then each node reads its three
// z contributions). A node's value is added to the block non-atomically: only
// this wave writes component q before the block's next barrier.
__device__ __forceinline__ void p2g_cell_flush(float (&sum)[27], int cx, int cy, int cz, float* __restrict__ smq,
                                               float* __restrict__ stage) {
    const float mx1 = cx >= 1 ? 1.f : 0.f, mx2 = cx >= 2 ? 1.f : 0.f;
#pragma unroll
    for (int cb = 0; cb < 9; ++cb) {
        float* r = &sum[cb * 3];
        const float s1 = r[1], s2 = r[2];
        r[0] = fmaf(mx2, dpp_f<kQuadUp2>(s2), fmaf(mx1, dpp_f<kQuadUp1>(s1), r[0]));
        r[1] = fmaf(mx1, dpp_f<kQuadUp1>(s2), s1);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            float* r0 = &sum[(c * 3 + 0) * 3 + i];
            float* r1 = &sum[(c * 3 + 1) * 3 + i];
            float* r2 = &sum[(c * 3 + 2) * 3 + i];
            const float t1 = *r1, t2 = *r2;
            *r0 += dpp_f<kRowUp4>(t1) + dpp_f<kRowUp8>(t2);
            *r1 = t1 + dpp_f<kRowUp4>(t2);
        }
    // stage[c][z][y][x] over the 6 x 6 (x, y) nodes of each cell layer z
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int i = 0; i < 3; ++i)
                if ((i == 0 || cx == kTile - 1) && (j == 0 || cy == kTile - 1))
                    stage[((c * kTile + cz) * kSpan + cy + j) * kSpan + cx + i] = sum[(c * 3 + j) * 3 + i];
    __builtin_amdgcn_wave_barrier();
    const int lane = (cz * kTile + cy) * kTile + cx;
    for (int n = lane; n < kSpan * kSpan * kSpan; n += 64) {
        const int nx = n % kSpan, ny = (n / kSpan) % kSpan, nz = n / (kSpan * kSpan);
        float v = 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int z = nz - c;
            if (z >= 0 && z < kTile) v += stage[((c * kTile + z) * kSpan + ny) * kSpan + nx];
        }
        smq[((nz + 1) * kBN + ny + 1) * kBN + nx + 1] += v;
    }
}

template <int kP2gSplit>  // walks per (component, cell): a block is 4 x kP2gSplit waves
__global__ void __launch_bounds__(256 * kP2gSplit, 4)
k_p2g(const float* __restrict__ x, const float* __restrict__ v, const float* __restrict__ Q,
      long long P, const DevEnv* __restrict__ envs, int n_envs, const unsigned* __restrict__ ptile_id,
      const unsigned* __restrict__ ptile_beg, const unsigned* __restrict__ keys,
      float4* __restrict__ blkbuf, float4* __restrict__ acc, unsigned* __restrict__ tile_flag,
      unsigned* __restrict__ active, DevCounters* cnt) {
    __shared__ float sm[4][kBN3];
    __shared__ float stage[4][3 * kTile * kSpan * kSpan];  // per wave: the cell flush's z staging
    __shared__ unsigned cbeg[64], cend[64];
    __shared__ unsigned drift[kDriftMax];
    __shared__ unsigned n_drift;
    __shared__ unsigned din[kP2gSplit][64][kDinCap];  // per walk and cell: tile-relative particles that drifted into it
    __shared__ unsigned din_cnt[kP2gSplit][64];
    __shared__ float comb[kP2gSplit > 1 ? (kP2gSplit - 1) * 4 : 1][kP2gSplit > 1 ? 27 : 1][64];  // the later walks' sums
    // the first kPreCap particles of the tile: the offset f of their stencil
    // base and that base as a cell of the tile (64: outside the tile)
    __shared__ float4 pinfo[kPreCap];
    if (cnt->abort_step) return;
    const unsigned n_tiles = cnt->n_ptiles;
    // the component and the walk are uniform over a wave: scalar branches below.
    // Walk `part` of a (component, cell) takes every kP2gSplit-th of the cell's
    // particles; the walks' sums are added in walk order before the flush.
    const int q = __builtin_amdgcn_readfirstlane((int)((threadIdx.x >> 6) & 3u)), cell = threadIdx.x & 63;
    const int part = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 8));
    const int cx = cell & 3, cy = (cell >> 2) & 3, cz = cell >> 4;
    bool clamped = false;
    for (unsigned t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        for (int n = threadIdx.x; n < kBN3; n += blockDim.x) {
            sm[0][n] = 0.f; sm[1][n] = 0.f; sm[2][n] = 0.f; sm[3][n] = 0.f;
        }
        if (threadIdx.x < 64) {
            cbeg[threadIdx.x] = 0u;
            cend[threadIdx.x] = 0u;
#pragma unroll
            for (int h = 0; h < kP2gSplit; ++h) din_cnt[h][threadIdx.x] = 0u;
        }
        if (threadIdx.x == 0) n_drift = 0u;
        __syncthreads();
        const unsigned gt = ptile_id[t];
        const long long pb = ptile_beg[t], pe = ptile_beg[t + 1];
        const DevEnv& E = envs[env_of_tile(envs, n_envs, (int)gt)];
        int tx, ty, tz;
        tile_coords(E, gt, &tx, &ty, &tz);
        // a stencil base as a cell of this tile, 64 when it lies outside
        auto tile_cell = [&](const int b[3]) -> int {
            const int rx = b[0] - tx * kTile, ry = b[1] - ty * kTile, rz = b[2] - tz * kTile;
            return (rx >= 0 && rx < kTile && ry >= 0 && ry < kTile && rz >= 0 && rz < kTile)
                       ? (rz * kTile + ry) * kTile + rx : 64;
        };
        // 1. cell ranges: the bounds of every run of equal keys; and each of
        // the first kPreCap particles' stencil base, formed once for the four
        // components
        for (long long p = pb + threadIdx.x; p < pe; p += blockDim.x) {
            const unsigned k = keys[p];
            if (p == pb || keys[p - 1] != k) cbeg[k & 63u] = (unsigned)(p - pb);
            if (p == pe - 1 || keys[p + 1] != k) cend[k & 63u] = (unsigned)(p - pb + 1);
            if (p - pb < kPreCap) {
                const float xp[3] = {x[p], x[P + p], x[2 * P + p]};
                int b[3];
                float f[3];
                stencil_base(E, xp, b, f, &clamped);
                pinfo[p - pb] = make_float4(f[0], f[1], f[2], __int_as_float(tile_cell(b)));
            }
        }
        __syncthreads();
        const int ox = tx * kTile - 1, oy = ty * kTile - 1, oz = tz * kTile - 1;
        const float dx = E.dx, mp = E.m_p;
        float sum[27];
#pragma unroll
        for (int o = 0; o < 27; ++o) sum[o] = 0.f;
        // 2. the walk over the cell's particles, the next one's loads issued first
        const unsigned k0 = cbeg[cell] + (unsigned)part, k1 = cend[cell];
        float nx0 = 0.f, nx1 = 0.f, nx2 = 0.f, nv = 0.f, nq0 = 0.f, nq1 = 0.f, nq2 = 0.f;
        if (k0 < k1) {
            const long long p = pb + k0;
            if (k0 >= (unsigned)kPreCap) { nx0 = x[p]; nx1 = x[P + p]; nx2 = x[2 * P + p]; }
            if (q > 0) {
                nv = v[(q - 1) * P + p];
                nq0 = Q[(3 * (q - 1) + 0) * P + p];
                nq1 = Q[(3 * (q - 1) + 1) * P + p];
                nq2 = Q[(3 * (q - 1) + 2) * P + p];
            }
        }
        // component q of a particle whose stencil base is this cell, into the sums
        // (the node's term w_a w_b w_c (base + q0 dx_a + q1 dy_b + q2 dz_c) is
        // formed as (w_b w_c) (w_a s_bc + w_a q0 dx_a), s_bc = base + q1 dy_b +
        // q2 dz_c: two FMAs per node)
        auto accumulate = [&](const float xp[3], const float f[3], float vq, float q0, float q1, float q2) {
            float wx[3], wy[3], wz[3];
            bspline_w(f[0], wx);
            bspline_w(f[1], wy);
            bspline_w(f[2], wz);
            const float base_val = q > 0 ? mp * vq : mp;
            float hx[3], sy[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                hx[a] = wx[a] * (q0 * (((float)a - f[0]) * dx));
                sy[a] = fmaf(q1, ((float)a - f[1]) * dx, base_val);
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float dz = q2 * (((float)c - f[2]) * dx);
#pragma unroll
                for (int bb = 0; bb < 3; ++bb) {
                    const float t = wy[bb] * wz[c];
                    const float sbc = sy[bb] + dz;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const int o = (c * 3 + bb) * 3 + a;
                        sum[o] = fmaf(t, fmaf(wx[a], sbc, hx[a]), sum[o]);
                    }
                }
            }
        };
        auto queue_drift = [&](unsigned kk, int qq) {
            const unsigned slot = atomicAdd(&n_drift, 1u);
            if (slot < (unsigned)kDriftMax) {
                drift[slot] = (kk << 2) | (unsigned)qq;
            } else {
                p2g_scatter_one(E, x, v, Q, P, pb + kk, qq, ox, oy, oz, sm, acc, tile_flag, active, cnt, &clamped);
            }
        };
        for (unsigned kk = k0; kk < k1; kk += kP2gSplit) {
            const float xp[3] = {nx0, nx1, nx2};
            const float vq = nv, q0 = nq0, q1 = nq1, q2 = nq2;
            if (kk + kP2gSplit < k1) {
                const long long pn = pb + kk + kP2gSplit;
                if (kk + kP2gSplit >= (unsigned)kPreCap) { nx0 = x[pn]; nx1 = x[P + pn]; nx2 = x[2 * P + pn]; }
                if (q > 0) {
                    nv = v[(q - 1) * P + pn];
                    nq0 = Q[(3 * (q - 1) + 0) * P + pn];
                    nq1 = Q[(3 * (q - 1) + 1) * P + pn];
                    nq2 = Q[(3 * (q - 1) + 2) * P + pn];
                }
            }
            float f[3];
            int to;
            if (kk < (unsigned)kPreCap) {
                const float4 in = pinfo[kk];
                f[0] = in.x; f[1] = in.y; f[2] = in.z;
                to = __float_as_int(in.w);
            } else {
                int b[3];
                stencil_base(E, xp, b, f, &clamped);
                to = tile_cell(b);
            }
            if (to != cell) {
                // drifted since the sort: into another cell of the tile, listed
                // there (by the mass wave, for all four components), else queued
                if (to < 64) {
                    if (q == 0) {
                        const unsigned slot = atomicAdd(&din_cnt[part][to], 1u);
                        if (slot < (unsigned)kDinCap) {
                            din[part][to][slot] = kk;
                        } else {
                            for (int qq = 0; qq < 4; ++qq) queue_drift(kk, qq);
                        }
                    }
                } else {
                    queue_drift(kk, q);
                }
                continue;
            }
            accumulate(xp, f, vq, q0, q1, q2);
        }
        __syncthreads();
        // 2b. the particles that drifted into this cell from another of the tile
        const unsigned n_in = min(din_cnt[part][cell], (unsigned)kDinCap);
        for (unsigned i = 0; i < n_in; ++i) {
            const long long p = pb + din[part][cell][i];
            const float xp[3] = {x[p], x[P + p], x[2 * P + p]};
            float vq = 0.f, q0 = 0.f, q1 = 0.f, q2 = 0.f;
            if (q > 0) {
                vq = v[(q - 1) * P + p];
                q0 = Q[(3 * (q - 1) + 0) * P + p];
                q1 = Q[(3 * (q - 1) + 1) * P + p];
                q2 = Q[(3 * (q - 1) + 2) * P + p];
            }
            int b[3];
            float f[3];
            stencil_base(E, xp, b, f, &clamped);
            accumulate(xp, f, vq, q0, q1, q2);
        }
        // 3. the later walks' sums added to the first's in walk order, then the
        // cells' sums into the LDS block (the first walk's whole wave, empty
        // cells too)
        if constexpr (kP2gSplit > 1) {
            if (part > 0) {
#pragma unroll
                for (int o = 0; o < 27; ++o) comb[(part - 1) * 4 + q][o][cell] = sum[o];
            }
            __syncthreads();
            if (part == 0) {
                for (int h = 1; h < kP2gSplit; ++h)
#pragma unroll
                    for (int o = 0; o < 27; ++o) sum[o] += comb[(h - 1) * 4 + q][o][cell];
            }
        }
        if (part == 0) p2g_cell_flush(sum, cx, cy, cz, sm[q], stage[q]);
        __syncthreads();
        // 4. the queued drifted particles, one (particle, component) per thread
        const unsigned nd = min(n_drift, (unsigned)kDriftMax);
        for (unsigned i = threadIdx.x; i < nd; i += blockDim.x) {
            const unsigned e = drift[i];
            p2g_scatter_one(E, x, v, Q, P, pb + (e >> 2), (int)(e & 3u), ox, oy, oz, sm, acc, tile_flag, active,
                            cnt, &clamped);
        }
        __syncthreads();
        // 5. atomic-free block store
        float4* out = blkbuf + (size_t)t * kBN3;
        for (int n = threadIdx.x; n < kBN3; n += blockDim.x)
            out[n] = make_float4(sm[0][n], sm[1][n], sm[2][n], sm[3][n]);
        __syncthreads();
    }
    if (clamped) atomicOr(&cnt->flags, kFlagDomain);
}

hipError_t launch_p2g(const Work& w, const float* x, const float* v, hipStream_t s) {
    const unsigned blocks = (unsigned)std::max<long long>(1, std::min<long long>(w.n_tiles, w.transfer_blocks));
    if (w.p2g_walks == 2)
        hipLaunchKernelGGL(k_p2g<2>, dim3(blocks), dim3(512), 0, s, x, v, w.Q, w.P, w.envs, w.n_envs,
                           w.ptile_id, w.ptile_beg, w.keys_sorted, w.blkbuf, w.acc, w.tile_flag,
                           w.active_tiles, w.cnt);
    else
        hipLaunchKernelGGL(k_p2g<1>, dim3(blocks), dim3(256), 0, s, x, v, w.Q, w.P, w.envs, w.n_envs,
                           w.ptile_id, w.ptile_beg, w.keys_sorted, w.blkbuf, w.acc, w.tile_flag,
                           w.active_tiles, w.cnt);
    return hipGetLastError();
}

// The tiled P2G's walks per (component, cell) for the next host step, from
// the particles per non-empty tile of the last sort: one walk per (component,
// cell) up to 16 particles per cell on average, two beyond (each walk then
// takes every other particle of the cell, and the block has twice the waves).
// Measured on the granular pour: at about 7 particles per cell one walk is
// faster (79 against 94 us at 1M particles), at about 28 two are (378
// against 661 us at 4M).
void p2g_adapt(Work& w, unsigned n_ptiles) {
    if (w.p2g_walks_fixed || n_ptiles == 0u) return;
    w.p2g_walks = (double)w.P > 16.0 * 64.0 * (double)n_ptiles ? 2 : 1;
}

// ---------------------------------------------------------------------------
// Grid update: sum the overlapping P2G blocks of every node (fixed order),
// v* = p/m + h g, boundary band. Node tiles next to a particle tile come from
// the static list; tiles reached only by drifted particles from the dynamic
// list, whose accumulator is read and cleared here.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float4 grid_node_update(const DevEnv& E, int i, int j, int k, float4 a,
                                                   float hf, double* psum) {
    float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
    if (a.x > 0.f) {
        float vv[3] = {a.y / a.x + hf * E.gravity[0], a.z / a.x + hf * E.gravity[1],
                       a.w / a.x + hf * E.gravity[2]};
        const int idx[3] = {i, j, k};
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            if (idx[ax] < 3 && vv[ax] < 0.f) vv[ax] = 0.f;
            if (idx[ax] >= E.dims[ax] - 3 && vv[ax] > 0.f) vv[ax] = 0.f;
        }
        out = make_float4(vv[0], vv[1], vv[2], a.x);
        *psum += (double)a.x * ((double)vv[0] * vv[0] + (double)vv[1] * vv[1] + (double)vv[2] * vv[2]);
    }
    return out;
}

// One FP64 atomic per block and environment (the block is one wave).
__device__ __forceinline__ void flush_env_sum(double psum, double* dst) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) psum += __shfl_down(psum, o, 64);
    if (threadIdx.x == 0 && psum != 0.0) atomicAdd(dst, psum);
}

__global__ void __launch_bounds__(64)
k_grid_update(const DevEnv* __restrict__ envs, int n_envs, double h, const float4* __restrict__ blkbuf,
              const int* __restrict__ ptile_of, const unsigned* __restrict__ ntile_list,
              const unsigned* __restrict__ ntile_mark, float4* __restrict__ acc,
              float4* __restrict__ vel, unsigned* __restrict__ tile_flag,
              const unsigned* __restrict__ active, double* __restrict__ env_pnorm, DevCounters* cnt) {
    __shared__ int nb[27];
    if (cnt->abort_step) return;
    const unsigned n_static = cnt->n_ntiles, n_dyn = cnt->n_active;
    double psum = 0.0;  // sum m |v*|^2 of environment psum_env, flushed when the environment changes
    int psum_env = -1;
    const float hf = (float)h;
    const int rx = threadIdx.x & 3, ry = (threadIdx.x >> 2) & 3, rz = threadIdx.x >> 4;
    for (unsigned t = blockIdx.x; t < n_static + n_dyn; t += gridDim.x) {
        const bool is_static = t < n_static;
        const unsigned gt = is_static ? ntile_list[t] : active[t - n_static];
        const int env = env_of_tile(envs, n_envs, (int)gt);
        if (env != psum_env) {  // uniform over the block (one tile at a time)
            if (psum_env >= 0) flush_env_sum(psum, env_pnorm + psum_env);
            psum = 0.0;
            psum_env = env;
        }
        const DevEnv& E = envs[env];
        int tx, ty, tz;
        tile_coords(E, gt, &tx, &ty, &tz);
        if (is_static) {
            __syncthreads();
            if (threadIdx.x < 27) {
                const int nx = tx + (int)(threadIdx.x % 3) - 1, ny = ty + (int)((threadIdx.x / 3) % 3) - 1,
                          nz = tz + (int)(threadIdx.x / 9) - 1;
                int pt = -1;
                if (nx >= 0 && ny >= 0 && nz >= 0 && nx < E.ntile[0] && ny < E.ntile[1] && nz < E.ntile[2])
                    pt = ptile_of[E.tile_base + nx + E.ntile[0] * (ny + E.ntile[1] * nz)];
                nb[threadIdx.x] = pt;
            }
            __syncthreads();
        } else if (threadIdx.x == 0) {
            tile_flag[gt] = 0u;
        }
        if (!is_static && ntile_mark[gt]) continue;  // already updated through the static list
        const int i = tx * 4 + rx, j = ty * 4 + ry, k = tz * 4 + rz;
        if (i >= E.dims[0] || j >= E.dims[1] || k >= E.dims[2]) continue;
        const long long gi = node_index(E, i, j, k);
        float4 sum = make_float4(0.f, 0.f, 0.f, 0.f);
        if (is_static) {
            // the node lies in the blocks of tiles {T-1, T} (r <= 2) or {T, T+1} (r == 3) per axis
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int bb = 0; bb < 2; ++bb)
#pragma unroll
                    for (int a = 0; a < 2; ++a) {
                        const int ofx = (rx == 3 ? a : a - 1), ofy = (ry == 3 ? bb : bb - 1), ofz = (rz == 3 ? c : c - 1);
                        const int pt = nb[(ofz + 1) * 9 + (ofy + 1) * 3 + (ofx + 1)];
                        if (pt < 0) continue;
                        const int lx = i - (4 * (tx + ofx) - 1), ly = j - (4 * (ty + ofy) - 1), lz = k - (4 * (tz + ofz) - 1);
                        const float4 q = blkbuf[(size_t)pt * kBN3 + (lz * kBN + ly) * kBN + lx];
                        sum.x += q.x; sum.y += q.y; sum.z += q.z; sum.w += q.w;
                    }
        }
        const float4 ac = acc[gi];
        if (ac.x != 0.f || ac.y != 0.f || ac.z != 0.f || ac.w != 0.f) {
            sum.x += ac.x; sum.y += ac.y; sum.z += ac.z; sum.w += ac.w;
            acc[gi] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        vel[gi] = grid_node_update(E, i, j, k, sum, hf, &psum);
    }
    if (psum_env >= 0) flush_env_sum(psum, env_pnorm + psum_env);
}

hipError_t launch_grid_update(const Work& w, double h, hipStream_t s) {
    const unsigned blocks = (unsigned)std::min<long long>(w.n_tiles, 4096);
    hipLaunchKernelGGL(k_grid_update, dim3(blocks), dim3(64), 0, s, w.envs, w.n_envs, h, w.blkbuf,
                       w.ptile_of, w.ntile_list, w.ntile_mark, w.acc, w.vel, w.tile_flag,
                       w.active_tiles, w.env_pnorm, w.cnt);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// G2P: v_p = sum w v_i, C_p = (4/dx^2) sum w v_i (x_i - x_p)^T,
// F <- (I + h C) F, x <- x + h v_p; return map for sand; Q for the next P2G
// ---------------------------------------------------------------------------
// G2P of one particle p with stencil fractions f and weights w[axis][3]:
// v_p = sum w v_i, C_p = D sum w v_i (x_i - x_p)^T, F <- (I + h C) F,
// x <- x + h v_p, the return map for sand, and Q for the next P2G. near(a, b,
// c) and far(a, b, c) return the velocity of stencil node (a, b, c), the
// first used when `local` holds. Idx: the index type of the particle arrays
// (32-bit when every index fits, so stores take a scalar base and one offset).
template <typename Idx, typename NearV, typename FarV>
__device__ __forceinline__ void g2p_particle(const DevEnv& E, Idx P, Idx p, const float xp[3],
                                             const float f[3], const float* const w[3], const float Fp[9],
                                             float hf, bool local, NearV near, FarV far, float* x_out,
                                             float* v_out, float* F_out, float* C_out, float* Q, bool* bad_out) {
    const float* wx = w[0];
    const float* wy = w[1];
    const float* wz = w[2];
    const float dx = E.dx, D = E.D;
    bool bad = false;
    // v_p = sum w v_i and C_p = D sum w v_i (x_i - x_p)^T, summed axis by axis
    // (the weights and offsets factor per axis): along x for each (y, z)
    // row of the stencil, then along y, then along z
    float wxd[3], wyd[3], wzd[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        wxd[a] = wx[a] * (((float)a - f[0]) * dx);
        wyd[a] = wy[a] * (((float)a - f[1]) * dx);
        wzd[a] = wz[a] * (((float)a - f[2]) * dx);
    }
    float vp[3] = {0.f, 0.f, 0.f};
    float Cp[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    auto gather = [&](auto node_v) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float q0[3] = {0.f, 0.f, 0.f}, q1[3] = {0.f, 0.f, 0.f}, q2[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) {
                float p0[3] = {0.f, 0.f, 0.f}, p1[3] = {0.f, 0.f, 0.f};
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const float4 g = node_v(a, bb, c);
                    const float vi[3] = {g.x, g.y, g.z};
#pragma unroll
                    for (int r = 0; r < 3; ++r) {
                        p0[r] = fmaf(wx[a], vi[r], p0[r]);
                        p1[r] = fmaf(wxd[a], vi[r], p1[r]);
                    }
                }
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    q0[r] = fmaf(wy[bb], p0[r], q0[r]);
                    q1[r] = fmaf(wy[bb], p1[r], q1[r]);
                    q2[r] = fmaf(wyd[bb], p0[r], q2[r]);
                }
            }
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                vp[r] = fmaf(wz[c], q0[r], vp[r]);
                Cp[r * 3 + 0] = fmaf(wz[c], q1[r], Cp[r * 3 + 0]);
                Cp[r * 3 + 1] = fmaf(wz[c], q2[r], Cp[r * 3 + 1]);
                Cp[r * 3 + 2] = fmaf(wzd[c], q0[r], Cp[r * 3 + 2]);
            }
        }
    };
    if (local) {
        gather(near);
    } else {
        gather(far);
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) Cp[k] *= D;
    // F <- (I + h C) F
    float Fn[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            Fn[r * 3 + c] = Fp[r * 3 + c] + hf * (Cp[r * 3 + 0] * Fp[0 * 3 + c] +
                                                  Cp[r * 3 + 1] * Fp[1 * 3 + c] +
                                                  Cp[r * 3 + 2] * Fp[2 * 3 + c]);
    float U[9], s[3], V[9], tau[9];
    // Drucker-Prager sand in tension (J = det F >= 1: the Hencky strain's trace
    // is not negative) returns to the cone tip: zero strain, F its rotation,
    // no stress. After such a substep F is a rotation up to h C, so the
    // rotation comes from a few Newton steps of the polar decomposition; F
    // farther from a rotation, and compression, take the SVD.
    bool done = false;
    if (E.mat.type == 1) {
        const float J = Fn[0] * (Fn[4] * Fn[8] - Fn[5] * Fn[7]) - Fn[1] * (Fn[3] * Fn[8] - Fn[5] * Fn[6]) +
                        Fn[2] * (Fn[3] * Fn[7] - Fn[4] * Fn[6]);
        float R[9];
        if (J >= 1.0f && polar_rotation_near(Fn, R)) {
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                Fn[k] = R[k];
                tau[k] = 0.0f;
            }
            done = true;
        }
    }
    if (!done) {
        svd3(Fn, U, s, V);
        if (E.mat.type == 1) {
            float eps[3];
            if (dp_return_map(E.mat, U, s, V, Fn, eps)) {
#pragma unroll
                for (int k = 0; k < 9; ++k) tau[k] = 0.0f;  // tension: eps = 0, no stress
            } else {
                hencky_tau(E.mat, U, eps[0], eps[1], eps[2], tau);
            }
        } else {
            kirchhoff_from_svd(E.mat, Fn, U, s, V, tau);
        }
    }
    const float cq = hf * E.V0 * D;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        x_out[a * P + p] = xp[a] + hf * vp[a];
        v_out[a * P + p] = vp[a];
        bad |= !isfinite(vp[a]);
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        F_out[k * P + p] = Fn[k];
        Q[k * P + p] = E.m_p * Cp[k] - cq * tau[k];
        bad |= !isfinite(Fn[k]);
    }
    if (C_out) {
#pragma unroll
        for (int k = 0; k < 9; ++k) C_out[k * P + p] = Cp[k];
    }
    *bad_out |= bad;
}

template <typename Idx>
__global__ void __launch_bounds__(256)
k_g2p(const float* x_in, const float* F_in, float* x_out, float* v_out, float* F_out,
      float* __restrict__ C_out, float* __restrict__ Q, const int* __restrict__ pid_in,
      int* __restrict__ pid_out, Idx P, const DevEnv* __restrict__ envs, int n_envs,
      const unsigned* __restrict__ ptile_id, const unsigned* __restrict__ ptile_beg,
      const float4* __restrict__ vel, double h, DevCounters* cnt) {
    __shared__ float4 sv[kBN3];  // node velocities of the tile's block (w unused)
    if (cnt->abort_step) return;
    const unsigned n_tiles = cnt->n_ptiles;
    const float hf = (float)h;
    bool bad = false;
    for (unsigned t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const unsigned gt = ptile_id[t];
        const Idx pb = ptile_beg[t], pe = ptile_beg[t + 1];
        const DevEnv& E = envs[env_of_tile(envs, n_envs, (int)gt)];
        int tx, ty, tz;
        tile_coords(E, gt, &tx, &ty, &tz);
        const int ox = tx * kTile - 1, oy = ty * kTile - 1, oz = tz * kTile - 1;
        __syncthreads();
        for (int n = threadIdx.x; n < kBN3; n += blockDim.x) {
            const int i = ox + (n % kBN), j = oy + ((n / kBN) % kBN), k = oz + n / (kBN * kBN);
            float4 vv = make_float4(0.f, 0.f, 0.f, 0.f);
            if (i >= 0 && j >= 0 && k >= 0 && i < E.dims[0] && j < E.dims[1] && k < E.dims[2])
                vv = vel[node_index(E, i, j, k)];
            sv[n] = vv;
        }
        __syncthreads();
        for (Idx p = pb + threadIdx.x; p < pe; p += blockDim.x) {
            float xp[3] = {x_in[p], x_in[P + p], x_in[2 * P + p]};
            float Fp[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) Fp[k] = F_in[k * P + p];
            int b[3];
            float f[3];
            bool clamped = false;
            stencil_base(E, xp, b, f, &clamped);
            float wx[3], wy[3], wz[3];
            bspline_w(f[0], wx);
            bspline_w(f[1], wy);
            bspline_w(f[2], wz);
            const int lx = b[0] - ox, ly = b[1] - oy, lz = b[2] - oz;
            const bool local = lx >= 0 && lx <= kBN - 3 && ly >= 0 && ly <= kBN - 3 && lz >= 0 && lz <= kBN - 3;
            const float* wv[3] = {wx, wy, wz};
            // a stencil that left the tile's block (drift of more than a cell) reads memory
            g2p_particle(
                E, P, p, xp, f, wv, Fp, hf, local,
                [&](int a, int bb, int c) { return sv[((lz + c) * kBN + (ly + bb)) * kBN + (lx + a)]; },
                [&](int a, int bb, int c) { return vel[node_index(E, b[0] + a, b[1] + bb, b[2] + c)]; }, x_out,
                v_out, F_out, C_out, Q, &bad);
            if (pid_in && pid_out) pid_out[p] = pid_in[p];
        }
    }
    if (bad) atomicOr(&cnt->flags, kFlagNan);
}

hipError_t launch_g2p(const Work& w, const float* x_in, const float* F_in, float* x_out,
                      float* v_out, float* F_out, float* C_out, const int* pid_in, int* pid_out,
                      double h, hipStream_t s) {
    const unsigned blocks = (unsigned)std::max<long long>(1, std::min<long long>(w.n_tiles, w.transfer_blocks));
    if (24 * w.P < (1ll << 32))
        hipLaunchKernelGGL(k_g2p<unsigned>, dim3(blocks), dim3(256), 0, s, x_in, F_in, x_out, v_out, F_out,
                           C_out, w.Q, pid_in, pid_out, (unsigned)w.P, w.envs, w.n_envs, w.ptile_id,
                           w.ptile_beg, w.vel, h, w.cnt);
    else
        hipLaunchKernelGGL(k_g2p<long long>, dim3(blocks), dim3(256), 0, s, x_in, F_in, x_out, v_out, F_out,
                           C_out, w.Q, pid_in, pid_out, w.P, w.envs, w.n_envs, w.ptile_id,
                           w.ptile_beg, w.vel, h, w.cnt);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sort-policy arms (the ablation of Sec. V-A's sorting): with the particles
// ordered by truncated keys or not reordered at all there are no particle
// tiles, so P2G is a plain scatter, one thread per particle and 27 x 4 float
// atomics into the dense accumulator (activating the node tiles the stencil
// touches, which the grid update then visits), and G2P a plain gather from
// the dense node velocities; the per-particle arithmetic is the tiled
// kernels'.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_p2g_plain(const float* __restrict__ x, const float* __restrict__ v, const float* __restrict__ Q,
            long long P, const DevEnv* __restrict__ envs, int n_envs, float4* __restrict__ acc,
            unsigned* __restrict__ tile_flag, unsigned* __restrict__ active, DevCounters* cnt) {
    if (cnt->abort_step) return;
    bool clamped = false;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < P;
         p += (long long)gridDim.x * blockDim.x) {
        const DevEnv& E = envs[env_of_particle(envs, n_envs, p)];
        const float xp[3] = {x[p], x[P + p], x[2 * P + p]};
        int b[3];
        float f[3];
        stencil_base(E, xp, b, f, &clamped);
        float wx[3], wy[3], wz[3];
        bspline_w(f[0], wx);
        bspline_w(f[1], wy);
        bspline_w(f[2], wz);
        const float dx = E.dx, mp = E.m_p;
        float mv[3], Qp[9];
#pragma unroll
        for (int a = 0; a < 3; ++a) mv[a] = mp * v[a * P + p];
#pragma unroll
        for (int k = 0; k < 9; ++k) Qp[k] = Q[k * P + p];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int bb = 0; bb < 3; ++bb)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const float w = wx[a] * wy[bb] * wz[c];
                    const float d[3] = {((float)a - f[0]) * dx, ((float)bb - f[1]) * dx, ((float)c - f[2]) * dx};
                    float* g = reinterpret_cast<float*>(&acc[node_index(E, b[0] + a, b[1] + bb, b[2] + c)]);
                    atomicAdd(g, w * mp);
#pragma unroll
                    for (int r = 0; r < 3; ++r)
                        atomicAdd(g + 1 + r, w * (mv[r] + Qp[3 * r] * d[0] + Qp[3 * r + 1] * d[1] + Qp[3 * r + 2] * d[2]));
                }
        for (int c = 0; c < 2; ++c)
            for (int bb = 0; bb < 2; ++bb)
                for (int a = 0; a < 2; ++a) {
                    const unsigned t = node_tile(E, b[0] + 2 * a, b[1] + 2 * bb, b[2] + 2 * c);
                    if (tile_flag[t] == 0u) activate_tile(t, tile_flag, active, cnt);
                }
    }
    if (clamped) atomicOr(&cnt->flags, kFlagDomain);
}

__global__ void __launch_bounds__(256)
k_g2p_plain(const float* x_in, const float* F_in, float* x_out, float* v_out, float* F_out,
            float* __restrict__ C_out, float* __restrict__ Q, const int* __restrict__ pid_in,
            int* __restrict__ pid_out, long long P, const DevEnv* __restrict__ envs, int n_envs,
            const float4* __restrict__ vel, double h, DevCounters* cnt) {
    if (cnt->abort_step) return;
    const float hf = (float)h;
    bool bad = false;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < P;
         p += (long long)gridDim.x * blockDim.x) {
        const DevEnv& E = envs[env_of_particle(envs, n_envs, p)];
        float xp[3] = {x_in[p], x_in[P + p], x_in[2 * P + p]};
        float Fp[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) Fp[k] = F_in[k * P + p];
        int b[3];
        float f[3];
        bool clamped = false;
        stencil_base(E, xp, b, f, &clamped);
        float wx[3], wy[3], wz[3];
        bspline_w(f[0], wx);
        bspline_w(f[1], wy);
        bspline_w(f[2], wz);
        const float* wv[3] = {wx, wy, wz};
        auto from_mem = [&](int a, int bb, int c) { return vel[node_index(E, b[0] + a, b[1] + bb, b[2] + c)]; };
        g2p_particle(E, P, p, xp, f, wv, Fp, hf, false, from_mem, from_mem, x_out, v_out, F_out, C_out, Q, &bad);
        if (pid_in && pid_out) pid_out[p] = pid_in[p];
    }
    if (bad) atomicOr(&cnt->flags, kFlagNan);
}

hipError_t launch_p2g_plain(const Work& w, const float* x, const float* v, hipStream_t s) {
    const unsigned blocks = (unsigned)std::min<long long>((w.P + 255) / 256, 16384);
    hipLaunchKernelGGL(k_p2g_plain, dim3(blocks), dim3(256), 0, s, x, v, w.Q, w.P, w.envs, w.n_envs, w.acc,
                       w.tile_flag, w.active_tiles, w.cnt);
    return hipGetLastError();
}

hipError_t launch_g2p_plain(const Work& w, const float* x_in, const float* F_in, float* x_out, float* v_out,
                            float* F_out, float* C_out, const int* pid_in, int* pid_out, double h, hipStream_t s) {
    const unsigned blocks = (unsigned)std::min<long long>((w.P + 255) / 256, 16384);
    hipLaunchKernelGGL(k_g2p_plain, dim3(blocks), dim3(256), 0, s, x_in, F_in, x_out, v_out, F_out, C_out, w.Q,
                       pid_in, pid_out, w.P, w.envs, w.n_envs, w.vel, h, w.cnt);
    return hipGetLastError();
}

// No particle tiles this host step (the sort-policy arms): the grid update
// then visits only the node tiles the scatter activates.
__global__ void k_no_tiles(DevCounters* cnt) {
    cnt->n_ptiles = 0u;
    cnt->n_ntiles = 0u;
}

hipError_t launch_no_tiles(const Work& w, hipStream_t s) {
    hipLaunchKernelGGL(k_no_tiles, dim3(1), dim3(1), 0, s, w.cnt);
    return hipGetLastError();
}

// C = (Q + h V0 D tau(F)) / m_p: recovers the affine matrix from the fused
// matrix when a step stops early, so the caller's state stays consistent.
__global__ void __launch_bounds__(256)
k_recover_C(const float* __restrict__ F, const float* __restrict__ Q, float* __restrict__ C,
            long long P, const DevEnv* __restrict__ envs, int n_envs, double h) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const DevEnv& E = envs[env_of_particle(envs, n_envs, i)];
    float Fp[9], U[9], s[3], V[9], tau[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Fp[k] = F[k * P + i];
    svd3(Fp, U, s, V);
    kirchhoff_from_svd(E.mat, Fp, U, s, V, tau);
    const float cq = (float)h * E.V0 * E.D;
#pragma unroll
    for (int k = 0; k < 9; ++k) C[k * P + i] = (Q[k * P + i] + cq * tau[k]) / E.m_p;
}

hipError_t launch_recover_C(const Work& w, const float* F, float* C, double h, hipStream_t s) {
    const unsigned blocks = (unsigned)((w.P + 255) / 256);
    hipLaunchKernelGGL(k_recover_C, dim3(blocks), dim3(256), 0, s, F, w.Q, C, w.P, w.envs,
                       w.n_envs, h);
    return hipGetLastError();
}

// Start of a host step: flags, impulse accumulators and per-substep stats.
// Start of a host step: flags, the abort state and the impulse sums (all but
// stats_only), and the substep statistics. A graph of several host steps
// clears everything once and only the statistics per host step, so flags and
// impulses accumulate and a stopped step stops the ones after it.
__global__ void k_clear_step(DevCounters* cnt, double* rigid_acc, int n_acc, SubstepStats* st, int n_st,
                             int stats_only) {
    const int t = threadIdx.x;
    if (!stats_only) {
        if (t == 0) {
            cnt->flags = 0u;
            cnt->abort_step = 0u;
            cnt->abort_substep = 0u;
        }
        for (int i = t; i < n_acc; i += blockDim.x) rigid_acc[i] = 0.0;
    }
    for (int i = t; i < n_st; i += blockDim.x) {
        SubstepStats z;
        z.n_contacts = z.n_slots = z.iterations = z.converged = z.ls_rounds = z.pad = 0;
        z.inner_iterations = z.pad2 = 0;
        z.residual = z.threshold = 0.0;
        for (int q = 0; q < 8; ++q) z.t_phase[q] = 0ull;
        st[i] = z;
    }
}

// Start of a substep: counters rebuilt every substep (a fill kernel rather
// than a memset, so the sequence can be captured in a graph).
__global__ void k_clear_substep(DevCounters* cnt, double* env_pnorm, int n_envs) {
    if (threadIdx.x == 0) {
        cnt->n_active = 0u;
        cnt->n_contacts = 0u;
        cnt->n_pairs = 0u;
        cnt->n_slots = 0u;
    }
    for (int e = threadIdx.x; e < n_envs; e += blockDim.x) env_pnorm[e] = 0.0;
}

hipError_t launch_clear_step(const Work& w, int N, bool stats_only, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_step, dim3(1), dim3(256), 0, s, w.cnt, w.rigid_acc, 6 * 256,
                       w.sstats, N * w.n_envs, stats_only ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_clear_substep(const Work& w, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_substep, dim3(1), dim3(256), 0, s, w.cnt, w.env_pnorm, w.n_envs);
    return hipGetLastError();
}

}  // namespace mpm
