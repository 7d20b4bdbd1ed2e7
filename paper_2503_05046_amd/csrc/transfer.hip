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
       unsigned* __restrict__ keys, unsigned* __restrict__ idx, DevCounters* cnt) {
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
    keys[i] = (tile << 6) | cell;
    idx[i] = (unsigned)i;
}

hipError_t launch_keys(const Work& w, const float* x, hipStream_t s) {
    const unsigned blocks = (unsigned)((w.P + 255) / 256);
    hipLaunchKernelGGL(k_keys, dim3(blocks), dim3(256), 0, s, x, w.P, w.envs, w.n_envs, w.key_a,
                       w.idx_a, w.cnt);
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
// P2G: m_i += w m_p, p_i += w (m_p v_p + Q_p (x_i - x_p))
//
// One block per particle tile, one thread per (cell of the tile, component):
// thread q*64 + c sums component q (0: mass, 1-3: momentum) of every particle
// sorted into cell c over the 27 stencil nodes in registers (the particles of
// a cell share one stencil), then adds its 27 sums into the tile's 8x8x8 LDS
// node block; the 64 lanes of a wave hold 64 different cells, so those LDS
// atomics never collide within an instruction. A particle whose stencil base
// has drifted from its sort-time cell adds to the LDS block directly, or, if it
// left the block, to the global accumulator. The block is stored atomic-free to
// the tile's slot of the block buffer; the grid update sums the 8 blocks that
// overlap each node in a fixed order.
// ---------------------------------------------------------------------------
// P2G, one particle tile per block: 256 threads, thread (q, cell) with
// component q = tid / 64 (mass, then the three momentum components) and cell
// = tid % 64 of the 4x4x4 tile. Each thread walks the particles of its cell
// (contiguous after the sort) and keeps in registers its component of the
// contributions of those whose stencil base is still the cell; it then adds
// its 27 sums into the tile's 8x8x8-node LDS block. The 64 lanes of a wave
// own 64 different cells, so those atomics never collide. Particles that
// drifted to another base since the sort are scattered directly, into LDS
// when their stencil lies inside the block, else into the global accumulator
// (activating the node tiles). The block is stored without atomics; the grid
// update sums the overlapping blocks of every node.
__global__ void __launch_bounds__(256)
k_p2g(const float* __restrict__ x, const float* __restrict__ v, const float* __restrict__ Q,
      long long P, const DevEnv* __restrict__ envs, int n_envs, const unsigned* __restrict__ ptile_id,
      const unsigned* __restrict__ ptile_beg, const unsigned* __restrict__ keys,
      float4* __restrict__ blkbuf, float4* __restrict__ acc, unsigned* __restrict__ tile_flag,
      unsigned* __restrict__ active, DevCounters* cnt) {
    __shared__ float sm[4][kBN3];
    __shared__ unsigned ccount[64], cstart[64];
    if (cnt->abort_step) return;
    const unsigned n_tiles = cnt->n_ptiles;
    const int q = threadIdx.x >> 6, cell = threadIdx.x & 63;
    const int cx = cell & 3, cy = (cell >> 2) & 3, cz = cell >> 4;
    for (unsigned t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        for (int n = threadIdx.x; n < kBN3; n += blockDim.x) {
            sm[0][n] = 0.f; sm[1][n] = 0.f; sm[2][n] = 0.f; sm[3][n] = 0.f;
        }
        if (threadIdx.x < 64) ccount[threadIdx.x] = 0u;
        __syncthreads();
        const unsigned gt = ptile_id[t];
        const long long pb = ptile_beg[t], pe = ptile_beg[t + 1];
        for (long long p = pb + threadIdx.x; p < pe; p += blockDim.x) atomicAdd(&ccount[keys[p] & 63u], 1u);
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned run = 0;
            for (int c = 0; c < 64; ++c) {
                cstart[c] = run;
                run += ccount[c];
            }
        }
        __syncthreads();
        const DevEnv& E = envs[env_of_tile(envs, n_envs, (int)gt)];
        int tx, ty, tz;
        tile_coords(E, gt, &tx, &ty, &tz);
        const int ox = tx * kTile - 1, oy = ty * kTile - 1, oz = tz * kTile - 1;
        const int nbx = tx * kTile + cx, nby = ty * kTile + cy, nbz = tz * kTile + cz;  // this cell's base
        const float dx = E.dx, mp = E.m_p;
        float sum[27];
#pragma unroll
        for (int o = 0; o < 27; ++o) sum[o] = 0.f;
        const unsigned cnt_c = ccount[cell];
        const long long p0 = pb + cstart[cell];
        bool clamped = false;
        for (unsigned kk = 0; kk < cnt_c; ++kk) {
            const long long p = p0 + kk;
            const float xp[3] = {x[p], x[P + p], x[2 * P + p]};
            int b[3];
            float f[3];
            stencil_base(E, xp, b, f, &clamped);
            float wx[3], wy[3], wz[3];
            bspline_w(f[0], wx);
            bspline_w(f[1], wy);
            bspline_w(f[2], wz);
            // component q of the particle's contribution: m_p, or m_p v_q + Q_q . (x_i - x_p)
            float base_val = mp, qr0 = 0.f, qr1 = 0.f, qr2 = 0.f;
            if (q > 0) {
                base_val = mp * v[(q - 1) * P + p];
                qr0 = Q[(3 * (q - 1) + 0) * P + p];
                qr1 = Q[(3 * (q - 1) + 1) * P + p];
                qr2 = Q[(3 * (q - 1) + 2) * P + p];
            }
            const bool same = b[0] == nbx && b[1] == nby && b[2] == nbz;
            const int lx = b[0] - ox, ly = b[1] - oy, lz = b[2] - oz;
            const bool local = lx >= 0 && lx <= kBN - 3 && ly >= 0 && ly <= kBN - 3 && lz >= 0 && lz <= kBN - 3;
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int bb = 0; bb < 3; ++bb)
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const int o = (c * 3 + bb) * 3 + a;
                        const float w = wx[a] * wy[bb] * wz[c];
                        const float val = w * (base_val + qr0 * (((float)a - f[0]) * dx) +
                                               qr1 * (((float)bb - f[1]) * dx) + qr2 * (((float)c - f[2]) * dx));
                        if (same) {
                            sum[o] += val;
                        } else if (local) {
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
                            activate_tile(node_tile(E, b[0] + 2 * a, b[1] + 2 * bb, b[2] + 2 * c),
                                          tile_flag, active, cnt);
            }
        }
        if (cnt_c > 0) {
            const int lx = nbx - ox, ly = nby - oy, lz = nbz - oz;  // in [1, 4]
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int bb = 0; bb < 3; ++bb)
#pragma unroll
                    for (int a = 0; a < 3; ++a)
                        atomicAdd(&sm[q][((lz + c) * kBN + (ly + bb)) * kBN + (lx + a)], sum[(c * 3 + bb) * 3 + a]);
        }
        if (clamped) atomicOr(&cnt->flags, kFlagDomain);
        __syncthreads();
        float4* out = blkbuf + (size_t)t * kBN3;
        for (int n = threadIdx.x; n < kBN3; n += blockDim.x)
            out[n] = make_float4(sm[0][n], sm[1][n], sm[2][n], sm[3][n]);
        __syncthreads();
    }
}

hipError_t launch_p2g(const Work& w, const float* x, const float* v, hipStream_t s) {
    const unsigned blocks = (unsigned)std::min<long long>(w.n_tiles, 8192);
    hipLaunchKernelGGL(k_p2g, dim3(blocks), dim3(256), 0, s, x, v, w.Q, w.P, w.envs, w.n_envs,
                       w.ptile_id, w.ptile_beg, w.keys_sorted, w.blkbuf, w.acc, w.tile_flag,
                       w.active_tiles, w.cnt);
    return hipGetLastError();
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
__global__ void __launch_bounds__(256)
k_g2p(const float* x_in, const float* F_in, float* x_out, float* v_out, float* F_out,
      float* __restrict__ C_out, float* __restrict__ Q, const int* __restrict__ pid_in,
      int* __restrict__ pid_out, long long P, const DevEnv* __restrict__ envs, int n_envs,
      const unsigned* __restrict__ ptile_id, const unsigned* __restrict__ ptile_beg,
      const float4* __restrict__ vel, double h, DevCounters* cnt) {
    __shared__ float sv[3][kBN3];
    if (cnt->abort_step) return;
    const unsigned n_tiles = cnt->n_ptiles;
    const float hf = (float)h;
    bool bad = false;
    for (unsigned t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const unsigned gt = ptile_id[t];
        const long long pb = ptile_beg[t], pe = ptile_beg[t + 1];
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
            sv[0][n] = vv.x;
            sv[1][n] = vv.y;
            sv[2][n] = vv.z;
        }
        __syncthreads();
        const float dx = E.dx, D = E.D;
        for (long long p = pb + threadIdx.x; p < pe; p += blockDim.x) {
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
            float vp[3] = {0.f, 0.f, 0.f};
            float Cp[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int bb = 0; bb < 3; ++bb)
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const float w = wx[a] * wy[bb] * wz[c];
                        float vi[3];
                        if (local) {
                            const int n = ((lz + c) * kBN + (ly + bb)) * kBN + (lx + a);
                            vi[0] = sv[0][n]; vi[1] = sv[1][n]; vi[2] = sv[2][n];
                        } else {
                            const float4 g = vel[node_index(E, b[0] + a, b[1] + bb, b[2] + c)];
                            vi[0] = g.x; vi[1] = g.y; vi[2] = g.z;
                        }
                        const float d[3] = {((float)a - f[0]) * dx, ((float)bb - f[1]) * dx,
                                            ((float)c - f[2]) * dx};
#pragma unroll
                        for (int r = 0; r < 3; ++r) {
                            const float wv = w * vi[r];
                            vp[r] += wv;
                            Cp[r * 3 + 0] += wv * d[0];
                            Cp[r * 3 + 1] += wv * d[1];
                            Cp[r * 3 + 2] += wv * d[2];
                        }
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
            svd3(Fn, U, s, V);
            if (E.mat.type == 1) dp_return_map(E.mat, U, s, V, Fn);
            kirchhoff_from_svd(E.mat, Fn, U, s, V, tau);
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
            if (pid_in && pid_out) pid_out[p] = pid_in[p];
        }
    }
    if (bad) atomicOr(&cnt->flags, kFlagNan);
}

hipError_t launch_g2p(const Work& w, const float* x_in, const float* F_in, float* x_out,
                      float* v_out, float* F_out, float* C_out, const int* pid_in, int* pid_out,
                      double h, hipStream_t s) {
    const unsigned blocks = (unsigned)std::min<long long>(w.n_tiles, 4096);
    hipLaunchKernelGGL(k_g2p, dim3(blocks), dim3(256), 0, s, x_in, F_in, x_out, v_out, F_out,
                       C_out, w.Q, pid_in, pid_out, w.P, w.envs, w.n_envs, w.ptile_id,
                       w.ptile_beg, w.vel, h, w.cnt);
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
