// sort_util.h -- chunking and block-scan helpers (wave64) used by the sort,
// the tile list, contact registration and the contact-node table.
#pragma once
#include <hip/hip_runtime.h>

namespace mpm {

// Contiguous chunk [beg, end) of n elements for block b of nb; chunks are
// multiples of 256 so that rounds of 256 stay aligned.
__device__ __forceinline__ void chunk_range(long long n, int b, int nb, long long* beg,
                                            long long* end) {
    long long per = (n + nb - 1) / nb;
    per = (per + 255) & ~255ll;
    long long s = per * b;
    long long e = s + per;
    *beg = s < n ? s : n;
    *end = e < n ? e : n;
}

__device__ __forceinline__ unsigned wave_inclusive_scan(unsigned v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        unsigned t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan across a block of up to 1024 threads (wsum: >= 16 entries).
__device__ __forceinline__ unsigned block_exclusive_scan_1024(unsigned v, unsigned* wsum) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    unsigned inc = wave_inclusive_scan(v);
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    if (wave == 0) {
        unsigned s = lane < nw ? wsum[lane] : 0u;
        unsigned si = wave_inclusive_scan(s);
        if (lane < nw) wsum[lane] = si - s;
    }
    __syncthreads();
    unsigned r = wsum[wave] + inc - v;
    __syncthreads();
    return r;
}

// Same with a total (wsum: >= 17 entries).
__device__ __forceinline__ unsigned block_exclusive_scan_total(unsigned v, unsigned* wsum,
                                                               unsigned* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    unsigned inc = wave_inclusive_scan(v);
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    if (wave == 0) {
        unsigned s = lane < nw ? wsum[lane] : 0u;
        unsigned si = wave_inclusive_scan(s);
        if (lane < nw) wsum[lane] = si - s;
        if (lane == nw - 1) wsum[16] = si;
    }
    __syncthreads();
    unsigned r = wsum[wave] + inc - v;
    *total = wsum[16];
    __syncthreads();
    return r;
}

}  // namespace mpm
