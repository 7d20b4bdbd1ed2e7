// sort.hip -- stable LSD radix sort of (key, value) pairs and device-wide
// chunked scans for gfx950 (wave64).
//
// A fixed grid of kSortBlocks blocks splits the input into contiguous chunks,
// so the element count may live in device memory (it is read by every kernel
// at start) and nothing needs a host round trip. Per 8-bit digit pass:
//   hist:    per-block digit histogram in LDS -> hist[digit][block]
//   rowscan: one block per digit scans its row of block counts (coalesced)
//            and stores the digit's total
//   scatter: each block first turns the 256 digit totals into digit offsets
//            (one block scan), then walks its chunk in order in 256-element
//            rounds; the
//            rank of an element among equal digits of its wave comes from
//            eight ballots, ranks across the block's four waves from a small
//            LDS table, so the pass is stable and the result bit-exact.
#include "mpm_internal.h"
#include "sort_util.h"

namespace mpm {

__global__ void __launch_bounds__(kSortThreads)
k_rs_hist(const unsigned* __restrict__ keys, const unsigned* count_dev, long long count_host,
          int shift, unsigned* __restrict__ hist) {
    __shared__ unsigned h[256];
    const long long n = count_dev ? (long long)*count_dev : count_host;
    long long beg, end;
    chunk_range(n, blockIdx.x, gridDim.x, &beg, &end);
    h[threadIdx.x] = 0;
    __syncthreads();
    for (long long i = beg + threadIdx.x; i < end; i += blockDim.x)
        atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    __syncthreads();
    hist[threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of one digit's row of per-block counts, in place; the row
// total goes to totals[digit]. One block of kSortBlocks threads per digit.
__global__ void __launch_bounds__(kSortBlocks)
k_rs_rowscan(unsigned* __restrict__ hist, unsigned* __restrict__ totals) {
    __shared__ unsigned wsum[17];
    unsigned* row = hist + (size_t)blockIdx.x * kSortBlocks;
    const unsigned v = row[threadIdx.x];
    unsigned total;
    const unsigned ex = block_exclusive_scan_total(v, wsum, &total);
    row[threadIdx.x] = ex;
    if (threadIdx.x == 0) totals[blockIdx.x] = total;
}

// Exclusive scan of n_items unsigned values in place by one block of 1024
// threads (used for n_items <= a few thousand); optionally stores the total.
__global__ void __launch_bounds__(1024)
k_scan_one_block(unsigned* __restrict__ data, int n_items, unsigned* total) {
    __shared__ unsigned wsum[16];
    const int T = blockDim.x;
    const int per = (n_items + T - 1) / T;
    const int beg = threadIdx.x * per;
    const int end = min(n_items, beg + per);
    unsigned local = 0;
    for (int i = beg; i < end; ++i) local += data[i];
    unsigned excl = block_exclusive_scan_1024(local, wsum);
    unsigned run = excl;
    for (int i = beg; i < end; ++i) {
        unsigned v = data[i];
        data[i] = run;
        run += v;
    }
    if (total && threadIdx.x == T - 1) *total = run;
}

__global__ void __launch_bounds__(kSortThreads)
k_rs_scatter(const unsigned* __restrict__ kin, const unsigned* __restrict__ vin,
             unsigned* __restrict__ kout, unsigned* __restrict__ vout,
             const unsigned* count_dev, long long count_host, int shift,
             const unsigned* __restrict__ hist, const unsigned* __restrict__ totals) {
    static_assert(kSortThreads == 256, "one thread per digit");
    __shared__ unsigned running[256];
    __shared__ unsigned wcnt[kSortThreads / 64][256];
    __shared__ unsigned wsum[16];
    const long long n = count_dev ? (long long)*count_dev : count_host;
    long long beg, end;
    chunk_range(n, blockIdx.x, gridDim.x, &beg, &end);
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const unsigned digit_off = block_exclusive_scan_1024(totals[tid], wsum);
    running[tid] = digit_off + hist[tid * gridDim.x + blockIdx.x];
    for (long long base = beg; base < end; base += kSortThreads) {
        for (int w = 0; w < kSortThreads / 64; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        const long long i = base + tid;
        const bool valid = i < end;
        unsigned key = valid ? kin[i] : 0u;
        unsigned val = valid ? vin[i] : 0u;
        unsigned d = (key >> shift) & 255u;
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            unsigned long long m = __ballot(valid && bit);
            peers &= bit ? m : ~m;
        }
        const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        const unsigned rank = (unsigned)__popcll(peers & lt);
        if (valid && rank == 0) wcnt[wave][d] = (unsigned)__popcll(peers);
        __syncthreads();
        if (valid) {
            unsigned off = running[d] + rank;
            for (int w = 0; w < wave; ++w) off += wcnt[w][d];
            kout[off] = key;
            vout[off] = val;
        }
        __syncthreads();
        unsigned tot = 0;
        for (int w = 0; w < kSortThreads / 64; ++w) tot += wcnt[w][tid];
        running[tid] += tot;
        __syncthreads();
    }
}

hipError_t launch_scan_blocks(unsigned* data, int n_items, unsigned* total, hipStream_t s) {
    hipLaunchKernelGGL(k_scan_one_block, dim3(1), dim3(1024), 0, s, data, n_items, total);
    return hipGetLastError();
}

hipError_t radix_sort(const Work& w, unsigned* keys, unsigned* vals, unsigned* keys_tmp,
                      unsigned* vals_tmp, const unsigned* count_dev, long long count_host,
                      int bits, hipStream_t s, unsigned** keys_out, unsigned** vals_out) {
    unsigned *ki = keys, *vi = vals, *ko = keys_tmp, *vo = vals_tmp;
    const int passes = (bits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_rs_hist, dim3(kSortBlocks), dim3(kSortThreads), 0, s, ki, count_dev,
                           count_host, shift, w.blk);
        unsigned* totals = w.blk + 256 * kSortBlocks;
        hipLaunchKernelGGL(k_rs_rowscan, dim3(256), dim3(kSortBlocks), 0, s, w.blk, totals);
        hipLaunchKernelGGL(k_rs_scatter, dim3(kSortBlocks), dim3(kSortThreads), 0, s, ki, vi, ko,
                           vo, count_dev, count_host, shift, w.blk, (const unsigned*)totals);
        unsigned* t = ki; ki = ko; ko = t;
        t = vi; vi = vo; vo = t;
    }
    *keys_out = ki;
    *vals_out = vi;
    return hipGetLastError();
}

}  // namespace mpm
