// sem_reduce.h -- deterministic reductions: every reduction kernel writes
// one FP64 partial per block; a one-block finalize kernel that follows in
// stream order sums the partials in index order.  (No grid-wide fences: on
// a chip whose L2 caches are private to each XCD an agent-scope fence per
// block costs an L2 write-back per block.)
#pragma once

#include <hip/hip_runtime.h>

namespace sem {

constexpr int kFinalizeThreads = 1024;

// Sum of one double per thread in a fixed order; the result is valid in
// thread 0 only.  Every thread of the block must call it.
__device__ __forceinline__ double block_sum_f64(double v, double *red /* >= 16 */) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int q = 0; q < nw; ++q) s += red[q];
    }
    __syncthreads();
    return s;
}

// Fixed-order sum of partial[0..cnt) by one block: thread t sums the
// entries t, t + blockDim, ... in order, then the block sums the threads.
// The loads of a batch of kBatch entries are issued before they are added,
// so the one block keeps many loads in flight.
__device__ __forceinline__ double sum_partials(const double *partial, int64_t cnt, double *red) {
    constexpr int kBatch = 8;
    double v = 0.0;
    const int64_t step = (int64_t)blockDim.x * kBatch;
    for (int64_t q0 = threadIdx.x; q0 < cnt; q0 += step) {
        double t[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int64_t q = q0 + (int64_t)u * blockDim.x;
            t[u] = q < cnt ? partial[q] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) v += t[u];
    }
    return block_sum_f64(v, red);
}

}  // namespace sem
