// sem_reduce.h -- deterministic block and grid reductions used by the
// reduction kernels (one FP64 partial per block, the last block to finish
// sums the partials in index order).
#pragma once

#include <hip/hip_runtime.h>

namespace sem {

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

// Publishes this block's partial and tells whether this block is the last
// one of the grid to do so (then every partial is visible to it).  The
// counter is reset by the last block, so the next launch starts from zero
// without a memset.  Every thread of the block must call it.
__device__ __forceinline__ bool publish_partial(double s, double *partial, unsigned int *counter,
                                                unsigned int nblocks, int *flag_lds) {
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = s;
        __threadfence();
        const unsigned int prev = atomicAdd(counter, 1u);
        *flag_lds = (prev == nblocks - 1) ? 1 : 0;
    }
    __syncthreads();
    const bool last = *flag_lds != 0;
    if (last) {
        __threadfence();
        if (threadIdx.x == 0) *counter = 0u;
    }
    return last;
}

// Fixed-order sum of partial[0..cnt) by one block: thread t sums the
// entries t, t + blockDim, ... in order, then the block sums the threads.
// The caller has executed the acquire fence of publish_partial.
__device__ __forceinline__ double sum_partials(const double *partial, int cnt, double *red) {
    double v = 0.0;
    for (int q = threadIdx.x; q < cnt; q += blockDim.x) v += partial[q];
    return block_sum_f64(v, red);
}

}  // namespace sem
