// sem_gs_body.h -- device code of the gather-scatter shared by the
// single-mesh and the batched kernels.
#pragma once

#include "sem_internal.h"

namespace sem {
namespace gsb {

constexpr int kGsThreads = 256;
constexpr int kXcds = 8;                          // MI355X: 8 XCDs, blocks dealt round-robin

// groups per thread for a group size: about 8 copies per thread in flight
__host__ __device__ constexpr int gs_per_thread(int M) { return M >= 8 ? 1 : (M >= 4 ? 2 : 4); }
__host__ __device__ constexpr int64_t gs_per_block(int M) {
    return (int64_t)kGsThreads * gs_per_thread(M);
}

template <int M>
struct alignas(M * 4 <= 16 ? M * 4 : 16) IdxVec {
    int32_t v[M];
};

// Groups of a compile-time size M: every lane first issues the index loads
// of all its groups, then all value loads, so each lane keeps
// kGsPerThread * M independent loads in flight (groups are disjoint, so the
// stores of one group never alias the loads of another).
template <typename T, int M>
__device__ __forceinline__ void gs_groups_fixed(const int32_t *__restrict__ ib, int64_t g0,
                                                int64_t ng, T *__restrict__ w) {
    constexpr int kGsPerThread = gs_per_thread(M);
    int32_t q[kGsPerThread][M];
    bool ok[kGsPerThread];
#pragma unroll
    for (int it = 0; it < kGsPerThread; ++it) {
        const int64_t g = g0 + (int64_t)it * kGsThreads;
        ok[it] = g < ng;
        if (ok[it]) {
            const IdxVec<M> *src = reinterpret_cast<const IdxVec<M> *>(ib + g * M);
            const IdxVec<M> iv = *src;
#pragma unroll
            for (int t = 0; t < M; ++t) q[it][t] = iv.v[t];
        } else {
#pragma unroll
            for (int t = 0; t < M; ++t) q[it][t] = 0;
        }
    }
    T v[kGsPerThread][M];
#pragma unroll
    for (int it = 0; it < kGsPerThread; ++it)
#pragma unroll
        for (int t = 0; t < M; ++t) v[it][t] = ok[it] ? w[q[it][t]] : T(0);
#pragma unroll
    for (int it = 0; it < kGsPerThread; ++it) {
        if (!ok[it]) continue;
        T s = v[it][0];
#pragma unroll
        for (int t = 1; t < M; ++t) s += v[it][t];
#pragma unroll
        for (int t = 0; t < M; ++t) w[q[it][t]] = s;
    }
}

template <typename T>
__device__ __forceinline__ void gs_groups_any(const int32_t *__restrict__ ib, int M, int64_t g0,
                                              int64_t ng, T *__restrict__ w) {
    for (int it = 0; it < gs_per_thread(M); ++it) {
        const int64_t g = g0 + (int64_t)it * kGsThreads;
        if (g >= ng) break;
        const int32_t *gi = ib + g * M;
        T s = w[gi[0]];
        for (int t = 1; t < M; ++t) s += w[gi[t]];
        for (int t = 0; t < M; ++t) w[gi[t]] = s;
    }
}

// Sums only: out[g] = sum of the copies of group g (ascending local index,
// the order of gs_groups_fixed); w is read, not written.  Loads of all of a
// lane's groups are issued before any sum, as in gs_groups_fixed.
template <typename T, int M>
__device__ __forceinline__ void gs_sums_fixed(const int32_t *__restrict__ ib, int64_t g0,
                                              int64_t ng, const T *__restrict__ w,
                                              T *__restrict__ out) {
    constexpr int kGsPerThread = gs_per_thread(M);
    int32_t q[kGsPerThread][M];
    bool ok[kGsPerThread];
#pragma unroll
    for (int it = 0; it < kGsPerThread; ++it) {
        const int64_t g = g0 + (int64_t)it * kGsThreads;
        ok[it] = g < ng;
        if (ok[it]) {
            const IdxVec<M> iv = *reinterpret_cast<const IdxVec<M> *>(ib + g * M);
#pragma unroll
            for (int t = 0; t < M; ++t) q[it][t] = iv.v[t];
        } else {
#pragma unroll
            for (int t = 0; t < M; ++t) q[it][t] = 0;
        }
    }
    T v[kGsPerThread][M];
#pragma unroll
    for (int it = 0; it < kGsPerThread; ++it)
#pragma unroll
        for (int t = 0; t < M; ++t) v[it][t] = ok[it] ? w[q[it][t]] : T(0);
#pragma unroll
    for (int it = 0; it < kGsPerThread; ++it) {
        if (!ok[it]) continue;
        T s = v[it][0];
#pragma unroll
        for (int t = 1; t < M; ++t) s += v[it][t];
        out[g0 + (int64_t)it * kGsThreads] = s;
    }
}

template <typename T>
__device__ __forceinline__ void gs_sums_any(const int32_t *__restrict__ ib, int M, int64_t g0,
                                            int64_t ng, const T *__restrict__ w,
                                            T *__restrict__ out) {
    for (int it = 0; it < gs_per_thread(M); ++it) {
        const int64_t g = g0 + (int64_t)it * kGsThreads;
        if (g >= ng) break;
        const int32_t *gi = ib + g * M;
        T s = w[gi[0]];
        for (int t = 1; t < M; ++t) s += w[gi[t]];
        out[g] = s;
    }
}

// One logical block lb of a mesh's group sums over the classes with
// M >= mmin (3: the groups of more than two copies of the full class list;
// 2: every class of the edge-node list of the table-free gather).  The
// copies of class c's groups are read from w at the indices
// idx[cls.io[c] - io0 ...] (gs_idx and the local w, or the compact edge
// array and its positions); the sums go to out + (groups of the classes
// with M >= mmin before c).
template <typename T>
__device__ __forceinline__ void gs_sums_logical_block(const GsClasses &cls, int64_t lb,
                                                      const int32_t *__restrict__ idx,
                                                      int64_t io0, const T *__restrict__ w,
                                                      T *__restrict__ out, int mmin = 3) {
    int c = 0;
    while (c + 1 < cls.ncls && lb >= cls.blk0[c + 1]) ++c;
    int64_t goff = 0;
    for (int q = 0; q < c; ++q)
        if (cls.M[q] >= mmin) goff += cls.ng[q];
    const int M = cls.M[c];
    const int64_t g0 = (lb - cls.blk0[c]) * gs_per_block(M) + threadIdx.x;
    const int32_t *ib = idx + (cls.io[c] - io0);
    const int64_t ng = cls.ng[c];
    switch (M) {
        case 2: gs_sums_fixed<T, 2>(ib, g0, ng, w, out + goff); break;
        case 4: gs_sums_fixed<T, 4>(ib, g0, ng, w, out + goff); break;
        case 8: gs_sums_fixed<T, 8>(ib, g0, ng, w, out + goff); break;
        default: gs_sums_any<T>(ib, M, g0, ng, w, out + goff); break;
    }
}

// The logical block at position lb of a gather-scatter launch (uniform
// across the block), in the class-major block numbering after the mesh's
// block order, if it has one.
template <typename T>
__device__ __forceinline__ void gs_logical_block(const GsClasses &cls, int64_t lb,
                                                 const int32_t *__restrict__ idx,
                                                 T *__restrict__ w) {
    if (cls.lb_order) lb = cls.lb_order[lb];
    int c = 0;
    while (c + 1 < cls.ncls && lb >= cls.blk0[c + 1]) ++c;
    const int M = cls.M[c];
    const int64_t g0 = (lb - cls.blk0[c]) * gs_per_block(M) + threadIdx.x;
    const int32_t *ib = idx + cls.io[c];
    const int64_t ng = cls.ng[c];
    switch (M) {
        case 2: gs_groups_fixed<T, 2>(ib, g0, ng, w); break;
        case 4: gs_groups_fixed<T, 4>(ib, g0, ng, w); break;
        case 8: gs_groups_fixed<T, 8>(ib, g0, ng, w); break;
        default: gs_groups_any<T>(ib, M, g0, ng, w); break;
    }
}

}  // namespace gsb
}  // namespace sem
