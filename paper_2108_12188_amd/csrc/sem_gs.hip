// sem_gs.hip -- gather-scatter QQ^T, Dirichlet mask, and the fused
// <p, w, c> reduction of Algorithm 1.
//
// Gather-scatter (Sec. 3.1, Sec. 4.3): every global point held by m > 1
// local copies forms a group; the copies' values are summed in ascending
// local index and the sum is written back to every copy.  Groups are stored
// by size class (all groups of one class have the same m), so a block only
// ever sees one m: no divergence across lanes, and the index list needs no
// offsets array.  Inside a class, groups are in ascending order of their
// first local index, which keeps neighbouring lanes on neighbouring faces.
#include "sem_internal.h"
#include "sem_reduce.h"

namespace sem {
namespace {

constexpr int kGsThreads = 256;
constexpr int kGsPerThread = 4;                   // groups per thread
constexpr int kGsPerBlock = kGsThreads * kGsPerThread;

template <typename T, int M>
__device__ __forceinline__ void group_sum(const int32_t *__restrict__ idx, T *__restrict__ w,
                                          const T *__restrict__ p, double &acc, bool dot) {
    int32_t q[M];
#pragma unroll
    for (int t = 0; t < M; ++t) q[t] = idx[t];
    T v[M];
#pragma unroll
    for (int t = 0; t < M; ++t) v[t] = w[q[t]];
    T s = v[0];
#pragma unroll
    for (int t = 1; t < M; ++t) s += v[t];
#pragma unroll
    for (int t = 0; t < M; ++t) w[q[t]] = s;
    if (dot) acc += (double)p[q[0]] * (double)s;
}

template <typename T>
__device__ __forceinline__ void group_sum_any(const int32_t *__restrict__ idx, int M,
                                              T *__restrict__ w, const T *__restrict__ p,
                                              double &acc, bool dot) {
    T s = w[idx[0]];
    for (int t = 1; t < M; ++t) s += w[idx[t]];
    for (int t = 0; t < M; ++t) w[idx[t]] = s;
    if (dot) acc += (double)p[idx[0]] * (double)s;
}

struct GsCfg {
    GsClasses cls;
    int64_t total_blocks;
};

template <typename T, bool FUSED>
__global__ void __launch_bounds__(kGsThreads)
gs_kernel(const GsClasses cls, const int32_t *__restrict__ idx, T *__restrict__ w,
          const T *__restrict__ p, CgState *st, const double *__restrict__ ax_partial,
          int n_ax_partial, double *gs_partial) {
    if constexpr (FUSED) {
        if (st->stop) return;
    }
    // locate the size class of this block (uniform)
    const int64_t b = blockIdx.x;
    int c = 0;
    while (c + 1 < cls.ncls && b >= cls.blk0[c + 1]) ++c;
    double acc = 0.0;
    if (c < cls.ncls && cls.ng[c] > 0) {
        const int M = cls.M[c];
        const int64_t g_first = (b - cls.blk0[c]) * kGsPerBlock;
        const int32_t *ib = idx + cls.io[c];
#pragma unroll
        for (int it = 0; it < kGsPerThread; ++it) {
            const int64_t g = g_first + (int64_t)it * kGsThreads + threadIdx.x;
            if (g < cls.ng[c]) {
                const int32_t *gi = ib + g * M;
                switch (M) {
                    case 2: group_sum<T, 2>(gi, w, p, acc, FUSED); break;
                    case 4: group_sum<T, 4>(gi, w, p, acc, FUSED); break;
                    case 8: group_sum<T, 8>(gi, w, p, acc, FUSED); break;
                    default: group_sum_any<T>(gi, M, w, p, acc, FUSED); break;
                }
            }
        }
    }
    if constexpr (FUSED) {
        __shared__ double red[16];
        __shared__ int last_flag;
        const double s = block_sum_f64(acc, red);
        if (publish_partial(s, gs_partial, &st->cnt_gs, gridDim.x, &last_flag)) {
            // <p, w, c> = interior part (from the Ax kernel) + shared part
            const double a1 = sum_partials(ax_partial, n_ax_partial, red);
            const double a2 = sum_partials(gs_partial, (int)gridDim.x, red);
            if (threadIdx.x == 0) {
                const double pw = a1 + a2;
                const double alpha = st->rho / pw;
                st->pw = pw;
                st->alpha = alpha;
                if (!(pw > 0.0) || !isfinite(alpha)) st->stop = 3;
                const int i = st->iter + 1;
                if (st->hist_alpha && i < st->hist_len) st->hist_alpha[i] = alpha;
            }
        }
    }
}

template <typename T>
__global__ void mask_kernel(const int32_t *__restrict__ dir, int64_t n_dir, T *__restrict__ w) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_dir) w[dir[t]] = T(0);
}

}  // namespace

int gs_cg_blocks(const Mesh &m) {
    int64_t b = m.gs.ncls > 0 ? m.gs.blk0[m.gs.ncls - 1] +
                                    (m.gs.ng[m.gs.ncls - 1] + kGsPerBlock - 1) / kGsPerBlock
                              : 0;
    return (int)(b > 0 ? b : 1);
}

void gs_classes_finish(GsClasses &c) {
    int64_t blk = 0;
    for (int q = 0; q < c.ncls; ++q) {
        c.blk0[q] = blk;
        blk += (c.ng[q] + kGsPerBlock - 1) / kGsPerBlock;
    }
}

template <typename T>
void launch_gs(const Mesh &m, T *w, hipStream_t s) {
    if (m.n_groups == 0) return;
    const int nb = gs_cg_blocks(m);
    hipLaunchKernelGGL((gs_kernel<T, false>), dim3(nb), dim3(kGsThreads), 0, s, m.gs, m.gs_idx,
                       w, (const T *)nullptr, (CgState *)nullptr, (const double *)nullptr, 0,
                       (double *)nullptr);
    check_hip(hipGetLastError(), "gs kernel launch");
}

template <typename T>
void launch_mask(const Mesh &m, T *w, hipStream_t s) {
    if (m.n_dir == 0) return;
    const int64_t nb = (m.n_dir + 255) / 256;
    hipLaunchKernelGGL((mask_kernel<T>), dim3((unsigned)nb), dim3(256), 0, s, m.dir_idx, m.n_dir, w);
    check_hip(hipGetLastError(), "mask kernel launch");
}

template <typename T>
void launch_gs_cg(const Mesh &m, T *w, const T *p, CgState *st, const double *ax_partial,
                  int n_ax_partial, double *gs_partial, hipStream_t s) {
    const int nb = gs_cg_blocks(m);
    hipLaunchKernelGGL((gs_kernel<T, true>), dim3(nb), dim3(kGsThreads), 0, s, m.gs, m.gs_idx, w,
                       p, st, ax_partial, n_ax_partial, gs_partial);
    check_hip(hipGetLastError(), "gs/cg kernel launch");
}

template void launch_gs<float>(const Mesh &, float *, hipStream_t);
template void launch_gs<double>(const Mesh &, double *, hipStream_t);
template void launch_mask<float>(const Mesh &, float *, hipStream_t);
template void launch_mask<double>(const Mesh &, double *, hipStream_t);
template void launch_gs_cg<float>(const Mesh &, float *, const float *, CgState *,
                                  const double *, int, double *, hipStream_t);
template void launch_gs_cg<double>(const Mesh &, double *, const double *, CgState *,
                                   const double *, int, double *, hipStream_t);

}  // namespace sem
