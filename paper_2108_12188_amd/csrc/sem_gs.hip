// sem_gs.hip -- gather-scatter QQ^T and the Dirichlet mask.
//
// Gather-scatter (Sec. 3.1, Sec. 4.3): every global point held by m > 1
// local copies forms a group; the copies' values are summed in ascending
// local index and the sum is written back to every copy.  Groups are stored
// by size class (all groups of one class have the same m), so a block only
// ever sees one m: no divergence across lanes, and the index list needs no
// offsets array.  Inside a class, groups are in ascending order of their
// first local index, which keeps neighbouring lanes on neighbouring faces.
#include "sem_gs_body.h"
#include "sem_internal.h"
#include "sem_vec_body.h"

namespace sem {
namespace {

using namespace gsb;

// Physical block b runs logical block lb: the blocks that land on one XCD
// (b mod 8) take one contiguous range of the group list, i.e. one region
// of the mesh, so the neighbouring copies they touch share that XCD's L2.
__device__ __forceinline__ int64_t logical_block(int64_t b, int64_t nb_phys) {
    const int64_t per = nb_phys / kXcds;
    return (b % kXcds) * per + b / kXcds;
}

// Logical blocks lb0 .. lb0 + nb_logical - 1.  st (may be null): a stopped
// CG state makes the whole grid exit at once.  With part_ax, the grid has
// one more block, which forms alpha from the operator's partials (Algorithm
// 1; it needs none of this kernel's results).
template <typename T>
__global__ void __launch_bounds__(kGsThreads)
gs_kernel(const GsClasses cls, int64_t lb0, int64_t nb_logical, const int32_t *__restrict__ idx,
          T *__restrict__ w, CgState *st, const double *part_ax, int64_t n_ax) {
    if (st && st->stop) return;
    int64_t nb = gridDim.x;
    if (part_ax) {
        if (blockIdx.x == gridDim.x - 1) {
            vecb::finalize_alpha_body(st, part_ax, n_ax);
            return;
        }
        --nb;
    }
    const int64_t b = logical_block(blockIdx.x, nb);
    if (b < nb_logical) gs_logical_block<T>(cls, lb0 + b, idx, w);
}

// Group sums of the classes with M >= mmin: logical blocks lb0 .. lb0 +
// nb_logical - 1 of the class list's block numbering; the last block forms
// alpha from the operator's partials.
template <typename T>
__global__ void __launch_bounds__(kGsThreads)
group_sums_kernel(const GsClasses cls, int64_t lb0, int64_t nb_logical,
                  const int32_t *__restrict__ idx, int64_t io0, const T *__restrict__ src,
                  T *__restrict__ out, CgState *st, const double *part_ax, int64_t n_ax,
                  int mmin) {
    if (st->stop) return;
    if (blockIdx.x == gridDim.x - 1) {
        vecb::finalize_alpha_body(st, part_ax, n_ax);
        return;
    }
    const int64_t b = logical_block(blockIdx.x, gridDim.x - 1);
    if (b < nb_logical) gs_sums_logical_block<T>(cls, lb0 + b, idx, io0, src, out, mmin);
}

template <typename T>
__global__ void mask_kernel(const int32_t *__restrict__ dir, int64_t n_dir, T *__restrict__ w) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_dir) w[dir[t]] = T(0);
}

}  // namespace

int64_t gs_logical_blocks(const Mesh &m) { return gs_total_blocks(m.gs); }

namespace {
// physical grid: a logical block count rounded up to a multiple of the XCD count
int gs_phys_blocks(int64_t b) { return (int)(b > 0 ? ((b + kXcds - 1) / kXcds) * kXcds : 1); }
}  // namespace

int gs_cg_blocks(const Mesh &m) { return gs_phys_blocks(gs_logical_blocks(m)); }

template <typename T>
void launch_gs(const Mesh &m, T *w, hipStream_t s) {
    if (m.n_groups == 0) return;
    const int nb = gs_cg_blocks(m);
    hipLaunchKernelGGL((gs_kernel<T>), dim3(nb), dim3(kGsThreads), 0, s, m.gs, (int64_t)0,
                       gs_logical_blocks(m), m.gs_idx, w, (CgState *)nullptr,
                       (const double *)nullptr, (int64_t)0);
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
void launch_gs_cg(const Mesh &m, T *w, CgState *st, const double *ax_partial, int n_ax_partial,
                  hipStream_t s) {
    const int64_t nlb = gs_logical_blocks(m);
    if (nlb > 0) {
        hipLaunchKernelGGL((gs_kernel<T>), dim3(gs_phys_blocks(nlb) + 1), dim3(kGsThreads), 0, s,
                           m.gs, (int64_t)0, nlb, m.gs_idx, w, st, ax_partial,
                           (int64_t)n_ax_partial);
        check_hip(hipGetLastError(), "gs/cg kernel launch");
    } else {
        launch_finalize_alpha(st, ax_partial, n_ax_partial, s);
    }
}

template <typename T>
void launch_group_sums_cg(const Mesh &m, const T *w, const T *wedge, T *gsum, CgState *st,
                          const double *ax_partial, int n_ax_partial, hipStream_t s) {
    const int64_t nlb = gs_logical_blocks(m) - m.gs_blk_multi;
    if (nlb > 0) {
        const bool compact = m.gsum_wedge;
        hipLaunchKernelGGL((group_sums_kernel<T>), dim3(gs_phys_blocks(nlb) + 1),
                           dim3(kGsThreads), 0, s, m.gs, m.gs_blk_multi, nlb,
                           compact ? m.wedge_idx : m.gs_idx, compact ? m.wedge_io0 : (int64_t)0,
                           compact ? wedge : w, gsum, st, ax_partial, (int64_t)n_ax_partial, 3);
        check_hip(hipGetLastError(), "group sums kernel launch");
    } else {
        launch_finalize_alpha(st, ax_partial, n_ax_partial, s);
    }
}

template <typename T>
void launch_edge_sums_cg(const Mesh &m, const T *wedge, T *gsum, CgState *st,
                         const double *ax_partial, int n_ax_partial, hipStream_t s) {
    const int64_t nlb = gs_total_blocks(m.ecls);
    if (nlb > 0) {
        hipLaunchKernelGGL((group_sums_kernel<T>), dim3(gs_phys_blocks(nlb) + 1),
                           dim3(kGsThreads), 0, s, m.ecls, (int64_t)0, nlb, m.ewedge_idx,
                           (int64_t)0, wedge, gsum, st, ax_partial, (int64_t)n_ax_partial, 2);
        check_hip(hipGetLastError(), "edge sums kernel launch");
    } else {
        launch_finalize_alpha(st, ax_partial, n_ax_partial, s);
    }
}

template void launch_gs<float>(const Mesh &, float *, hipStream_t);
template void launch_gs<double>(const Mesh &, double *, hipStream_t);
template void launch_mask<float>(const Mesh &, float *, hipStream_t);
template void launch_mask<double>(const Mesh &, double *, hipStream_t);
template void launch_gs_cg<float>(const Mesh &, float *, CgState *, const double *, int,
                                  hipStream_t);
template void launch_gs_cg<double>(const Mesh &, double *, CgState *, const double *, int,
                                   hipStream_t);
template void launch_edge_sums_cg<float>(const Mesh &, const float *, float *, CgState *,
                                         const double *, int, hipStream_t);
template void launch_edge_sums_cg<double>(const Mesh &, const double *, double *, CgState *,
                                          const double *, int, hipStream_t);
template void launch_group_sums_cg<float>(const Mesh &, const float *, const float *, float *,
                                          CgState *, const double *, int, hipStream_t);
template void launch_group_sums_cg<double>(const Mesh &, const double *, const double *,
                                           double *, CgState *, const double *, int,
                                           hipStream_t);

}  // namespace sem
