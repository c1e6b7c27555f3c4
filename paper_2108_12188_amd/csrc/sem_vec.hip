// sem_vec.hip -- the vector updates and weighted reductions of Algorithm 1.
//
// All reductions accumulate in FP64 (a product of two FP32 values is exact
// in FP64) with the weights c_l = 1/m_l of the weighted inner product
// <a, b, c>; the per-point code holds m_l and the Dirichlet flag.  The grid
// size depends only on n, and the block partials are summed in index order
// by the last block, so every result is bitwise reproducible.
#include <mutex>

#include "sem_vec_body.h"

namespace sem {
namespace {

using namespace vecb;

template <typename T, bool PC>
__global__ void __launch_bounds__(kVecThreads)
update_kernel(int64_t n, T *__restrict__ r, const T *__restrict__ w,
              const uint8_t *__restrict__ mcode, CgState *st, double *partial, PcArgs<T> pc) {
    update_body<T, false, PC>(n, nullptr, r, nullptr, w, mcode, st, partial, blockIdx.x,
                              gridDim.x, pc);
}

// x += alpha p when the state says the last update's step is pending
template <typename T>
__global__ void __launch_bounds__(kVecThreads)
x_flush_kernel(int64_t n, T *__restrict__ x, const T *__restrict__ p, const CgState *st) {
    if (!st->x_lag) return;
    const T a = (T)st->alpha;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride)
        x[q] += a * p[q];
}

template <typename T, bool PC>
__global__ void __launch_bounds__(kVecThreads)
update_gather_kernel(int64_t n, T *__restrict__ r, const T *__restrict__ w,
                     const T *__restrict__ gsum, const uint8_t *__restrict__ mcode,
                     const GatherMap gm, CgState *st, double *partial, PcArgs<T> pc) {
    update_gather_body<T, PC>(n, r, w, gsum, mcode, gm, st, partial, blockIdx.x, gridDim.x, pc);
}

template <typename T, bool PC>
__global__ void __launch_bounds__(kVecThreads)
update_struct_kernel(int64_t n, T *__restrict__ r, const T *__restrict__ wg,
                     const StructMap sm, CgState *st, double *partial, PcArgs<T> pc) {
    update_struct_body<T, PC>(n, r, wg, sm, st, partial, blockIdx.x, gridDim.x, pc);
}

__global__ void __launch_bounds__(kFinalizeThreads)
finalize_rho_kernel(CgState *st, const double *partial, int cnt, const double *partial2) {
    finalize_rho_body(st, partial, cnt, partial2);
}

// Jacobi preconditioner from the assembled diagonal d (local form):
// minv = 1/d on the free points, 0 on the Dirichlet points.
__global__ void __launch_bounds__(kVecThreads)
jacobi_invert_kernel(int64_t n, const double *__restrict__ d, const uint8_t *__restrict__ mcode,
                     double *__restrict__ minv64, float *__restrict__ minv32) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
        const double v = (mcode[q] & kDirichletBit) ? 0.0 : 1.0 / d[q];
        minv64[q] = v;
        minv32[q] = (float)v;
    }
}

__global__ void __launch_bounds__(kFinalizeThreads)
finalize_alpha_kernel(CgState *st, const double *part_ax, int64_t n_ax) {
    finalize_alpha_body(st, part_ax, n_ax);
}

// r0 = b - A x0 (w holds A x0, or is null for x0 = 0); p0 = 0; beta_0 = 0;
// rho_0 = <r0, r0, c>; the threshold becomes tol^2 rho_0.  With pc.minv:
// z0 = minv r0, rho = <r0, z0, c> (partial) and <r0, r0, c> (partial2).
template <typename T>
__global__ void __launch_bounds__(kVecThreads)
cg_init_kernel(int64_t n, const T *__restrict__ b, const T *__restrict__ w, T *__restrict__ r,
               T *__restrict__ p, const uint8_t *__restrict__ mcode, CgState *st,
               double *partial, PcArgs<T> pc) {
    __shared__ double cw[kVecThreads];
    __shared__ double red[16];
    weights_lds(cw);
    double acc = 0.0, acc2 = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
        const T rv = w ? b[q] - w[q] : b[q];
        r[q] = rv;
        p[q] = T(0);
        if (pc.minv) {
            const T zv = pc.minv[q] * rv;
            pc.z[q] = zv;
            acc += (double)rv * (double)zv * cw[mcode[q]];
            acc2 += (double)rv * (double)rv * cw[mcode[q]];
        } else {
            acc += (double)rv * (double)rv * cw[mcode[q]];
        }
    }
    const double s = block_sum_f64(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
    if (pc.minv) {
        const double s2 = block_sum_f64(acc2, red);
        if (threadIdx.x == 0) pc.partial2[blockIdx.x] = s2;
    }
}

__global__ void __launch_bounds__(kFinalizeThreads)
finalize_init_kernel(CgState *st, const double *partial, int cnt, const double *partial2) {
    __shared__ double red[16];
    const double rz0 = sum_partials(partial, cnt, red);
    const double rho0 = partial2 ? sum_partials(partial2, cnt, red) : rz0;
    if (threadIdx.x == 0) {
        st->rho = rz0;
        st->rr = rho0;
        st->rho0 = rho0;
        st->thresh = st->thresh * rho0;
        st->beta = 0.0;
        st->alpha = 0.0;
        st->x_lag = 0;
        st->iter = 0;
        if (st->hist_rho && st->hist_len > 0) st->hist_rho[0] = rho0;
        int stop = 0;
        if (!isfinite(rho0) || !isfinite(rz0)) stop = 3;
        else if (rho0 == 0.0) stop = 1;
        else if (st->max_iter <= 0) stop = 2;
        st->stop = stop;
    }
}

template <typename T>
__global__ void __launch_bounds__(kVecThreads)
dot_kernel(int64_t n, const T *__restrict__ a, const T *__restrict__ b,
           const uint8_t *__restrict__ mcode, double *partial) {
    __shared__ double cw[kVecThreads];
    __shared__ double red[16];
    weights_lds(cw);
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride)
        acc += (double)a[q] * (double)b[q] * cw[mcode[q]];
    const double s = block_sum_f64(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kVecThreads)
residual64_kernel(int64_t n, const double *__restrict__ b, const double *__restrict__ w,
                  double *__restrict__ r, const uint8_t *__restrict__ mcode, double *partial) {
    __shared__ double cw[kVecThreads];
    __shared__ double red[16];
    weights_lds(cw);
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
        const double rv = b[q] - w[q];
        r[q] = rv;
        acc += rv * rv * cw[mcode[q]];
    }
    const double s = block_sum_f64(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kFinalizeThreads)
finalize_sum_kernel(double *out, const double *partial, int cnt) {
    __shared__ double red[16];
    const double v = sum_partials(partial, cnt, red);
    if (threadIdx.x == 0) *out = v;
}

__global__ void scale_to_f32_kernel(int64_t n, const double *__restrict__ src,
                                    const double *__restrict__ nrm2, float *__restrict__ dst) {
    const double inv = 1.0 / sqrt(*nrm2);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride)
        dst[q] = (float)(src[q] * inv);
}

__global__ void axpy_from_f32_kernel(int64_t n, double *__restrict__ x,
                                     const double *__restrict__ nrm2, const float *__restrict__ d) {
    const double sc = sqrt(*nrm2);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride)
        x[q] += sc * (double)d[q];
}

template <typename Ts, typename Td>
__global__ void convert_kernel(int64_t n, const Ts *__restrict__ src, Td *__restrict__ dst) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride)
        dst[q] = (Td)src[q];
}

__global__ void mul64_kernel(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                             double *__restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride)
        out[q] = a[q] * b[q];
}

int elem_blocks(int64_t n) {
    int64_t b = (n + kVecThreads - 1) / kVecThreads;
    if (b > 8192) b = 8192;
    return (int)(b > 0 ? b : 1);
}

}  // namespace

int vec_blocks(int64_t n) {
    int64_t b = (n + 4 * kVecThreads - 1) / (4 * kVecThreads);
    if (b > kVecMaxBlocks) {
        // as many blocks as give every block the same number of grid-stride
        // steps (at most kVecMaxBlocks): the XCD-contiguous block ranges of
        // the updates then end together (24^3 N = 9: 3375 blocks of four
        // steps, update 42.1 against 45.5 us with 4096 of three or four)
        const int64_t steps = (b + kVecMaxBlocks - 1) / kVecMaxBlocks;
        b = (b + steps - 1) / steps;
    }
    return (int)(b > 0 ? b : 1);
}

template <typename T>
void launch_update(const Mesh &m, T *r, const T *w, CgState *st, double *partial,
                   hipStream_t s, PcArgs<T> pc) {
    const int nb = vec_blocks(m.n);
    if (pc.minv)
        hipLaunchKernelGGL((update_kernel<T, true>), dim3(nb), dim3(kVecThreads), 0, s, m.n, r, w,
                           m.mcode, st, partial, pc);
    else
        hipLaunchKernelGGL((update_kernel<T, false>), dim3(nb), dim3(kVecThreads), 0, s, m.n, r,
                           w, m.mcode, st, partial, pc);
    hipLaunchKernelGGL(finalize_rho_kernel, dim3(1), dim3(kFinalizeThreads), 0, s, st,
                       (const double *)partial, nb, (const double *)pc.partial2);
    check_hip(hipGetLastError(), "update kernel launch");
}

void launch_jacobi_invert(const Mesh &m, const double *d, double *minv64, float *minv32,
                          hipStream_t s) {
    hipLaunchKernelGGL(jacobi_invert_kernel, dim3(elem_blocks(m.n)), dim3(kVecThreads), 0, s,
                       m.n, d, m.mcode, minv64, minv32);
    check_hip(hipGetLastError(), "jacobi invert kernel launch");
}

template <typename T>
void launch_x_flush(const Mesh &m, T *x, const T *p, const CgState *st, hipStream_t s) {
    hipLaunchKernelGGL((x_flush_kernel<T>), dim3(elem_blocks(m.n)), dim3(kVecThreads), 0, s, m.n,
                       x, p, st);
    check_hip(hipGetLastError(), "x flush kernel launch");
}

template <typename T>
void launch_update_gather(const Mesh &m, T *r, const T *w, const T *gsum, CgState *st,
                          double *partial, hipStream_t s, PcArgs<T> pc) {
    if (!m.gs_in_update)
        fail(SEM_EUNSUPPORTED, "mesh shares points inside elements: no gather in the update");
    if (!m.gsrc) fail(SEM_EUNSUPPORTED, "mesh holds no per-point gather table");
    const GatherMap gm{m.gsrc};
    const int nb = vec_blocks(m.n);
    if (pc.minv)
        hipLaunchKernelGGL((update_gather_kernel<T, true>), dim3(nb), dim3(kVecThreads), 0, s,
                           m.n, r, w, gsum, m.mcode, gm, st, partial, pc);
    else
        hipLaunchKernelGGL((update_gather_kernel<T, false>), dim3(nb), dim3(kVecThreads), 0, s,
                           m.n, r, w, gsum, m.mcode, gm, st, partial, pc);
    hipLaunchKernelGGL(finalize_rho_kernel, dim3(1), dim3(kFinalizeThreads), 0, s, st,
                       (const double *)partial, nb, (const double *)pc.partial2);
    check_hip(hipGetLastError(), "update kernel launch");
}

template <typename T>
void launch_update_struct(const Mesh &m, T *r, const T *wg, CgState *st, double *partial,
                          hipStream_t s, PcArgs<T> pc) {
    if (!m.gs_struct) fail(SEM_EUNSUPPORTED, "mesh has no table-free gather");
    if (m.P3 > kMaxPosTab || m.n % 4) fail(SEM_EUNSUPPORTED, "table-free gather: bad order");
    const StructMap sm{m.erec, m.pos_tab, m.P3, 6 + edge_slots(m.N), m.p3_magic, m.p3_shift};
    const int nb = vec_blocks(m.n);
    if (pc.minv)
        hipLaunchKernelGGL((update_struct_kernel<T, true>), dim3(nb), dim3(kVecThreads), 0, s,
                           m.n, r, wg, sm, st, partial, pc);
    else
        hipLaunchKernelGGL((update_struct_kernel<T, false>), dim3(nb), dim3(kVecThreads), 0, s,
                           m.n, r, wg, sm, st, partial, pc);
    hipLaunchKernelGGL(finalize_rho_kernel, dim3(1), dim3(kFinalizeThreads), 0, s, st,
                       (const double *)partial, nb, (const double *)pc.partial2);
    check_hip(hipGetLastError(), "update kernel launch");
}

template <typename T>
void launch_cg_init(const Mesh &m, const T *b, const T *w, T *r, T *p, CgState *st,
                    double *partial, hipStream_t s, PcArgs<T> pc) {
    const int nb = vec_blocks(m.n);
    hipLaunchKernelGGL((cg_init_kernel<T>), dim3(nb), dim3(kVecThreads), 0, s, m.n, b, w, r, p,
                       m.mcode, st, partial, pc);
    hipLaunchKernelGGL(finalize_init_kernel, dim3(1), dim3(kFinalizeThreads), 0, s, st,
                       (const double *)partial, nb, (const double *)pc.partial2);
    check_hip(hipGetLastError(), "cg init kernel launch");
}

template <typename T>
void launch_dot(const Mesh &m, const T *a, const T *b, double *out, double *partial,
                hipStream_t s) {
    const int nb = vec_blocks(m.n);
    hipLaunchKernelGGL((dot_kernel<T>), dim3(nb), dim3(kVecThreads), 0, s, m.n, a, b, m.mcode,
                       partial);
    hipLaunchKernelGGL(finalize_sum_kernel, dim3(1), dim3(kFinalizeThreads), 0, s, out,
                       (const double *)partial, nb);
    check_hip(hipGetLastError(), "dot kernel launch");
}

void launch_residual64(const Mesh &m, const double *b, const double *w, double *r, double *out,
                       double *partial, hipStream_t s) {
    const int nb = vec_blocks(m.n);
    hipLaunchKernelGGL(residual64_kernel, dim3(nb), dim3(kVecThreads), 0, s, m.n, b, w, r,
                       m.mcode, partial);
    hipLaunchKernelGGL(finalize_sum_kernel, dim3(1), dim3(kFinalizeThreads), 0, s, out,
                       (const double *)partial, nb);
    check_hip(hipGetLastError(), "residual kernel launch");
}

void launch_scale_to_f32(int64_t n, const double *src, const double *nrm2, float *dst,
                         hipStream_t s) {
    hipLaunchKernelGGL(scale_to_f32_kernel, dim3(elem_blocks(n)), dim3(kVecThreads), 0, s, n, src,
                       nrm2, dst);
    check_hip(hipGetLastError(), "scale kernel launch");
}

void launch_axpy_from_f32(int64_t n, double *x, const double *nrm2, const float *d,
                          hipStream_t s) {
    hipLaunchKernelGGL(axpy_from_f32_kernel, dim3(elem_blocks(n)), dim3(kVecThreads), 0, s, n, x,
                       nrm2, d);
    check_hip(hipGetLastError(), "axpy kernel launch");
}

template <typename Ts, typename Td>
void launch_convert(int64_t n, const Ts *src, Td *dst, hipStream_t s) {
    hipLaunchKernelGGL((convert_kernel<Ts, Td>), dim3(elem_blocks(n)), dim3(kVecThreads), 0, s, n,
                       src, dst);
    check_hip(hipGetLastError(), "convert kernel launch");
}

void launch_mul64(int64_t n, const double *a, const double *b, double *out, hipStream_t s) {
    hipLaunchKernelGGL(mul64_kernel, dim3(elem_blocks(n)), dim3(kVecThreads), 0, s, n, a, b, out);
    check_hip(hipGetLastError(), "mul kernel launch");
}

template void launch_update<float>(const Mesh &, float *, const float *, CgState *, double *,
                                   hipStream_t, PcArgs<float>);
template void launch_update<double>(const Mesh &, double *, const double *, CgState *, double *,
                                    hipStream_t, PcArgs<double>);
template void launch_x_flush<float>(const Mesh &, float *, const float *, const CgState *,
                                    hipStream_t);
template void launch_x_flush<double>(const Mesh &, double *, const double *, const CgState *,
                                     hipStream_t);
template void launch_update_gather<float>(const Mesh &, float *, const float *, const float *,
                                          CgState *, double *, hipStream_t, PcArgs<float>);
template void launch_update_gather<double>(const Mesh &, double *, const double *,
                                           const double *, CgState *, double *, hipStream_t,
                                           PcArgs<double>);
template void launch_update_struct<float>(const Mesh &, float *, const float *, CgState *,
                                          double *, hipStream_t, PcArgs<float>);
template void launch_update_struct<double>(const Mesh &, double *, const double *, CgState *,
                                           double *, hipStream_t, PcArgs<double>);
template void launch_cg_init<float>(const Mesh &, const float *, const float *, float *, float *,
                                    CgState *, double *, hipStream_t, PcArgs<float>);
template void launch_cg_init<double>(const Mesh &, const double *, const double *, double *,
                                     double *, CgState *, double *, hipStream_t, PcArgs<double>);
// ---------------------------------------------------------------------------
// sem_dot_noalloc: the weighted inner product with its block partials in
// `scratch`, a file-scope device array (one copy per GPU, held until the
// process ends), so the call allocates nothing.  Every block writes its own
// partial before the finalize kernel reads exactly those, so nothing needs
// clearing between calls.  Calls that overlap on one GPU share the array and
// race.
// ---------------------------------------------------------------------------
namespace {
constexpr int kNoAllocPartials = 4096;          // 32 KiB of FP64 partials
static_assert(kVecMaxBlocks <= kNoAllocPartials,
              "the no-allocation dot needs one scratch slot per vector block");
static __device__ __align__(256) double scratch[kNoAllocPartials];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[kMaxScratchDevices] = {};

// Device address of this GPU's copy of `scratch` (the array's name is only a
// host-side stand-in); looked up once per device with that device current.
double *noalloc_scratch() {
    int dev = 0;
    check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxScratchDevices)
        fail(SEM_EUNSUPPORTED, "device ordinal beyond the no-allocation table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        check_hip(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!ptr) fail(SEM_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_dev[dev] = static_cast<double *>(ptr);
    }
    return g_scratch_dev[dev];
}
}  // namespace

template <typename T>
void launch_dot_noalloc(const Mesh &m, const T *a, const T *b, double *out, hipStream_t s) {
    const int nb = vec_blocks(m.n);
    if (nb > kNoAllocPartials)
        fail(SEM_EINVAL, "sem_dot_noalloc: " + std::to_string(nb) +
                             " block partials exceed the static scratch of " +
                             std::to_string(kNoAllocPartials));
    double *part = noalloc_scratch();
    hipLaunchKernelGGL((dot_kernel<T>), dim3(nb), dim3(kVecThreads), 0, s, m.n, a, b, m.mcode,
                       part);
    hipLaunchKernelGGL(finalize_sum_kernel, dim3(1), dim3(kFinalizeThreads), 0, s, out,
                       (const double *)part, nb);
    check_hip(hipGetLastError(), "dot kernel launch");
}
template void launch_dot_noalloc<float>(const Mesh &, const float *, const float *, double *,
                                        hipStream_t);
template void launch_dot_noalloc<double>(const Mesh &, const double *, const double *, double *,
                                         hipStream_t);

template void launch_dot<float>(const Mesh &, const float *, const float *, double *, double *,
                                hipStream_t);
template void launch_dot<double>(const Mesh &, const double *, const double *, double *,
                                 double *, hipStream_t);

void launch_finalize_alpha(CgState *st, const double *part_ax, int64_t n_ax, hipStream_t s) {
    hipLaunchKernelGGL(finalize_alpha_kernel, dim3(1), dim3(kFinalizeThreads), 0, s, st, part_ax,
                       n_ax);
    check_hip(hipGetLastError(), "finalize kernel launch");
}
template void launch_convert<float, double>(int64_t, const float *, double *, hipStream_t);
template void launch_convert<double, float>(int64_t, const double *, float *, hipStream_t);
template void launch_convert<double, double>(int64_t, const double *, double *, hipStream_t);

}  // namespace sem
