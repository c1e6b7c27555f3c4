// sem_vec_body.h -- device code of the Algorithm 1 vector update and the
// one-block finalize steps, shared by the single-mesh and batched kernels.
#pragma once

#include "sem_internal.h"
#include "sem_reduce.h"

namespace sem {
namespace vecb {

constexpr int kVecThreads = 256;
constexpr int kVecMaxBlocks = 2048;

template <typename T>
struct alignas(4 * sizeof(T)) Pack4 {
    T v[4];
};
struct alignas(4) Code4 {
    uint8_t v[4];
};

__device__ __forceinline__ void weights_lds(double *cw) {
    // weight 1/m for every code (m in the low bits; exact for powers of two)
    const int m = threadIdx.x & kMultMask;
    cw[threadIdx.x] = m ? 1.0 / (double)m : 0.0;
    __syncthreads();
}

// x += alpha p; r -= alpha w; rho_i = <r, r, c>  (Algorithm 1, fused updates
// and reduction), then beta_i = rho_i / rho_{i-1} and the convergence test.
// Virtual block vb of a grid of vgrid blocks; the partial goes to
// partial[vb].
template <typename T>
__device__ __forceinline__ void update_body(int64_t n, T *__restrict__ x, T *__restrict__ r,
                                            const T *__restrict__ p, const T *__restrict__ w,
                                            const uint8_t *__restrict__ mcode, CgState *st,
                                            double *partial, int64_t vb, int64_t vgrid) {
    if (st->stop) return;
    __shared__ double cw[kVecThreads];
    __shared__ double red[16];
    weights_lds(cw);
    const T a = (T)st->alpha;
    double acc = 0.0;
    const int64_t n4 = n >> 2;
    const int64_t stride = vgrid * blockDim.x;
    const int64_t tid = vb * blockDim.x + threadIdx.x;
    for (int64_t q = tid; q < n4; q += stride) {
        Pack4<T> xv = reinterpret_cast<const Pack4<T> *>(x)[q];
        Pack4<T> rv = reinterpret_cast<const Pack4<T> *>(r)[q];
        const Pack4<T> pv = reinterpret_cast<const Pack4<T> *>(p)[q];
        const Pack4<T> wv = reinterpret_cast<const Pack4<T> *>(w)[q];
        const Code4 mv = reinterpret_cast<const Code4 *>(mcode)[q];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            xv.v[t] += a * pv.v[t];
            rv.v[t] -= a * wv.v[t];
            const double rd = (double)rv.v[t];
            acc += rd * rd * cw[mv.v[t]];
        }
        reinterpret_cast<Pack4<T> *>(x)[q] = xv;
        reinterpret_cast<Pack4<T> *>(r)[q] = rv;
    }
    for (int64_t q = 4 * n4 + tid; q < n; q += stride) {
        x[q] += a * p[q];
        const T rn = r[q] - a * w[q];
        r[q] = rn;
        acc += (double)rn * (double)rn * cw[mcode[q]];
    }
    const double s = block_sum_f64(acc, red);
    if (threadIdx.x == 0) partial[vb] = s;
}

// rho_i = sum of the update partials; beta_i = rho_i / rho_{i-1}; the
// iteration count, the history and the stopping test (Algorithm 1, last
// two steps).  One block.
__device__ __forceinline__ void finalize_rho_body(CgState *st, const double *partial, int cnt) {
    if (st->stop) return;
    __shared__ double red[16];
    const double rho = sum_partials(partial, cnt, red);
    if (threadIdx.x == 0) {
        const double beta = rho / st->rho;
        st->beta = beta;
        st->rho = rho;
        const int it = st->iter + 1;
        st->iter = it;
        if (st->hist_rho && it < st->hist_len) st->hist_rho[it] = rho;
        if (!isfinite(rho)) st->stop = 3;
        else if (!st->fixed && rho <= st->thresh) st->stop = 1;
        else if (it >= st->max_iter) st->stop = 2;
    }
}

// alpha_i = rho_{i-1} / <p, w, c>, the inner product being the sum of the
// operator kernel's partials (see the CgFused mode of the local operator).
// One block.
__device__ __forceinline__ void finalize_alpha_body(CgState *st, const double *part_ax,
                                                    int64_t n_ax) {
    if (st->stop) return;
    __shared__ double red[16];
    const double pw = sum_partials(part_ax, n_ax, red);
    if (threadIdx.x == 0) {
        const double alpha = st->rho / pw;
        st->pw = pw;
        st->alpha = alpha;
        if (!(pw > 0.0) || !isfinite(alpha)) st->stop = 3;
        const int i = st->iter + 1;
        if (st->hist_alpha && i < st->hist_len) st->hist_alpha[i] = alpha;
    }
}

}  // namespace vecb
}  // namespace sem
