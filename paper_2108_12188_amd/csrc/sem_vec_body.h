// sem_vec_body.h -- device code of the Algorithm 1 vector update and the
// one-block finalize steps, shared by the single-mesh and batched kernels.
#pragma once

#include "sem_internal.h"
#include "sem_reduce.h"

namespace sem {
namespace vecb {

constexpr int kVecThreads = 256;
#ifndef SEM_VEC_MAX_BLOCKS
#define SEM_VEC_MAX_BLOCKS 4096
#endif
constexpr int kVecMaxBlocks = SEM_VEC_MAX_BLOCKS;
// packs of 4 points a thread of the gather update keeps in flight per step
#ifndef SEM_UPD_PACKS
#define SEM_UPD_PACKS 2
#endif
constexpr int kUpdPacks = SEM_UPD_PACKS;
// the same for the table-free gather, whose records already keep loads in
// flight (one pack per step measured faster there); the per-thread packs
// and their order are those of every K, so both forms agree bitwise
#ifndef SEM_UPD_STRUCT_PACKS
#define SEM_UPD_STRUCT_PACKS 1
#endif
constexpr int kUpdStructPacks = SEM_UPD_STRUCT_PACKS;

// Blocks are dealt to the 8 XCDs round-robin (block b on XCD b mod 8): the
// vector updates give each XCD a contiguous range of the logical blocks
// instead (a bijection on [0, vgrid); the last vgrid mod 8 blocks keep
// their place), so that the face partners a block reads in neighbouring
// elements were mostly brought in through the same L2.  The ρ partial of a
// block stays at its own index vb.
__device__ __forceinline__ int64_t xcd_block(int64_t vb, int64_t vgrid) {
    const int64_t full = vgrid & ~int64_t(7);
    if (vb >= full) return vb;
    return (vb & 7) * (full >> 3) + (vb >> 3);
}

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

// [x += alpha p;] r -= alpha mask(w); rho_i = <r, r, c>  (Algorithm 1:
// mask, fused updates and reduction; the operator leaves w unmasked).
// WithX = false leaves x to the next operator launch (single-mesh solves).
// PC: also z = minv r, partial <- <r, z, c>, partial2 <- <r, r, c>.
// Virtual block vb of a grid of vgrid blocks; the partial goes to
// partial[vb].
template <typename T, bool WithX, bool PC = false>
__device__ __forceinline__ void update_body(int64_t n, T *__restrict__ x, T *__restrict__ r,
                                            const T *__restrict__ p, const T *__restrict__ w,
                                            const uint8_t *__restrict__ mcode, CgState *st,
                                            double *partial, int64_t vb, int64_t vgrid,
                                            PcArgs<T> pc = PcArgs<T>{}) {
    // the state's loads go out with the block's set-up; a stopped state
    // returns before the first store to global memory (uniform)
    const int stopped = st->stop;
    const T a = (T)st->alpha;
    __shared__ double cw[kVecThreads];
    __shared__ double red[16];
    weights_lds(cw);
    if (stopped) return;
    double acc = 0.0, acc2 = 0.0;
    const int64_t n4 = n >> 2;
    const int64_t stride = vgrid * blockDim.x;
    const int64_t tid = xcd_block(vb, vgrid) * blockDim.x + threadIdx.x;
    for (int64_t q = tid; q < n4; q += stride) {
        Pack4<T> rv = reinterpret_cast<const Pack4<T> *>(r)[q];
        const Pack4<T> wv = reinterpret_cast<const Pack4<T> *>(w)[q];
        const Code4 mv = reinterpret_cast<const Code4 *>(mcode)[q];
        if constexpr (WithX) {
            Pack4<T> xv = reinterpret_cast<const Pack4<T> *>(x)[q];
            const Pack4<T> pv = reinterpret_cast<const Pack4<T> *>(p)[q];
#pragma unroll
            for (int t = 0; t < 4; ++t) xv.v[t] += a * pv.v[t];
            reinterpret_cast<Pack4<T> *>(x)[q] = xv;
        }
        Pack4<T> mi{}, zv{};
        if constexpr (PC) mi = reinterpret_cast<const Pack4<T> *>(pc.minv)[q];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const T wm = (mv.v[t] & kDirichletBit) ? T(0) : wv.v[t];
            rv.v[t] -= a * wm;
            const double rd = (double)rv.v[t];
            if constexpr (PC) {
                zv.v[t] = mi.v[t] * rv.v[t];
                acc += rd * (double)zv.v[t] * cw[mv.v[t]];
                acc2 += rd * rd * cw[mv.v[t]];
            } else {
                acc += rd * rd * cw[mv.v[t]];
            }
        }
        reinterpret_cast<Pack4<T> *>(r)[q] = rv;
        if constexpr (PC) reinterpret_cast<Pack4<T> *>(pc.z)[q] = zv;
    }
    for (int64_t q = 4 * n4 + tid; q < n; q += stride) {
        const uint8_t c = mcode[q];
        if constexpr (WithX) x[q] += a * p[q];
        const T rn = r[q] - a * ((c & kDirichletBit) ? T(0) : w[q]);
        r[q] = rn;
        if constexpr (PC) {
            const T zn = pc.minv[q] * rn;
            pc.z[q] = zn;
            acc += (double)rn * (double)zn * cw[c];
            acc2 += (double)rn * (double)rn * cw[c];
        } else {
            acc += (double)rn * (double)rn * cw[c];
        }
    }
    const double s = block_sum_f64(acc, red);
    if (threadIdx.x == 0) partial[vb] = s;
    if constexpr (PC) {
        const double s2 = block_sum_f64(acc2, red);
        if (threadIdx.x == 0) pc.partial2[vb] = s2;
    }
}

// Where the sums over the copies are formed inside the update: per local
// point the partner of a pair point, the group rank of a point in a larger
// group, else the point's own index (see Mesh::gsrc).
struct GatherMap {
    const int32_t *gsrc;         // [n]
};

// Code of a pair point off the Dirichlet boundary: m = 2, flag clear.
constexpr uint8_t kPairCode = 2;

__host__ __device__ __forceinline__ bool is_group_code(uint8_t code) {
    return (code & kMultMask) > 2 && !(code & kDirichletBit);
}

// The one value point l loads besides its own: its partner's w (pairs), its
// group's sum (larger groups), else its own w again.
template <typename T>
__host__ __device__ __forceinline__ const T *gather_source(const T *w, const T *gsum,
                                                           uint8_t code, int32_t lk, int64_t l) {
    const bool group = is_group_code(code);
    const T *base = group ? gsum : w;
    const int64_t off = (code == kPairCode || group) ? (int64_t)(uint32_t)lk : l;
    return base + off;
}

// mask(QQ^T w)_l: a pair adds its partner's value (a + b == b + a in IEEE
// arithmetic, so both copies get the sum the gather-scatter forms); a point
// of a larger group takes the group's sum (formed in the gather-scatter's
// order); points with m = 1 keep their own value, Dirichlet points get 0.
// src: the value at gather_source.
template <typename T>
__host__ __device__ __forceinline__ T copies_sum(T own, uint8_t code, T src) {
    // selects, not branches: src is consumed on every path
    const T pair_sum = own + src;
    T v = code == kPairCode ? pair_sum : own;
    v = is_group_code(code) ? src : v;
    return (code & kDirichletBit) ? T(0) : v;
}

// update_body<T, false> with w replaced by QQ^T w (w itself is not
// modified).  Same grid, same per-thread order and the same sums as
// gather-scatter + update_body, so the results are bitwise those of the
// two-pass form.  All loads are unconditional: two packs (q, q + stride)
// per step, each costing two dependent rounds of loads (r, w, the codes and
// the 4 gather-table entries of a pack, then the 4 gathered values), all
// loads of both packs issued before any result is used; the sum of r^2/m
// still runs pack by pack in the thread's order q, q + stride, ...
template <typename T, bool PC = false>
__device__ __forceinline__ void update_gather_body(int64_t n, T *__restrict__ r,
                                                   const T *__restrict__ w,
                                                   const T *__restrict__ gsum,
                                                   const uint8_t *__restrict__ mcode,
                                                   const GatherMap &gm, CgState *st,
                                                   double *partial, int64_t vb, int64_t vgrid,
                                                   PcArgs<T> pc = PcArgs<T>{}) {
    // the state's loads go out with the block's set-up; a stopped state
    // returns before the first store to global memory (uniform)
    const int stopped = st->stop;
    const T a = (T)st->alpha;
    __shared__ double cw[kVecThreads];
    __shared__ double red[16];
    weights_lds(cw);
    if (stopped) return;
    double acc = 0.0, acc2 = 0.0;
    const int64_t n4 = n >> 2;
    const int64_t stride = vgrid * blockDim.x;
    const int64_t tid = xcd_block(vb, vgrid) * blockDim.x + threadIdx.x;
    constexpr int K = kUpdPacks;
    for (int64_t q = tid; q < n4; q += K * stride) {
        int64_t qq[K];
        bool live[K];
#pragma unroll
        for (int h = 0; h < K; ++h) {
            live[h] = q + h * stride < n4;
            qq[h] = live[h] ? q + h * stride : q;
        }
        int32_t lk[K][4];
        Pack4<T> rv[K], wv[K];
        Code4 mv[K];
#pragma unroll
        for (int h = 0; h < K; ++h) {
            const int4 g4 = reinterpret_cast<const int4 *>(gm.gsrc)[qq[h]];
            lk[h][0] = g4.x, lk[h][1] = g4.y, lk[h][2] = g4.z, lk[h][3] = g4.w;
            rv[h] = reinterpret_cast<const Pack4<T> *>(r)[qq[h]];
            wv[h] = reinterpret_cast<const Pack4<T> *>(w)[qq[h]];
            mv[h] = reinterpret_cast<const Code4 *>(mcode)[qq[h]];
        }
        T src[K][4];
#pragma unroll
        for (int h = 0; h < K; ++h)
#pragma unroll
            for (int t = 0; t < 4; ++t)
                src[h][t] = *gather_source<T>(w, gsum, mv[h].v[t], lk[h][t],
                                              (int64_t)(4 * qq[h] + t));
        // a pack past the end (!live) repeats the first: it stores the same
        // values and adds exactly 0 to the sums (every result is consumed on
        // every path, so no load of this step is still pending when the next
        // step reuses its registers)
#pragma unroll
        for (int h = 0; h < K; ++h) {
            Pack4<T> mi{}, zv{};
            if constexpr (PC) mi = reinterpret_cast<const Pack4<T> *>(pc.minv)[qq[h]];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const T wg = copies_sum<T>(wv[h].v[t], mv[h].v[t], src[h][t]);
                rv[h].v[t] -= a * wg;
                const double rd = (double)rv[h].v[t];
                if constexpr (PC) {
                    zv.v[t] = mi.v[t] * rv[h].v[t];
                    acc += live[h] ? rd * (double)zv.v[t] * cw[mv[h].v[t]] : 0.0;
                    acc2 += live[h] ? rd * rd * cw[mv[h].v[t]] : 0.0;
                } else {
                    acc += live[h] ? rd * rd * cw[mv[h].v[t]] : 0.0;
                }
            }
            reinterpret_cast<Pack4<T> *>(r)[qq[h]] = rv[h];
            if constexpr (PC) reinterpret_cast<Pack4<T> *>(pc.z)[qq[h]] = zv;
        }
    }
    for (int64_t q = 4 * n4 + tid; q < n; q += stride) {
        const uint8_t c = mcode[q];
        const int32_t lk = gm.gsrc[q];
        const T wg = copies_sum<T>(w[q], c, *gather_source<T>(w, gsum, c, lk, q));
        const T rn = r[q] - a * wg;
        r[q] = rn;
        if constexpr (PC) {
            const T zn = pc.minv[q] * rn;
            pc.z[q] = zn;
            acc += (double)rn * (double)zn * cw[c];
            acc2 += (double)rn * (double)rn * cw[c];
        } else {
            acc += (double)rn * (double)rn * cw[c];
        }
    }
    const double s = block_sum_f64(acc, red);
    if (threadIdx.x == 0) partial[vb] = s;
    if constexpr (PC) {
        const double s2 = block_sum_f64(acc2, red);
        if (threadIdx.x == 0) pc.partial2[vb] = s2;
    }
}

// Table-free form of the same gather (Mesh::gs_struct): a point's copies
// follow from its position in the element and the element's records.
struct StructMap {
    const ElemRec *rec;         // [E][nrec]
    const uint32_t *pos_tab;    // [p3] (pos_entry)
    int p3, nrec;               // P^3, 6 + edge_slots(N)
    uint32_t magic;             // element of local index l: (l * magic) >> shift
    int shift;
};
constexpr int kMaxPosTab = kMaxP * kMaxP * kMaxP;

__host__ __device__ __forceinline__ int64_t struct_elem(const StructMap &sm, int64_t l) {
    return (int64_t)(((uint64_t)l * sm.magic) >> sm.shift);
}

// The record point l (element e, position entry pe) needs: its face's or
// its edge slot's (face 0's for an interior point, which uses none).
// Loaded first: the address of the value the point gathers depends on it.
__host__ __device__ __forceinline__ ElemRec struct_record(const StructMap &sm, int64_t e,
                                                          uint32_t pe) {
    return sm.rec[e * sm.nrec + (pe >> 12)];
}

// Where point l finds the value it loads besides its own w, as an index
// into wg = [w | the edge-group sums] (the sums sit right after the n local
// values): a face point the copy on the neighbour's face (its own index
// when it has none), a shared edge or corner node n + its group's rank, any
// other point its own index; and its code byte.  Every path gives an index
// inside wg.
struct StructSrc {
    int32_t idx;      // n + the number of edge groups stays below 2^31 (host check)
    uint8_t code;
    bool edge;
};
__host__ __device__ __forceinline__ StructSrc struct_source(const StructMap &sm, int64_t n,
                                                            int64_t l, uint32_t pe,
                                                            const ElemRec &rc) {
    const int kind = (int)(pe & 3);
    const int a = (int)((pe >> 2) & 31), b = (int)((pe >> 7) & 31);
    const uint8_t code = (uint8_t)(rc.hi & 255);
    const int32_t sa = (int32_t)((uint32_t)rc.hi << 12) >> 20;   // bits 8-19, signed
    const int32_t sb = rc.hi >> 20;                               // bits 20-31, signed
    const int32_t q = rc.lo + sa * a + sb * b;
    const bool eshared = (code & kMultMask) >= 2 && !(code & kDirichletBit);
    StructSrc s;
    const int32_t own_or_face = kind == 1 ? q : (int32_t)l;
    s.idx = (kind == 2 && eshared) ? (int32_t)n + rc.lo : own_or_face;
    s.code = kind == 0 ? (uint8_t)1 : code;
    s.edge = kind == 2;
    return s;
}
// mask(QQ^T w)_l from the loaded value: a face pair adds its partner (the
// sum a + b == b + a of the gather-scatter), a shared edge or corner node
// takes its group's sum (the gather-scatter's ascending order), points with
// m = 1 keep their own value, Dirichlet points get 0.
template <typename T>
__host__ __device__ __forceinline__ T struct_sum(T own, uint8_t code, bool edge, T src) {
    const bool shared = (code & kMultMask) >= 2;
    const T pair_sum = own + src;
    T v = edge ? (shared ? src : own) : (code == kPairCode ? pair_sum : own);
    return (code & kDirichletBit) ? T(0) : v;
}

// update_gather_body with the table-free gather: the same per-thread packs,
// the same values and the same sums, so bitwise the same results.  n is a
// multiple of 4 (P^3 is), and the 4 points of a pack lie in one element.
// wg: w followed by the edge-group sums.  Load order: the element records
// first (pinned there by a compiler fence, so none is moved into a branch),
// then r and w, then the gathered values, whose addresses need only
// the records (loads complete in issue order, so the gathers wait for the
// records, not for r and w).
template <typename T, bool PC = false>
__device__ __forceinline__ void update_struct_body(int64_t n, T *__restrict__ r,
                                                   const T *__restrict__ wg,
                                                   const StructMap &sm, CgState *st,
                                                   double *partial, int64_t vb, int64_t vgrid,
                                                   PcArgs<T> pc = PcArgs<T>{}) {
    // the state's loads go out with the block's set-up; a stopped state
    // returns before the first store to global memory (uniform)
    const int stopped = st->stop;
    const T a = (T)st->alpha;
    __shared__ double cw[kVecThreads];
    __shared__ double red[16];
    __shared__ __align__(16) uint32_t pos[kMaxPosTab];
    for (int q = threadIdx.x; q < sm.p3; q += blockDim.x) pos[q] = sm.pos_tab[q];
    weights_lds(cw);
    if (stopped) return;
    double acc = 0.0, acc2 = 0.0;
    const int64_t n4 = n >> 2;
    const int64_t stride = vgrid * blockDim.x;
    const int64_t tid = xcd_block(vb, vgrid) * blockDim.x + threadIdx.x;
    constexpr int K = kUpdStructPacks;
    for (int64_t q = tid; q < n4; q += K * stride) {
        int64_t qq[K];
        bool live[K];
#pragma unroll
        for (int h = 0; h < K; ++h) {
            live[h] = q + h * stride < n4;
            qq[h] = live[h] ? q + h * stride : q;
        }
        uint32_t pv[K][4];
        ElemRec rc[K][4];
#pragma unroll
        for (int h = 0; h < K; ++h) {
            const int64_t l0 = 4 * qq[h];
            const int64_t e = struct_elem(sm, l0);
            // 16-byte entries (P^3 and l0 are multiples of 4): one ds_read_b128
            const uint4 pe = reinterpret_cast<const uint4 *>(pos)[(l0 - e * sm.p3) >> 2];
            pv[h][0] = pe.x, pv[h][1] = pe.y, pv[h][2] = pe.z, pv[h][3] = pe.w;
#pragma unroll
            for (int t = 0; t < 4; ++t) rc[h][t] = struct_record(sm, e, pv[h][t]);
        }
        __asm__ volatile("" ::: "memory");
        Pack4<T> rv[K], wv[K];
#pragma unroll
        for (int h = 0; h < K; ++h) {
            rv[h] = reinterpret_cast<const Pack4<T> *>(r)[qq[h]];
            wv[h] = reinterpret_cast<const Pack4<T> *>(wg)[qq[h]];
        }
        int32_t ix[K][4];
        uint8_t cd[K][4];
        bool ed[K][4];
#pragma unroll
        for (int h = 0; h < K; ++h)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const StructSrc ss = struct_source(sm, n, 4 * qq[h] + t, pv[h][t], rc[h][t]);
                ix[h][t] = ss.idx;
                cd[h][t] = ss.code;
                ed[h][t] = ss.edge;
            }
        T src[K][4];
#pragma unroll
        for (int h = 0; h < K; ++h)
#pragma unroll
            for (int t = 0; t < 4; ++t) src[h][t] = wg[ix[h][t]];
        // a pack past the end (!live) repeats the first: it stores the same
        // values and adds exactly 0 to the sums
#pragma unroll
        for (int h = 0; h < K; ++h) {
            Pack4<T> mi{}, zv{};
            if constexpr (PC) mi = reinterpret_cast<const Pack4<T> *>(pc.minv)[qq[h]];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const T wg = struct_sum<T>(wv[h].v[t], cd[h][t], ed[h][t], src[h][t]);
                rv[h].v[t] -= a * wg;
                const double rd = (double)rv[h].v[t];
                if constexpr (PC) {
                    zv.v[t] = mi.v[t] * rv[h].v[t];
                    acc += live[h] ? rd * (double)zv.v[t] * cw[cd[h][t]] : 0.0;
                    acc2 += live[h] ? rd * rd * cw[cd[h][t]] : 0.0;
                } else {
                    acc += live[h] ? rd * rd * cw[cd[h][t]] : 0.0;
                }
            }
            reinterpret_cast<Pack4<T> *>(r)[qq[h]] = rv[h];
            if constexpr (PC) reinterpret_cast<Pack4<T> *>(pc.z)[qq[h]] = zv;
        }
    }
    const double s = block_sum_f64(acc, red);
    if (threadIdx.x == 0) partial[vb] = s;
    if constexpr (PC) {
        const double s2 = block_sum_f64(acc2, red);
        if (threadIdx.x == 0) pc.partial2[vb] = s2;
    }
}

// rho_i = sum of the update partials; beta_i = rho_i / rho_{i-1}; the
// iteration count, the history and the stopping test (Algorithm 1, last
// two steps).  One block.
// partial2 (may be null): the partials of <r, r, c> when rho is the
// preconditioned <r, z, c>; the stopping test and the history use <r, r, c>.
__device__ __forceinline__ void finalize_rho_body(CgState *st, const double *partial, int cnt,
                                                  const double *partial2 = nullptr) {
    // the state is read with the partials (one round of loads instead of
    // three); a stopped state sums them and stores nothing
    const int stopped = st->stop;
    const double rho_prev = st->rho;
    const int it = st->iter + 1;
    const int fixed = st->fixed, max_iter = st->max_iter, hist_len = st->hist_len;
    const double thresh = st->thresh;
    double *const hist_rho = st->hist_rho;
    __shared__ double red[16];
    const double rho = sum_partials(partial, cnt, red);
    const double rr = partial2 ? sum_partials(partial2, cnt, red) : rho;
    if (stopped) return;
    if (threadIdx.x == 0) {
        const double beta = rho / rho_prev;
        st->beta = beta;
        st->rho = rho;
        st->rr = rr;
        st->x_lag = 1;
        st->iter = it;
        if (hist_rho && it < hist_len) hist_rho[it] = rr;
        if (!isfinite(rho) || !isfinite(rr)) st->stop = 3;
        else if (!fixed && rr <= thresh) st->stop = 1;
        else if (it >= max_iter) st->stop = 2;
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
        st->x_lag = 0;     // the operator launch before this one applied it
        if (!(pw > 0.0) || !isfinite(alpha)) st->stop = 3;
        const int i = st->iter + 1;
        if (st->hist_alpha && i < st->hist_len) st->hist_alpha[i] = alpha;
    }
}

}  // namespace vecb
}  // namespace sem
