// sem_ax_order.hip -- the local operator A_L for one polynomial order.
//
// Compiled once per order with -DSEM_ORDER=N.  Implements Eq. 4-5 of the
// paper (w_e = D^T G^e D u_e, per element, no gather-scatter) in two forms:
//   * precomputed G: the six symmetric factors are streamed from HBM
//     (Sec. 4.2: 6 words per point, the HBM-bound form);
//   * on-the-fly G (rematerialization, Sec. 5.1, Eq. 13-14): G is rebuilt
//     at every point from the element's 8 vertices, so only u and w move.
// and two modes:
//   * Plain: w = A_L u;
//   * CgFused: the p-update of Algorithm 1 is the prologue (p <- r + beta p,
//     the loop fusion of Sec. 5.1), the block's FP64 partial of
//     sum_l p_l w_l is reduced, and (optionally) the values of the edge and
//     corner nodes are also written to a compact per-element array for the
//     group sums of the gather-scatter.  Because p is continuous (p = Q p_g), zero on
//     the Dirichlet points, and the weights of every group add up to one,
//     <p, mask(QQ^T w), c> = p_g^T Q^T w = sum_l p_l w_l over the local, not
//     yet gathered or masked w: the whole alpha reduction of Algorithm 1
//     happens here, before the gather-scatter, instead of after it as in
//     Sec. 5.1.  The mask itself is applied where w is next read (the
//     vector update), which already holds the point codes.
//
// Work decomposition (gfx950, 64-lane waves): a block holds `epb` elements;
// one thread owns one (i, j) column of one element and walks the k
// direction in registers.  The i- and j-direction contractions read the
// element tile from LDS; the k-direction contraction is register-only with
// D entries that are wave-uniform (kernel-argument / scalar registers).
#include "sem_internal.h"
#include "sem_reduce.h"

#ifndef SEM_ORDER
#error "compile with -DSEM_ORDER=<N>"
#endif

namespace sem {
namespace {

constexpr int kOrder = SEM_ORDER;
constexpr int kP = kOrder + 1;

// Precomputed form: issue the loads of all 6 P factors of a column before
// the first barrier (more loads in flight per wave) when the registers allow.
#ifndef SEM_AX_PREFETCH_G
#define SEM_AX_PREFETCH_G 0
#endif
template <typename T>
constexpr bool prefetch_g() {
    return SEM_AX_PREFETCH_G && 6 * kP * sizeof(T) <= 6 * 8 * 4;
}

// The precomputed factors are read once per application and are the largest
// stream (24 B of 32 per point in FP32): non-temporal loads keep them from
// displacing the vectors (u, w and, in CG, r, p, x: 268 MB in FP32) that the
// next kernels read again from the 256 MB Infinity Cache.  FP64 vectors
// (537 MB) do not fit it either way, and there the hint costs a little.
#ifndef SEM_AX_G_STREAM
#define SEM_AX_G_STREAM 1
#endif
template <typename T>
__device__ __forceinline__ T load_g(const T *p) {
    if constexpr (SEM_AX_G_STREAM && sizeof(T) == 4) return __builtin_nontemporal_load(p);
    else return *p;
}

// Kernel-argument copy of the basis: indexed only with compile-time
// constants, so every access is a scalar load.
template <typename T>
struct BasisK {
    T D[kP * kP];   // D[k*P + l] = l_l'(xi_k)
    T xi[kP];
    T w[kP];
};

template <typename T>
__device__ __forceinline__ T rcp(T x) { return T(1) / x; }
template <>
__device__ __forceinline__ float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }

// a * b + c with one rounding.
template <typename T>
__device__ __forceinline__ T fmadd(T a, T b, T c) {
    if constexpr (sizeof(T) == 4) return __builtin_fmaf(a, b, c);
    else return __builtin_fma(a, b, c);
}

template <typename T>
struct Vec3 {
    T x, y, z;
};
template <typename T>
__device__ __forceinline__ Vec3<T> cross(const Vec3<T> &a, const Vec3<T> &b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <typename T>
__device__ __forceinline__ T dot3(const Vec3<T> &a, const Vec3<T> &b) {
    return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <typename T>
__device__ __forceinline__ Vec3<T> axpy3(T s, const Vec3<T> &a, const Vec3<T> &b) {
    return {b.x + s * a.x, b.y + s * a.y, b.z + s * a.z};   // b + s a
}
template <typename T>
__device__ __forceinline__ Vec3<T> add3(const Vec3<T> &a, const Vec3<T> &b) {
    return {a.x + b.x, a.y + b.y, a.z + b.z};
}

// Per-thread constants of the trilinear map along one (i, j) column.
// Along the column only gamma varies, and
//   x_xi(gamma) = A0 + gamma A1,  x_eta(gamma) = B0 + gamma B1,  x_gamma = C,
// so the cofactor rows r0 = x_eta x x_gamma, r1 = x_gamma x x_xi,
// r2 = x_xi x x_eta and |J| = x_xi . r0 are low-degree polynomials in gamma.
template <typename T>
struct ColumnGeom {
    Vec3<T> R00, R01, R10, R11, R20, R21, R22;
    T d0, d1, d2, wij;
};

// The 12 edge vectors of an element from its 8 vertices, in the order the
// column geometry uses them: along xi (v1 - v0, v3 - v2, v5 - v4, v7 - v6),
// along eta (v2 - v0, v3 - v1, v6 - v4, v7 - v5), along gamma (v4 - v0,
// v5 - v1, v6 - v2, v7 - v3); ed[t * 3 + d].  The host builds the same
// FP32 array per element (Mesh::vedge32) with the same subtractions.
template <typename T>
__device__ __forceinline__ void element_edges(const T *__restrict__ ve, T (&ed)[36]) {
    constexpr int kA[12] = {1, 3, 5, 7, 2, 3, 6, 7, 4, 5, 6, 7};
    constexpr int kB[12] = {0, 2, 4, 6, 0, 1, 4, 5, 0, 1, 2, 3};
#pragma unroll
    for (int t = 0; t < 12; ++t)
#pragma unroll
        for (int d = 0; d < 3; ++d) ed[t * 3 + d] = ve[kA[t] * 3 + d] - ve[kB[t] * 3 + d];
}

template <typename T, typename EdgePtr>
__device__ __forceinline__ ColumnGeom<T> column_geom_edges(EdgePtr ed, T xi_i, T eta_j, T wij) {
    const T fi0 = T(0.5) * (T(1) - xi_i), fi1 = T(0.5) * (T(1) + xi_i);
    const T fj0 = T(0.5) * (T(1) - eta_j), fj1 = T(0.5) * (T(1) + eta_j);
    T A0[3], A1[3], B0[3], B1[3], Cc[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        // Every product-sum here is an explicit fused multiply-add: the
        // edges may sit in scalar registers (matrix-core operator) or come
        // out of subtractions (VALU operator), and both must round alike.
        // d/dxi at (eta_j, gamma corner c)
        const T a0 = T(0.5) * fmadd(ed[0 * 3 + d], fj0, ed[1 * 3 + d] * fj1);
        const T a1 = T(0.5) * fmadd(ed[2 * 3 + d], fj0, ed[3 * 3 + d] * fj1);
        // d/deta at (xi_i, gamma corner c)
        const T b0 = T(0.5) * fmadd(ed[4 * 3 + d], fi0, ed[5 * 3 + d] * fi1);
        const T b1 = T(0.5) * fmadd(ed[6 * 3 + d], fi0, ed[7 * 3 + d] * fi1);
        A0[d] = T(0.5) * (a0 + a1);
        A1[d] = T(0.5) * (a1 - a0);
        B0[d] = T(0.5) * (b0 + b1);
        B1[d] = T(0.5) * (b1 - b0);
        const T c4 = fmadd(ed[9 * 3 + d] * fi1, fj0, ed[8 * 3 + d] * fi0 * fj0);
        const T c6 = fmadd(ed[10 * 3 + d] * fi0, fj1, c4);
        Cc[d] = T(0.5) * fmadd(ed[11 * 3 + d] * fi1, fj1, c6);
    }
    const Vec3<T> a0{A0[0], A0[1], A0[2]}, a1{A1[0], A1[1], A1[2]};
    const Vec3<T> b0{B0[0], B0[1], B0[2]}, b1{B1[0], B1[1], B1[2]};
    const Vec3<T> c{Cc[0], Cc[1], Cc[2]};
    ColumnGeom<T> g;
    g.R00 = cross(b0, c);
    g.R01 = cross(b1, c);
    g.R10 = cross(c, a0);
    g.R11 = cross(c, a1);
    g.R20 = cross(a0, b0);
    g.R21 = add3(cross(a0, b1), cross(a1, b0));
    g.R22 = cross(a1, b1);
    g.d0 = dot3(a0, g.R00);
    g.d1 = dot3(a0, g.R01) + dot3(a1, g.R00);
    g.d2 = dot3(a1, g.R01);
    g.wij = wij;
    return g;
}

template <typename T>
__device__ __forceinline__ ColumnGeom<T> column_geom(const T *__restrict__ ve, T xi_i, T eta_j,
                                                     T wij) {
    T ed[36];
    element_edges<T>(ve, ed);
    return column_geom_edges<T>(ed, xi_i, eta_j, wij);
}

// The pointwise step of A_L at level k of a column: (vr, vs, vt) = G (ur, us, ut)
// with G rebuilt from the column geometry (on the fly) or read from HBM
// (precomputed: gq when prefetched, else Ge = this column's factors).
template <typename T, bool OTF, bool kPre>
__device__ __forceinline__ void point_flux(const ColumnGeom<T> &cg, const BasisK<T> &bk, int k,
                                           const T (&gq)[kPre ? 6 : 1][kPre ? kP : 1],
                                           const T *__restrict__ Ge, T ur, T us, T ut, T &vr,
                                           T &vs, T &vt) {
    constexpr int P2 = kP * kP, P3 = P2 * kP;
    if constexpr (OTF) {
        const T gam = bk.xi[k];
        const Vec3<T> r0 = axpy3(gam, cg.R01, cg.R00);
        const Vec3<T> r1 = axpy3(gam, cg.R11, cg.R10);
        const Vec3<T> r2 = axpy3(gam, axpy3(gam, cg.R22, cg.R21), cg.R20);
        const T det = cg.d0 + gam * (cg.d1 + gam * cg.d2);
        const T s = cg.wij * bk.w[k] * rcp<T>(det);
        const Vec3<T> g{r0.x * ur + r1.x * us + r2.x * ut, r0.y * ur + r1.y * us + r2.y * ut,
                        r0.z * ur + r1.z * us + r2.z * ut};
        vr = s * dot3(r0, g);
        vs = s * dot3(r1, g);
        vt = s * dot3(r2, g);
    } else {
        T g11, g12, g13, g22, g23, g33;
        if constexpr (kPre) {
            g11 = gq[0][k], g12 = gq[1][k], g13 = gq[2][k];
            g22 = gq[3][k], g23 = gq[4][k], g33 = gq[5][k];
        } else {
            const T *G = Ge + k * P2;
            g11 = load_g(G), g12 = load_g(G + P3), g13 = load_g(G + 2 * P3);
            g22 = load_g(G + 3 * P3), g23 = load_g(G + 4 * P3), g33 = load_g(G + 5 * P3);
        }
        // fused multiply-adds in a fixed order, so that every kernel (and
        // both engines) rounds this product the same way
        vr = fmadd(g13, ut, fmadd(g12, us, g11 * ur));
        vs = fmadd(g23, ut, fmadd(g22, us, g12 * ur));
        vt = fmadd(g33, ut, fmadd(g23, us, g13 * ur));
    }
}

__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[16];
    return block_sum_f64(v, red);
}

// FP32 kernels up to N = 7 are held to 128 VGPRs (4 waves per SIMD): the
// on-the-fly form is latency-bound below that occupancy.  Higher orders and
// FP64 keep their registers (capping them spills).
template <typename T>
constexpr int ax_min_waves() { return (sizeof(T) == 4 && kP <= 8) ? 4 : 1; }

// FP32 CG-fused tiles stage the next tile's r, p and vertices in LDS with
// gfx950's direct global-to-LDS loads (16 bytes per lane, no registers held
// while in flight), issued while the current tile computes; x (when the
// previous step is applied here) lands in the operator tile itself, issued
// once the tile is free.  Needs 16-byte aligned element blocks: P^3 a
// multiple of 4 (odd N).
template <typename T, bool FUSED>
__host__ __device__ constexpr bool ax_dma() {
    return FUSED && sizeof(T) == 4 && (kP * kP * kP) % 4 == 0;
}

// Dynamic LDS of a block: the two operator tiles, plus the staging buffers.
template <typename T, bool OTF, bool FUSED>
__host__ __device__ constexpr size_t ax_lds_bytes(int epb) {
    constexpr size_t P3 = (size_t)kP * kP * kP;
    return 2 * sizeof(T) * epb * P3 +
           (ax_dma<T, FUSED>() ? 2 * sizeof(float) * epb * P3 + (OTF ? 24 * 4 * (size_t)epb : 0)
                               : 0);
}

// s_waitcnt immediates (gfx9 encoding): vmcnt(0) alone, lgkmcnt(0) alone
constexpr int kWaitVmcnt0 = 0x0F70;
constexpr int kWaitVmcnt8 = 0x0F78;
constexpr int kWaitLgkmcnt0 = 0xC07F;

// Barrier for LDS traffic only: the wave's own LDS accesses complete
// before it, but global loads and stores -- and the staging loads, which
// write LDS -- keep flying across it (a fenced __syncthreads would wait for
// all of them).  The memory clobber keeps the compiler from moving any
// memory access across the barrier.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_s_waitcnt(kWaitLgkmcnt0);
    __asm__ volatile("s_barrier" ::: "memory");
}

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;

// In a CG iteration the search direction p and the solution x are read
// and written by the CG-fused operator alone, once per iteration, one
// iteration apart.  When the iteration's vectors, records and edge copy
// exceed the 256 MB Infinity Cache (AxArgs::stream, set by the host; in
// FP64 only with G on the fly), those accesses are non-temporal
// (cache-policy bit NT on the loads, non-temporal stores), so that p and x
// take no cache space from r, w, the edge copy and the gather records, which
// the group sums and the update read again within the iteration.  A smaller
// iteration fits the cache as it is and keeps plain accesses.
constexpr int kCpolNt = 2;       // NT bit of the load cache-policy operand

// First tile of block vb in a grid-stride walk over vgrid blocks: blocks
// are dealt to the 8 XCDs round-robin (block b on XCD b mod 8), and each
// XCD takes a contiguous range of the first tiles instead (a bijection on
// [0, vgrid); the last vgrid mod 8 blocks keep their place).
__device__ __forceinline__ int64_t xcd_first_tile(int64_t vb, int64_t vgrid) {
    const int64_t full = vgrid & ~int64_t(7);
    return vb < full ? (vb & 7) * (full >> 3) + (vb >> 3) : vb;
}

// read-only data that every lane of a wave reads at one address, loaded
// into scalar registers (constant address space)
typedef __attribute__((address_space(4))) const float kconst_float;
// The choice is a template argument: a runtime flag lets the compiler merge
// the two stores into one plain store before the flag is known.
template <bool NT, typename T>
__device__ __forceinline__ void store_nt(T *p, T v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}
template <bool NT, typename T>
__device__ __forceinline__ T load_nt(const T *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// The block's nwave waves copy nf floats (a multiple of 4; src and dst
// 16-byte aligned) from global memory to LDS: every wave moves 64 x 16
// bytes per instruction, lane q of a wave landing at the wave's (uniform)
// LDS base + 16 q.  Completion is tracked by vmcnt.  (The wave count is an
// argument: the block size lives in memory, and loading it would make the
// wave wait for all of its outstanding stores.)
template <int kCpol = 0>
__device__ __forceinline__ void dma_to_lds(const float *src, float *dst, int nf, int nwave) {
    const int pieces = nf >> 2;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & 63);
    for (int q0 = wave * 64; q0 < pieces; q0 += nwave * 64) {
        if (q0 + lane < pieces)
            __builtin_amdgcn_global_load_lds((glb_void_t *)(src + 4 * (q0 + lane)),
                                             (lds_void_t *)(dst + 4 * q0), 16, 0, kCpol);
    }
}
template <bool NT>
__device__ __forceinline__ void dma_to_lds_nt(const float *src, float *dst, int nf, int nwave) {
    dma_to_lds<NT ? kCpolNt : 0>(src, dst, nf, nwave);
}

// Tiles vb, vb + vgrid, vb + 2 vgrid, ... of one problem; in the fused mode
// the block's partial goes to a.partial[vb].  Every thread of the block
// calls it.
template <typename T, bool OTF, bool FUSED, bool NT = false>
__device__ __forceinline__ void ax_body(const AxArgs<T> &a, const BasisK<T> &bk, int64_t ntiles,
                                        int64_t vb, int64_t vgrid) {
    constexpr int P = kP, P2 = P * P, P3 = P2 * P;
    constexpr bool kDma = ax_dma<T, FUSED>();
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T *const sA = reinterpret_cast<T *>(lds_raw);
    T *const sB = sA + a.epb * P3;
    // staging (kDma): r and p of a tile, then its vertices; x goes to sA
    float *const sR = reinterpret_cast<float *>(sB + a.epb * P3);
    float *const sP = sR + a.epb * P3;
    float *const sV = sP + a.epb * P3;
    float *const sX = reinterpret_cast<float *>(sA);

    // the CG state in one round of loads: stop, beta, the lagged x step
    T beta = T(0);
    // single-mesh CG: x += alpha_{i-1} p_{i-1} of the previous iteration,
    // applied here where p_{i-1} is read anyway
    bool xlag = false;
    T aprev = T(0);
    if constexpr (FUSED) {
        const int stopped = a.st->stop;
        beta = (T)a.st->beta;
        xlag = a.x != nullptr && a.st->x_lag != 0;
        aprev = (T)a.st->alpha;
        if (stopped) return;             // uniform: the whole grid exits
    }

    const int t = threadIdx.x;
    const int el = t / P2;
    const int col = t - el * P2;
    const int nwave = (a.epb * P2 + 63) >> 6;   // the launch's block size in waves
    const int i = col % P;
    const int j = col / P;
    T *const sa = sA + el * P3;
    T *const sb = sB + el * P3;

    // per-lane rows of D and D^T for the i and j contractions
    T Di[P], Dj[P], DiT[P], DjT[P];
#pragma unroll
    for (int l = 0; l < P; ++l) {
        Di[l] = a.D[i * P + l];
        Dj[l] = a.D[j * P + l];
        DiT[l] = a.Dt[i * P + l];
        DjT[l] = a.Dt[j * P + l];
    }
    constexpr bool strm = FUSED && NT;   // p and x non-temporal
    // edge-array slots of the column (edge_slot): base ecb (-1 off the
    // border) holds k = 0, ecb + 1 holds k = N, and corner columns keep
    // k = 1 .. N-1 at ecb + 1 + k
    const int ecb = edge_column_base(kOrder, i, j);
    const bool ecorner = (i == 0 || i == P - 1) && (j == 0 || j == P - 1);

    // per-lane GLL abscissae and weight product of the column
    T xi_i = T(0), eta_j = T(0), wij = T(0);
    if constexpr (OTF) {
        xi_i = a.xi[i];
        eta_j = a.xi[j];
        wij = a.wq[i] * a.wq[j];
    }

    // stage tile tl (its valid elements only): r, p, vertices; x separately
    auto stage = [&](int64_t tl) {
        if constexpr (kDma) {
            const int64_t e0 = tl * a.epb;
            const int nval = (int)(a.E - e0 < a.epb ? a.E - e0 : a.epb);
            dma_to_lds(reinterpret_cast<const float *>(a.u) + e0 * P3, sR, nval * P3, nwave);
            dma_to_lds_nt<strm>(reinterpret_cast<const float *>(a.p) + e0 * P3, sP, nval * P3,
                               nwave);
            if constexpr (OTF)
                dma_to_lds(reinterpret_cast<const float *>(a.vert) + e0 * 24, sV, nval * 24,
                           nwave);
        }
    };
    auto stage_x = [&](int64_t tl) {
        if constexpr (kDma) {
            const int64_t e0 = tl * a.epb;
            const int nval = (int)(a.E - e0 < a.epb ? a.E - e0 : a.epb);
            if (xlag)
                dma_to_lds_nt<strm>(reinterpret_cast<const float *>(a.x) + e0 * P3, sX, nval * P3,
                                   nwave);
        }
    };
    if constexpr (kDma) {
        if (vb < ntiles) {
            stage(vb);
            stage_x(vb);
        }
    }

    double acc = 0.0;
    // a tile is `epb` consecutive elements; the grid strides over tiles (in
    // launch order: the XCD-contiguous walk of the N = 7 matrix-core kernel
    // measured slower here at every order)
    for (int64_t tile = vb; tile < ntiles; tile += vgrid) {
        const int64_t e = tile * a.epb + el;
        const bool valid = (el < a.epb) && (e < a.E);
        const int64_t base = e * P3 + col;   // global index of (i, j, k=0)
        T *const wep = (FUSED && a.wedge && valid && ecb >= 0)
                           ? a.wedge + e * edge_slots(kOrder) + ecb
                           : nullptr;
        if constexpr (kDma) {
            // this tile's staged data has landed (every wave's share)
            __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
            lds_barrier();
        }

        T uc[P];
        if (valid) {
            if constexpr (kDma) {
                const float *const rr = sR + el * P3 + col;
                const float *const pp = sP + el * P3 + col;
#pragma unroll
                for (int k = 0; k < P; ++k) uc[k] = rr[k * P2] + beta * pp[k * P2];
#pragma unroll
                for (int k = 0; k < P; ++k) store_nt<strm>(a.p + base + k * P2, uc[k]);
                if (xlag) {
                    // x was staged in this thread's own slots of the tile,
                    // which the p-update below overwrites
                    const float *const xx = sX + el * P3 + col;
#pragma unroll
                    for (int k = 0; k < P; ++k)
                        store_nt<strm>(a.x + base + k * P2, xx[k * P2] + aprev * pp[k * P2]);
                }
            } else if constexpr (FUSED) {
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    const T r = a.u[base + k * P2];
                    const T pold = load_nt<strm>(a.p + base + k * P2);
                    uc[k] = r + beta * pold;
                    if (xlag)
                        store_nt<strm>(a.x + base + k * P2,
                                load_nt<strm>(a.x + base + k * P2) +
                                    aprev * pold);
                }
#pragma unroll
                for (int k = 0; k < P; ++k) store_nt<strm>(a.p + base + k * P2, uc[k]);
            } else {
#pragma unroll
                for (int k = 0; k < P; ++k) uc[k] = a.u[base + k * P2];
            }
#pragma unroll
            for (int k = 0; k < P; ++k) sa[k * P2 + col] = uc[k];
        }

        ColumnGeom<T> cg;
        if constexpr (OTF) {
            if (valid) {
                if constexpr (kDma)
                    cg = column_geom<T>(reinterpret_cast<const T *>(sV) + el * 24, xi_i, eta_j,
                                        wij);
                else
                    cg = column_geom<T>(a.vert + e * 24, xi_i, eta_j, wij);
            }
        }
        constexpr bool kPre = !OTF && prefetch_g<T>();
        T gq[kPre ? 6 : 1][kPre ? P : 1];
        if constexpr (kPre) {
            if (valid) {
                const T *Ge = a.G + e * (6 * P3) + col;
#pragma unroll
                for (int c = 0; c < 6; ++c)
#pragma unroll
                    for (int k = 0; k < P; ++k) gq[c][k] = load_g(Ge + c * P3 + k * P2);
            }
        }
        lds_barrier();
        // every thread is done with the staged tile: stage the next one
        if constexpr (kDma) {
            if (tile + vgrid < ntiles) stage(tile + vgrid);
        }

        T vsr[P], vtr[P];
        if (valid) {
#pragma unroll
            for (int k = 0; k < P; ++k) {
                T ur = T(0), us = T(0), ut = T(0);
#pragma unroll
                for (int l = 0; l < P; ++l) {
                    ur += Di[l] * sa[k * P2 + j * P + l];
                    us += Dj[l] * sa[k * P2 + l * P + i];
                    ut += bk.D[k * P + l] * uc[l];
                }
                T vr, vs, vt;
                point_flux<T, OTF, kPre>(cg, bk, k, gq, OTF ? nullptr : a.G + e * (6 * P3) + col,
                                         ur, us, ut, vr, vs, vt);
                sb[k * P2 + col] = vr;
                vsr[k] = vs;
                vtr[k] = vt;
            }
        }
        lds_barrier();
        if (valid) {
#pragma unroll
            for (int k = 0; k < P; ++k) sa[k * P2 + col] = vsr[k];
        }
        lds_barrier();

        if (valid) {
#pragma unroll
            for (int k = 0; k < P; ++k) {
                // three chains, one per direction, summed (r + s) + t (the
                // order of the matrix-core form, which gives the same bits)
                T wr = T(0), ws = T(0), wt = T(0);
#pragma unroll
                for (int l = 0; l < P; ++l) {
                    wr += DiT[l] * sb[k * P2 + j * P + l];
                    ws += DjT[l] * sa[k * P2 + l * P + i];
                    wt += bk.D[l * P + k] * vtr[l];
                }
                const T wv = (wr + ws) + wt;
                if constexpr (FUSED) {
                    acc += (double)uc[k] * (double)wv;
                    // compact copy of the edge and corner nodes
                    if (wep && (k == 0 || k == P - 1 || ecorner))
                        wep[k == 0 ? 0 : (k == P - 1 ? 1 : 1 + k)] = wv;
                }
                a.w[base + k * P2] = wv;
            }
        }
        lds_barrier();   // the next tile overwrites the LDS tile
        if constexpr (kDma) {
            if (tile + vgrid < ntiles) stage_x(tile + vgrid);
        }
    }
    if constexpr (FUSED) {
        const double s = block_sum(acc);
        if (threadIdx.x == 0) a.partial[vb] = s;
    }
}

// ---------------------------------------------------------------------------
// Matrix-core form (FP32, N = 7): one wave per element, so P^2 = 64 columns
// fill the wave exactly and no barrier is needed (a wave's LDS accesses
// complete in issue order).  Every contraction with D or D^T runs on the
// 16-block 4x4x1 FP32 MFMA: block b of a wave multiplies the 4-vector of
// operand A with each of its lanes' own value (operand B), so after 8
// steps l = 0..7 on the two row quads, lane q holds sum_l M[r][l] x_q[l]
// for r = 0..7 and its own 8-vector x_q: the whole 8 x 8 product of M with
// the lane's vector.  The accumulation is one fused multiply-add per step
// in the order l = 0..7, which is bitwise the VALU loop of ax_body.  For
// the i- and j-directions the lanes take the element's pencils along that
// direction from an LDS tile, and the results return to the column layout
// through the same tile.
// ---------------------------------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));

// One wave copies one element's P^3 = 512 floats from global memory to LDS:
// two 16-byte-per-lane direct loads, tracked by vmcnt.  The source base is
// made wave-uniform (scalar base + the lane's constant offset), so the
// loads hold no per-lane 64-bit address registers.
template <int kCpol = 0>
__device__ __forceinline__ void dma_elem_to_lds(const float *src, float *dst) {
    const int lane = (int)(threadIdx.x & 63);
    const uint64_t pa = reinterpret_cast<uint64_t>(src);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)pa);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(pa >> 32));
    const float *su = reinterpret_cast<const float *>(((uint64_t)hi << 32) | lo);
    // the immediate offset (1024 bytes) applies to the global and the LDS
    // address alike; kCpol: the cache-policy bits of the loads
    __builtin_amdgcn_global_load_lds((glb_void_t *)(su + 4 * lane), (lds_void_t *)dst, 16, 0,
                                     kCpol);
    __builtin_amdgcn_global_load_lds((glb_void_t *)(su + 4 * lane), (lds_void_t *)dst, 16, 1024,
                                     kCpol);
}
template <bool NT>
__device__ __forceinline__ void dma_elem_to_lds_nt(const float *src, float *dst) {
    dma_elem_to_lds<NT ? kCpolNt : 0>(src, dst);
}


// Element tile in LDS (512 floats): point (i, j, k) at
//   (i ^ 4 (j >> 2)) + 8 (j ^ (k & 3)) + 64 k.
// With 32 banks of 4 bytes, and 16-byte accesses served 8 lanes at a time,
// the three access patterns are conflict-free: a column access (lanes over
// (i, j) at one k) covers a whole slice; a j-pencil access (lanes over
// (i, k) at one j) puts the 4 levels k of a 32-lane half on 4 different
// rows j ^ (k & 3); and the 16-byte i-pencil accesses of 8 lanes (one k,
// j = 0..7) hit 8 different 4-bank groups because rows j >= 4 swap their
// two halves.
__host__ __device__ constexpr int mfma_slot(int i, int j, int k) {
    return (i ^ (4 * (j >> 2))) + 8 * (j ^ (k & 3)) + 64 * k;
}

// Exchange through LDS inside one wave: the wave's earlier LDS accesses
// complete before its later ones issue, and the compiler moves no memory
// access across this point (lanes read what other lanes of the wave wrote).
__device__ __forceinline__ void wave_lds_sync() {
    __asm__ volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(kWaitLgkmcnt0);
    __asm__ volatile("" ::: "memory");
}

// out = M x for the lane's own 8-vector x.  The rows of M come from one
// register per step l: every block takes operand A from the 4 lanes of
// block AB (rows 0..3 of M) and AB + 1 (rows 4..7) through the MFMA's
// A-operand broadcast (CBSZ = 4: all 16 blocks; ABID selects the block).
// Lanes 0..7 hold the rows of D, lanes 8..15 the rows of D^T (AB = 0, 2).
template <int AB>
__device__ __forceinline__ void mfma_apply8(const float (&m)[kP], const float (&x)[kP],
                                            float (&out)[kP]) {
    v4f c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int l = 0; l < kP; ++l) {
        c0 = __builtin_amdgcn_mfma_f32_4x4x1f32(m[l], x[l], c0, 4, AB, 0);
        c1 = __builtin_amdgcn_mfma_f32_4x4x1f32(m[l], x[l], c1, 4, AB + 1, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        out[r] = c0[r];
        out[4 + r] = c1[r];
    }
}

// The lane's pencil along i (lane q is (j, k) = (q & 7, q >> 3)) and along
// j (lane q is (i, k) = (q & 7, q >> 3)): tile offsets.
struct MfmaPencils {
    int ilo, ihi;          // the two 16-byte halves i = 0..3 and 4..7
    int j0, j1, jx;        // element l along j: (l < 4 ? j0 : j1) + ((8 l) ^ jx)
    __device__ __forceinline__ int jslot(int l) const { return (l < 4 ? j0 : j1) + ((8 * l) ^ jx); }
};

__device__ __forceinline__ MfmaPencils mfma_pencils(int q) {
    const int a = q & 7, k = q >> 3;
    MfmaPencils pc;
    const int row = 8 * (a ^ (k & 3)) + 64 * k;      // i-pencil: row j = a at level k
    const int sw = a >> 2;
    pc.ilo = row + 4 * sw;
    pc.ihi = row + 4 * (1 - sw);
    pc.j0 = a + 64 * k;                               // j-pencil: column i = a at level k
    pc.j1 = (a ^ 4) + 64 * k;
    pc.jx = 8 * (k & 3);
    return pc;
}

template <bool OTF, bool FUSED, bool NT = false>
__device__ __forceinline__ void ax_mfma_body(const AxArgs<float> &a, const BasisK<float> &bk,
                                             int64_t ntiles, int64_t vb, int64_t vgrid) {
    if constexpr (kP == 8) {
        using T = float;
        constexpr int P = kP, P2 = P * P, P3 = P2 * P;
        constexpr bool kDma = FUSED;
        // Separate LDS objects: the compiler can then tell which accesses
        // the staging loads in flight may touch (with one array every tile
        // access would wait for them).  2 tiles + 3 staging buffers of
        // 2 KB: 16 waves of a CU fit in its 160 KB.
        __shared__ __align__(16) float sA[P3];
        __shared__ __align__(16) float sB[P3];
        __shared__ __align__(16) float sR[FUSED ? P3 : 4];   // next element's r
        __shared__ __align__(16) float sP[FUSED ? P3 : 4];   // next element's p
        __shared__ __align__(16) float sX[FUSED ? P3 : 4];   // next element's x

        // the CG state in one round of loads: stop, beta, the lagged x step
        T beta = T(0);
        bool xlag = false;
        T aprev = T(0);
        if constexpr (FUSED) {
            const int stopped = a.st->stop;
            beta = (T)a.st->beta;
            xlag = a.x != nullptr && a.st->x_lag != 0;
            aprev = (T)a.st->alpha;
            if (stopped) return;
        }
        const int q = threadIdx.x;        // column (i, j) = (q & 7, q >> 3)
        const int i = q & 7, j = q >> 3;
        const int cq = q ^ ((q >> 5) << 2);                  // mfma_slot(i, j, 0) ^ row swizzle
        auto cslot = [&](int k) { return (cq ^ (8 * (k & 3))) + 64 * k; };   // = mfma_slot(i, j, k)
        const MfmaPencils pc = mfma_pencils(q);
        // operand-A table: lane r < 8 holds row r of D, lane 8 + r row r of
        // D^T, at step l in Dtab[l] (other lanes unused)
        float Dtab[P];
#pragma unroll
        for (int l = 0; l < P; ++l)
            Dtab[l] = q < 8 ? a.D[q * P + l] : (q < 16 ? a.Dt[(q - 8) * P + l] : 0.f);
        constexpr bool strm = FUSED && NT;   // p and x non-temporal
        const int ecb = edge_column_base(kOrder, i, j);
        const bool ecorner = (i == 0 || i == P - 1) && (j == 0 || j == P - 1);
        T xi_i = T(0), eta_j = T(0), wij = T(0);
        if constexpr (OTF) {
            xi_i = a.xi[i];
            eta_j = a.xi[j];
            wij = a.wq[i] * a.wq[j];
        }
        auto stage = [&](int64_t e) {
            if constexpr (kDma) {
                dma_elem_to_lds(reinterpret_cast<const float *>(a.u) + e * P3, sR);
                dma_elem_to_lds_nt<strm>(
                    reinterpret_cast<const float *>(a.p) + e * P3, sP);
                if (xlag)
                    dma_elem_to_lds_nt<strm>(
                        reinterpret_cast<const float *>(a.x) + e * P3, sX);
            }
        };
        // the CG-fused form walks XCD-contiguously when every block takes
        // the same number of elements (measured faster there; with a
        // remainder, the contiguous ranges would leave the last round's
        // elements to the first XCDs, and launch order spreads them); the
        // plain operators, precomputed G most, keep launch order
        const int64_t ev0 =
            (FUSED && ntiles % vgrid == 0) ? xcd_first_tile(vb, vgrid) : vb;
        if (ev0 < ntiles) {
            if constexpr (kDma) stage(ev0);
        }

        double acc = 0.0;
        for (int64_t e = ev0; e < ntiles; e += vgrid) {
            const int64_t base = e * P3 + q;
            T *const wep = (FUSED && a.wedge && ecb >= 0) ? a.wedge + e * edge_slots(kOrder) + ecb
                                                          : nullptr;
            // this element's staged data has landed: on the first element
            // every load; later, all but the previous element's last 8
            // vector-memory operations (its w stores, issued after the
            // staging loads; vector-memory operations complete in order)
            if constexpr (kDma) {
                if (e == vb) __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
                else __builtin_amdgcn_s_waitcnt(kWaitVmcnt8);
                __asm__ volatile("" ::: "memory");
            }

            T uc[P];
            if constexpr (kDma) {
#pragma unroll
                for (int k = 0; k < P; ++k) uc[k] = sR[q + k * P2] + beta * sP[q + k * P2];
#pragma unroll
                for (int k = 0; k < P; ++k)
                    store_nt<strm>(a.p + base + k * P2, uc[k]);
                if (xlag) {
#pragma unroll
                    for (int k = 0; k < P; ++k)
                        store_nt<strm>(a.x + base + k * P2, sX[q + k * P2] + aprev * sP[q + k * P2]);
                }
            } else {
#pragma unroll
                for (int k = 0; k < P; ++k) uc[k] = a.u[base + k * P2];
            }
#pragma unroll
            for (int k = 0; k < P; ++k) sA[cslot(k)] = uc[k];
            wave_lds_sync();

            constexpr bool kPre = !OTF && prefetch_g<T>();
            T gq[kPre ? 6 : 1][kPre ? P : 1];
            if constexpr (kPre) {
                const T *Ge = a.G + e * (6 * P3) + q;
#pragma unroll
                for (int c = 0; c < 6; ++c)
#pragma unroll
                    for (int k = 0; k < P; ++k) gq[c][k] = load_g(Ge + c * P3 + k * P2);
            }

            // gradient: k in the column's registers, i and j on pencils
            T ut[P], pi[P], pj[P], dri[P], dsj[P];
            mfma_apply8<0>(Dtab, uc, ut);
            {
                const float4 lo = *reinterpret_cast<const float4 *>(sA + pc.ilo);
                const float4 hi = *reinterpret_cast<const float4 *>(sA + pc.ihi);
                pi[0] = lo.x, pi[1] = lo.y, pi[2] = lo.z, pi[3] = lo.w;
                pi[4] = hi.x, pi[5] = hi.y, pi[6] = hi.z, pi[7] = hi.w;
            }
#pragma unroll
            for (int l = 0; l < P; ++l) pj[l] = sA[pc.jslot(l)];
            mfma_apply8<0>(Dtab, pi, dri);
            mfma_apply8<0>(Dtab, pj, dsj);
            *reinterpret_cast<float4 *>(sB + pc.ilo) = make_float4(dri[0], dri[1], dri[2], dri[3]);
            *reinterpret_cast<float4 *>(sB + pc.ihi) = make_float4(dri[4], dri[5], dri[6], dri[7]);
#pragma unroll
            for (int l = 0; l < P; ++l) sA[pc.jslot(l)] = dsj[l];
            wave_lds_sync();
            // every read of this element's staging is long done: stage the next
            if constexpr (kDma) {
                if (e + vgrid < ntiles) stage(e + vgrid);
            }
            // column geometry (after the gradient: fewer registers live)
            ColumnGeom<T> cg;
            if constexpr (OTF) {
                // the element's 12 edge vectors (36 values, precomputed from
                // the FP32 vertices with the same subtractions) in scalar
                // registers: read through the constant address space (they
                // are read-only here; a C-style cast is the form clang
                // accepts for the address-space conversion), so no VALU
                // instruction forms or broadcasts them
                const kconst_float *es = (const kconst_float *)(a.edge + e * 36);
                T ed[36];
#pragma unroll
                for (int m = 0; m < 36; ++m) ed[m] = es[m];
                cg = column_geom_edges<T>(ed, xi_i, eta_j, wij);
            }

            // pointwise G, back in the column layout
            T vt[P];
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const int cs = cslot(k);
                const T ur = sB[cs], us = sA[cs];
                T vr, vs;
                point_flux<T, OTF, kPre>(cg, bk, k, gq, OTF ? nullptr : a.G + e * (6 * P3) + q,
                                         ur, us, ut[k], vr, vs, vt[k]);
                sB[cs] = vr;
                sA[cs] = vs;
            }
            wave_lds_sync();

            // divergence: D^T along k in registers, along i and j on pencils
            T wt[P];
            mfma_apply8<2>(Dtab, vt, wt);
            {
                const float4 lo = *reinterpret_cast<const float4 *>(sB + pc.ilo);
                const float4 hi = *reinterpret_cast<const float4 *>(sB + pc.ihi);
                pi[0] = lo.x, pi[1] = lo.y, pi[2] = lo.z, pi[3] = lo.w;
                pi[4] = hi.x, pi[5] = hi.y, pi[6] = hi.z, pi[7] = hi.w;
            }
#pragma unroll
            for (int l = 0; l < P; ++l) pj[l] = sA[pc.jslot(l)];
            mfma_apply8<2>(Dtab, pi, dri);
            mfma_apply8<2>(Dtab, pj, dsj);
            *reinterpret_cast<float4 *>(sB + pc.ilo) = make_float4(dri[0], dri[1], dri[2], dri[3]);
            *reinterpret_cast<float4 *>(sB + pc.ihi) = make_float4(dri[4], dri[5], dri[6], dri[7]);
#pragma unroll
            for (int l = 0; l < P; ++l) sA[pc.jslot(l)] = dsj[l];
            wave_lds_sync();

#pragma unroll
            for (int k = 0; k < P; ++k) {
                const int cs = cslot(k);
                const T wv = (sB[cs] + sA[cs]) + wt[k];
                if constexpr (FUSED) {
                    acc += (double)uc[k] * (double)wv;
                    if (wep && (k == 0 || k == P - 1 || ecorner))
                        wep[k == 0 ? 0 : (k == P - 1 ? 1 : 1 + k)] = wv;
                }
                a.w[base + k * P2] = wv;
            }
        }
        if constexpr (FUSED) {
            // the block is one wave: a shuffle reduction in a fixed order
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
            if (threadIdx.x == 0) a.partial[vb] = acc;
        }
    }
}

// ---------------------------------------------------------------------------
// Matrix-core form for N = 9: P^2 = 100 columns, one element per block of
// two waves (threads 100..127 shadow thread 99: they compute its values
// and store nothing).  The contractions are those of ax_mfma_body with
// three row quads (rows 10, 11 of the operand table are zero): lanes 0..11
// of each wave hold the rows of D, lanes 12..23 those of D^T.  The waves
// exchange pencils through LDS with barriers.  Tile: point (i, j, k) at
// i + 10 j + 106 k (a column access covers consecutive words; a j-pencil
// access of 32 lanes (i, k) lands on 32 consecutive banks because
// 106 = 10 mod 32).  Same accumulation order as the VALU engine.
// ---------------------------------------------------------------------------
template <int AB>
__device__ __forceinline__ void mfma_apply10(const float (&m)[kP], const float (&x)[kP],
                                             float (&out)[kP]) {
    v4f c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f}, c2 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int l = 0; l < kP; ++l) {
        c0 = __builtin_amdgcn_mfma_f32_4x4x1f32(m[l], x[l], c0, 4, AB, 0);
        c1 = __builtin_amdgcn_mfma_f32_4x4x1f32(m[l], x[l], c1, 4, AB + 1, 0);
        c2 = __builtin_amdgcn_mfma_f32_4x4x1f32(m[l], x[l], c2, 4, AB + 2, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        out[r] = c0[r];
        out[4 + r] = c1[r];
        if (8 + r < kP) out[8 + r] = c2[r];
    }
}

template <bool OTF, bool FUSED, bool NT = false>
__device__ __forceinline__ void ax_mfma10_body(const AxArgs<float> &a, const BasisK<float> &bk,
                                               int64_t ntiles, int64_t vb, int64_t vgrid) {
    if constexpr (kP == 10) {
        using T = float;
        constexpr int P = kP, P2 = P * P, P3 = P2 * P, S = 106;
        constexpr bool kDma = FUSED;
        __shared__ __align__(16) float sA[P * S];
        __shared__ __align__(16) float sB[P * S];
        __shared__ __align__(16) float sC[P * S];
        __shared__ __align__(16) float sR[FUSED ? P3 : 4];   // next element's r
        __shared__ __align__(16) float sP[FUSED ? P3 : 4];   // next element's p
        __shared__ __align__(16) float sX[FUSED ? P3 : 4];   // next element's x
        __shared__ __align__(16) float sV[FUSED ? 32 : 4];   // next element's vertices

        // the CG state in one round of loads: stop, beta, the lagged x step
        T beta = T(0);
        bool xlag = false;
        T aprev = T(0);
        if constexpr (FUSED) {
            const int stopped = a.st->stop;
            beta = (T)a.st->beta;
            xlag = a.x != nullptr && a.st->x_lag != 0;
            aprev = (T)a.st->alpha;
            if (stopped) return;
        }
        const int t = threadIdx.x;
        const bool active = t < P2;
        const int c = active ? t : P2 - 1;             // column, i-pencil or j-pencil index
        const int i = c % P, j = c / P;                 // column (i, j)
        const int qw = t & 63;                          // lane in the wave
        // operand-A table: lane r < 12 of each wave holds row r of D, lane
        // 12 + r row r of D^T (rows 10, 11 zero), at step l in Dtab[l]
        float Dtab[P];
#pragma unroll
        for (int l = 0; l < P; ++l)
            Dtab[l] = qw < P ? a.D[qw * P + l]
                             : (qw >= 12 && qw < 12 + P ? a.Dt[(qw - 12) * P + l] : 0.f);
        // pencils: along i, index c is (j, k) = (c % P, c / P); along j,
        // index c is (i, k) = (c % P, c / P)
        const int ipen = P * (c % P) + S * (c / P);     // + i
        const int jpen = (c % P) + S * (c / P);         // + P j
        constexpr bool strm = FUSED && NT;   // p and x non-temporal
        const int ecb = edge_column_base(kOrder, i, j);
        const bool ecorner = (i == 0 || i == P - 1) && (j == 0 || j == P - 1);
        T xi_i = T(0), eta_j = T(0), wij = T(0);
        if constexpr (OTF) {
            xi_i = a.xi[i];
            eta_j = a.xi[j];
            wij = a.wq[i] * a.wq[j];
        }
        auto stage = [&](int64_t e) {
            if constexpr (kDma) {
                dma_to_lds(reinterpret_cast<const float *>(a.u) + e * P3, sR, P3, 2);
                dma_to_lds_nt<strm>(reinterpret_cast<const float *>(a.p) + e * P3, sP, P3, 2);
                if (xlag)
                    dma_to_lds_nt<strm>(reinterpret_cast<const float *>(a.x) + e * P3, sX, P3, 2);
            }
        };
        auto stage_vert = [&](int64_t e) {
            if constexpr (kDma && OTF)
                dma_to_lds(reinterpret_cast<const float *>(a.vert) + e * 24, sV, 24, 2);
        };
        // blocks in launch order here (xcd_first_tile measured 9% slower
        // for this two-wave kernel)
        if constexpr (kDma) {
            if (vb < ntiles) {
                stage(vb);
                stage_vert(vb);
            }
        }

        double acc = 0.0;
        for (int64_t e = vb; e < ntiles; e += vgrid) {
            const int64_t base = e * P3 + c;
            T *const wep = (FUSED && active && a.wedge && ecb >= 0)
                               ? a.wedge + e * edge_slots(kOrder) + ecb
                               : nullptr;
            if constexpr (kDma) {
                __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
                lds_barrier();                          // every wave's share has landed
            }
            T uc[P];
            if constexpr (kDma) {
#pragma unroll
                for (int k = 0; k < P; ++k) uc[k] = sR[c + k * P2] + beta * sP[c + k * P2];
                if (active) {
#pragma unroll
                    for (int k = 0; k < P; ++k) store_nt<strm>(a.p + base + k * P2, uc[k]);
                    if (xlag) {
#pragma unroll
                        for (int k = 0; k < P; ++k)
                            store_nt<strm>(a.x + base + k * P2, sX[c + k * P2] + aprev * sP[c + k * P2]);
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < P; ++k) uc[k] = a.u[base + k * P2];
            }
            if (active) {
#pragma unroll
                for (int k = 0; k < P; ++k) sA[c + k * S] = uc[k];
            }
            lds_barrier();                              // (1) sA holds u; staging reads done
            // every read of this element's r, p, x staging is done: stage the next
            if constexpr (kDma) {
                if (e + vgrid < ntiles) stage(e + vgrid);
            }
            constexpr bool kPre = !OTF && prefetch_g<T>();
            T gq[kPre ? 6 : 1][kPre ? P : 1];
            if constexpr (kPre) {
                const T *Ge = a.G + e * (6 * P3) + c;
#pragma unroll
                for (int cc = 0; cc < 6; ++cc)
#pragma unroll
                    for (int k = 0; k < P; ++k) gq[cc][k] = load_g(Ge + cc * P3 + k * P2);
            }

            // gradient: i- and j-pencils of sA into sB and sC
            T ut[P];
            mfma_apply10<0>(Dtab, uc, ut);
            {
                T pi[P], pj[P], dri[P], dsj[P];
#pragma unroll
                for (int l = 0; l < P; ++l) {
                    pi[l] = sA[ipen + l];
                    pj[l] = sA[jpen + P * l];
                }
                mfma_apply10<0>(Dtab, pi, dri);
                mfma_apply10<0>(Dtab, pj, dsj);
                if (active) {
#pragma unroll
                    for (int l = 0; l < P; ++l) {
                        sB[ipen + l] = dri[l];
                        sC[jpen + P * l] = dsj[l];
                    }
                }
            }
            lds_barrier();                              // (2)

            // column geometry, then G pointwise: each thread rewrites only
            // its own column's slots, in place
            ColumnGeom<T> cg;
            if constexpr (OTF) {
                if constexpr (kDma) cg = column_geom<T>(sV, xi_i, eta_j, wij);
                else cg = column_geom<T>(a.vert + e * 24, xi_i, eta_j, wij);
            }
            T vt[P];
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const int cs = c + k * S;
                const T ur = sB[cs], us = sC[cs];
                T vr, vs;
                point_flux<T, OTF, kPre>(cg, bk, k, gq, OTF ? nullptr : a.G + e * (6 * P3) + c,
                                         ur, us, ut[k], vr, vs, vt[k]);
                if (active) {
                    sB[cs] = vr;
                    sC[cs] = vs;
                }
            }
            lds_barrier();                              // (3) the vertices were read too
            if constexpr (kDma) {
                if (e + vgrid < ntiles) stage_vert(e + vgrid);
            }

            // divergence: i-pencils of sB into sA, j-pencils of sC kept
            // until every pencil read of sC is done
            T wt[P];
            mfma_apply10<3>(Dtab, vt, wt);
            {
                T pi[P], pj[P], dri[P], dsj[P];
#pragma unroll
                for (int l = 0; l < P; ++l) {
                    pi[l] = sB[ipen + l];
                    pj[l] = sC[jpen + P * l];
                }
                mfma_apply10<3>(Dtab, pi, dri);
                mfma_apply10<3>(Dtab, pj, dsj);
                if (active) {
#pragma unroll
                    for (int l = 0; l < P; ++l) sA[ipen + l] = dri[l];
                }
                lds_barrier();                          // (4)
                if (active) {
#pragma unroll
                    for (int l = 0; l < P; ++l) sB[jpen + P * l] = dsj[l];
                }
            }
            lds_barrier();                              // (5)
            if (active) {
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    const int cs = c + k * S;
                    const T wv = (sA[cs] + sB[cs]) + wt[k];
                    if constexpr (FUSED) {
                        acc += (double)uc[k] * (double)wv;
                        if (wep && (k == 0 || k == P - 1 || ecorner))
                            wep[k == 0 ? 0 : (k == P - 1 ? 1 : 1 + k)] = wv;
                    }
                    a.w[base + k * P2] = wv;
                }
            }
            lds_barrier();                              // (6) the next element rewrites sA
        }
        if constexpr (FUSED) {
            const double sum = block_sum(acc);
            if (threadIdx.x == 0) a.partial[vb] = sum;
        }
    }
}

// Matrix-core kernels: N = 7 on single-wave blocks, N = 9 on two-wave blocks.
constexpr int kMfmaThreads = kP == 10 ? 128 : 64;
constexpr int kMfmaWaves = kP == 10 ? 3 : 4;

template <bool OTF, bool FUSED, bool NT>
__device__ __forceinline__ void ax_mfma_any(const AxArgs<float> &a, const BasisK<float> &bk,
                                            int64_t ntiles, int64_t vb, int64_t vgrid) {
    if constexpr (kP == 10) ax_mfma10_body<OTF, FUSED, NT>(a, bk, ntiles, vb, vgrid);
    else ax_mfma_body<OTF, FUSED, NT>(a, bk, ntiles, vb, vgrid);
}

// NT: the CG-fused form with p and x non-temporal (AxArgs::stream)
template <bool OTF, bool FUSED, bool NT = false>
__global__ void __launch_bounds__(kMfmaThreads, kMfmaWaves)
ax_mfma_kernel(const AxArgs<float> a, const BasisK<float> bk, int64_t ntiles) {
    ax_mfma_any<OTF, FUSED, NT>(a, bk, ntiles, blockIdx.x, gridDim.x);
}

template <bool OTF, bool NT = false>
__global__ void __launch_bounds__(kMfmaThreads, kMfmaWaves)
ax_mfma_batch_kernel(const AxArgs<float> *__restrict__ descs, const int2 *__restrict__ blk,
                     const BasisK<float> bk) {
    const int2 pv = blk[blockIdx.x];
    const AxArgs<float> a = descs[pv.x];
    ax_mfma_any<OTF, true, NT>(a, bk, a.E, pv.y, a.vgrid);
}

template <typename T, bool OTF, bool FUSED, bool NT = false>
__global__ void __launch_bounds__(512, ax_min_waves<T>())
ax_kernel(const AxArgs<T> a, const BasisK<T> bk, int64_t ntiles) {
    ax_body<T, OTF, FUSED, NT>(a, bk, ntiles, blockIdx.x, gridDim.x);
}

// Many problems of this order in one launch: block b runs virtual block
// blk[b].y of problem blk[b].x, exactly the block that problem's own launch
// would run, so every problem's partials (and results) are bitwise those
// of its solo solve.
template <typename T, bool OTF, bool NT = false>
__global__ void __launch_bounds__(512, ax_min_waves<T>())
ax_batch_kernel(const AxArgs<T> *__restrict__ descs, const int2 *__restrict__ blk,
                const BasisK<T> bk) {
    const int2 pv = blk[blockIdx.x];
    const AxArgs<T> a = descs[pv.x];
    ax_body<T, OTF, true, NT>(a, bk, (a.E + a.epb - 1) / a.epb, pv.y, a.vgrid);
}

template <typename T>
BasisK<T> make_basis(const double *D, const double *xi, const double *w) {
    BasisK<T> b;
    for (int q = 0; q < kP * kP; ++q) b.D[q] = (T)D[q];
    for (int q = 0; q < kP; ++q) {
        b.xi[q] = (T)xi[q];
        b.w[q] = (T)w[q];
    }
    return b;
}

template <typename T, bool OTF, bool FUSED>
void launch(const AxArgs<T> &a, const BasisK<T> &bk, int64_t grid, hipStream_t s) {
    constexpr bool kMayStream = FUSED;
    const bool nt = kMayStream && a.stream != 0;
    if constexpr (sizeof(T) == 4 && (kP == 8 || kP == 10)) {
        if (a.mfma) {
            // one element per block (one wave at N = 7, two at N = 9)
            if (nt)
                hipLaunchKernelGGL((ax_mfma_kernel<OTF, FUSED, kMayStream>), dim3((unsigned)grid),
                                   dim3(kMfmaThreads), 0, s, a, bk, a.E);
            else
                hipLaunchKernelGGL((ax_mfma_kernel<OTF, FUSED>), dim3((unsigned)grid),
                                   dim3(kMfmaThreads), 0, s, a, bk, a.E);
            return;
        }
    }
    const int threads = ((a.epb * kP * kP + 63) / 64) * 64;
    const size_t lds = ax_lds_bytes<T, OTF, FUSED>(a.epb);
    const int64_t ntiles = (a.E + a.epb - 1) / a.epb;
    if (nt)
        hipLaunchKernelGGL((ax_kernel<T, OTF, FUSED, kMayStream>), dim3((unsigned)grid),
                           dim3(threads), lds, s, a, bk, ntiles);
    else
        hipLaunchKernelGGL((ax_kernel<T, OTF, FUSED>), dim3((unsigned)grid), dim3(threads), lds,
                           s, a, bk, ntiles);
}

}  // namespace

#define SEM_CAT3_(a, b, c) a##b##c
#define SEM_CAT3(a, b, c) SEM_CAT3_(a, b, c)

template <typename T>
static void ax_entry(bool otf, AxMode mode, const AxArgs<T> &a, const double *D,
                     const double *xi, const double *w, int64_t grid, hipStream_t s) {
    const BasisK<T> bk = make_basis<T>(D, xi, w);
    const bool fused = mode == AxMode::CgFused;
    if (otf) {
        if (fused) launch<T, true, true>(a, bk, grid, s);
        else launch<T, true, false>(a, bk, grid, s);
    } else {
        if (fused) launch<T, false, true>(a, bk, grid, s);
        else launch<T, false, false>(a, bk, grid, s);
    }
}

template <typename T, bool NT>
static void ax_batch_launch(bool otf, bool mfma, const AxArgs<T> *descs, const int2 *blk,
                            int64_t nblk, int epb, const BasisK<T> &bk, hipStream_t s) {
    if constexpr (sizeof(T) == 4 && (kP == 8 || kP == 10)) {
        if (mfma) {
            // static LDS only
            if (otf)
                hipLaunchKernelGGL((ax_mfma_batch_kernel<true, NT>), dim3((unsigned)nblk),
                                   dim3(kMfmaThreads), 0, s, descs, blk, bk);
            else
                hipLaunchKernelGGL((ax_mfma_batch_kernel<false, NT>), dim3((unsigned)nblk),
                                   dim3(kMfmaThreads), 0, s, descs, blk, bk);
            return;
        }
    }
    const int threads = ((epb * kP * kP + 63) / 64) * 64;
    const size_t lds_otf = ax_lds_bytes<T, true, true>(epb);
    const size_t lds_pre = ax_lds_bytes<T, false, true>(epb);
    if (otf)
        hipLaunchKernelGGL((ax_batch_kernel<T, true, NT>), dim3((unsigned)nblk), dim3(threads),
                           lds_otf, s, descs, blk, bk);
    else
        hipLaunchKernelGGL((ax_batch_kernel<T, false, NT>), dim3((unsigned)nblk), dim3(threads),
                           lds_pre, s, descs, blk, bk);
}

template <typename T>
static void ax_batch_entry(bool otf, bool mfma, bool stream, const AxArgs<T> *descs,
                           const int2 *blk, int64_t nblk, int epb, const double *D,
                           const double *xi, const double *w, hipStream_t s) {
    const BasisK<T> bk = make_basis<T>(D, xi, w);
    if (stream) ax_batch_launch<T, true>(otf, mfma, descs, blk, nblk, epb, bk, s);
    else ax_batch_launch<T, false>(otf, mfma, descs, blk, nblk, epb, bk, s);
}

void SEM_CAT3(ax_batch_order_, SEM_ORDER, _f32)(bool otf, bool mfma, bool stream,
                                                 const AxArgs<float> *descs, const int2 *blk,
                                                 int64_t nblk, int epb, const double *D,
                                                 const double *xi, const double *w,
                                                 hipStream_t s) {
    ax_batch_entry<float>(otf, mfma, stream, descs, blk, nblk, epb, D, xi, w, s);
}

void SEM_CAT3(ax_order_, SEM_ORDER, _f32)(bool otf, AxMode mode, const AxArgs<float> &a,
                                           const double *D, const double *xi, const double *w,
                                           int64_t grid, hipStream_t s) {
    ax_entry<float>(otf, mode, a, D, xi, w, grid, s);
}
void SEM_CAT3(ax_order_, SEM_ORDER, _f64)(bool otf, AxMode mode, const AxArgs<double> &a,
                                           const double *D, const double *xi, const double *w,
                                           int64_t grid, hipStream_t s) {
    ax_entry<double>(otf, mode, a, D, xi, w, grid, s);
}

}  // namespace sem
