// sem_ax_dispatch.cpp -- order dispatch and launch shapes of the local operator.
#include "sem_internal.h"

#include <atomic>
#include <cstdlib>

namespace sem {

#define SEM_DECL_ORDER(N)                                                                       \
    void ax_order_##N##_f32(bool, AxMode, const AxArgs<float> &, const double *, const double *, \
                            const double *, int64_t, hipStream_t);                              \
    void ax_order_##N##_f64(bool, AxMode, const AxArgs<double> &, const double *,               \
                            const double *, const double *, int64_t, hipStream_t);
SEM_DECL_ORDER(1)
SEM_DECL_ORDER(2)
SEM_DECL_ORDER(3)
SEM_DECL_ORDER(4)
SEM_DECL_ORDER(5)
SEM_DECL_ORDER(6)
SEM_DECL_ORDER(7)
SEM_DECL_ORDER(8)
SEM_DECL_ORDER(9)
SEM_DECL_ORDER(10)
SEM_DECL_ORDER(11)
#undef SEM_DECL_ORDER

#define SEM_DECL_BATCH(N)                                                                      \
    void ax_batch_order_##N##_f32(bool, bool, bool, const AxArgs<float> *, const int2 *,       \
                                  int64_t, int, const double *, const double *, const double *, \
                                  hipStream_t);
SEM_DECL_BATCH(1)
SEM_DECL_BATCH(2)
SEM_DECL_BATCH(3)
SEM_DECL_BATCH(4)
SEM_DECL_BATCH(5)
SEM_DECL_BATCH(6)
SEM_DECL_BATCH(7)
SEM_DECL_BATCH(8)
SEM_DECL_BATCH(9)
SEM_DECL_BATCH(10)
SEM_DECL_BATCH(11)
#undef SEM_DECL_BATCH

using FnB = void (*)(bool, bool, bool, const AxArgs<float> *, const int2 *, int64_t, int,
                     const double *, const double *, const double *, hipStream_t);
static const FnB kFnB[kMaxOrder + 1] = {
    nullptr,           ax_batch_order_1_f32, ax_batch_order_2_f32, ax_batch_order_3_f32,
    ax_batch_order_4_f32, ax_batch_order_5_f32, ax_batch_order_6_f32, ax_batch_order_7_f32,
    ax_batch_order_8_f32, ax_batch_order_9_f32, ax_batch_order_10_f32, ax_batch_order_11_f32};

using Fn32 = void (*)(bool, AxMode, const AxArgs<float> &, const double *, const double *,
                      const double *, int64_t, hipStream_t);
using Fn64 = void (*)(bool, AxMode, const AxArgs<double> &, const double *, const double *,
                      const double *, int64_t, hipStream_t);

// The CG-fused operator writes one FP64 partial per block; its grid is
// capped so that the partial sum stays short (tiles are then strided).
#ifndef SEM_AX_FUSED_MAX_BLOCKS
#define SEM_AX_FUSED_MAX_BLOCKS 2048
#endif
constexpr int64_t kAxFusedMaxBlocks = SEM_AX_FUSED_MAX_BLOCKS;
// the matrix-core form: blocks of one wave (N = 7; measured best of 8192,
// 16384 and 32768) and of two waves (N = 9: 1536, the blocks resident at
// once at 3 waves per SIMD and 6 blocks per CU, ahead of 3072 and 4096 at
// 10^3 ... 28^3 elements: every block walks its share of the elements
// without a partial last round)
#ifndef SEM_AX_MFMA_MAX_BLOCKS
#define SEM_AX_MFMA_MAX_BLOCKS 16384
#endif
#ifndef SEM_AX_MFMA2_MAX_BLOCKS
#define SEM_AX_MFMA2_MAX_BLOCKS 1536
#endif
constexpr int64_t kAxMfmaMaxBlocks = SEM_AX_MFMA_MAX_BLOCKS;
constexpr int64_t kAxMfma2MaxBlocks = SEM_AX_MFMA2_MAX_BLOCKS;

// the plain (stand-alone) operator: one tile per block unless capped
#ifndef SEM_AX_PLAIN_MAX_BLOCKS
#define SEM_AX_PLAIN_MAX_BLOCKS 0
#endif
constexpr int64_t kAxPlainMaxBlocks = SEM_AX_PLAIN_MAX_BLOCKS;

static int64_t ax_grid(int64_t ntiles, AxMode mode, bool mfma, int threads = 64) {
    const int64_t cap =
        mfma ? (threads == 64 ? kAxMfmaMaxBlocks : kAxMfma2MaxBlocks) : kAxFusedMaxBlocks;
    if (mode == AxMode::CgFused && ntiles > cap) return cap;
    if (mode != AxMode::CgFused && kAxPlainMaxBlocks > 0 && ntiles > kAxPlainMaxBlocks)
        return kAxPlainMaxBlocks;
    return ntiles;
}

static const Fn32 kFn32[kMaxOrder + 1] = {nullptr,        ax_order_1_f32, ax_order_2_f32,
                                          ax_order_3_f32, ax_order_4_f32, ax_order_5_f32,
                                          ax_order_6_f32, ax_order_7_f32, ax_order_8_f32,
                                          ax_order_9_f32, ax_order_10_f32, ax_order_11_f32};
static const Fn64 kFn64[kMaxOrder + 1] = {nullptr,        ax_order_1_f64, ax_order_2_f64,
                                          ax_order_3_f64, ax_order_4_f64, ax_order_5_f64,
                                          ax_order_6_f64, ax_order_7_f64, ax_order_8_f64,
                                          ax_order_9_f64, ax_order_10_f64, ax_order_11_f64};

// Default elements per block: fill a multiple of 64 lanes with (i, j)
// columns as tightly as possible, at most 512 threads and 64 KiB of LDS.
// The autotuner (sem_ax_shape_set) overrides them per order, precision
// and geometric-factor form.
static const int kEpb32[kMaxOrder + 1] = {0, 64, 28, 16, 10, 7, 5, 4, 3, 2, 2, 3};
static const int kEpb64[kMaxOrder + 1] = {0, 64, 28, 16, 10, 7, 5, 4, 3, 3, 2, 1};

// Process-wide tile shapes set by the autotuner (0: built-in default),
// indexed [on-the-fly][fp64][N], and a generation counter that tells cached
// graphs and batch tables that a shape changed.
static std::atomic<int> g_epb[2][2][kMaxOrder + 1];
static std::atomic<int> g_engine[2][2][kMaxOrder + 1];
static std::atomic<int> g_shape_gen{0};

int ax_shape_generation() { return g_shape_gen.load(); }

static std::atomic<int64_t> g_cache_bytes{kInfinityCacheBytes};

bool cg_streams_vectors(int64_t footprint) { return footprint > g_cache_bytes.load(); }

void cache_bytes_set(int64_t bytes) {
    g_cache_bytes.store(bytes > 0 ? bytes : kInfinityCacheBytes);
    g_shape_gen.fetch_add(1);
}

void ax_shape_set(int N, bool fp64, bool otf, int epb) {
    g_epb[otf ? 1 : 0][fp64 ? 1 : 0][N].store(epb > 0 ? epb : 0);
    g_shape_gen.fetch_add(1);
}

bool ax_mfma_available(int N, bool fp64) { return (N == 7 || N == 9) && !fp64; }

void ax_engine_set(int N, bool fp64, bool otf, int engine) {
    g_engine[otf ? 1 : 0][fp64 ? 1 : 0][N].store(engine);
    g_shape_gen.fetch_add(1);
}

AxShape ax_shape(int N, bool fp64, bool otf, int epb_override) {
    const int P = N + 1, P2 = P * P, P3 = P2 * P;
    const size_t tsz = fp64 ? 8 : 4;
    // default: the matrix cores where they are built (FP32, N = 7: the
    // fused operator is 14% faster there than with VALU FMA)
    const int engine = g_engine[otf ? 1 : 0][fp64 ? 1 : 0][N].load();
    // built-in choice: the matrix cores wherever they measured faster than
    // the best VALU tile (N = 7 in both G forms, N = 9 with G on the fly;
    // at N = 9 with G read from HBM two VALU elements per block are ahead)
    const bool mfma = engine == kAxEngineMfma ||
                      (engine == kAxEngineDefault && !(N == 9 && !otf));
    if (mfma && ax_mfma_available(N, fp64)) {
        // one element per block (one wave at N = 7, two at N = 9): the
        // operator tiles (two unpadded at N = 7, three of slices of 106
        // floats at N = 9) and the staging of r, p, x and the vertices
        AxShape s;
        s.epb = 1;
        s.threads = N == 9 ? 128 : 64;
        s.lds = N == 9 ? 4 * (3 * (size_t)P * 106 + 3 * (size_t)P3 + 32)
                       : 4 * (5 * (size_t)P3);
        s.mfma = true;
        return s;
    }
    int epb = epb_override > 0 ? epb_override : g_epb[otf ? 1 : 0][fp64 ? 1 : 0][N].load();
    if (epb <= 0) epb = fp64 ? kEpb64[N] : kEpb32[N];
    // clamp to the kernel limits (FP32 CG-fused tiles of odd N also stage
    // the next tile's r, p and vertices in LDS)
    const bool staged = !fp64 && P3 % 4 == 0;
    auto lds = [&](int q) {
        return 2 * tsz * (size_t)q * P3 + (staged ? 8 * (size_t)q * P3 + 96 * (size_t)q : 0);
    };
    while (epb > 1 && (((epb * P2 + 63) / 64) * 64 > 512 || lds(epb) > 65536)) --epb;
    AxShape s;
    s.epb = epb;
    s.threads = ((epb * P2 + 63) / 64) * 64;
    s.lds = lds(epb);
    s.mfma = false;
    return s;
}

template <>
void launch_ax<float>(const Mesh &m, bool otf, AxMode mode, AxArgs<float> a, hipStream_t s) {
    const AxShape sh = ax_shape(m.N, false, otf, a.epb);
    a.epb = sh.epb;
    a.mfma = sh.mfma ? 1 : 0;
    a.E = m.E;
    a.D = m.b32.D;
    a.Dt = m.b32.Dt;
    a.xi = m.b32.xi;
    a.wq = m.b32.w;
    a.vert = m.vert32;
    a.edge = m.edge32;
    if (!otf) a.G = m.G32;
    const int64_t ntiles = (m.E + sh.epb - 1) / sh.epb;
    kFn32[m.N](otf, mode, a, m.h_D.data(), m.h_xi.data(), m.h_w.data(),
               ax_grid(ntiles, mode, sh.mfma, sh.threads), s);
    check_hip(hipGetLastError(), "ax kernel launch (fp32)");
}

template <>
void launch_ax<double>(const Mesh &m, bool otf, AxMode mode, AxArgs<double> a, hipStream_t s) {
    const AxShape sh = ax_shape(m.N, true, otf, a.epb);
    a.epb = sh.epb;
    a.mfma = 0;
    a.E = m.E;
    a.D = m.b64.D;
    a.Dt = m.b64.Dt;
    a.xi = m.b64.xi;
    a.wq = m.b64.w;
    a.vert = m.vert64;
    a.edge = nullptr;
    if (!otf) a.G = m.G64;
    const int64_t ntiles = (m.E + sh.epb - 1) / sh.epb;
    kFn64[m.N](otf, mode, a, m.h_D.data(), m.h_xi.data(), m.h_w.data(),
               ax_grid(ntiles, mode, false), s);
    check_hip(hipGetLastError(), "ax kernel launch (fp64)");
}

void ax_batch_desc(const Mesh &m, bool otf, AxArgs<float> &a) {
    const AxShape sh = ax_shape(m.N, false, otf, 0);
    a.epb = sh.epb;
    a.mfma = sh.mfma ? 1 : 0;
    a.E = m.E;
    a.D = m.b32.D;
    a.Dt = m.b32.Dt;
    a.xi = m.b32.xi;
    a.wq = m.b32.w;
    a.vert = m.vert32;
    a.edge = m.edge32;
    a.G = otf ? nullptr : m.G32;
    a.vgrid = ax_grid((m.E + sh.epb - 1) / sh.epb, AxMode::CgFused, sh.mfma, sh.threads);
}

void launch_ax_batch(int N, bool otf, bool mfma, bool stream, const AxArgs<float> *descs,
                     const int2 *blk, int64_t nblk, int epb, const double *D, const double *xi,
                     const double *w,
                     hipStream_t s) {
    if (nblk <= 0) return;
    kFnB[N](otf, mfma, stream, descs, blk, nblk, epb, D, xi, w, s);
    check_hip(hipGetLastError(), "batched ax kernel launch");
}

int64_t cg_footprint(const Mesh &m, int tsz, bool table_free) {
    const int64_t es = edge_slots(m.N);
    int64_t b = 4 * tsz * m.n;                                          // r, p, x, w
    if (table_free) b += m.E * (6 + es) * 8 + tsz * m.n_egroups;       // records, edge sums
    else if (m.gs_in_update) b += 4 * m.n + tsz * m.n_groups_multi;    // table, group sums
    if (m.gsum_wedge || table_free) b += m.E * es * tsz;                // edge copy
    // vertices (the matrix-core operator at N = 7 reads the element edge
    // vectors instead), point codes
    b += (m.edge32 && tsz == 4 ? m.E * 36 * 4 : m.E * 24 * tsz) + m.n;
    return b;
}

int64_t ax_blocks(const Mesh &m, bool fp64, bool otf, int epb_override) {
    const AxShape sh = ax_shape(m.N, fp64, otf, epb_override);
    return ax_grid((m.E + sh.epb - 1) / sh.epb, AxMode::CgFused, sh.mfma, sh.threads);
}

}  // namespace sem
