// sem_batch.hip -- many independent meshes advanced together.
//
// One batched CG iteration is a fixed sequence of launches that each cover
// every problem, the same schedule as a single-mesh solve: the fused local
// operator once per polynomial order (p-update, the previous iteration's x
// step, <p,w,c> partials), the edge/vertex group sums (or, for a mesh that
// shares element-interior nodes, the whole gather-scatter), the alpha
// finalize (one block per problem), the r update with the gather and the rho
// finalize (one block per problem).  Block b of a
// launch runs "virtual block" blk[b].y of problem blk[b].x -- exactly the
// block that the problem's own single-mesh launch would run, with the same
// tiles, the same grid stride and the same partial slot -- so every
// problem's reductions happen in the same order as in its solo solve and
// its result is bitwise identical.  Problems that have stopped exit at the
// first instruction of their blocks.  The sequence is captured once in a
// HIP graph and replayed.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>

#include "sem_cg_internal.h"
#include "sem_gs_body.h"
#include "sem_vec_body.h"

namespace sem {
namespace {

struct GsBatchDesc {
    const GsClasses *cls;
    const int32_t *idx;
    float *w;
    const CgState *st;
};

struct UpdBatchDesc {
    int64_t n;
    float *r;
    const float *w;
    const uint8_t *mcode;
    CgState *st;
    double *partial;
    int64_t vgrid;
};

// group sums of one problem (see launch_group_sums_cg / launch_edge_sums_cg)
struct GsumBatchDesc {
    const GsClasses *cls;
    const int32_t *idx;
    int64_t io0;
    const float *src;
    float *out;
    const CgState *st;
    int mmin;
};

// update with gather of one problem (see launch_update_gather)
struct UpdGBatchDesc {
    int64_t n;
    float *r;
    const float *w;
    const float *gsum;
    const uint8_t *mcode;
    vecb::GatherMap gm;
    CgState *st;
    double *partial;
    int64_t vgrid;
};

// update with the table-free gather of one problem (see launch_update_struct)
struct UpdSBatchDesc {
    int64_t n;
    float *r;
    const float *wg;
    vecb::StructMap sm;
    CgState *st;
    double *partial;
    int64_t vgrid;
};

struct FinBatchDesc {
    CgState *st;
    const double *part_ax;
    int64_t n_ax;
    const double *part_vec;
    int n_vec;
};

__global__ void __launch_bounds__(gsb::kGsThreads)
gs_batch_kernel(const GsBatchDesc *__restrict__ d, const int2 *__restrict__ blk) {
    const int2 pv = blk[blockIdx.x];
    const GsBatchDesc g = d[pv.x];
    if (g.st->stop) return;
    gsb::gs_logical_block<float>(*g.cls, pv.y, g.idx, g.w);
}

__global__ void __launch_bounds__(kFinalizeThreads)
finalize_alpha_batch_kernel(const FinBatchDesc *__restrict__ d) {
    const FinBatchDesc f = d[blockIdx.x];
    vecb::finalize_alpha_body(f.st, f.part_ax, f.n_ax);
}

__global__ void __launch_bounds__(gsb::kGsThreads)
group_sums_batch_kernel(const GsumBatchDesc *__restrict__ d, const int2 *__restrict__ blk) {
    const int2 pv = blk[blockIdx.x];
    const GsumBatchDesc g = d[pv.x];
    if (g.st->stop) return;
    gsb::gs_sums_logical_block<float>(*g.cls, pv.y, g.idx, g.io0, g.src, g.out, g.mmin);
}

__global__ void __launch_bounds__(vecb::kVecThreads)
update_batch_kernel(const UpdBatchDesc *__restrict__ d, const int2 *__restrict__ blk) {
    const int2 pv = blk[blockIdx.x];
    const UpdBatchDesc u = d[pv.x];
    vecb::update_body<float, false>(u.n, nullptr, u.r, nullptr, u.w, u.mcode, u.st, u.partial,
                                    pv.y, u.vgrid);
}

__global__ void __launch_bounds__(vecb::kVecThreads)
update_gather_batch_kernel(const UpdGBatchDesc *__restrict__ d, const int2 *__restrict__ blk) {
    const int2 pv = blk[blockIdx.x];
    const UpdGBatchDesc u = d[pv.x];
    vecb::update_gather_body<float>(u.n, u.r, u.w, u.gsum, u.mcode, u.gm, u.st, u.partial, pv.y,
                                    u.vgrid);
}

__global__ void __launch_bounds__(vecb::kVecThreads)
update_struct_batch_kernel(const UpdSBatchDesc *__restrict__ d, const int2 *__restrict__ blk) {
    const int2 pv = blk[blockIdx.x];
    const UpdSBatchDesc u = d[pv.x];
    vecb::update_struct_body<float>(u.n, u.r, u.wg, u.sm, u.st, u.partial, pv.y, u.vgrid);
}

__global__ void __launch_bounds__(kFinalizeThreads)
finalize_rho_batch_kernel(const FinBatchDesc *__restrict__ d) {
    const FinBatchDesc f = d[blockIdx.x];
    vecb::finalize_rho_body(f.st, f.part_vec, f.n_vec);
}

// What the host reads of every problem's CG state after a chunk of batched
// iterations: one array, one copy.
struct StateRow {
    int stop;
    int iter;
    double rr;       // <r, r, c> of the current residual
    double rho0;     // <r0, r0, c>
};

__global__ void gather_states_kernel(const FinBatchDesc *__restrict__ d, int count,
                                     StateRow *out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < count) {
        const CgState *st = d[q].st;
        out[q] = StateRow{st->stop, st->iter, st->rr, st->rho0};
    }
}

template <typename T>
T *dalloc(size_t count, size_t &bytes) {
    void *p = nullptr;
    const size_t b = std::max<size_t>(count, 1) * sizeof(T);
    if (hipMalloc(&p, b) != hipSuccess) {
        (void)hipGetLastError();
        fail(SEM_ENOMEM, "batch allocation of " + std::to_string(b) + " bytes failed");
    }
    bytes += b;
    return static_cast<T *>(p);
}

template <typename T>
void upload_sync(T *dst, const std::vector<T> &src) {
    if (!src.empty())
        SEM_HIP(hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
}

}  // namespace

struct BatchImpl {
    int device = 0;
    std::vector<Mesh *> meshes;
    struct OrderGroup {
        int N;
        int epb;
        bool mfma = false;
        int2 *blk = nullptr;
        int64_t nblk = 0;
    };
    std::vector<OrderGroup> groups[2];              // [precomputed, on the fly]
    bool stream_vectors = false;                    // p and x non-temporal (footprint)
    struct BlkTable {
        int2 *blk = nullptr;
        size_t cap = 0;
    };
    std::map<int, BlkTable> blk_tab[2];              // per order; owns the group tables
    AxArgs<float> *d_ax[2] = {nullptr, nullptr};   // [precomputed, on the fly]
    GsClasses *d_cls = nullptr;
    GsBatchDesc *d_gs = nullptr;
    int2 *d_gs_blk = nullptr;
    int64_t n_gs_blk = 0;
    UpdBatchDesc *d_upd = nullptr;
    int2 *d_upd_blk = nullptr;
    int64_t n_upd_blk = 0;
    GsumBatchDesc *d_gsum = nullptr;
    int2 *d_gsum_blk = nullptr;
    int64_t n_gsum_blk = 0;
    UpdGBatchDesc *d_updg = nullptr;
    int2 *d_updg_blk = nullptr;
    int64_t n_updg_blk = 0;
    UpdSBatchDesc *d_upds = nullptr;
    int2 *d_upds_blk = nullptr;
    int64_t n_upds_blk = 0;
    FinBatchDesc *d_fin[2] = {nullptr, nullptr};   // [precomputed, on the fly]
    StateRow *d_states = nullptr;
    StateRow *h_states = nullptr;                    // pinned
    size_t cap_ax[2] = {0, 0}, cap_fin[2] = {0, 0}, cap_cls = 0, cap_gs = 0, cap_gs_blk = 0,
           cap_upd = 0, cap_upd_blk = 0, cap_gsum = 0, cap_gsum_blk = 0, cap_updg = 0,
           cap_updg_blk = 0, cap_upds = 0, cap_upds_blk = 0, cap_states = 0, cap_h_states = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    std::map<GraphKey, hipGraphExec_t> graphs;
    size_t bytes = 0;
    int shape_gen = -1;       // tile-shape generation the tables were built for

    ~BatchImpl() {
        (void)hipDeviceSynchronize();
        for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
        for (int f = 0; f < 2; ++f)
            for (auto &kv : blk_tab[f])
                if (kv.second.blk) (void)hipFree(kv.second.blk);
        void *ptrs[] = {d_ax[0],   d_ax[1], d_cls,      d_gs,   d_gs_blk,   d_upd,
                        d_upd_blk, d_gsum,  d_gsum_blk, d_updg, d_updg_blk, d_upds, d_upds_blk,
                        d_fin[0],
                        d_fin[1],  d_states};
        for (void *q : ptrs)
            if (q) (void)hipFree(q);
        if (h_states) (void)hipHostFree(h_states);
        if (ev) (void)hipEventDestroy(ev);
        if (stream) (void)hipStreamDestroy(stream);
    }

    int count() const { return (int)meshes.size(); }

    void rebuild(const std::vector<Mesh *> &ms);

    // one batched CG iteration of every problem
    void enqueue_iteration(bool otf, hipStream_t s) {
        if (count() == 0) return;
        const int f = otf ? 1 : 0;
        for (const auto &g : groups[f]) {
            launch_ax_batch(g.N, otf, g.mfma, stream_vectors, d_ax[f], g.blk, g.nblk, g.epb,
                            order_D[g.N].data(), order_xi[g.N].data(), order_w[g.N].data(), s);
        }
        if (n_gs_blk > 0)
            hipLaunchKernelGGL(gs_batch_kernel, dim3((unsigned)n_gs_blk), dim3(gsb::kGsThreads), 0,
                               s, d_gs, d_gs_blk);
        if (n_gsum_blk > 0)
            hipLaunchKernelGGL(group_sums_batch_kernel, dim3((unsigned)n_gsum_blk),
                               dim3(gsb::kGsThreads), 0, s, d_gsum, d_gsum_blk);
        hipLaunchKernelGGL(finalize_alpha_batch_kernel, dim3(count()), dim3(kFinalizeThreads), 0,
                           s, d_fin[f]);
        if (n_upd_blk > 0)
            hipLaunchKernelGGL(update_batch_kernel, dim3((unsigned)n_upd_blk),
                               dim3(vecb::kVecThreads), 0, s, d_upd, d_upd_blk);
        if (n_updg_blk > 0)
            hipLaunchKernelGGL(update_gather_batch_kernel, dim3((unsigned)n_updg_blk),
                               dim3(vecb::kVecThreads), 0, s, d_updg, d_updg_blk);
        if (n_upds_blk > 0)
            hipLaunchKernelGGL(update_struct_batch_kernel, dim3((unsigned)n_upds_blk),
                               dim3(vecb::kVecThreads), 0, s, d_upds, d_upds_blk);
        hipLaunchKernelGGL(finalize_rho_batch_kernel, dim3(count()), dim3(kFinalizeThreads), 0, s,
                           d_fin[f]);
        check_hip(hipGetLastError(), "batched iteration launch");
    }

    void run_chunk(bool otf, int chunk, bool use_graph) {
        if (!use_graph) {
            for (int c = 0; c < chunk; ++c) enqueue_iteration(otf, stream);
            return;
        }
        const GraphKey key{otf, chunk, ax_shape_generation()};
        auto it = graphs.find(key);
        if (it == graphs.end()) {
            hipGraph_t g = nullptr;
            SEM_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
            try {
                for (int c = 0; c < chunk; ++c) enqueue_iteration(otf, stream);
            } catch (...) {
                hipGraph_t junk = nullptr;
                (void)hipStreamEndCapture(stream, &junk);
                if (junk) (void)hipGraphDestroy(junk);
                throw;
            }
            SEM_HIP(hipStreamEndCapture(stream, &g));
            hipGraphExec_t ge = nullptr;
            const hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            check_hip(e, "hipGraphInstantiate (batch)");
            it = graphs.emplace(key, ge).first;
        }
        SEM_HIP(hipGraphLaunch(it->second, stream));
    }

    // the state of every member into the pinned h_states (stream-ordered)
    void enqueue_read_states() {
        hipLaunchKernelGGL(gather_states_kernel, dim3((count() + 255) / 256), dim3(256), 0, stream,
                           d_fin[0], count(), d_states);
        SEM_HIP(hipMemcpyAsync(h_states, d_states, sizeof(StateRow) * count(), hipMemcpyDeviceToHost,
                               stream));
    }
    // ... and wait for it
    void read_states() {
        enqueue_read_states();
        SEM_HIP(hipStreamSynchronize(stream));
    }

    // per order: host basis copies (FP64) for the kernel-argument basis
    std::map<int, std::vector<double>> order_D, order_xi, order_w;
};

namespace {

// Device array with a capacity; grows (and drops its contents) on demand.
template <typename T>
void ensure_cap(T *&ptr, size_t &cap, size_t need, size_t &bytes) {
    if (need <= cap && ptr) return;
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    cap = 0;
    ptr = dalloc<T>(need, bytes);
    cap = std::max<size_t>(need, 1);
}

BatchImpl *batch_create(int count, const sem_mesh_t *handles) {
    if (count <= 0) fail(SEM_EINVAL, "count must be positive");
    if (!handles) fail(SEM_EINVAL, "meshes must not be NULL");
    std::vector<Mesh *> ms;
    for (int q = 0; q < count; ++q) {
        Mesh *m = as_mesh(handles[q]);
        for (Mesh *o : ms)
            if (o == m) fail(SEM_EINVAL, "a mesh appears twice in the batch");
        ms.push_back(m);
    }
    for (Mesh *m : ms)
        if (m->device != ms[0]->device) fail(SEM_EINVAL, "all meshes of a batch must share a device");
    std::unique_ptr<BatchImpl> b(new BatchImpl());
    b->device = ms[0]->device;
    SEM_HIP(hipSetDevice(b->device));
    SEM_HIP(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    SEM_HIP(hipEventCreateWithFlags(&b->ev, hipEventDisableTiming));
    b->rebuild(ms);
    return b.release();
}

}  // namespace

// Rebuilds every descriptor and block table for a new member list (the
// captured graphs refer to the old tables and are dropped).
void BatchImpl::rebuild(const std::vector<Mesh *> &ms) {
    SEM_HIP(hipStreamSynchronize(stream));
    shape_gen = ax_shape_generation();
    for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
    meshes = ms;
    const int count = (int)ms.size();
    std::vector<AxArgs<float>> ax[2];
    std::vector<GsClasses> cls;
    std::vector<GsBatchDesc> gsd;
    std::vector<UpdBatchDesc> upd;
    std::vector<GsumBatchDesc> gsumd;
    std::vector<UpdGBatchDesc> updg;
    std::vector<UpdSBatchDesc> upds;
    std::vector<FinBatchDesc> fin[2];
    std::vector<int2> gs_blk, upd_blk, gsum_blk, updg_blk, upds_blk;
    std::map<int, std::vector<int2>> order_blk[2];
    std::map<int, int> order_epb[2];
    std::map<int, bool> order_mfma[2];
    ensure_cap(d_cls, cap_cls, count, bytes);
    // one batched iteration touches every member's vectors
    int64_t footprint = 0;
    for (int q = 0; q < count; ++q) footprint += cg_footprint(*ms[q], 4, ms[q]->gs_struct);
    const int stream = cg_streams_vectors(footprint) ? 1 : 0;
    stream_vectors = stream != 0;
    for (int q = 0; q < count; ++q) {
        Mesh &m = *ms[q];
        Workspace &ws = cg_workspace(m, false);
        for (int otf = 0; otf < 2; ++otf) {
            AxArgs<float> a{};
            ax_batch_desc(m, otf != 0, a);
            a.stream = stream;
            a.u = static_cast<float *>(ws.r);
            a.p = static_cast<float *>(ws.p);
            a.w = static_cast<float *>(ws.w);
            a.st = ws.st;
            a.partial = ws.part_ax;
            a.x = static_cast<float *>(ws.x);
            a.wedge = (m.gsum_wedge || m.gs_struct) ? static_cast<float *>(ws.wedge) : nullptr;
            ax[otf].push_back(a);
        }
        for (int f = 0; f < 2; ++f) {
            const AxArgs<float> &af = ax[f].back();
            order_epb[f][m.N] = af.epb;
            order_mfma[f][m.N] = af.mfma != 0;
            for (int64_t vb = 0; vb < af.vgrid; ++vb)
                order_blk[f][m.N].push_back(make_int2(q, (int)vb));
        }
        if (!order_D.count(m.N)) {
            order_D[m.N] = m.h_D;
            order_xi[m.N] = m.h_xi;
            order_w[m.N] = m.h_w;
        }
        cls.push_back(m.gs_struct ? m.ecls : m.gs);
        const int64_t nlb = m.n_groups > 0 ? gs_logical_blocks(m) : 0;
        const int nv = vec_blocks(m.n);
        if (m.gs_struct) {
            // the single-mesh schedule with the table-free gather: sums of
            // every edge-node group after w, then the update
            float *wg = static_cast<float *>(ws.w);
            gsumd.push_back({d_cls + q, m.ewedge_idx, (int64_t)0,
                             static_cast<const float *>(ws.wedge), wg + m.n, ws.st, 2});
            const int64_t nelb = gs_total_blocks(m.ecls);
            for (int64_t lb = 0; lb < nelb; ++lb)
                gsum_blk.push_back(make_int2((int)gsumd.size() - 1, (int)lb));
            const vecb::StructMap sm{m.erec, m.pos_tab, m.P3, 6 + edge_slots(m.N), m.p3_magic,
                                     m.p3_shift};
            upds.push_back({m.n, static_cast<float *>(ws.r), wg, sm, ws.st, ws.part_vec, nv});
            for (int vb = 0; vb < nv; ++vb)
                upds_blk.push_back(make_int2((int)upds.size() - 1, vb));
        } else if (m.gs_in_update) {
            // the single-mesh schedule: group sums of the edge and vertex
            // groups, update with gather (the same logical and virtual blocks)
            const bool compact = m.gsum_wedge;
            gsumd.push_back({d_cls + q, compact ? m.wedge_idx : m.gs_idx,
                             compact ? m.wedge_io0 : (int64_t)0,
                             compact ? static_cast<const float *>(ws.wedge)
                                     : static_cast<const float *>(ws.w),
                             static_cast<float *>(ws.gsum), ws.st, 3});
            for (int64_t lb = m.gs_blk_multi; lb < nlb; ++lb)
                gsum_blk.push_back(make_int2((int)gsumd.size() - 1, (int)lb));
            const vecb::GatherMap gm{m.gsrc};
            updg.push_back({m.n, static_cast<float *>(ws.r), static_cast<const float *>(ws.w),
                            static_cast<const float *>(ws.gsum), m.mcode, gm, ws.st, ws.part_vec,
                            nv});
            for (int vb = 0; vb < nv; ++vb)
                updg_blk.push_back(make_int2((int)updg.size() - 1, vb));
        } else {
            gsd.push_back({d_cls + q, m.gs_idx, static_cast<float *>(ws.w), ws.st});
            for (int64_t lb = 0; lb < nlb; ++lb)
                gs_blk.push_back(make_int2((int)gsd.size() - 1, (int)lb));
            upd.push_back({m.n, static_cast<float *>(ws.r), static_cast<const float *>(ws.w),
                           m.mcode, ws.st, ws.part_vec, nv});
            for (int vb = 0; vb < nv; ++vb)
                upd_blk.push_back(make_int2((int)upd.size() - 1, vb));
        }
        for (int f = 0; f < 2; ++f)
            fin[f].push_back({ws.st, ws.part_ax, ax[f].back().vgrid, ws.part_vec, nv});
    }
    for (int otf = 0; otf < 2; ++otf) {
        ensure_cap(d_ax[otf], cap_ax[otf], count, bytes);
        upload_sync(d_ax[otf], ax[otf]);
    }
    upload_sync(d_cls, cls);
    ensure_cap(d_gs, cap_gs, count, bytes);
    upload_sync(d_gs, gsd);
    ensure_cap(d_upd, cap_upd, count, bytes);
    upload_sync(d_upd, upd);
    ensure_cap(d_gsum, cap_gsum, count, bytes);
    upload_sync(d_gsum, gsumd);
    ensure_cap(d_updg, cap_updg, count, bytes);
    upload_sync(d_updg, updg);
    ensure_cap(d_upds, cap_upds, count, bytes);
    upload_sync(d_upds, upds);
    for (int f = 0; f < 2; ++f) {
        ensure_cap(d_fin[f], cap_fin[f], count, bytes);
        upload_sync(d_fin[f], fin[f]);
    }
    ensure_cap(d_states, cap_states, count, bytes);
    if (cap_h_states < (size_t)count) {
        if (h_states) (void)hipHostFree(h_states);
        h_states = nullptr;
        SEM_HIP(hipHostMalloc((void **)&h_states, sizeof(StateRow) * std::max(count, 1)));
        cap_h_states = std::max(count, 1);
    }
    n_gs_blk = (int64_t)gs_blk.size();
    ensure_cap(d_gs_blk, cap_gs_blk, gs_blk.size(), bytes);
    upload_sync(d_gs_blk, gs_blk);
    n_upd_blk = (int64_t)upd_blk.size();
    ensure_cap(d_upd_blk, cap_upd_blk, upd_blk.size(), bytes);
    upload_sync(d_upd_blk, upd_blk);
    n_gsum_blk = (int64_t)gsum_blk.size();
    ensure_cap(d_gsum_blk, cap_gsum_blk, gsum_blk.size(), bytes);
    upload_sync(d_gsum_blk, gsum_blk);
    n_updg_blk = (int64_t)updg_blk.size();
    ensure_cap(d_updg_blk, cap_updg_blk, updg_blk.size(), bytes);
    upload_sync(d_updg_blk, updg_blk);
    n_upds_blk = (int64_t)upds_blk.size();
    ensure_cap(d_upds_blk, cap_upds_blk, upds_blk.size(), bytes);
    upload_sync(d_upds_blk, upds_blk);
    for (int f = 0; f < 2; ++f) {
        // each order's block table (and its capacity) persists across
        // rebuilds: the serving loop rebuilds whenever its member set changes
        groups[f].clear();
        for (auto &kv : order_blk[f]) {
            BlkTable &t = blk_tab[f][kv.first];
            ensure_cap(t.blk, t.cap, kv.second.size(), bytes);
            upload_sync(t.blk, kv.second);
            OrderGroup g;
            g.N = kv.first;
            g.epb = order_epb[f][kv.first];
            g.mfma = order_mfma[f][kv.first];
            g.nblk = (int64_t)kv.second.size();
            g.blk = t.blk;
            groups[f].push_back(g);
        }
    }
}

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// Sets the FP32 CG state of problem q: fresh solve (todo) or stopped.
// idle: the caller knows no copy from or to the workspace's pinned state is
// still in flight (else the stream is synchronised first).
void set_state(Mesh &m, bool active, double tol, int max_iter, int fixed, hipStream_t s,
               bool idle = false) {
    Workspace &ws = cg_workspace(m, false);
    CgState h{};
    h.thresh = tol * tol;
    h.max_iter = fixed > 0 ? fixed : max_iter;
    h.fixed = fixed > 0 ? 1 : 0;
    h.stop = active ? 0 : 1;
    if (!idle) SEM_HIP(hipStreamSynchronize(s));
    *ws.h_st = h;
    SEM_HIP(hipMemcpyAsync(ws.st, ws.h_st, sizeof(CgState), hipMemcpyHostToDevice, s));
}

// Batched FP32 iterations until every problem has stopped.  Problems that
// have stopped leave the launches: once a quarter of the current members
// have stopped, the tables are rebuilt for the running ones (a running
// problem's blocks, partial slots and results stay those of its solo solve;
// the caller restores the full member list afterwards).
void iterate_all(BatchImpl &B, bool otf, int chunk, bool use_graph, int max_iter) {
    int64_t last_sum = -1;
    const int64_t guard = (int64_t)max_iter / std::max(chunk, 1) + 8;
    for (int64_t round = 0;; ++round) {
        B.read_states();
        int running = 0;
        int64_t sum = 0;
        for (int q = 0; q < B.count(); ++q) {
            running += B.h_states[q].stop == 0;
            sum += B.h_states[q].iter;
        }
        if (!running) break;
        if (sum <= last_sum || round > guard)
            fail(SEM_EDEVICE, "batched CG state did not advance");
        last_sum = sum;
        if (4 * (B.count() - running) >= B.count()) {
            std::vector<Mesh *> keep;
            for (int q = 0; q < B.count(); ++q)
                if (B.h_states[q].stop == 0) keep.push_back(B.meshes[q]);
            B.rebuild(keep);
            last_sum = -1;      // the sum now runs over fewer members
        }
        B.run_chunk(otf, chunk, use_graph);
    }
}

}  // namespace

struct ServerImpl;
ServerImpl *server_new(const sem_cg_opts &o, int round_iters);
void server_delete(ServerImpl *sv);
void server_add(ServerImpl &sv, Mesh *m, const double *b, double *x, int64_t tag,
                hipStream_t user_s);
int server_step(ServerImpl &sv, int64_t *tags, sem_cg_result *results, int cap, int *n_done);

sem_status batch_solve(BatchImpl &B, const sem_cg_opts &o, const void *const *b_dev,
                       void *const *x_dev, sem_cg_result *res, hipStream_t user_s) {
    const double t0 = now_s();
    const bool otf = o.geom == SEM_G_ON_THE_FLY;
    const int P = B.count();
    for (int q = 0; q < P; ++q) {
        if (!b_dev[q] || !x_dev[q]) fail(SEM_EINVAL, "b and x of every problem must be set");
        if (!otf && !B.meshes[q]->G32)
            fail(SEM_EUNSUPPORTED, "precomputed FP32 G was not built for a mesh of the batch");
    }
    if (o.kernel_ms || o.hist_rho || o.hist_alpha)
        fail(SEM_EUNSUPPORTED, "histories and kernel timing are single-mesh options");
    hipStream_t s = B.stream;
    if (B.shape_gen != ax_shape_generation()) B.rebuild(B.meshes);
    SEM_HIP(hipEventRecord(B.ev, user_s));
    SEM_HIP(hipStreamWaitEvent(s, B.ev, 0));
    int64_t nmax = 0;
    for (Mesh *m : B.meshes) nmax = std::max(nmax, m->n);
    const int chunk = o.poll_every > 0 ? o.poll_every : cg_auto_chunk(nmax, o.fixed_iters);
    const bool graph = o.use_graph != 0;
    bool breakdown = false;

    const std::vector<Mesh *> all = B.meshes;   // iterate_all may drop stopped members
    if (o.prec == SEM_FP32) {
        for (int q = 0; q < P; ++q) {
            Mesh &m = *all[q];
            Workspace &ws = cg_workspace(m, false);
            set_state(m, true, o.tol, o.max_iter, o.fixed_iters, s);
            SEM_HIP(hipMemcpyAsync(ws.x, x_dev[q], sizeof(float) * m.n, hipMemcpyDeviceToDevice, s));
            launch_mask<float>(m, static_cast<float *>(ws.x), s);
            AxArgs<float> a{};
            a.u = static_cast<const float *>(ws.x);
            a.w = static_cast<float *>(ws.w);
            launch_ax<float>(m, otf, AxMode::Plain, a, s);
            launch_gs<float>(m, static_cast<float *>(ws.w), s);
            launch_mask<float>(m, static_cast<float *>(ws.w), s);
            launch_cg_init<float>(m, static_cast<const float *>(b_dev[q]),
                                  static_cast<const float *>(ws.w), static_cast<float *>(ws.r),
                                  static_cast<float *>(ws.p), ws.st, ws.part_vec, s);
        }
        iterate_all(B, otf, chunk, graph, o.fixed_iters > 0 ? o.fixed_iters : o.max_iter);
        if (B.meshes != all) B.rebuild(all);
        for (int q = 0; q < P; ++q) {
            Mesh &m = *all[q];
            Workspace &ws = cg_workspace(m, false);
            launch_x_flush<float>(m, static_cast<float *>(ws.x), static_cast<const float *>(ws.p),
                                  ws.st, s);
            SEM_HIP(hipMemcpyAsync(x_dev[q], ws.x, sizeof(float) * m.n, hipMemcpyDeviceToDevice, s));
            SEM_HIP(hipMemcpyAsync(ws.h_st, ws.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
            SEM_HIP(hipStreamSynchronize(s));
            const CgState &h = *ws.h_st;
            res[q] = sem_cg_result{};
            res[q].iters = h.iter;
            res[q].status = h.stop;
            res[q].converged = h.stop == 1;
            res[q].rel_res_recursive = h.rho0 > 0 ? std::sqrt(h.rr / h.rho0) : 0.0;
            res[q].rel_res_true = -1.0;
            breakdown |= h.stop == 3;
        }
    } else if (o.prec == SEM_MIXED) {
        // every problem runs the refinement of sem_cg_solve(SEM_MIXED) with
        // outer steps of its own: the serving loop with all problems added
        // at once.  The inner FP32 iterations of the problems in their inner
        // solve advance together; a problem leaves the launches when its
        // inner solve stops (its FP64 outer residual runs between rounds)
        // and joins them again for its next inner solve.
        std::unique_ptr<ServerImpl, void (*)(ServerImpl *)> sv(server_new(o, chunk),
                                                                server_delete);
        for (int q = 0; q < P; ++q)
            server_add(*sv, all[q], static_cast<const double *>(b_dev[q]),
                       static_cast<double *>(x_dev[q]), q, user_s);
        std::vector<int64_t> tags(P);
        std::vector<sem_cg_result> out(P);
        for (int left = P; left > 0;) {
            int nd = 0;
            left = server_step(*sv, tags.data(), out.data(), P, &nd);
            for (int k = 0; k < nd; ++k) {
                res[tags[k]] = out[k];
                breakdown |= out[k].status == 3;
            }
        }
    } else {
        fail(SEM_EUNSUPPORTED, "batched solves run in SEM_FP32 or SEM_MIXED");
    }
    const double dt = now_s() - t0;
    for (int q = 0; q < P; ++q) res[q].seconds = dt;
    return breakdown ? SEM_EBREAKDOWN : SEM_OK;
}

BatchImpl *batch_new(int count, const sem_mesh_t *meshes) { return batch_create(count, meshes); }
void batch_delete(BatchImpl *b) { delete b; }

}  // namespace sem

// ---------------------------------------------------------------------------
// Continuous-batching server: requests join and leave at round boundaries.
// Every request runs the mixed-precision refinement of sem_cg_solve (FP64
// outer residual per request, FP32 inner CG); the inner iterations of all
// requests that are in their inner phase advance together in batched
// launches.  A request's arithmetic and reduction order do not depend on
// which other requests share its launches, so its result is bitwise that of
// its own sem_cg_solve.
//
// The loop is pipelined over two streams.  Each call of server_step ends by
// launching the next round of inner iterations (main stream) and returns
// while it runs; the next call first computes, on the side stream and
// concurrently with that round, the FP64 outer residuals of the requests
// that are between inner solves (new ones, and those whose inner solve
// stopped), decides which are done, then waits for the round, reads the
// state of every member in one copy, restarts the inner solves of the
// requests that go on (they join the next round) and launches it.
// ---------------------------------------------------------------------------
namespace sem {

struct ServerReq {
    uint64_t uid = 0;       // unique per request (mesh addresses can be reused)
    Mesh *m = nullptr;
    const double *b = nullptr;
    double *x = nullptr;
    int64_t tag = 0;
    int phase = 0;          // 0: outer residual pending; 1: inner CG running (member of
                            // the round in flight); 2: to restart its inner solve
    int outer = 0, total = 0, last_stop = 0;
    bool broken = false;    // the inner CG broke down
    double rel = 0.0, inner_rel = 0.0;
};

struct ServerImpl {
    sem_cg_opts o{};
    int round_iters = 16;
    BatchImpl batch;                    // its stream is the main stream
    hipStream_t side = nullptr;         // request set-up, outer residuals, result copies
    hipEvent_t ev_side = nullptr, ev_round = nullptr;
    bool round_in_flight = false;
    std::vector<ServerReq> reqs;
    uint64_t next_uid = 1;
    std::vector<uint64_t> batch_uids;   // requests the batch tables were built for
    std::vector<uint64_t> round_uids;   // members of the round in flight, in table order
    double inner_tol = 1e-5;
    int max_outer = 20, inner_cap = 100000;

    ~ServerImpl() {
        (void)hipDeviceSynchronize();
        if (ev_side) (void)hipEventDestroy(ev_side);
        if (ev_round) (void)hipEventDestroy(ev_round);
        if (side) (void)hipStreamDestroy(side);
    }
};

ServerImpl *server_new(const sem_cg_opts &o, int round_iters) {
    if (o.prec != SEM_MIXED) fail(SEM_EUNSUPPORTED, "the server runs SEM_MIXED solves");
    if (!(o.tol > 0)) fail(SEM_EINVAL, "tol must be positive");
    if (o.geom != SEM_G_PRECOMPUTED && o.geom != SEM_G_ON_THE_FLY)
        fail(SEM_EINVAL, "unknown geometry form");
    std::unique_ptr<ServerImpl> sv(new ServerImpl());
    sv->o = o;
    sv->round_iters = round_iters > 0 ? round_iters : 16;
    sv->inner_tol = o.inner_tol > 0 ? o.inner_tol : 1e-5;
    sv->max_outer = o.max_outer > 0 ? o.max_outer : 20;
    sv->inner_cap = o.max_iter > 0 ? o.max_iter : 100000;
    SEM_HIP(hipGetDevice(&sv->batch.device));
    SEM_HIP(hipStreamCreateWithFlags(&sv->batch.stream, hipStreamNonBlocking));
    SEM_HIP(hipEventCreateWithFlags(&sv->batch.ev, hipEventDisableTiming));
    SEM_HIP(hipStreamCreateWithFlags(&sv->side, hipStreamNonBlocking));
    SEM_HIP(hipEventCreateWithFlags(&sv->ev_side, hipEventDisableTiming));
    SEM_HIP(hipEventCreateWithFlags(&sv->ev_round, hipEventDisableTiming));
    sv->batch.rebuild({});
    return sv.release();
}

void server_delete(ServerImpl *sv) { delete sv; }

void server_add(ServerImpl &sv, Mesh *m, const double *b, double *x, int64_t tag,
                hipStream_t user_s) {
    if (!b || !x) fail(SEM_EINVAL, "b and x must not be NULL");
    for (const ServerReq &r : sv.reqs)
        if (r.m == m) fail(SEM_EINVAL, "the mesh already has a request in the server");
    if (m->device != sv.batch.device) fail(SEM_EINVAL, "the mesh lives on another device");
    if (sv.o.geom == SEM_G_PRECOMPUTED && !m->G32)
        fail(SEM_EUNSUPPORTED, "precomputed FP32 G was not built for the mesh");
    // the request's set-up runs on the side stream (a round may be in
    // flight on the main one); b and x may still be in flight on the
    // caller's stream, which the side stream waits for
    hipStream_t s = sv.side;
    SEM_HIP(hipEventRecord(sv.batch.ev, user_s));
    SEM_HIP(hipStreamWaitEvent(s, sv.batch.ev, 0));
    Workspace &w64 = cg_workspace(*m, true);
    (void)cg_workspace(*m, false);
    double *x64 = static_cast<double *>(w64.x);
    SEM_HIP(hipMemcpyAsync(x64, x, sizeof(double) * m->n, hipMemcpyDeviceToDevice, s));
    launch_mask<double>(*m, x64, s);
    launch_dot<double>(*m, b, b, w64.dval + 1, w64.part_vec, s);
    ServerReq r;
    r.uid = sv.next_uid++;
    r.m = m;
    r.b = b;
    r.x = x;
    r.tag = tag;
    sv.reqs.push_back(r);
}

// One step.  Returns the number of requests still in the server; finished
// requests are written to (tags, results) up to cap (the rest stay queued
// as finished and are returned by the next call).  The round it launches
// is still running when it returns.
int server_step(ServerImpl &sv, int64_t *tags, sem_cg_result *results, int cap, int *n_done) {
    hipStream_t s = sv.batch.stream, s2 = sv.side;
    const bool otf = sv.o.geom == SEM_G_ON_THE_FLY;
    *n_done = 0;
    // 1. outer FP64 residuals of the requests between inner solves, on the
    // side stream while the round launched by the previous step runs
    bool any_outer = false;
    for (ServerReq &r : sv.reqs) {
        if (r.phase != 0) continue;
        any_outer = true;
        Workspace &w64 = cg_workspace(*r.m, true);
        api_apply_A64(*r.m, static_cast<const double *>(w64.x), static_cast<double *>(w64.w), s2);
        launch_residual64(*r.m, r.b, static_cast<const double *>(w64.w),
                          static_cast<double *>(w64.r), w64.dval + 0, w64.part_vec, s2);
        SEM_HIP(hipMemcpyAsync(w64.h_val, w64.dval, 2 * sizeof(double), hipMemcpyDeviceToHost, s2));
    }
    if (any_outer) {
        SEM_HIP(hipEventRecord(sv.ev_side, s2));
        SEM_HIP(hipEventSynchronize(sv.ev_side));
    }
    // 2. the stopping test of those requests: finished ones copy their x
    // out (side stream) and leave; the others will restart their inner solve
    std::vector<ServerReq> keep;
    for (ServerReq &r : sv.reqs) {
        if (r.phase == 0) {
            Workspace &w64 = cg_workspace(*r.m, true);
            const double rr = w64.h_val[0], bb = w64.h_val[1];
            r.rel = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
            int done = 0;
            if (r.broken || !std::isfinite(r.rel)) done = 3;
            else if (r.rel <= sv.o.tol || rr == 0.0) done = 1;
            else if (r.outer >= sv.max_outer) done = 2;
            if (done && *n_done < cap) {
                SEM_HIP(hipMemcpyAsync(r.x, w64.x, sizeof(double) * r.m->n,
                                       hipMemcpyDeviceToDevice, s2));
                sem_cg_result &o = results[*n_done];
                o = sem_cg_result{};
                o.iters = r.total;
                o.outer = r.outer;
                o.converged = done == 1;
                o.status = done == 1 ? 1 : (done == 3 ? 3 : (r.last_stop ? r.last_stop : 2));
                o.rel_res_recursive = r.inner_rel;
                o.rel_res_true = r.rel;
                tags[*n_done] = r.tag;
                ++*n_done;
                continue;
            }
            if (!done) r.phase = 2;
            // done but no room to report it: kept (phase 0) for the next call
        }
        keep.push_back(r);
    }
    sv.reqs.swap(keep);
    // 3. the round in flight: wait for it and read every member's state
    // (gathered into one array at its end)
    if (sv.round_in_flight) {
        SEM_HIP(hipEventSynchronize(sv.ev_round));
        sv.round_in_flight = false;
        for (ServerReq &r : sv.reqs) {
            if (r.phase != 1) continue;
            const auto it = std::find(sv.round_uids.begin(), sv.round_uids.end(), r.uid);
            if (it == sv.round_uids.end()) fail(SEM_EDEVICE, "a running request missed its round");
            const StateRow h = sv.batch.h_states[it - sv.round_uids.begin()];
            if (!h.stop) continue;
            Workspace &w32 = cg_workspace(*r.m, false);
            Workspace &w64 = cg_workspace(*r.m, true);
            r.total += h.iter;
            r.last_stop = h.stop;
            r.inner_rel = h.rho0 > 0 ? std::sqrt(h.rr / h.rho0) : 0.0;
            if (h.stop == 3) {
                r.broken = true;
            } else {
                // the round is complete: x64 += ||r||_c d on the side
                // stream, ahead of this request's next outer residual there
                launch_x_flush<float>(*r.m, static_cast<float *>(w32.x),
                                      static_cast<const float *>(w32.p), w32.st, s2);
                launch_axpy_from_f32(r.m->n, static_cast<double *>(w64.x), w64.dval + 0,
                                     static_cast<const float *>(w32.x), s2);
                ++r.outer;
            }
            r.phase = 0;   // next step: outer residual and the stopping test
        }
    }
    // 4. restart the inner FP32 solves of A d = r / ||r||_c that go on, on
    // the main stream ahead of the next round (the residual they start from
    // is complete: the side stream was waited for above; no round in
    // flight touches their state)
    for (ServerReq &r : sv.reqs) {
        if (r.phase != 2) continue;
        Workspace &w32 = cg_workspace(*r.m, false);
        Workspace &w64 = cg_workspace(*r.m, true);
        float *b32 = static_cast<float *>(w32.b);
        launch_scale_to_f32(r.m->n, static_cast<const double *>(w64.r), w64.dval + 0, b32, s);
        set_state(*r.m, true, refine_inner_tol(sv.inner_tol, sv.o.tol, r.rel), sv.inner_cap, 0,
                  s, true);
        SEM_HIP(hipMemsetAsync(w32.x, 0, sizeof(float) * r.m->n, s));
        launch_cg_init<float>(*r.m, b32, nullptr, static_cast<float *>(w32.r),
                              static_cast<float *>(w32.p), w32.st, w32.part_vec, s);
        r.phase = 1;
    }
    // 5. launch the next round for every request in its inner solve (the
    // tables rebuilt when the member set changed), with the gather of all
    // members' states at its end; it runs while the caller goes on
    std::vector<Mesh *> inner;
    std::vector<uint64_t> inner_uids;
    for (ServerReq &r : sv.reqs)
        if (r.phase == 1) {
            inner.push_back(r.m);
            inner_uids.push_back(r.uid);
        }
    if (!inner.empty()) {
        if (inner_uids != sv.batch_uids || sv.batch.shape_gen != ax_shape_generation()) {
            sv.batch.rebuild(inner);
            sv.batch_uids = inner_uids;
        }
        for (int c = 0; c < sv.round_iters; ++c) sv.batch.enqueue_iteration(otf, s);
        sv.batch.enqueue_read_states();
        SEM_HIP(hipEventRecord(sv.ev_round, s));
        sv.round_uids = inner_uids;
        sv.round_in_flight = true;
    }
    // the finished requests' x copies (and the set-up of new ones) are done
    SEM_HIP(hipStreamSynchronize(s2));
    return (int)sv.reqs.size();
}

}  // namespace sem
