// sem_cg.cpp -- the CG driver (Algorithm 1) and the mixed-precision
// refinement built on it.
//
// One CG iteration is three kernels:
//   1. p <- r + beta p fused with w <- A_L p and the block partials of
//      <p, w, c> (Algorithm 1: p-update and operator steps); the same pass
//      applies the previous iteration's x += alpha p while p_old is at hand;
//   2. w <- QQ^T w on the shared points, and one block forms
//      alpha = rho / <p, w, c>;
//   3. r -= alpha mask(w) and the partials of rho = <r, r, c>, then a
//      one-block kernel forms beta and runs the convergence test.
// After the last iteration a flush applies the pending x += alpha p.
// With the Jacobi preconditioner step 3 also writes z = M^-1 r and reduces
// <r, z, c> (which drives beta) beside <r, r, c> (the stopping test), and
// step 1 forms p from z.
// When every shared point lies on an element's surface (any conforming
// mesh), step 2 only writes the sums of the groups of more than two copies
// (edge and vertex nodes) to a compact array, and step 3 forms (QQ^T w)_l
// itself: a face node adds its partner's w, an edge or vertex node takes its
// group's sum.  The summed w is never written back, and the results are
// bitwise those of the three-pass form.
// The CG scalars never leave the device.  Iterations are enqueued in chunks
// (replayed HIP graphs by default); after each chunk the host reads the
// state once.  Kernels of iterations past convergence exit at their first
// instruction.
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>

#include "sem_cg_internal.h"

namespace sem {

namespace {

void ws_free(Workspace *ws) {
    if (!ws) return;
    for (auto &kv : ws->graphs) (void)hipGraphExecDestroy(kv.second);
    void *dev[] = {ws->x,       ws->r,        ws->p,  ws->w,    ws->b,   ws->gsum,
                   ws->wedge,   ws->part_ax,  ws->part_vec, ws->z, ws->part_vec2, ws->st,
                   ws->hist,    ws->dval};
    for (void *q : dev)
        if (q) (void)hipFree(q);
    if (ws->h_st) (void)hipHostFree(ws->h_st);
    if (ws->h_val) (void)hipHostFree(ws->h_val);
    if (ws->ev) (void)hipEventDestroy(ws->ev);
    for (hipEvent_t e : ws->tev) (void)hipEventDestroy(e);
    if (ws->stream) (void)hipStreamDestroy(ws->stream);
    delete ws;
}

template <typename T>
T *ws_alloc(Workspace &ws, size_t count) {
    void *q = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    if (hipMalloc(&q, bytes) != hipSuccess) {
        (void)hipGetLastError();
        fail(SEM_ENOMEM, "workspace allocation of " + std::to_string(bytes) + " bytes failed");
    }
    ws.bytes += bytes;
    return static_cast<T *>(q);
}

Workspace *ws_create(const Mesh &m, bool fp64) {
    Workspace *ws = new Workspace();
    try {
        ws->fp64 = fp64;
        ws->n = m.n;
        ws->device = m.device;
        const size_t tsz = fp64 ? 8 : 4;
        const size_t nv = (size_t)m.n * tsz;
        ws->x = ws_alloc<char>(*ws, nv);
        ws->r = ws_alloc<char>(*ws, nv);
        ws->p = ws_alloc<char>(*ws, nv);
        // table-free gather: the edge-group sums sit right after w
        ws->w = ws_alloc<char>(*ws, nv + (m.gs_struct ? (size_t)m.n_egroups * tsz : 0));
        ws->b = ws_alloc<char>(*ws, nv);
        if (m.gs_in_update)
            ws->gsum = ws_alloc<char>(*ws, (size_t)m.n_groups_multi * tsz);
        if (m.gsum_wedge || m.gs_struct)
            ws->wedge = ws_alloc<char>(*ws, (size_t)m.E * edge_slots(m.N) * tsz);
        // the smallest shape (1 element per block) bounds the Ax partial count
        ws->cap_ax = m.E;
        ws->cap_vec = vec_blocks(m.n);
        ws->part_ax = ws_alloc<double>(*ws, ws->cap_ax);
        ws->part_vec = ws_alloc<double>(*ws, ws->cap_vec);
        ws->st = ws_alloc<CgState>(*ws, 1);
        ws->dval = ws_alloc<double>(*ws, 8);
        SEM_HIP(hipHostMalloc((void **)&ws->h_st, sizeof(CgState)));
        SEM_HIP(hipHostMalloc((void **)&ws->h_val, 8 * sizeof(double)));
        SEM_HIP(hipStreamCreateWithFlags(&ws->stream, hipStreamNonBlocking));
        SEM_HIP(hipEventCreateWithFlags(&ws->ev, hipEventDisableTiming));
        SEM_HIP(hipMemset(ws->st, 0, sizeof(CgState)));
    } catch (...) {
        ws_free(ws);
        throw;
    }
    return ws;
}

Workspace &get_ws(Mesh &m, bool fp64) {
    Workspace *&slot = fp64 ? m.ws64 : m.ws32;
    if (!slot) slot = ws_create(m, fp64);
    return *slot;
}

// Jacobi preconditioner of the mesh (both precisions) and the workspace's
// z vector and second partial set, built on first use.  M = diag(Q^T A_L Q):
// element diagonals from the FP64 geometry, summed over the copies of each
// global point by the gather-scatter; minv = 1/M on the free points.
void ensure_jacobi(Mesh &m, Workspace &ws) {
    if (!m.minv64) {
        hipStream_t s = ws.stream;
        double *d = nullptr, *m64 = nullptr;
        float *m32 = nullptr;
        auto alloc = [&](void **q, size_t bytes) {
            if (hipMalloc(q, bytes) != hipSuccess) {
                (void)hipGetLastError();
                if (d) (void)hipFree(d);
                if (m64) (void)hipFree(m64);
                fail(SEM_ENOMEM, "Jacobi preconditioner allocation failed");
            }
        };
        alloc((void **)&d, sizeof(double) * m.n);
        alloc((void **)&m64, sizeof(double) * m.n);
        alloc((void **)&m32, sizeof(float) * m.n);
        launch_diag_local(m, d, s);
        launch_gs<double>(m, d, s);
        launch_jacobi_invert(m, d, m64, m32, s);
        const hipError_t e = hipStreamSynchronize(s);
        (void)hipFree(d);
        if (e != hipSuccess) {
            (void)hipFree(m64);
            (void)hipFree(m32);
            check_hip(e, "Jacobi preconditioner setup");
        }
        m.minv64 = m64;
        m.minv32 = m32;
        m.device_bytes += 12 * (size_t)m.n;
    }
    if (!ws.z) {
        ws.z = ws_alloc<char>(ws, (size_t)m.n * (ws.fp64 ? 8 : 4));
        ws.part_vec2 = ws_alloc<double>(ws, ws.cap_vec);
    }
}

template <typename T>
PcArgs<T> pc_args(const Mesh &m, Workspace &ws, bool pc) {
    PcArgs<T> a{};
    if (!pc) return a;
    if constexpr (sizeof(T) == 8) a.minv = m.minv64;
    else a.minv = m.minv32;
    a.z = static_cast<T *>(ws.z);
    a.partial2 = ws.part_vec2;
    return a;
}

void ensure_hist(Workspace &ws, int len) {
    if (len <= ws.hist_cap) return;
    if (ws.hist) {
        // histories are captured by pointer in no graph (read from the state)
        SEM_HIP(hipStreamSynchronize(ws.stream));
        (void)hipFree(ws.hist);
        ws.hist = nullptr;
        ws.hist_cap = 0;
    }
    ws.hist = ws_alloc<double>(ws, 2 * (size_t)len);
    ws.hist_cap = len;
}

// ---------------------------------------------------------------------------
// one CG iteration (three steps) on stream s; ev (may be null): events
// recorded before and after each step
// ---------------------------------------------------------------------------
template <typename T>
void enqueue_iteration(const Mesh &m, Workspace &ws, bool otf, bool pc, hipStream_t s,
                       hipEvent_t *ev = nullptr) {
    T *x = static_cast<T *>(ws.x), *r = static_cast<T *>(ws.r);
    T *p = static_cast<T *>(ws.p), *w = static_cast<T *>(ws.w);
    T *gsum = static_cast<T *>(ws.gsum), *wedge = static_cast<T *>(ws.wedge);
    const PcArgs<T> pa = pc_args<T>(m, ws, pc);
    AxArgs<T> a{};
    a.u = pc ? pa.z : r;
    a.p = p;
    a.w = w;
    a.st = ws.st;
    a.partial = ws.part_ax;
    a.wedge = (m.gsum_wedge || m.gs_struct_solo) ? wedge : nullptr;
    a.x = x;
    a.stream = ((sizeof(T) == 4 || otf) &&
                cg_streams_vectors(cg_footprint(m, (int)sizeof(T), m.gs_struct_solo)))
                   ? 1
                   : 0;
    if (ev) SEM_HIP(hipEventRecord(ev[0], s));
    launch_ax<T>(m, otf, AxMode::CgFused, a, s);
    if (ev) SEM_HIP(hipEventRecord(ev[1], s));
    const int64_t nax = ax_blocks(m, sizeof(T) == 8, otf, 0);
    if (m.gs_struct_solo)
        launch_edge_sums_cg<T>(m, wedge, w + m.n, ws.st, ws.part_ax, (int)nax, s);
    else if (m.gs_in_update)
        launch_group_sums_cg<T>(m, w, wedge, gsum, ws.st, ws.part_ax, (int)nax, s);
    else launch_gs_cg<T>(m, w, ws.st, ws.part_ax, (int)nax, s);
    if (ev) SEM_HIP(hipEventRecord(ev[2], s));
    if (m.gs_struct_solo) launch_update_struct<T>(m, r, w, ws.st, ws.part_vec, s, pa);
    else if (m.gs_in_update) launch_update_gather<T>(m, r, w, gsum, ws.st, ws.part_vec, s, pa);
    else launch_update<T>(m, r, w, ws.st, ws.part_vec, s, pa);
    if (ev) SEM_HIP(hipEventRecord(ev[3], s));
}

struct KernelTimes {
    double ms[3] = {0, 0, 0};
    long count = 0;
};

template <typename T>
void run_chunk_timed(const Mesh &m, Workspace &ws, bool otf, bool pc, int chunk,
                     int iter_before, KernelTimes &kt) {
    hipStream_t s = ws.stream;
    while ((int)ws.tev.size() < 4 * chunk) {
        hipEvent_t e = nullptr;
        SEM_HIP(hipEventCreate(&e));
        ws.tev.push_back(e);
    }
    for (int c = 0; c < chunk; ++c) enqueue_iteration<T>(m, ws, otf, pc, s, &ws.tev[4 * c]);
    SEM_HIP(hipMemcpyAsync(ws.h_st, ws.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
    const int done = std::min(chunk, ws.h_st->iter - iter_before);
    for (int c = 0; c < done; ++c)
        for (int k = 0; k < 3; ++k) {
            float ms = 0.f;
            SEM_HIP(hipEventElapsedTime(&ms, ws.tev[4 * c + k], ws.tev[4 * c + k + 1]));
            kt.ms[k] += ms;
        }
    kt.count += done;
}

template <typename T>
void run_chunk(const Mesh &m, Workspace &ws, bool otf, bool pc, int chunk, bool use_graph) {
    hipStream_t s = ws.stream;
    if (!use_graph) {
        for (int c = 0; c < chunk; ++c) enqueue_iteration<T>(m, ws, otf, pc, s);
        return;
    }
    const GraphKey key{otf, chunk, ax_shape_generation(), pc};
    auto it = ws.graphs.find(key);
    if (it == ws.graphs.end()) {
        hipGraph_t g = nullptr;
        SEM_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        try {
            for (int c = 0; c < chunk; ++c) enqueue_iteration<T>(m, ws, otf, pc, s);
        } catch (...) {
            hipGraph_t junk = nullptr;
            (void)hipStreamEndCapture(s, &junk);
            if (junk) (void)hipGraphDestroy(junk);
            throw;
        }
        SEM_HIP(hipStreamEndCapture(s, &g));
        hipGraphExec_t ge = nullptr;
        hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        check_hip(e, "hipGraphInstantiate");
        it = ws.graphs.emplace(key, ge).first;
    }
    SEM_HIP(hipGraphLaunch(it->second, s));
}

int auto_chunk(int64_t n, int fixed) {
    int c = n < (1 << 20) ? 32 : (n < (1 << 23) ? 16 : 8);
    if (fixed > 0) c = std::min(std::max(fixed, 1), 50);
    return c;
}

// FP64 operator w = mask(QQ^T A_L u): precomputed G64 if present, else on the fly
void apply_A64(const Mesh &m, const double *u, double *w, hipStream_t s) {
    AxArgs<double> a{};
    a.u = u;
    a.w = w;
    launch_ax<double>(m, m.G64 == nullptr, AxMode::Plain, a, s);
    launch_gs<double>(m, w, s);
    launch_mask<double>(m, w, s);
}

template <typename T>
void apply_A(const Mesh &m, bool otf, const T *u, T *w, hipStream_t s) {
    AxArgs<T> a{};
    a.u = u;
    a.w = w;
    launch_ax<T>(m, otf, AxMode::Plain, a, s);
    launch_gs<T>(m, w, s);
    launch_mask<T>(m, w, s);
}

struct InnerOut {
    int iters;
    int stop;
    double rel;
};

// Runs Algorithm 1 on ws (x, r, p, w) for right-hand side b_dev (device, T).
// x0_zero: the initial guess is zero (r0 = b, no operator application).
// pc: Jacobi-preconditioned (ensure_jacobi has run for m and ws).
template <typename T>
InnerOut cg_core(const Mesh &m, Workspace &ws, const T *b_dev, bool x0_zero, bool otf, bool pc,
                 double tol, int max_iter, int fixed, int chunk, bool use_graph, int hist_len,
                 KernelTimes *kt = nullptr) {
    hipStream_t s = ws.stream;
    CgState h{};
    h.thresh = tol * tol;
    h.max_iter = fixed > 0 ? fixed : max_iter;
    h.fixed = fixed > 0 ? 1 : 0;
    if (hist_len > 0) {
        ensure_hist(ws, hist_len);
        h.hist_len = hist_len;
        h.hist_rho = ws.hist;
        h.hist_alpha = ws.hist + ws.hist_cap;
    }
    SEM_HIP(hipStreamSynchronize(s));   // h_st may still be the target of a copy
    *ws.h_st = h;
    SEM_HIP(hipMemcpyAsync(ws.st, ws.h_st, sizeof(CgState), hipMemcpyHostToDevice, s));
    T *x = static_cast<T *>(ws.x), *r = static_cast<T *>(ws.r);
    T *p = static_cast<T *>(ws.p), *w = static_cast<T *>(ws.w);
    const PcArgs<T> pa = pc_args<T>(m, ws, pc);
    if (x0_zero) {
        SEM_HIP(hipMemsetAsync(x, 0, sizeof(T) * m.n, s));
        launch_cg_init<T>(m, b_dev, nullptr, r, p, ws.st, ws.part_vec, s, pa);
    } else {
        launch_mask<T>(m, x, s);
        apply_A<T>(m, otf, x, w, s);
        launch_cg_init<T>(m, b_dev, w, r, p, ws.st, ws.part_vec, s, pa);
    }
    // every chunk advances the iteration count by `chunk` until the state
    // stops; a chunk that does not advance it means the device state is
    // inconsistent, which ends the loop with an error instead of spinning
    int last_iter = -1;
    for (;;) {
        SEM_HIP(hipMemcpyAsync(ws.h_st, ws.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
        SEM_HIP(hipStreamSynchronize(s));
        if (ws.h_st->stop) break;
        if (ws.h_st->iter <= last_iter)
            fail(SEM_EDEVICE, "CG state did not advance (iteration " +
                                  std::to_string(ws.h_st->iter) + ")");
        last_iter = ws.h_st->iter;
        if (kt) run_chunk_timed<T>(m, ws, otf, pc, chunk, last_iter, *kt);
        else run_chunk<T>(m, ws, otf, pc, chunk, use_graph);
    }
    // the last completed iteration's x step
    launch_x_flush<T>(m, x, p, ws.st, s);
    InnerOut o;
    o.iters = ws.h_st->iter;
    o.stop = ws.h_st->stop;
    o.rel = ws.h_st->rho0 > 0 ? std::sqrt(ws.h_st->rr / ws.h_st->rho0) : 0.0;
    return o;
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

void copy_hist(Workspace &ws, const sem_cg_opts &o, int iters) {
    if (o.hist_len <= 0) return;
    const int cnt = std::min(o.hist_len, iters + 1);
    if (o.hist_rho)
        SEM_HIP(hipMemcpy(o.hist_rho, ws.hist, cnt * sizeof(double), hipMemcpyDeviceToHost));
    if (o.hist_alpha)
        SEM_HIP(hipMemcpy(o.hist_alpha, ws.hist + ws.hist_cap, cnt * sizeof(double),
                          hipMemcpyDeviceToHost));
}

// FP64 true relative residual ||b - A x||_c / ||b||_c of device vectors
// (b64, x64 double); uses ws64 r/w as scratch.
double true_residual64(Mesh &m, const double *b64, const double *x64, Workspace &w64) {
    hipStream_t s = w64.stream;
    double *r = static_cast<double *>(w64.r), *wv = static_cast<double *>(w64.w);
    apply_A64(m, x64, wv, s);
    launch_residual64(m, b64, wv, r, w64.dval + 0, w64.part_vec, s);
    launch_dot<double>(m, b64, b64, w64.dval + 1, w64.part_vec, s);
    SEM_HIP(hipMemcpyAsync(w64.h_val, w64.dval, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
    const double rr = w64.h_val[0], bb = w64.h_val[1];
    return bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
}

}  // namespace

void destroy_workspaces(Mesh *m) {
    ws_free(m->ws32);
    ws_free(m->ws64);
    m->ws32 = m->ws64 = nullptr;
}

// ---------------------------------------------------------------------------
// entry: plain FP32 / FP64 CG
// ---------------------------------------------------------------------------
template <typename T>
static sem_status cg_plain(Mesh &m, const sem_cg_opts &o, const void *b_user, void *x_user,
                           sem_cg_result &res, hipStream_t user_s) {
    const bool fp64 = sizeof(T) == 8;
    const bool otf = o.geom == SEM_G_ON_THE_FLY;
    if (!otf && (fp64 ? m.G64 == nullptr : m.G32 == nullptr))
        fail(SEM_EUNSUPPORTED, "precomputed G of this precision was not built for the mesh");
    Workspace &ws = get_ws(m, fp64);
    const bool pc = o.precond == SEM_PRECOND_JACOBI;
    if (pc) ensure_jacobi(m, ws);
    SEM_HIP(hipEventRecord(ws.ev, user_s));
    SEM_HIP(hipStreamWaitEvent(ws.stream, ws.ev, 0));
    const T *b = static_cast<const T *>(b_user);
    SEM_HIP(hipMemcpyAsync(ws.x, x_user, sizeof(T) * m.n, hipMemcpyDeviceToDevice, ws.stream));
    const int chunk = o.poll_every > 0 ? o.poll_every : auto_chunk(m.n, o.fixed_iters);
    const int hist_len = (o.hist_rho || o.hist_alpha) ? o.hist_len : 0;
    KernelTimes kt;
    InnerOut io = cg_core<T>(m, ws, b, false, otf, pc, o.tol, o.max_iter, o.fixed_iters, chunk,
                             o.use_graph != 0, hist_len, o.kernel_ms ? &kt : nullptr);
    if (o.kernel_ms)
        for (int k = 0; k < 3; ++k) o.kernel_ms[k] = kt.count ? kt.ms[k] / kt.count : 0.0;
    SEM_HIP(hipMemcpyAsync(x_user, ws.x, sizeof(T) * m.n, hipMemcpyDeviceToDevice, ws.stream));
    SEM_HIP(hipStreamSynchronize(ws.stream));
    copy_hist(ws, o, io.iters);
    res.iters = io.iters;
    res.outer = 0;
    res.status = io.stop;
    res.converged = io.stop == 1 ? 1 : 0;
    res.rel_res_recursive = io.rel;
    res.rel_res_true = -1.0;
    if (o.true_residual) {
        Workspace &w64 = get_ws(m, true);
        double *b64 = static_cast<double *>(w64.b), *x64 = static_cast<double *>(w64.x);
        SEM_HIP(hipStreamSynchronize(ws.stream));
        launch_convert<T, double>(m.n, b, b64, w64.stream);
        launch_convert<T, double>(m.n, static_cast<const T *>(x_user), x64, w64.stream);
        res.rel_res_true = true_residual64(m, b64, x64, w64);
    }
    return io.stop == 3 ? SEM_EBREAKDOWN : SEM_OK;
}

// ---------------------------------------------------------------------------
// entry: mixed precision (FP32 inner CG, FP64 outer residual)
// ---------------------------------------------------------------------------
static sem_status cg_mixed(Mesh &m, const sem_cg_opts &o, const double *b, double *x_user,
                           sem_cg_result &res, hipStream_t user_s) {
    const bool otf = o.geom == SEM_G_ON_THE_FLY;
    if (!otf && m.G32 == nullptr)
        fail(SEM_EUNSUPPORTED, "precomputed FP32 G was not built for the mesh");
    Workspace &w64 = get_ws(m, true);
    Workspace &w32 = get_ws(m, false);
    const bool pc = o.precond == SEM_PRECOND_JACOBI;
    if (pc) ensure_jacobi(m, w32);
    SEM_HIP(hipEventRecord(w64.ev, user_s));
    SEM_HIP(hipStreamWaitEvent(w64.stream, w64.ev, 0));
    hipStream_t s = w64.stream;
    double *x64 = static_cast<double *>(w64.x), *r64 = static_cast<double *>(w64.r);
    double *t64 = static_cast<double *>(w64.w);
    SEM_HIP(hipMemcpyAsync(x64, x_user, sizeof(double) * m.n, hipMemcpyDeviceToDevice, s));
    launch_mask<double>(m, x64, s);
    launch_dot<double>(m, b, b, w64.dval + 1, w64.part_vec, s);
    const double inner_tol = o.inner_tol > 0 ? o.inner_tol : 1e-5;
    const int max_outer = o.max_outer > 0 ? o.max_outer : 20;
    const int chunk = o.poll_every > 0 ? o.poll_every : auto_chunk(m.n, 0);
    const int inner_cap = o.max_iter > 0 ? o.max_iter : 100000;
    int total = 0, outer = 0, last_stop = 0;
    double rel = 0.0, last_inner_rel = 0.0;
    KernelTimes kt;
    bool converged = false, breakdown = false;
    for (;;) {
        apply_A64(m, x64, t64, s);
        launch_residual64(m, b, t64, r64, w64.dval + 0, w64.part_vec, s);
        SEM_HIP(hipMemcpyAsync(w64.h_val, w64.dval, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        SEM_HIP(hipStreamSynchronize(s));
        const double rr = w64.h_val[0], bb = w64.h_val[1];
        rel = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
        if (!std::isfinite(rel)) {
            breakdown = true;
            break;
        }
        if (rel <= o.tol || rr == 0.0) {
            converged = true;
            break;
        }
        if (outer >= max_outer) break;
        // inner FP32 solve of A d = r / ||r||_c  (x0 = 0)
        float *b32 = static_cast<float *>(w32.b);
        launch_scale_to_f32(m.n, r64, w64.dval + 0, b32, s);
        SEM_HIP(hipEventRecord(w64.ev, s));
        SEM_HIP(hipStreamWaitEvent(w32.stream, w64.ev, 0));
        InnerOut io = cg_core<float>(m, w32, b32, true, otf, pc,
                                     refine_inner_tol(inner_tol, o.tol, rel), inner_cap, 0, chunk,
                                     o.use_graph != 0, 0, o.kernel_ms ? &kt : nullptr);
        total += io.iters;
        last_stop = io.stop;
        last_inner_rel = io.rel;
        SEM_HIP(hipEventRecord(w32.ev, w32.stream));
        SEM_HIP(hipStreamWaitEvent(s, w32.ev, 0));
        if (io.stop == 3) {
            breakdown = true;
            break;
        }
        launch_axpy_from_f32(m.n, x64, w64.dval + 0, static_cast<const float *>(w32.x), s);
        ++outer;
    }
    SEM_HIP(hipMemcpyAsync(x_user, x64, sizeof(double) * m.n, hipMemcpyDeviceToDevice, s));
    SEM_HIP(hipStreamSynchronize(s));
    if (o.kernel_ms)
        for (int k = 0; k < 3; ++k) o.kernel_ms[k] = kt.count ? kt.ms[k] / kt.count : 0.0;
    res.iters = total;
    res.outer = outer;
    res.converged = converged ? 1 : 0;
    res.status = converged ? 1 : (breakdown ? 3 : (last_stop ? last_stop : 2));
    res.rel_res_recursive = last_inner_rel;
    res.rel_res_true = rel;
    return breakdown ? SEM_EBREAKDOWN : SEM_OK;
}

sem_status cg_solve(Mesh &m, const sem_cg_opts &o, const void *b, void *x, sem_cg_result &res,
                    hipStream_t user_s) {
    const double t0 = now_s();
    sem_status st;
    switch (o.prec) {
        case SEM_FP32: st = cg_plain<float>(m, o, b, x, res, user_s); break;
        case SEM_FP64: st = cg_plain<double>(m, o, b, x, res, user_s); break;
        case SEM_MIXED:
            st = cg_mixed(m, o, static_cast<const double *>(b), static_cast<double *>(x), res,
                          user_s);
            break;
        default: fail(SEM_EINVAL, "unknown precision");
    }
    res.seconds = now_s() - t0;
    return st;
}

// FP64 operator and helpers for the API layer and the batched driver
void api_apply_A64(const Mesh &m, const double *u, double *w, hipStream_t s) {
    apply_A64(m, u, w, s);
}
Workspace &cg_workspace(Mesh &m, bool fp64) { return get_ws(m, fp64); }
size_t workspace_bytes(const Mesh &m) {
    return (m.ws32 ? m.ws32->bytes : 0) + (m.ws64 ? m.ws64->bytes : 0);
}
int cg_auto_chunk(int64_t n, int fixed) { return auto_chunk(n, fixed); }

}  // namespace sem
