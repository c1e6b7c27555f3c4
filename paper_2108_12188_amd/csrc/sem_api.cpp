// sem_api.cpp -- the extern "C" boundary: argument checks, error codes and
// the thread-local error message.  No C++ exception crosses it.
#include <cstring>
#include <exception>
#include <new>
#include <string>

#include "sem_internal.h"

namespace sem {

namespace {
thread_local std::string g_last_error;

struct SemException {
    sem_status code;
    std::string msg;
};
}  // namespace

void set_error(const std::string &msg) { g_last_error = msg; }

[[noreturn]] void fail(sem_status code, const std::string &msg) { throw SemException{code, msg}; }

void check_hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return;
    (void)hipGetLastError();
    const sem_status code = (e == hipErrorOutOfMemory) ? SEM_ENOMEM : SEM_EDEVICE;
    fail(code, std::string(what) + ": " + hipGetErrorString(e));
}

Mesh *as_mesh(sem_mesh_t m) {
    if (!m) fail(SEM_EINVAL, "NULL mesh handle");
    return reinterpret_cast<Mesh *>(m);
}

Mesh *mesh_create(int64_t E, int N, const double *vert, const int64_t *gid, const uint8_t *dir,
                  uint32_t flags, hipStream_t s);
void element_order(int64_t E, const double *vert, int kind, int64_t *perm);
void mesh_destroy(Mesh *m);
sem_status cg_solve(Mesh &m, const sem_cg_opts &o, const void *b, void *x, sem_cg_result &res,
                    hipStream_t s);
void api_apply_A64(const Mesh &m, const double *u, double *w, hipStream_t s);
struct BatchImpl;
BatchImpl *batch_new(int count, const sem_mesh_t *meshes);
void batch_delete(BatchImpl *b);
sem_status batch_solve(BatchImpl &B, const sem_cg_opts &o, const void *const *b_dev,
                       void *const *x_dev, sem_cg_result *res, hipStream_t user_s);
struct ServerImpl;
ServerImpl *server_new(const sem_cg_opts &o, int round_iters);
void server_delete(ServerImpl *sv);
void server_add(ServerImpl &sv, Mesh *m, const double *b, double *x, int64_t tag,
                hipStream_t user_s);
int server_step(ServerImpl &sv, int64_t *tags, sem_cg_result *results, int cap, int *n_done);
size_t mesh_footprint(int64_t E, int N, uint32_t flags, sem_precision prec);
size_t workspace_bytes(const Mesh &m);

template <typename F>
static sem_status guarded(F &&f) {
    try {
        g_last_error.clear();
        return f();
    } catch (const SemException &e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return SEM_ENOMEM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return SEM_EDEVICE;
    } catch (...) {
        g_last_error = "unknown error";
        return SEM_EDEVICE;
    }
}

static void need(const void *p, const char *name) {
    if (!p) fail(SEM_EINVAL, std::string(name) + " must not be NULL");
}

// Runs device work on the mesh's device and restores the caller's device.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) check_hip(hipSetDevice(dev), "hipSetDevice");
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace sem

using namespace sem;

extern "C" {

sem_status sem_element_order(int64_t n_elem, const double *vert_xyz, int kind, int64_t *perm) {
    return guarded([&]() -> sem_status {
        element_order(n_elem, vert_xyz, kind, perm);
        return SEM_OK;
    });
}

sem_status sem_mesh_create(int64_t n_elem, int order_N, const double *vert_xyz,
                           const int64_t *glob_id, const uint8_t *dirichlet, uint32_t flags,
                           void *hip_stream, sem_mesh_t *out) {
    return guarded([&]() -> sem_status {
        need(out, "out");
        Mesh *m = mesh_create(n_elem, order_N, vert_xyz, glob_id, dirichlet, flags,
                              static_cast<hipStream_t>(hip_stream));
        *out = reinterpret_cast<sem_mesh_t>(m);
        return SEM_OK;
    });
}

void sem_mesh_destroy(sem_mesh_t mesh) {
    if (!mesh) return;
    mesh_destroy(reinterpret_cast<Mesh *>(mesh));
}

sem_status sem_mesh_info(sem_mesh_t mesh, sem_mesh_info_t *info) {
    return guarded([&]() -> sem_status {
        Mesh *m = as_mesh(mesh);
        need(info, "info");
        info->n_elem = m->E;
        info->order_N = m->N;
        info->n_local = m->n;
        info->n_glob = m->n_glob;
        info->n_shared = m->n_shared;
        info->n_groups = m->n_groups;
        info->n_dirichlet = m->n_dir;
        info->device_bytes = m->device_bytes + workspace_bytes(*m);
        info->gs_in_update = m->gs_in_update ? 1 : 0;
        info->gs_table_free = m->gs_struct_solo ? 1 : 0;
        return SEM_OK;
    });
}

static void check_prec(sem_precision prec) {
    if (prec != SEM_FP32 && prec != SEM_FP64) fail(SEM_EINVAL, "precision must be FP32 or FP64");
}

sem_status sem_ax(sem_mesh_t mesh, sem_precision prec, sem_geom geom, const void *u_dev,
                  void *w_dev, void *hip_stream) {
    return guarded([&]() -> sem_status {
        Mesh *m = as_mesh(mesh);
        need(u_dev, "u_dev");
        need(w_dev, "w_dev");
        check_prec(prec);
        if (geom != SEM_G_PRECOMPUTED && geom != SEM_G_ON_THE_FLY)
            fail(SEM_EINVAL, "unknown geometry form");
        if (u_dev == w_dev) fail(SEM_EINVAL, "u and w must not overlap");
        const bool otf = geom == SEM_G_ON_THE_FLY;
        DeviceGuard dg(m->device);
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        if (prec == SEM_FP32) {
            if (!otf && !m->G32) fail(SEM_EUNSUPPORTED, "mesh has no FP32 precomputed G");
            AxArgs<float> a{};
            a.u = static_cast<const float *>(u_dev);
            a.w = static_cast<float *>(w_dev);
            launch_ax<float>(*m, otf, AxMode::Plain, a, s);
        } else {
            if (!otf && !m->G64) fail(SEM_EUNSUPPORTED, "mesh has no FP64 precomputed G");
            AxArgs<double> a{};
            a.u = static_cast<const double *>(u_dev);
            a.w = static_cast<double *>(w_dev);
            launch_ax<double>(*m, otf, AxMode::Plain, a, s);
        }
        return SEM_OK;
    });
}

sem_status sem_gs(sem_mesh_t mesh, sem_precision prec, void *w_dev, int apply_mask,
                  void *hip_stream) {
    return guarded([&]() -> sem_status {
        Mesh *m = as_mesh(mesh);
        need(w_dev, "w_dev");
        check_prec(prec);
        DeviceGuard dg(m->device);
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        if (prec == SEM_FP32) {
            launch_gs<float>(*m, static_cast<float *>(w_dev), s);
            if (apply_mask) launch_mask<float>(*m, static_cast<float *>(w_dev), s);
        } else {
            launch_gs<double>(*m, static_cast<double *>(w_dev), s);
            if (apply_mask) launch_mask<double>(*m, static_cast<double *>(w_dev), s);
        }
        return SEM_OK;
    });
}

sem_status sem_dot(sem_mesh_t mesh, sem_precision prec, const void *a_dev, const void *b_dev,
                   double *out_dev, void *hip_stream) {
    return guarded([&]() -> sem_status {
        Mesh *m = as_mesh(mesh);
        need(a_dev, "a_dev");
        need(b_dev, "b_dev");
        need(out_dev, "out_dev");
        check_prec(prec);
        DeviceGuard dg(m->device);
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        if (prec == SEM_FP32)
            launch_dot<float>(*m, static_cast<const float *>(a_dev),
                              static_cast<const float *>(b_dev), out_dev, m->scratch, s);
        else
            launch_dot<double>(*m, static_cast<const double *>(a_dev),
                               static_cast<const double *>(b_dev), out_dev, m->scratch, s);
        return SEM_OK;
    });
}

sem_status sem_dot_noalloc(sem_mesh_t mesh, sem_precision prec, const void *a_dev,
                           const void *b_dev, double *out_dev, void *hip_stream) {
    return guarded([&]() -> sem_status {
        Mesh *m = as_mesh(mesh);
        need(a_dev, "a_dev");
        need(b_dev, "b_dev");
        need(out_dev, "out_dev");
        check_prec(prec);
        DeviceGuard dg(m->device);
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        if (prec == SEM_FP32)
            launch_dot_noalloc<float>(*m, static_cast<const float *>(a_dev),
                                      static_cast<const float *>(b_dev), out_dev, s);
        else
            launch_dot_noalloc<double>(*m, static_cast<const double *>(a_dev),
                                       static_cast<const double *>(b_dev), out_dev, s);
        return SEM_OK;
    });
}

sem_status sem_diag(sem_mesh_t mesh, double *diag_dev, void *hip_stream) {
    return guarded([&]() -> sem_status {
        Mesh *m = as_mesh(mesh);
        need(diag_dev, "diag_dev");
        DeviceGuard dg(m->device);
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        launch_diag_local(*m, diag_dev, s);
        launch_gs<double>(*m, diag_dev, s);
        return SEM_OK;
    });
}

sem_status sem_coords(sem_mesh_t mesh, double *xyz_dev, void *hip_stream) {
    return guarded([&]() -> sem_status {
        Mesh *m = as_mesh(mesh);
        need(xyz_dev, "xyz_dev");
        DeviceGuard dg(m->device);
        launch_coords(*m, xyz_dev, static_cast<hipStream_t>(hip_stream));
        return SEM_OK;
    });
}

sem_status sem_rhs(sem_mesh_t mesh, sem_precision prec, const double *f_dev, void *b_dev,
                   void *hip_stream) {
    return guarded([&]() -> sem_status {
        Mesh *m = as_mesh(mesh);
        need(f_dev, "f_dev");
        need(b_dev, "b_dev");
        if (prec != SEM_FP32 && prec != SEM_FP64 && prec != SEM_MIXED)
            fail(SEM_EINVAL, "unknown precision");
        DeviceGuard dg(m->device);
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        if (prec == SEM_FP32) {
            double *tmp = nullptr;
            SEM_HIP(hipMalloc(&tmp, sizeof(double) * m->n));
            launch_mul64(m->n, m->B64, f_dev, tmp, s);
            launch_gs<double>(*m, tmp, s);
            launch_mask<double>(*m, tmp, s);
            launch_convert<double, float>(m->n, tmp, static_cast<float *>(b_dev), s);
            const hipError_t e = hipStreamSynchronize(s);
            (void)hipFree(tmp);
            check_hip(e, "rhs");
        } else {
            double *b = static_cast<double *>(b_dev);
            launch_mul64(m->n, m->B64, f_dev, b, s);
            launch_gs<double>(*m, b, s);
            launch_mask<double>(*m, b, s);
        }
        return SEM_OK;
    });
}

sem_status sem_cg_solve(sem_mesh_t mesh, const sem_cg_opts *opts, const void *b_dev, void *x_dev,
                        sem_cg_result *result, void *hip_stream) {
    return guarded([&]() -> sem_status {
        Mesh *m = as_mesh(mesh);
        need(opts, "opts");
        need(b_dev, "b_dev");
        need(x_dev, "x_dev");
        need(result, "result");
        if (opts->fixed_iters <= 0 && !(opts->tol > 0.0))
            fail(SEM_EINVAL, "tol must be positive unless fixed_iters > 0");
        if (opts->fixed_iters <= 0 && opts->max_iter <= 0 && opts->prec != SEM_MIXED)
            fail(SEM_EINVAL, "max_iter must be positive");
        if (opts->geom != SEM_G_PRECOMPUTED && opts->geom != SEM_G_ON_THE_FLY)
            fail(SEM_EINVAL, "unknown geometry form");
        if (opts->hist_len < 0 || ((opts->hist_rho || opts->hist_alpha) && opts->hist_len == 0))
            fail(SEM_EINVAL, "history buffers need hist_len > 0");
        if (opts->precond != SEM_PRECOND_NONE && opts->precond != SEM_PRECOND_JACOBI)
            fail(SEM_EINVAL, "unknown preconditioner");
        DeviceGuard dg(m->device);
        sem_cg_result r{};
        const sem_status st =
            cg_solve(*m, *opts, b_dev, x_dev, r, static_cast<hipStream_t>(hip_stream));
        *result = r;
        if (st == SEM_EBREAKDOWN) set_error("CG breakdown: <p, w, c> <= 0 or a non-finite scalar");
        return st;
    });
}

sem_status sem_batch_create(int count, const sem_mesh_t *meshes, sem_batch_t *out) {
    return guarded([&]() -> sem_status {
        need(out, "out");
        need(meshes, "meshes");
        if (count <= 0) fail(SEM_EINVAL, "count must be positive");
        DeviceGuard dg(as_mesh(meshes[0])->device);
        *out = reinterpret_cast<sem_batch_t>(batch_new(count, meshes));
        return SEM_OK;
    });
}

void sem_batch_destroy(sem_batch_t batch) {
    if (batch) batch_delete(reinterpret_cast<BatchImpl *>(batch));
}

sem_status sem_batch_solve(sem_batch_t batch, const sem_cg_opts *opts, const void *const *b_dev,
                           void *const *x_dev, sem_cg_result *results, void *hip_stream) {
    return guarded([&]() -> sem_status {
        need(batch, "batch");
        need(opts, "opts");
        need(b_dev, "b_dev");
        need(x_dev, "x_dev");
        need(results, "results");
        if (opts->fixed_iters <= 0 && !(opts->tol > 0.0))
            fail(SEM_EINVAL, "tol must be positive unless fixed_iters > 0");
        if (opts->geom != SEM_G_PRECOMPUTED && opts->geom != SEM_G_ON_THE_FLY)
            fail(SEM_EINVAL, "unknown geometry form");
        if (opts->precond != SEM_PRECOND_NONE)
            fail(SEM_EUNSUPPORTED, "batched solves take no preconditioner");
        BatchImpl &B = *reinterpret_cast<BatchImpl *>(batch);
        const sem_status st =
            batch_solve(B, *opts, b_dev, x_dev, results, static_cast<hipStream_t>(hip_stream));
        if (st == SEM_EBREAKDOWN) set_error("CG breakdown in at least one problem of the batch");
        return st;
    });
}

sem_status sem_server_create(const sem_cg_opts *opts, int round_iters, sem_server_t *out) {
    return guarded([&]() -> sem_status {
        need(opts, "opts");
        need(out, "out");
        if (opts->precond != SEM_PRECOND_NONE)
            fail(SEM_EUNSUPPORTED, "the server takes no preconditioner");
        *out = reinterpret_cast<sem_server_t>(server_new(*opts, round_iters));
        return SEM_OK;
    });
}

void sem_server_destroy(sem_server_t server) {
    if (server) server_delete(reinterpret_cast<ServerImpl *>(server));
}

sem_status sem_server_add(sem_server_t server, sem_mesh_t mesh, const void *b_dev, void *x_dev,
                          int64_t tag, void *hip_stream) {
    return guarded([&]() -> sem_status {
        need(server, "server");
        Mesh *m = as_mesh(mesh);
        DeviceGuard dg(m->device);
        server_add(*reinterpret_cast<ServerImpl *>(server), m, static_cast<const double *>(b_dev),
                   static_cast<double *>(x_dev), tag, static_cast<hipStream_t>(hip_stream));
        return SEM_OK;
    });
}

sem_status sem_server_step(sem_server_t server, int64_t *done_tags, sem_cg_result *done_results,
                           int cap, int *n_done, int *n_active) {
    return guarded([&]() -> sem_status {
        need(server, "server");
        need(n_done, "n_done");
        if (cap > 0) {
            need(done_tags, "done_tags");
            need(done_results, "done_results");
        }
        const int left = server_step(*reinterpret_cast<ServerImpl *>(server), done_tags,
                                     done_results, cap, n_done);
        if (n_active) *n_active = left;
        return SEM_OK;
    });
}

sem_status sem_mesh_footprint(int64_t n_elem, int order_N, uint32_t flags, sem_precision prec,
                              size_t *bytes) {
    return guarded([&]() -> sem_status {
        need(bytes, "bytes");
        if (n_elem <= 0) fail(SEM_EINVAL, "n_elem must be positive");
        if (order_N < 1 || order_N > kMaxOrder) fail(SEM_EUNSUPPORTED, "order not built");
        *bytes = mesh_footprint(n_elem, order_N, flags, prec);
        return SEM_OK;
    });
}

sem_status sem_ax_shape_set(int order_N, sem_precision prec, sem_geom geom, int elems_per_block) {
    return guarded([&]() -> sem_status {
        if (order_N < 1 || order_N > kMaxOrder) fail(SEM_EUNSUPPORTED, "order not built");
        check_prec(prec);
        if (geom != SEM_G_PRECOMPUTED && geom != SEM_G_ON_THE_FLY)
            fail(SEM_EINVAL, "unknown geometry form");
        if (elems_per_block < 0) fail(SEM_EINVAL, "elems_per_block must be >= 0");
        ax_shape_set(order_N, prec == SEM_FP64, geom == SEM_G_ON_THE_FLY, elems_per_block);
        return SEM_OK;
    });
}

sem_status sem_set_cache_bytes(int64_t bytes) {
    return guarded([&]() -> sem_status {
        if (bytes < 0) fail(SEM_EINVAL, "bytes must be >= 0");
        cache_bytes_set(bytes);
        return SEM_OK;
    });
}

sem_status sem_ax_engine_set(int order_N, sem_precision prec, sem_geom geom, int engine) {
    return guarded([&]() -> sem_status {
        if (order_N < 1 || order_N > kMaxOrder) fail(SEM_EUNSUPPORTED, "order not built");
        check_prec(prec);
        if (geom != SEM_G_PRECOMPUTED && geom != SEM_G_ON_THE_FLY)
            fail(SEM_EINVAL, "unknown geometry form");
        if (engine != SEM_AX_ENGINE_DEFAULT && engine != SEM_AX_ENGINE_VALU &&
            engine != SEM_AX_ENGINE_MFMA)
            fail(SEM_EINVAL, "unknown engine");
        if (engine == SEM_AX_ENGINE_MFMA && !ax_mfma_available(order_N, prec == SEM_FP64))
            fail(SEM_EUNSUPPORTED, "the matrix-core engine is built for FP32 at N = 7 and 9 only");
        ax_engine_set(order_N, prec == SEM_FP64, geom == SEM_G_ON_THE_FLY, engine);
        return SEM_OK;
    });
}

sem_status sem_ax_engine_get(int order_N, sem_precision prec, sem_geom geom, int *engine) {
    return guarded([&]() -> sem_status {
        need(engine, "engine");
        if (order_N < 1 || order_N > kMaxOrder) fail(SEM_EUNSUPPORTED, "order not built");
        check_prec(prec);
        const AxShape sh = ax_shape(order_N, prec == SEM_FP64, geom == SEM_G_ON_THE_FLY, 0);
        *engine = sh.mfma ? SEM_AX_ENGINE_MFMA : SEM_AX_ENGINE_VALU;
        return SEM_OK;
    });
}

sem_status sem_ax_shape_get(int order_N, sem_precision prec, sem_geom geom, int *elems_per_block,
                            int *threads, size_t *lds_bytes) {
    return guarded([&]() -> sem_status {
        if (order_N < 1 || order_N > kMaxOrder) fail(SEM_EUNSUPPORTED, "order not built");
        check_prec(prec);
        const AxShape sh = ax_shape(order_N, prec == SEM_FP64, geom == SEM_G_ON_THE_FLY, 0);
        if (elems_per_block) *elems_per_block = sh.epb;
        if (threads) *threads = sh.threads;
        if (lds_bytes) *lds_bytes = sh.lds;
        return SEM_OK;
    });
}

const char *sem_last_error(void) { return g_last_error.c_str(); }

const char *sem_version(void) { return "sem-mi355x 0.1 (gfx950)"; }

}  // extern "C"
