// sem_mesh.cpp -- mesh handle: validation, device arrays and the
// geometric-factor setup.  The gather-scatter tables are built on the host
// by sem_tables.cpp.
#include <algorithm>
#include <cstring>
#include <memory>
#include <numeric>

#include "sem_internal.h"

namespace sem {

namespace {

template <typename T>
T *dev_alloc(Mesh &m, size_t count) {
    if (count == 0) return nullptr;
    void *p = nullptr;
    const size_t bytes = count * sizeof(T);
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        fail(SEM_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    m.device_bytes += bytes;
    return static_cast<T *>(p);
}

template <typename T>
void upload(T *dst, const T *src, size_t count, hipStream_t s) {
    if (count) SEM_HIP(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyHostToDevice, s));
}

// The gather-scatter runs its blocks in the order of GsClasses::lb_order
// (0: class-major order, for comparison).
#ifndef SEM_GS_BLOCK_ORDER
#define SEM_GS_BLOCK_ORDER 1
#endif

void free_mesh_arrays(Mesh *m) {
    void *ptrs[] = {m->vert64,     m->vert32,  m->edge32,  m->G32,     m->G64,       m->B64,
                    m->mcode,      m->gs_idx,  m->gs_lb_order, m->dir_idx, m->gsrc,
                    m->wedge_idx,  m->basis_blob, m->scratch, m->state,   m->minv64,
                    m->minv32,     m->erec,    m->pos_tab, m->ewedge_idx};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
}

}  // namespace

void destroy_workspaces(Mesh *m);   // sem_cg.cpp

void mesh_destroy(Mesh *m) {
    if (!m) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(m->device);
    (void)hipDeviceSynchronize();
    destroy_workspaces(m);
    free_mesh_arrays(m);
    (void)hipSetDevice(cur);
    delete m;
}

// Upper bound of the device bytes a mesh and the work vectors of a solve in
// precision prec will hold (for admission by memory footprint).
size_t mesh_footprint(int64_t E, int N, uint32_t flags, sem_precision prec) {
    const size_t P3 = (size_t)(N + 1) * (N + 1) * (N + 1);
    const size_t n = (size_t)E * P3;
    size_t b = (size_t)E * 24 * (8 + 4);          // vertices, FP64 and FP32
    if (N == 7) b += (size_t)E * 36 * 4;           // FP32 edge vectors
    b += n * 8;                                    // mass
    b += n * 1;                                    // point codes
    b += n * 4 * 2;                                // group index list and Dirichlet list (bounds)
    b += n * 4;                                        // table of the gather in the update
    b += n / 3 * 4;                                    // edge-array positions (bound)
    {   // table-free gather: element records and edge-group positions (bounds)
        const size_t ms = (size_t)edge_slots(N);
        b += (size_t)E * (6 + ms) * 8 + ((size_t)E * ms + 8 * kMaxGsClasses) * 4 + P3 * 4;
    }
    if (flags & SEM_MESH_G_FP32) b += n * 24;
    if (flags & SEM_MESH_G_FP64) b += n * 48;
    b += ((size_t)vec_blocks((int64_t)n) + 16) * 8 + sizeof(CgState) + 4096;
    // 5 vectors, the group sums (at most n / 3 groups of more than two
    // copies), reduction partials
    const size_t we = (size_t)E * edge_slots(N);      // compact edge array
    const size_t ws32 = n * 4 * 5 + n / 3 * 4 + we * 4 + (size_t)E * 8 + (size_t)vec_blocks((int64_t)n) * 8 + 1024;
    const size_t ws64 = n * 8 * 5 + n / 3 * 8 + we * 8 + (size_t)E * 8 + (size_t)vec_blocks((int64_t)n) * 8 + 1024;
    if (prec == SEM_FP32) b += ws32;
    else if (prec == SEM_FP64) b += ws64;
    else b += ws32 + ws64;
    return b;
}

Mesh *mesh_create(int64_t E, int N, const double *vert, const int64_t *gid, const uint8_t *dir,
                  uint32_t flags, hipStream_t s) {
    if (E <= 0) fail(SEM_EINVAL, "n_elem must be positive");
    if (N < 1 || N > kMaxOrder)
        fail(SEM_EUNSUPPORTED, "order N=" + std::to_string(N) + " is not built (1..11)");
    if (!vert || !gid) fail(SEM_EINVAL, "vert_xyz and glob_id must not be NULL");
    if (flags & ~(uint32_t)(SEM_MESH_G_FP32 | SEM_MESH_G_FP64 | SEM_MESH_GATHER_TABLE |
                            SEM_MESH_GATHER_TABLE_FREE | SEM_MESH_GATHER_PASS))
        fail(SEM_EINVAL, "unknown mesh flags");
    {
        const int forms = ((flags & SEM_MESH_GATHER_TABLE) ? 1 : 0) +
                          ((flags & SEM_MESH_GATHER_TABLE_FREE) ? 1 : 0) +
                          ((flags & SEM_MESH_GATHER_PASS) ? 1 : 0);
        if (forms > 1)
            fail(SEM_EINVAL, "SEM_MESH_GATHER_TABLE, SEM_MESH_GATHER_TABLE_FREE and "
                             "SEM_MESH_GATHER_PASS exclude each other");
    }
    const int P = N + 1, P3 = P * P * P;
    const int64_t n = E * P3;
    if (E > (int64_t(1) << 31) / P3 || n >= (int64_t(1) << 31))
        fail(SEM_EINVAL, "n_local must be below 2^31");

    std::unique_ptr<Mesh> m(new Mesh());
    SEM_HIP(hipGetDevice(&m->device));
    m->E = E;
    m->N = N;
    m->P = P;
    m->P3 = P3;
    m->n = n;

    HostTables t;
    build_tables(E, N, gid, dir, t);
    if (flags & SEM_MESH_GATHER_PASS) {
        // the paper's schedule: a gather-scatter pass of its own
        t.gs_in_update = false;
        t.gsum_wedge = false;
        t.gs_struct = false;
    }
    m->n_glob = t.n_glob;
    m->gs = t.gs;
    m->n_groups = t.n_groups;
    m->n_shared = t.n_shared;
    m->n_dir = t.n_dir;
    m->gs_in_update = t.gs_in_update;
    m->n_groups_multi = t.n_groups_multi;
    m->gs_blk_multi = t.gs_blk_multi;
    m->gsum_wedge = t.gsum_wedge;
    m->wedge_io0 = t.wedge_io0;
    // the table-free gather wherever it applies unless the table is asked
    // for; single-mesh solves use it when forced or by size (below about half
    // a million points its fixed per-block set-up costs more than the table's
    // bytes there), batched launches always (their blocks span every member)
    m->gs_struct = t.gs_struct && !(flags & SEM_MESH_GATHER_TABLE);
    m->gs_struct_solo =
        m->gs_struct && ((flags & SEM_MESH_GATHER_TABLE_FREE) || n >= kTableFreeMinPoints);
    if (m->gs_struct) {
        m->ecls = t.ecls;
        m->n_egroups = t.n_egroups;
        m->p3_magic = t.p3_magic;
        m->p3_shift = t.p3_shift;
    }

    // ---- basis ---------------------------------------------------------------
    gll_points(N, m->h_xi, m->h_w);
    derivative_matrix(m->h_xi, m->h_D);

    // ---- device arrays ---------------------------------------------------------
    try {
        m->vert64 = dev_alloc<double>(*m, (size_t)E * 24);
        m->vert32 = dev_alloc<float>(*m, (size_t)E * 24);
        if (N == 7) m->edge32 = dev_alloc<float>(*m, (size_t)E * 36);
        m->B64 = dev_alloc<double>(*m, (size_t)n);
        if (flags & SEM_MESH_G_FP32) m->G32 = dev_alloc<float>(*m, (size_t)n * 6);
        if (flags & SEM_MESH_G_FP64) m->G64 = dev_alloc<double>(*m, (size_t)n * 6);
        m->mcode = dev_alloc<uint8_t>(*m, (size_t)n);
        m->gs_idx = dev_alloc<int32_t>(*m, t.gs_idx.size());
        m->gs_lb_order = dev_alloc<int32_t>(*m, t.gs_lb_order.size());
        m->dir_idx = dev_alloc<int32_t>(*m, t.dir_idx.size());
        if (t.gs_in_update && !m->gs_struct_solo) m->gsrc = dev_alloc<int32_t>(*m, t.gsrc.size());
        if (t.gsum_wedge) m->wedge_idx = dev_alloc<int32_t>(*m, t.wedge_idx.size());
        if (m->gs_struct) {
            m->erec = dev_alloc<ElemRec>(*m, t.erec.size());
            m->pos_tab = dev_alloc<uint32_t>(*m, t.pos_tab.size());
            m->ewedge_idx = dev_alloc<int32_t>(*m, t.ewedge_idx.size());
        }
        // basis blob: FP64 D, Dt, xi, w then FP32 D, Dt, xi, w
        const size_t PP = (size_t)P * P;
        const size_t nd = 2 * PP + 2 * P;
        m->basis_blob = dev_alloc<double>(*m, nd + (nd + 1) / 2 + 1);
        double *b64 = static_cast<double *>(m->basis_blob);
        float *b32 = reinterpret_cast<float *>(b64 + nd);
        m->b64 = {b64, b64 + PP, b64 + 2 * PP, b64 + 2 * PP + P};
        m->b32 = {b32, b32 + PP, b32 + 2 * PP, b32 + 2 * PP + P};
        std::vector<double> h64(nd);
        std::vector<float> h32(nd);
        for (int i = 0; i < P; ++i)
            for (int j = 0; j < P; ++j) {
                h64[i * P + j] = m->h_D[i * P + j];
                h64[PP + i * P + j] = m->h_D[j * P + i];
            }
        for (int i = 0; i < P; ++i) {
            h64[2 * PP + i] = m->h_xi[i];
            h64[2 * PP + P + i] = m->h_w[i];
        }
        for (size_t q = 0; q < nd; ++q) h32[q] = (float)h64[q];
        // scratch for sem_dot: partials + a few scalars; device state block
        m->scratch_len = (size_t)vec_blocks(n) + 16;
        m->scratch = dev_alloc<double>(*m, m->scratch_len);
        m->state = dev_alloc<CgState>(*m, 1);

        std::vector<float> v32((size_t)E * 24);
        for (size_t q = 0; q < v32.size(); ++q) v32[q] = (float)vert[q];
        upload(m->vert64, vert, (size_t)E * 24, s);
        upload(m->vert32, v32.data(), v32.size(), s);
        std::vector<float> ed32;
        if (m->edge32) {
            // the 12 edge vectors of each element, subtracted in FP32 from
            // the FP32 vertices exactly as the on-the-fly geometry does: the
            // matrix-core operator at N = 7 reads these instead of the
            // vertices (same values, bit for bit)
            static const int kHead[12] = {1, 3, 5, 7, 2, 3, 6, 7, 4, 5, 6, 7};
            static const int kTail[12] = {0, 2, 4, 6, 0, 1, 4, 5, 0, 1, 2, 3};
            ed32.resize((size_t)E * 36);
            for (int64_t e = 0; e < E; ++e)
                for (int t = 0; t < 12; ++t)
                    for (int d = 0; d < 3; ++d)
                        ed32[(size_t)e * 36 + t * 3 + d] = v32[(size_t)e * 24 + kHead[t] * 3 + d] -
                                                           v32[(size_t)e * 24 + kTail[t] * 3 + d];
            upload(m->edge32, ed32.data(), ed32.size(), s);
        }
        upload(m->mcode, t.mcode.data(), t.mcode.size(), s);
        upload(m->gs_idx, t.gs_idx.data(), t.gs_idx.size(), s);
        upload(m->gs_lb_order, t.gs_lb_order.data(), t.gs_lb_order.size(), s);
        if (SEM_GS_BLOCK_ORDER) m->gs.lb_order = m->gs_lb_order;
        upload(m->dir_idx, t.dir_idx.data(), t.dir_idx.size(), s);
        if (t.gs_in_update && !m->gs_struct_solo) upload(m->gsrc, t.gsrc.data(), t.gsrc.size(), s);
        if (t.gsum_wedge) upload(m->wedge_idx, t.wedge_idx.data(), t.wedge_idx.size(), s);
        if (m->gs_struct) {
            upload(m->erec, t.erec.data(), t.erec.size(), s);
            upload(m->pos_tab, t.pos_tab.data(), t.pos_tab.size(), s);
            upload(m->ewedge_idx, t.ewedge_idx.data(), t.ewedge_idx.size(), s);
        }
        upload(b64, h64.data(), nd, s);
        upload(b32, h32.data(), nd, s);
        SEM_HIP(hipMemsetAsync(m->state, 0, sizeof(CgState), s));
        const int64_t bad = launch_geometry(*m, s);   // synchronises s (host vectors stay alive)
        if (bad >= 0)
            fail(SEM_EJACOBIAN,
                 "non-positive Jacobian determinant in element " + std::to_string(bad));
    } catch (...) {
        (void)hipStreamSynchronize(s);
        free_mesh_arrays(m.get());
        throw;
    }
    return m.release();
}

}  // namespace sem
