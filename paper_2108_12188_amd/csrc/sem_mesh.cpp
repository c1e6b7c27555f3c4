// sem_mesh.cpp -- mesh handle: validation, gather-scatter groups, device
// arrays and the geometric-factor setup.
//
// The scatter map Q of Sec. 3.1 arrives as one global id per local point.
// Local points sharing an id are the copies summed by the gather-scatter
// (Sec. 4.3: points with equal position).  They are grouped here, on the
// host, once per mesh: groups of m > 1 copies are bucketed by m, each
// group's local indices ascending, and groups inside a bucket in ascending
// order of their first local index.
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

void free_mesh_arrays(Mesh *m) {
    void *ptrs[] = {m->vert64, m->vert32, m->G32,     m->G64,      m->B64,  m->mcode,
                    m->gs_idx, m->dir_idx, m->basis_blob, m->scratch, m->state};
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
    b += n * 8;                                    // mass
    b += n * 1;                                    // point codes
    b += n * 4 * 2;                                // group index list and Dirichlet list (bounds)
    if (flags & SEM_MESH_G_FP32) b += n * 24;
    if (flags & SEM_MESH_G_FP64) b += n * 48;
    b += ((size_t)vec_blocks((int64_t)n) + 16) * 8 + sizeof(CgState) + 4096;
    const size_t ws32 = n * 4 * 5 + (size_t)E * 8 + (size_t)vec_blocks((int64_t)n) * 8 + 1024;
    const size_t ws64 = n * 8 * 5 + (size_t)E * 8 + (size_t)vec_blocks((int64_t)n) * 8 + 1024;
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
    if (flags & ~(uint32_t)(SEM_MESH_G_FP32 | SEM_MESH_G_FP64))
        fail(SEM_EINVAL, "unknown mesh flags");
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

    // ---- global ids: validate, count copies -------------------------------
    int64_t maxid = -1;
    for (int64_t l = 0; l < n; ++l) {
        if (gid[l] < 0) fail(SEM_EINVAL, "glob_id has a negative entry at " + std::to_string(l));
        maxid = std::max(maxid, gid[l]);
    }
    // compact ids to 0..n_glob-1 in order of first appearance
    std::vector<int32_t> cid(n);
    {
        const bool dense = maxid < 4 * n + 16;
        if (dense) {
            std::vector<int32_t> map(maxid + 1, -1);
            int32_t next = 0;
            for (int64_t l = 0; l < n; ++l) {
                int32_t &c = map[gid[l]];
                if (c < 0) c = next++;
                cid[l] = c;
            }
            m->n_glob = next;
        } else {
            std::vector<int64_t> order(n);
            std::iota(order.begin(), order.end(), 0);
            std::stable_sort(order.begin(), order.end(),
                             [&](int64_t a, int64_t b) { return gid[a] < gid[b]; });
            // first-appearance numbering: smallest l of each id
            std::vector<std::pair<int64_t, int64_t>> first;   // (first l, rank in sorted ids)
            int32_t rank = -1;
            std::vector<int32_t> rank_of(n);
            for (int64_t t = 0; t < n; ++t) {
                if (t == 0 || gid[order[t]] != gid[order[t - 1]]) {
                    ++rank;
                    first.push_back({order[t], rank});
                }
                rank_of[order[t]] = rank;
            }
            std::vector<int32_t> renum(first.size());
            std::sort(first.begin(), first.end());
            for (size_t q = 0; q < first.size(); ++q) renum[first[q].second] = (int32_t)q;
            for (int64_t l = 0; l < n; ++l) cid[l] = renum[rank_of[l]];
            m->n_glob = (int64_t)first.size();
        }
    }
    const int64_t G = m->n_glob;
    std::vector<int32_t> cnt(G, 0);
    for (int64_t l = 0; l < n; ++l) ++cnt[cid[l]];
    std::vector<int8_t> dflag(G, -1);
    for (int64_t l = 0; l < n; ++l) {
        const int8_t d = dir ? (dir[l] ? 1 : 0) : 0;
        int8_t &f = dflag[cid[l]];
        if (f < 0) f = d;
        else if (f != d)
            fail(SEM_EINVAL, "dirichlet flags differ between copies of a global point (local " +
                                 std::to_string(l) + ")");
    }
    std::vector<uint8_t> mcode(n);
    int64_t n_dir = 0;
    for (int64_t l = 0; l < n; ++l) {
        const int32_t c = cnt[cid[l]];
        if (c > kMaxMultiplicity)
            fail(SEM_EINVAL, "more than 127 local copies of one global point");
        const bool d = dflag[cid[l]] == 1;
        mcode[l] = (uint8_t)((d ? kDirichletBit : 0) | c);
        n_dir += d;
    }

    // ---- groups by size class ----------------------------------------------
    // CSR of local points by compact id (ascending l inside each id)
    std::vector<int64_t> start(G + 1, 0);
    for (int64_t g = 0; g < G; ++g) start[g + 1] = start[g] + cnt[g];
    std::vector<int32_t> byid(n);
    {
        std::vector<int64_t> fill(start.begin(), start.end() - 1);
        for (int64_t l = 0; l < n; ++l) byid[fill[cid[l]]++] = (int32_t)l;
    }
    // compact ids are numbered by first appearance, so ascending id order is
    // ascending first-local-index order
    int sizes_seen[256] = {0};
    for (int64_t g = 0; g < G; ++g)
        if (cnt[g] > 1) sizes_seen[cnt[g]] = 1;
    GsClasses cls{};
    int64_t n_shared = 0, n_groups = 0;
    std::vector<int32_t> gs_idx;
    for (int msz = 2; msz <= kMaxMultiplicity; ++msz) {
        if (!sizes_seen[msz]) continue;
        if (cls.ncls == kMaxGsClasses)
            fail(SEM_EUNSUPPORTED, "more than 32 distinct multiplicities");
        const int c = cls.ncls++;
        cls.M[c] = msz;
        // every class starts on a 32-byte boundary (vector index loads)
        while (gs_idx.size() % 8) gs_idx.push_back(0);
        cls.io[c] = (int64_t)gs_idx.size();
        int64_t ng = 0;
        for (int64_t g = 0; g < G; ++g) {
            if (cnt[g] != msz) continue;
            for (int64_t o = start[g]; o < start[g + 1]; ++o) gs_idx.push_back(byid[o]);
            ++ng;
        }
        cls.ng[c] = ng;
        n_groups += ng;
        n_shared += ng * msz;
    }
    while (gs_idx.size() % 8) gs_idx.push_back(0);
    gs_classes_finish(cls);
    m->gs = cls;
    m->n_groups = n_groups;
    m->n_shared = n_shared;
    m->n_dir = n_dir;
    std::vector<int32_t> dir_idx;
    dir_idx.reserve(n_dir);
    for (int64_t l = 0; l < n; ++l)
        if (mcode[l] & kDirichletBit) dir_idx.push_back((int32_t)l);

    // ---- basis ---------------------------------------------------------------
    gll_points(N, m->h_xi, m->h_w);
    derivative_matrix(m->h_xi, m->h_D);

    // ---- device arrays ---------------------------------------------------------
    try {
        m->vert64 = dev_alloc<double>(*m, (size_t)E * 24);
        m->vert32 = dev_alloc<float>(*m, (size_t)E * 24);
        m->B64 = dev_alloc<double>(*m, (size_t)n);
        if (flags & SEM_MESH_G_FP32) m->G32 = dev_alloc<float>(*m, (size_t)n * 6);
        if (flags & SEM_MESH_G_FP64) m->G64 = dev_alloc<double>(*m, (size_t)n * 6);
        m->mcode = dev_alloc<uint8_t>(*m, (size_t)n);
        m->gs_idx = dev_alloc<int32_t>(*m, gs_idx.size());
        m->dir_idx = dev_alloc<int32_t>(*m, dir_idx.size());
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
        upload(m->mcode, mcode.data(), mcode.size(), s);
        upload(m->gs_idx, gs_idx.data(), gs_idx.size(), s);
        upload(m->dir_idx, dir_idx.data(), dir_idx.size(), s);
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
