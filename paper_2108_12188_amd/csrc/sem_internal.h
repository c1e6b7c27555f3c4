// sem_internal.h -- shared host/device definitions of the SEM library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sem.h"

namespace sem {

constexpr int kMaxOrder = 11;
// Per-point code: multiplicity m (copies of the global point) in the low 7
// bits, the Dirichlet flag in bit 7.  The inner-product weight is 1/m.
constexpr int kMaxMultiplicity = 127;
constexpr uint8_t kDirichletBit = 0x80;
constexpr uint8_t kMultMask = 0x7F;
constexpr int kMaxP = kMaxOrder + 1;
// local points from which a mesh takes the table-free gather by default
// (below it, where a CG iteration is mostly launch latency, the table form
// measured up to 8% faster; from it on the table-free form is as fast or
// faster, alone and in batches)
constexpr int64_t kTableFreeMinPoints = int64_t(1) << 19;

// Edge and corner nodes of an element's P^3 block (on two or three of its
// faces): 12 N - 4 of them, numbered column by column (i, j on the border
// of the face square): every border column starts at its base with its
// k = 0 node, then k = N; the 4 corner columns (bases 0, P, 2P, 3P) follow
// with k = 1 .. N-1, the other border columns (bases 4P + 2s) have no more.
// -1 for other nodes.
__host__ __device__ inline int edge_slots(int N) { return 12 * N - 4; }
__host__ __device__ inline int edge_column_base(int N, int i, int j) {
    const int P = N + 1;
    const bool bi = i == 0 || i == N, bj = j == 0 || j == N;
    if (bi && bj) return ((i == N) + 2 * (j == N)) * P;
    if (!(bi || bj)) return -1;
    int s;
    if (j == 0) s = i - 1;
    else if (j == N) s = (P - 2) + i - 1;
    else if (i == 0) s = 2 * (P - 2) + j - 1;
    else s = 3 * (P - 2) + j - 1;
    return 4 * P + 2 * s;
}
__host__ __device__ inline int edge_slot(int N, int i, int j, int k) {
    const int cb = edge_column_base(N, i, j);
    if (cb < 0) return -1;
    if (k == 0 || k == N) return cb + (k == N);
    const bool corner = (i == 0 || i == N) && (j == 0 || j == N);
    return corner ? cb + 1 + k : -1;
}

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);
[[noreturn]] void fail(sem_status code, const std::string &msg);
void check_hip(hipError_t e, const char *what);

#define SEM_HIP(call) ::sem::check_hip((call), #call)

// ---------------------------------------------------------------------------
// Device-resident CG scalars of one solve (Algorithm 1: rho, alpha, beta).
// Written only by the one-block finalize kernels; read by every block of
// the kernels that follow in stream order.
// ---------------------------------------------------------------------------
struct CgState {
    double rho;        // rho_{i-1}: <r, r, c> of the current residual (<r, z, c>
                       // with a preconditioner)
    double rr;         // <r, r, c> of the current residual
    double rho0;       // <r0, r0, c>
    double alpha;      // alpha_i
    double beta;       // beta_{i-1} used by the next p-update
    double pw;         // <p, w, c> of the current iteration
    double thresh;     // stop when rr <= thresh (= tol^2 rho_0)
    int iter;          // completed iterations
    int max_iter;      // iteration cap
    int stop;          // 0 running, 1 converged, 2 cap reached, 3 breakdown
    int fixed;         // 1: no convergence test
    int x_lag;         // 1: x still lacks alpha_i p_i of the last completed
                       // update (single-mesh solves apply it in the next
                       // operator launch, or in the closing flush)
    int hist_len;      // capacity of the history arrays
    double *hist_rho;  // device history (may be null)
    double *hist_alpha;
};

// ---------------------------------------------------------------------------
// Mesh handle
// ---------------------------------------------------------------------------
template <typename T>
struct Basis {
    T *D = nullptr;    // [P][P]  D_ij = l_j'(xi_i)
    T *Dt = nullptr;   // [P][P]  transpose
    T *xi = nullptr;   // [P]
    T *w = nullptr;    // [P]
};

struct Workspace;      // CG vectors of one precision (sem_cg.cpp)

// Gather-scatter groups by size class (see sem_gs.hip).
constexpr int kMaxGsClasses = 32;
struct GsClasses {
    int ncls;
    int M[kMaxGsClasses];          // copies per group in this class
    int64_t ng[kMaxGsClasses];     // groups in this class
    int64_t io[kMaxGsClasses];     // offset of the class in gs_idx
    int64_t blk0[kMaxGsClasses];   // first block of the class in a gs launch
    // gather-scatter launches only (null: identity): DEVICE int32 [blocks],
    // the class-major logical block that position b of a launch runs; the
    // blocks sorted by the first local index of their first group, so the
    // classes of one region of the mesh run together.  A permutation of all
    // blocks: only launches that cover every block may apply it (the group
    // sums over a sub-range of classes do not).
    const int32_t *lb_order = nullptr;
};
void gs_classes_finish(GsClasses &c);
int64_t gs_total_blocks(const GsClasses &c);   // logical blocks of a whole gather-scatter

// Table-free gather inside the CG update (see Mesh::gs_struct): one record
// per face and per edge slot of an element, [E][6 + edge_slots(N)], faces
// first.  Face f = 2 d + (the face lies at coordinate N along d, its normal
// direction): the copies of its face-interior points, with face coordinates
// (a, b) (the two coordinates other than d, in i, j, k order), are
// lo + sa a + sb b, where hi = code | sa << 8 | sb << 20 with sa, sb 12-bit
// two's-complement strides (0, +-1, +-P or +-P^2; every partial sum fits
// in 32 bits); a face without a partner (or a Dirichlet face) has
// sa = sb = 0 and lo inside its own element.  Edge slot s (record 6 + s): lo = the rank of its group among the
// edge groups (0 when unshared or Dirichlet), hi = code.  code: the points'
// multiplicity | Dirichlet byte.
struct alignas(8) ElemRec {
    int32_t lo, hi;
};
// Per local position of the element (P^3 entries): bits 0-1 kind (0
// interior, 1 face interior, 2 edge or corner node), bits 2-6 and 7-11 the
// face coordinates a, b, bits 12-20 the record (face f, or 6 + edge slot).
__host__ __device__ inline uint32_t pos_entry(int kind, int a, int b, int rec) {
    return (uint32_t)kind | ((uint32_t)a << 2) | ((uint32_t)b << 7) | ((uint32_t)rec << 12);
}

struct Mesh {
    int device = 0;
    int64_t E = 0;
    int N = 0, P = 0, P3 = 0;
    int64_t n = 0;            // local points
    int64_t n_glob = 0;
    int64_t n_groups = 0, n_shared = 0, n_dir = 0;
    GsClasses gs{};           // shared-point groups by size class

    // host copies of the basis (FP64, this library's own construction)
    std::vector<double> h_xi, h_w, h_D;

    // device arrays
    double *vert64 = nullptr;     // [E][8][3]
    float *vert32 = nullptr;      // [E][8][3]
    float *edge32 = nullptr;      // N = 7: [E][12][3] element edge vectors from vert32
    float *G32 = nullptr;         // [E][6][P3]
    double *G64 = nullptr;        // [E][6][P3]
    double *B64 = nullptr;        // [E][P3] mass w_q |J_q|
    uint8_t *mcode = nullptr;     // [n]: multiplicity | Dirichlet bit
    int32_t *gs_idx = nullptr;    // [n_shared], class-major, groups of M ascending indices
    int32_t *gs_lb_order = nullptr;   // gs.lb_order's array
    int32_t *dir_idx = nullptr;   // [n_dir]
    // Shared sums inside the CG update (used when every shared point lies on
    // the surface of its element's P^3 block): gsrc[l] is the other copy of
    // a pair (m = 2), the rank of a larger group among the n_groups_multi
    // groups with m > 2 (whose sums a gather-scatter variant over blocks
    // gs_blk_multi.. writes to a compact array), else l itself.
    bool gs_in_update = false;
    int64_t n_groups_multi = 0, gs_blk_multi = 0;
    int32_t *gsrc = nullptr;       // [n]
    // When every copy of a group with m > 2 is an edge or corner node of its
    // element (edge_slot), the CG operator also writes those nodes' values
    // to a compact [E][edge_slots(N)] array and the group sums read it:
    // wedge_idx lists, for the groups with m > 2 in gs_idx's layout from
    // offset wedge_io0, the copies' positions e * edge_slots(N) + slot.
    bool gsum_wedge = false;
    int64_t wedge_io0 = 0;
    int32_t *wedge_idx = nullptr;
    // Table-free form of the same gather (odd N, conforming meshes, unless
    // SEM_MESH_GATHER_TABLE): the update derives every point's copies from
    // its position in the element (pos_tab) and the element's face and edge
    // records (ElemRec) instead of loading gsrc and mcode.  The sums of the
    // n_egroups edge and corner groups of two or more copies (ecls /
    // ewedge_idx: positions in the compact edge array) follow w in class
    // order.  Division of a local index by P^3: (l * p3_magic) >> p3_shift
    // (checked on the host for every l < n).  gs_struct: its tables are
    // present (batched and served solves use it then); gs_struct_solo: a
    // single-mesh solve uses it too (from kTableFreeMinPoints points on, or
    // when forced), else the per-point table gsrc, which is then present.
    // The two forms give bitwise identical results.
    bool gs_struct = false;
    bool gs_struct_solo = false;
    ElemRec *erec = nullptr;       // [E][6 + edge_slots(N)]
    uint32_t *pos_tab = nullptr;   // [P3]
    GsClasses ecls{};
    int64_t n_egroups = 0;
    int32_t *ewedge_idx = nullptr;
    uint32_t p3_magic = 0;
    int p3_shift = 0;
    // Jacobi preconditioner (built on first use): 1 / diag(A) on the free
    // points, 0 on the Dirichlet points, local form
    double *minv64 = nullptr;
    float *minv32 = nullptr;
    Basis<float> b32;
    Basis<double> b64;
    void *basis_blob = nullptr;
    double *scratch = nullptr;    // reduction partials / small scalars
    size_t scratch_len = 0;       // in doubles
    CgState *state = nullptr;     // device CG state for sem_dot / solves
    size_t device_bytes = 0;

    Workspace *ws32 = nullptr;
    Workspace *ws64 = nullptr;
};

Mesh *as_mesh(sem_mesh_t m);

// Relative tolerance of one inner FP32 solve of the mixed-precision
// refinement when the outer relative residual is rel and the target is tol:
// the reduction still needed, with a factor 10 to spare, but never tighter
// than the configured inner tolerance (nor looser than 1/2).  The last
// outer step then solves only as far as the target requires.
inline double refine_inner_tol(double inner_tol, double tol, double rel) {
    double t = rel > 0.0 ? 0.1 * tol / rel : inner_tol;
    if (t < inner_tol) t = inner_tol;
    if (t > 0.5) t = 0.5;
    return t;
}

// Host tables of a mesh's scatter map (sem_tables.cpp; no device calls).
struct HostTables {
    int64_t n_glob = 0, n_groups = 0, n_shared = 0, n_dir = 0;
    GsClasses gs{};
    std::vector<uint8_t> mcode;     // [n]
    std::vector<int32_t> gs_idx;    // class-major ascending member lists
    std::vector<int32_t> gs_lb_order;  // see GsClasses::lb_order
    std::vector<int32_t> dir_idx;   // Dirichlet local points
    bool gs_in_update = false;      // every shared point on its element's surface
    int64_t n_groups_multi = 0;     // groups with more than two copies
    int64_t gs_blk_multi = 0;       // their first gather-scatter block
    bool gsum_wedge = false;        // every copy of those groups an edge or corner node
    int64_t wedge_io0 = 0;          // gs_idx offset of the first such group
    std::vector<int32_t> wedge_idx; // copies' positions in the compact edge array
    std::vector<int32_t> gsrc;      // [n] (only when gs_in_update), see Mesh::gsrc
    bool gs_struct = false;         // the table-free form applies, see Mesh::gs_struct
    std::vector<ElemRec> erec;
    std::vector<uint32_t> pos_tab;
    GsClasses ecls{};
    int64_t n_egroups = 0;
    std::vector<int32_t> ewedge_idx;
    uint32_t p3_magic = 0;
    int p3_shift = 0;
};
// Validates glob_id / dirichlet (fail() on error) and fills t.
void build_tables(int64_t E, int N, const int64_t *gid, const uint8_t *dir, HostTables &t);

// ---------------------------------------------------------------------------
// Host basis construction (sem_basis.cpp)
// ---------------------------------------------------------------------------
void gll_points(int N, std::vector<double> &xi, std::vector<double> &w);
void derivative_matrix(const std::vector<double> &xi, std::vector<double> &D);

// ---------------------------------------------------------------------------
// Kernel launchers
// ---------------------------------------------------------------------------
enum class AxMode { Plain = 0, CgFused = 1 };

template <typename T>
struct AxArgs {
    int64_t E;
    int epb;                    // elements per block
    const T *u;                 // Plain: input u. CgFused: residual r
    T *p;                       // CgFused: search direction, updated in place
    T *w;                       // output
    const T *G;                 // precomputed factors [E][6][P3]
    const T *vert;              // vertices [E][8][3] (on-the-fly form)
    const T *edge;              // FP32, N = 7, may be null: edge vectors [E][12][3]
                                // (the matrix-core on-the-fly form reads these)
    const T *D;                 // [P][P]
    const T *Dt;                // [P][P]
    const T *xi;                // [P]
    const T *wq;                // [P]
    CgState *st;                // CgFused: beta, stop flag
    double *partial;            // CgFused: one FP64 partial of sum p w per block
    int64_t vgrid;              // batched launches: this problem's own grid size
    T *wedge;                   // CgFused, may be null: w of the edge and corner
                                // nodes, [E][edge_slots(N)]
    T *x;                       // CgFused, may be null: solution; when st->x_lag,
                                // x += alpha p_old (previous iteration's step)
    int mfma;                   // host side: launch the matrix-core form (FP32,
                                // N = 7; one element per wave-sized block)
    int stream;                 // CgFused FP32: p and x accesses non-temporal
                                // (cg_streams_vectors of the iteration's footprint)
};

// Jacobi preconditioning in the CG update (preconditioned CG, Sec. 3.2;
// Algorithm 1 is its unpreconditioned case): z = minv r is written, and the block partials of
// <r, z, c> (partial) and <r, r, c> (partial2) are reduced.
template <typename T>
struct PcArgs {
    const T *minv;      // null: no preconditioner
    T *z;
    double *partial2;
};

// Launch configuration chosen for an order (threads, elements per block,
// dynamic LDS bytes).
struct AxShape {
    int epb;
    int threads;
    size_t lds;
    bool mfma;                  // matrix-core form (epb 1, one wave per block)
};
AxShape ax_shape(int N, bool fp64, bool otf, int epb_override);
void ax_shape_set(int N, bool fp64, bool otf, int epb);
// Contraction engine per order, precision and G form: 0 default, 1 VALU FMA,
// 2 matrix cores (FP32, N = 7 only).
constexpr int kAxEngineDefault = 0, kAxEngineValu = 1, kAxEngineMfma = 2;
bool ax_mfma_available(int N, bool fp64);
void ax_engine_set(int N, bool fp64, bool otf, int engine);
int ax_shape_generation();

// Fills the basis / geometry pointers and the shape from the mesh; the
// caller sets u, p, w, mcode, st, partial (and epb to force a shape).
template <typename T>
void launch_ax(const Mesh &m, bool otf, AxMode mode, AxArgs<T> a, hipStream_t s);
int64_t ax_blocks(const Mesh &m, bool fp64, bool otf, int epb_override);
// Bytes a CG iteration of mesh m with tsz-byte vectors keeps touching: r,
// p, x, w, the gather records (table_free) or table, the operator's edge
// copy, vertices and codes.
int64_t cg_footprint(const Mesh &m, int tsz, bool table_free);

// The CG-fused operator reads and writes p and x non-temporally when the
// iteration (of one mesh, or of a whole batch) exceeds the 256 MB Infinity
// Cache, so that the cache keeps what the rest of the iteration reads again
// (in FP64 only with G on the fly: the precomputed FP64 factors, read with
// plain loads, fill the cache either way).
constexpr int64_t kInfinityCacheBytes = int64_t(256) << 20;
bool cg_streams_vectors(int64_t footprint);
// The cache size assumed by cg_streams_vectors (0: kInfinityCacheBytes);
// changing it invalidates captured graphs and batch tables like a new tile
// shape does.
void cache_bytes_set(int64_t bytes);

// Fills `a` (basis, geometry, epb, vgrid) for a batched FP32 launch of mesh m.
void ax_batch_desc(const Mesh &m, bool otf, AxArgs<float> &a);
// One FP32 CG-fused operator launch over many problems of order N:
// blk[b] = (descriptor index, virtual block).
// stream: p and x non-temporal (cg_streams_vectors of the batch's footprint)
void launch_ax_batch(int N, bool otf, bool mfma, bool stream, const AxArgs<float> *descs,
                     const int2 *blk, int64_t nblk, int epb, const double *D, const double *xi,
                     const double *w,
                     hipStream_t s);

// gather-scatter / mask / vector kernels (sem_gs.hip, sem_vec.hip)
template <typename T>
void launch_gs(const Mesh &m, T *w, hipStream_t s);
template <typename T>
void launch_mask(const Mesh &m, T *w, hipStream_t s);
// CG step after the fused operator: gather-scatter, then alpha from the
// operator kernel's partials of <p, w, c>
template <typename T>
void launch_gs_cg(const Mesh &m, T *w, CgState *st, const double *ax_partial, int n_ax_partial,
                  hipStream_t s);
// The same for the gather in the update: gsum[k] = sum of the copies of the
// k-th group with m > 2 (ascending local index; read from wedge, the
// operator's compact copy of the edge and corner nodes, when m.gsum_wedge,
// else from w; neither is modified), and alpha.
template <typename T>
void launch_group_sums_cg(const Mesh &m, const T *w, const T *wedge, T *gsum, CgState *st,
                          const double *ax_partial, int n_ax_partial, hipStream_t s);
// The same for the table-free gather (needs m.gs_struct): gsum[k] = sum of
// the copies of the k-th edge or corner group of two or more copies
// (ascending local index, read from wedge, the operator's compact edge
// array), then alpha.
template <typename T>
void launch_edge_sums_cg(const Mesh &m, const T *wedge, T *gsum, CgState *st,
                         const double *ax_partial, int n_ax_partial, hipStream_t s);
int gs_cg_blocks(const Mesh &m);
int64_t gs_logical_blocks(const Mesh &m);

// Algorithm 1 vector kernels (sem_vec.hip).  Reductions write one FP64
// partial per block (`partial`, at least vec_blocks(n) entries) and a
// one-block finalize kernel sums them in index order.
int vec_blocks(int64_t n);
// r -= alpha mask(w); rho = <r, r, c>; then beta, convergence, history (x is
// advanced by the next operator launch or launch_x_flush)
template <typename T>
void launch_update(const Mesh &m, T *r, const T *w, CgState *st, double *partial,
                   hipStream_t s, PcArgs<T> pc = PcArgs<T>{});
// x += alpha p when st->x_lag (the step of the last completed update)
template <typename T>
void launch_x_flush(const Mesh &m, T *x, const T *p, const CgState *st, hipStream_t s);
// The same with w read as QQ^T w, w holding the operator's masked local
// output and gsum the group sums of launch_group_sums_cg: pairs are summed
// inside the update (needs m.gs_in_update).
template <typename T>
void launch_update_gather(const Mesh &m, T *r, const T *w, const T *gsum, CgState *st,
                          double *partial, hipStream_t s, PcArgs<T> pc = PcArgs<T>{});
// The same with the table-free gather (needs m.gs_struct): wg holds w
// (n values) followed by the edge-group sums of launch_edge_sums_cg;
// bitwise the results of launch_update_gather.
template <typename T>
void launch_update_struct(const Mesh &m, T *r, const T *wg, CgState *st, double *partial,
                          hipStream_t s, PcArgs<T> pc = PcArgs<T>{});
// r = b - w (w may be null: r = b); p = 0; rho_0 = <r, r, c>; initial state.
// With pc.minv: z = minv r, rho = <r, z, c>, and the threshold and the
// reported residual use <r, r, c>.
template <typename T>
void launch_cg_init(const Mesh &m, const T *b, const T *w, T *r, T *p, CgState *st,
                    double *partial, hipStream_t s, PcArgs<T> pc = PcArgs<T>{});
// Jacobi: minv = 1/d on free points, 0 on Dirichlet points (both precisions)
void launch_jacobi_invert(const Mesh &m, const double *d, double *minv64, float *minv32,
                          hipStream_t s);
// d_l = (A_L)_{ll} of every local point from the geometry (FP64, unassembled)
void launch_diag_local(const Mesh &m, double *d, hipStream_t s);
// *out = <a, b, c>
template <typename T>
void launch_dot(const Mesh &m, const T *a, const T *b, double *out, double *partial,
                hipStream_t s);
// The same weighted inner product with its block partials in a file-scope
// device array of the library (no device allocation; sem_dot_noalloc).
template <typename T>
void launch_dot_noalloc(const Mesh &m, const T *a, const T *b, double *out, hipStream_t s);
// r = b - w and *out = <r, r, c>  (FP64 outer residual of the refinement)
void launch_residual64(const Mesh &m, const double *b, const double *w, double *r, double *out,
                       double *partial, hipStream_t s);
// alpha = rho / (sum of both partial sets)
void launch_finalize_alpha(CgState *st, const double *part_ax, int64_t n_ax, hipStream_t s);
// dst = (float)(src / sqrt(*nrm2))
void launch_scale_to_f32(int64_t n, const double *src, const double *nrm2, float *dst,
                         hipStream_t s);
// x += sqrt(*nrm2) * (double)d
void launch_axpy_from_f32(int64_t n, double *x, const double *nrm2, const float *d,
                          hipStream_t s);
// elementwise helpers
template <typename Ts, typename Td>
void launch_convert(int64_t n, const Ts *src, Td *dst, hipStream_t s);
void launch_mul64(int64_t n, const double *a, const double *b, double *out, hipStream_t s);

// FP64 geometry setup (sem_geom.hip)
int64_t launch_geometry(Mesh &m, hipStream_t s);
void launch_coords(const Mesh &m, double *xyz, hipStream_t s);
template <typename T>
void launch_rhs_mass(const Mesh &m, const double *f, T *b, hipStream_t s);

}  // namespace sem
