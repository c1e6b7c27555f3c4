/*
 * sem.h -- C ABI of the MI355X (gfx950) spectral-element Poisson CG library.
 *
 * The library implements the per-iteration hot path of the unpreconditioned
 * SEM conjugate-gradient solver of Karp et al., "A High-Fidelity Flow Solver
 * for Unstructured Meshes on Field-Programmable Gate Arrays" (HPC Asia 2022,
 * arXiv 2108.12188): the matrix-free local operator A_L (Sec. 3, Eq. 4-5),
 * gather-scatter QQ^T with Dirichlet masking (Sec. 3.1, Sec. 4.3) and the
 * CG vector updates and weighted reductions of Algorithm 1, with the
 * geometric factors either precomputed or recomputed on the fly from the
 * element vertices (Sec. 5.1, Eq. 13-14).
 *
 * General conventions
 *   - Order N, P = N + 1, P3 = P^3 local points per element; N in [1, 11].
 *   - Local (replicated) vectors have n_local = E * P3 entries, element-major,
 *     local point l = i + P*(j + P*k) inside an element (i fastest).  This is
 *     the local form u_L = Q u of a global vector u (Sec. 3.1).
 *   - Vectors passed as `void*` are caller-owned DEVICE buffers of n_local
 *     entries of the precision named by the call (double for SEM_FP64 and
 *     SEM_MIXED, float for SEM_FP32), at least 16-byte aligned.  The mesh
 *     handle owns every other device array and frees it in
 *     sem_mesh_destroy.
 *   - `hip_stream` is a hipStream_t (NULL = the default stream).  Every call
 *     except sem_mesh_create, sem_cg_solve and the batch solve is
 *     stream-ordered and returns before the work finishes.
 *   - No C++ exception crosses this boundary.  On an error the call returns
 *     a negative sem_status, leaves its outputs untouched, and
 *     sem_last_error() returns a message for the calling thread.
 *   - Calls that use the same mesh handle on overlapping streams race on the
 *     handle's internal work vectors; serialise them.
 */
#ifndef SEM_H
#define SEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sem_mesh_s *sem_mesh_t;
typedef struct sem_batch_s *sem_batch_t;

typedef enum {
    SEM_OK = 0,
    SEM_EINVAL = -1,       /* bad argument (NULL pointer, size, inconsistent mesh) */
    SEM_ENOMEM = -2,       /* device allocation failed */
    SEM_EDEVICE = -3,      /* a HIP runtime call failed */
    SEM_EJACOBIAN = -4,    /* |J| <= 0 at some GLL point; message names the element */
    SEM_EBREAKDOWN = -5,   /* CG breakdown: <p,w,c> <= 0 or a non-finite scalar */
    SEM_EUNSUPPORTED = -6  /* order, precision/geometry form or size not built */
} sem_status;

typedef enum { SEM_FP64 = 0, SEM_FP32 = 1, SEM_MIXED = 2 } sem_precision;
typedef enum { SEM_G_PRECOMPUTED = 0, SEM_G_ON_THE_FLY = 1 } sem_geom;

/* sem_mesh_create flags: which precomputed geometric-factor arrays to keep.
 * The on-the-fly form needs none of them (it reads the vertices; at N = 7 the
 * FP32 matrix-core operator reads 12 edge vectors per element, 144 B, that
 * mesh creation derives from them). */
#define SEM_MESH_G_FP32 0x1u   /* G as float [E][6][P3]  (24 B per point)  */
#define SEM_MESH_G_FP64 0x2u   /* G as double [E][6][P3] (48 B per point)  */
/* Form of the gather-scatter inside CG (the two give bitwise identical
 * results).  The table-free form applies to odd N on conforming meshes.
 * sem_cg_solve uses it by default from 2^19 local points on (smaller meshes
 * run faster alone with the per-point table, which such a mesh then holds
 * as well); batched and served solves use it wherever it applies.
 * SEM_MESH_GATHER_TABLE keeps the table form everywhere;
 * SEM_MESH_GATHER_TABLE_FREE takes the table-free form wherever it applies,
 * whatever the size.  Not both. */
#define SEM_MESH_GATHER_TABLE 0x4u
#define SEM_MESH_GATHER_TABLE_FREE 0x8u
/* The paper's schedule instead (Algorithm 1 with the gather-scatter QQ^T as a
 * pass of its own over w between the operator and the update, Sec. 4.3):
 * same results up to rounding order; for measuring the gather-scatter's own
 * bandwidth as the performance model of Sec. 5.2 (Eq. 15) does.  Excludes
 * the two flags above. */
#define SEM_MESH_GATHER_PASS 0x10u

/*
 * Build a mesh on the current HIP device (Sec. 3: decomposition into E
 * hexahedra with a tensor GLL basis of order N; Sec. 3.1: the scatter map Q).
 *   n_elem     E > 0.
 *   order_N    N in [1, 11].
 *   vert_xyz   HOST double [E][8][3]: element vertices; vertex a + 2b + 4c sits
 *              at reference corner (xi, eta, gamma) = (2a-1, 2b-1, 2c-1).
 *              Elements are trilinear: linearly deformed hexahedra (Sec. 5.1).
 *   glob_id    HOST int64 [E][P3]: global point of every local point (this is
 *              Q).  Ids are >= 0; points with equal id are summed by the
 *              gather-scatter.  Every id in [0, max id] need not be used.
 *   dirichlet  HOST uint8 [E][P3]: 1 on the Dirichlet boundary; must be equal
 *              on all copies of a global point.  May be NULL (no boundary).
 *   flags      bit set of SEM_MESH_G_FP32 / SEM_MESH_G_FP64 / one of
 *              SEM_MESH_GATHER_TABLE, SEM_MESH_GATHER_TABLE_FREE,
 *              SEM_MESH_GATHER_PASS.
 *   out        receives the handle.
 * Copies what it needs; the host arrays may be freed on return.  Blocks until
 * the device-side setup (geometric factors, Jacobian check) has finished.
 * Errors: SEM_EINVAL (NULL, E <= 0, bad ids, inconsistent Dirichlet flags,
 * more than 127 copies of a point, n_local >= 2^31), SEM_EUNSUPPORTED (N out
 * of range), SEM_EJACOBIAN, SEM_ENOMEM, SEM_EDEVICE.
 */
sem_status sem_mesh_create(int64_t n_elem, int order_N, const double *vert_xyz,
                           const int64_t *glob_id, const uint8_t *dirichlet,
                           uint32_t flags, void *hip_stream, sem_mesh_t *out);

/*
 * Element order for locality on unstructured meshes.  Sec. 4.3 notes that an
 * unstructured mesh guarantees no ordering or spatial locality of the
 * elements in the local vectors, which makes the gather-scatter's accesses
 * unaligned; Sec. 8.2 proposes partitioning or sorting the elements to
 * recover it.  This sorts the elements by their centroids, along a
 * space-filling curve or in rows.  Host only (no device work).
 *   n_elem, vert_xyz  as in sem_mesh_create.
 *   kind      SEM_ORDER_HILBERT or SEM_ORDER_MORTON (Z-order): elements whose
 *             centroids fall in one cell of the curve's 2^21-per-axis grid
 *             keep their input order; SEM_ORDER_ROWS: row-major order of the
 *             centroids quantized per axis to the elements' median vertex
 *             span along it, the axis with the most cells slowest (a structured box comes back in its
 *             row-major numbering; elements in one cell keep their input
 *             order; more than 2^21 cells along an axis is an error).
 *   perm      HOST int64 [n_elem], written: perm[k] is the input element
 *             placed at position k.
 * Applying perm to vert_xyz, glob_id and dirichlet (and to the element blocks
 * of every local vector) before sem_mesh_create gives the same operator with
 * the elements renumbered: every result equals that of the input order with
 * its element blocks permuted.
 * Errors: SEM_EINVAL (NULL, n_elem <= 0, non-finite coordinate, unknown kind,
 * zero-extent elements or too many cells for SEM_ORDER_ROWS).
 */
typedef enum {
    SEM_ORDER_HILBERT = 0,
    SEM_ORDER_MORTON = 1,
    SEM_ORDER_ROWS = 2
} sem_element_order_kind;
sem_status sem_element_order(int64_t n_elem, const double *vert_xyz, int kind, int64_t *perm);

/* Free every device array of the mesh (synchronises the device). NULL is a no-op. */
void sem_mesh_destroy(sem_mesh_t mesh);

typedef struct {
    int64_t n_elem;        /* E */
    int32_t order_N;       /* N */
    int64_t n_local;       /* E * P3 (the paper's n, Eq. 7) */
    int64_t n_glob;        /* distinct global points */
    int64_t n_shared;      /* local points with multiplicity > 1 */
    int64_t n_groups;      /* global points with multiplicity > 1 */
    int64_t n_dirichlet;   /* local points on the Dirichlet boundary */
    size_t device_bytes;   /* device memory held by the handle (mesh arrays and work vectors) */
    int32_t gs_in_update;  /* 1: every shared point lies on an element face, and sem_cg_solve
                              gathers the shared sums inside its vector update instead of a
                              separate gather-scatter pass (same results, bitwise) */
    int32_t gs_table_free; /* 1: sem_cg_solve's gather derives each point's copies from its
                              position in the element and per-element face and edge records
                              (see SEM_MESH_GATHER_TABLE_FREE) instead of a per-point table
                              (same results, bitwise) */
} sem_mesh_info_t;

sem_status sem_mesh_info(sem_mesh_t mesh, sem_mesh_info_t *info);

/*
 * Local operator, no gather-scatter, no mask (Eq. 4-5: w_e = D^T G^e D u_e
 * for every element e).  prec: SEM_FP32 or SEM_FP64 (buffers of that type).
 * geom: SEM_G_PRECOMPUTED reads the G array of that precision (it must have
 * been requested at mesh creation, else SEM_EUNSUPPORTED); SEM_G_ON_THE_FLY
 * recomputes G at every point from the 8 vertices (the paper's
 * rematerialization, Sec. 5.1).  u and w must not overlap.
 */
sem_status sem_ax(sem_mesh_t mesh, sem_precision prec, sem_geom geom,
                  const void *u_dev, void *w_dev, void *hip_stream);

/*
 * In-place gather-scatter w <- QQ^T w (Sec. 3.1 and 4.3): every copy of a
 * global point receives the sum of all copies, summed in ascending local
 * index.  apply_mask = 1 then zeroes the Dirichlet points (Algorithm 1, mask
 * step).  prec: SEM_FP32 or SEM_FP64.
 */
sem_status sem_gs(sem_mesh_t mesh, sem_precision prec, void *w_dev, int apply_mask,
                  void *hip_stream);

/*
 * Weighted inner product <a, b, c> = sum_l a_l b_l c_l with c_l = 1/m_l, m_l
 * the multiplicity of local point l (Algorithm 1; c removes the replicated
 * copies).  Accumulates in FP64 in a fixed order (deterministic).  Writes one
 * double to the DEVICE pointer out_dev.  prec: SEM_FP32 or SEM_FP64.
 */
sem_status sem_dot(sem_mesh_t mesh, sem_precision prec, const void *a_dev,
                   const void *b_dev, double *out_dev, void *hip_stream);

/*
 * sem_dot without device allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and result as
 * sem_dot (bitwise).  Its block partials live in a static device array of
 * the library, 4096 doubles (32 KiB) per GPU, held until the process ends;
 * the partial count is min(ceil(n_local / 1024), 4096), so every mesh fits,
 * and a larger count would return SEM_EINVAL.  The call makes no hipMalloc
 * or hipFree (its first call on a device looks the array's address up).
 * Calls that overlap on one GPU share the array and race: serialise them.
 */
sem_status sem_dot_noalloc(sem_mesh_t mesh, sem_precision prec, const void *a_dev,
                           const void *b_dev, double *out_dev, void *hip_stream);

/*
 * Diagonal of the assembled operator A = Q^T A_L Q (Eq. 4) in local form
 * (unmasked): the element diagonals (A_L)_qq = sum_{a,b} sum_q' (D_a)_{q'q}
 * G_ab(q') (D_b)_{q'q}, formed in FP64 from the vertices whatever G form the
 * mesh stores, summed over the copies of every global point in ascending
 * local index.  This is the M of the Jacobi preconditioner
 * (SEM_PRECOND_JACOBI).  diag_dev: DEVICE double [n_local], written.
 */
sem_status sem_diag(sem_mesh_t mesh, double *diag_dev, void *hip_stream);

/*
 * Physical coordinates of every local GLL point: xyz_dev is a DEVICE double
 * buffer [3][n_local] (x block, then y, then z).
 */
sem_status sem_coords(sem_mesh_t mesh, double *xyz_dev, void *hip_stream);

/*
 * Right-hand side of the weak form, Eq. 2: b = mask(QQ^T (B f)) with B the
 * diagonal GLL mass (w_q |J_q|) and f DEVICE double [n_local] the source at
 * every local point.  b: n_local entries of prec (SEM_FP32 or SEM_FP64;
 * SEM_MIXED writes double).  f and b may alias only if both are double.
 */
sem_status sem_rhs(sem_mesh_t mesh, sem_precision prec, const double *f_dev, void *b_dev,
                   void *hip_stream);

/*
 * Preconditioner of the CG (Sec. 3.2 introduces CG in its usual
 * preconditioned form and takes the unpreconditioned Algorithm 1 as the
 * first step; Sec. 10 leaves preconditioning open).
 * SEM_PRECOND_JACOBI: M = diagonal of the assembled operator A = Q^T A_L Q
 * (Eq. 4), formed once per mesh in FP64 from the vertices: the element
 * diagonals (A_L)_qq summed over the copies of every global point; the
 * update then applies z = M^-1 r on the free points (0 on Dirichlet
 * points), p = z + beta p, and alpha, beta use <r, z, c>.
 */
typedef enum { SEM_PRECOND_NONE = 0, SEM_PRECOND_JACOBI = 1 } sem_precond;

typedef struct {
    sem_precision prec;   /* SEM_FP64, SEM_FP32, or SEM_MIXED (FP32 inner CG + FP64 outer) */
    sem_geom geom;        /* form of the local operator in the (inner) CG */
    double tol;           /* stop when ||r||_c / ||r0||_c <= tol (MIXED: true FP64 residual / ||b||_c) */
    int max_iter;         /* iteration cap (MIXED: cap on inner iterations per outer step) */
    int fixed_iters;      /* > 0: run exactly this many iterations, no convergence test */
    double inner_tol;     /* MIXED: tightest relative tolerance of an inner FP32 solve
                             (0 -> 1e-5); each inner solve stops at
                             max(inner_tol, 0.1 tol / rel), rel the current outer
                             relative residual, so the last step solves only as far
                             as tol requires */
    int max_outer;        /* MIXED: cap on outer refinement steps (0 -> 20) */
    int poll_every;       /* iterations per graph launch between host checks (0 -> auto) */
    int use_graph;        /* 1: replay captured HIP graphs; 0: plain launches */
    int true_residual;    /* 1: also compute ||b - A x||_c / ||b||_c in FP64 at the end */
    double *hist_rho;     /* optional HOST buffer: rho_0..rho_iters (length hist_len) */
    double *hist_alpha;   /* optional HOST buffer: alpha_1..alpha_iters at [1..] */
    int hist_len;
    double *kernel_ms;    /* optional HOST [3]: mean duration (ms) of the operator kernel,
                             the gather-scatter kernel and the update kernel of one CG
                             iteration, timed with HIP events on the solver's stream.
                             When set, iterations are launched without graphs. */
    int precond;          /* sem_precond (sem_cg_solve only; batches and the server take
                             SEM_PRECOND_NONE).  With a preconditioner the stopping test,
                             rel_res_recursive and hist_rho stay on <r, r, c>. */
} sem_cg_opts;

typedef struct {
    int iters;                /* CG iterations done (MIXED: total inner iterations) */
    int outer;                /* MIXED: outer refinement steps; else 0 */
    int converged;            /* 1 if the tolerance was met */
    int status;               /* 0 running/ok, 1 converged, 2 iteration cap, 3 breakdown */
    double rel_res_recursive; /* sqrt(rho_i / rho_0) of the last (inner) solve */
    double rel_res_true;      /* FP64 ||b - A x||_c / ||b||_c (if requested; MIXED: always) */
    double seconds;           /* host wall time of the call */
} sem_cg_result;

/*
 * Solve A x = b with Algorithm 1 (CG; unpreconditioned unless opts->precond
 * names one): A = mask o QQ^T o A_L.
 * b, x: DEVICE buffers in local form (continuous, masked), double for
 * SEM_FP64 / SEM_MIXED, float for SEM_FP32.  x holds the initial guess on
 * entry (its Dirichlet entries are zeroed) and the iterate on return.
 * Readings of Algorithm 1 used: rho_0 = <r0, r0, c>; convergence when
 * sqrt(rho_i / rho_0) <= tol; CG scalars are kept in FP64 on the device.
 * SEM_MIXED: outer FP64 residual r = b - A x (FP64 operator), inner FP32 CG
 * on r / ||r||_c to inner_tol, x += ||r||_c d, until ||r||_c / ||b||_c <= tol.
 * Blocks until done.  Returns SEM_EBREAKDOWN if CG broke down (x holds the
 * last iterate).
 */
sem_status sem_cg_solve(sem_mesh_t mesh, const sem_cg_opts *opts, const void *b_dev,
                        void *x_dev, sem_cg_result *result, void *hip_stream);

/*
 * Batched solves: many independent meshes (any mix of E and N) advanced
 * together, one CG iteration of every active problem per step, with the
 * per-problem CG scalars on the device (each problem's arithmetic and
 * reduction order is the same as in its own sem_cg_solve, so its result is
 * bitwise identical).  The batch keeps pointers to the meshes; they must
 * outlive it.  Entries of `meshes` must be distinct.
 */
sem_status sem_batch_create(int count, const sem_mesh_t *meshes, sem_batch_t *out);
void sem_batch_destroy(sem_batch_t batch);

/* b[i], x[i]: DEVICE buffers of problem i (as in sem_cg_solve); results[i]
 * receives its outcome.  Blocks until every problem has stopped. */
sem_status sem_batch_solve(sem_batch_t batch, const sem_cg_opts *opts,
                           const void *const *b_dev, void *const *x_dev,
                           sem_cg_result *results, void *hip_stream);

/*
 * Continuous-batching server (mixed precision only: opts->prec = SEM_MIXED).
 * Requests join and leave at round boundaries; every request runs the
 * refinement of sem_cg_solve(SEM_MIXED) and the inner FP32 iterations of
 * all requests advance together in batched launches (round_iters per
 * round).  A request's result is bitwise that of its own sem_cg_solve.
 * sem_server_add: b_dev / x_dev are DEVICE double [n_local] of the mesh and
 * must stay valid until the request is reported done; x holds the initial
 * guess.  hip_stream is the stream that produced b and x: the server's own
 * stream waits for the work enqueued on it so far before reading them (the
 * call itself does not block).  One request per mesh at a time.
 * sem_server_step: runs one round on the server's own stream, blocks until
 * it is done, writes up to cap finished requests (their tags and results;
 * their x is final), and the number of requests still held.
 */
typedef struct sem_server_s *sem_server_t;
sem_status sem_server_create(const sem_cg_opts *opts, int round_iters, sem_server_t *out);
void sem_server_destroy(sem_server_t server);
sem_status sem_server_add(sem_server_t server, sem_mesh_t mesh, const void *b_dev, void *x_dev,
                          int64_t tag, void *hip_stream);
sem_status sem_server_step(sem_server_t server, int64_t *done_tags, sem_cg_result *done_results,
                           int cap, int *n_done, int *n_active);

/* Upper bound of the device bytes of a mesh of n_elem elements of order N
 * created with `flags`, plus the work vectors of a solve in `prec` (admission
 * by memory footprint). */
sem_status sem_mesh_footprint(int64_t n_elem, int order_N, uint32_t flags, sem_precision prec,
                              size_t *bytes);

/*
 * Tile shape of the local-operator kernels: elements per workgroup for an
 * order, precision (SEM_FP32 / SEM_FP64) and geometric-factor form; one
 * thread per (i, j) column, so a workgroup has roundup64(epb (N+1)^2)
 * threads.  0 restores the built-in default; values are clamped to 512
 * threads and 64 KiB of LDS.  Process-wide, used by later launches (the
 * shape fixes the grouping of the FP64 partial sums, so solves that must
 * agree bitwise need the same shapes).  For the autotuner.
 */
sem_status sem_ax_shape_set(int order_N, sem_precision prec, sem_geom geom, int elems_per_block);
sem_status sem_ax_shape_get(int order_N, sem_precision prec, sem_geom geom, int *elems_per_block,
                            int *threads, size_t *lds_bytes);

/*
 * Contraction engine of the local operator for an order, precision and
 * G form: SEM_AX_ENGINE_VALU runs the D contractions as FP32/FP64 FMAs
 * (one thread per (i, j) column, sem_ax_shape_set picks elements per
 * block); SEM_AX_ENGINE_MFMA runs them on the FP32 matrix cores (16-block
 * 4x4x1 MFMA, one element per workgroup of 64 (N = 7) or 128 (N = 9)
 * threads; available for SEM_FP32 at N = 7 and N = 9, else
 * SEM_EUNSUPPORTED).  The two engines accumulate every
 * contraction in the same order with fused multiply-adds, so their results
 * are bitwise identical.  SEM_AX_ENGINE_DEFAULT restores the built-in
 * choice: the matrix cores at N = 7 in both G forms and at N = 9 with G on
 * the fly, the VALU engine elsewhere.  Process-wide, used by later
 * launches.  For the autotuner.
 */
typedef enum {
    SEM_AX_ENGINE_DEFAULT = 0,
    SEM_AX_ENGINE_VALU = 1,
    SEM_AX_ENGINE_MFMA = 2
} sem_ax_engine;
sem_status sem_ax_engine_set(int order_N, sem_precision prec, sem_geom geom, int engine);
/* The engine later launches use (SEM_AX_ENGINE_VALU or SEM_AX_ENGINE_MFMA). */
sem_status sem_ax_engine_get(int order_N, sem_precision prec, sem_geom geom, int *engine);

/*
 * Cache size the CG drivers assume (process-wide).  MI355X holds a 256 MB
 * Infinity Cache in front of HBM; a CG iteration whose vectors, gather
 * records and edge copy (of one mesh, or of all members of a batch) exceed
 * it runs the CG-fused operator with non-temporal accesses to p and x, the
 * two vectors nothing else reads within an iteration, so that the cache
 * keeps what the group sums and the update read again (FP32; FP64 with G on
 * the fly).  The results are bitwise the same either way.
 *   bytes   > 0: the size assumed; 0: back to 256 MiB.
 * Applies to solves started afterwards (captured iteration graphs and batch
 * tables are rebuilt).  Errors: SEM_EINVAL (bytes < 0).
 */
sem_status sem_set_cache_bytes(int64_t bytes);

/* Message for the last failing call on this thread ("" if none). */
const char *sem_last_error(void);

/* Library version string. */
const char *sem_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SEM_H */
