/*
 * sem_oracle.c -- plain FP64 CPU reference of the spectral-element Poisson
 * CG hot path (Karp et al., HPC Asia 2022, arXiv 2108.12188).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this file's library.  It shares
 * no code with the HIP library: GLL points, the derivative matrix, the
 * geometric factors, the operator, gather-scatter and CG are all written
 * here again, in the plainest form, straight from their definitions.
 *
 * Conventions
 *   P = N+1, local point l = i + P*(j + P*k) inside an element, elements
 *   stored one after the other (element-major).
 *   vert[e][v][d]: vertex v = a + 2b + 4c sits at reference corner
 *   (xi, eta, gamma) = (2a-1, 2b-1, 2c-1).
 *   G[e][c][q] with component order c = (G11, G12, G13, G22, G23, G33).
 *
 * Readings of the paper that this file takes (the paper leaves them open):
 *   - the problem is -Laplace(u) = f (the weak form of Eq. 2 is that of
 *     the negative Laplacian, Sec. 3);
 *   - G = w_q |J| J^-1 J^-T, the standard SEM geometric factors that Eq. 4
 *     leaves undefined;
 *   - D_ij = l_j'(xi_i), Lagrange interpolants through the GLL points;
 *   - c = 1/multiplicity in the weighted inner product of Algorithm 1;
 *   - rho_0 = <r0, r0, c>; stop when sqrt(rho_i / rho_0) <= tol;
 *   - the Dirichlet mask is applied to b (and x0) as well as to w.
 *
 * Every function is pinned by tests against closed forms, invariants and an
 * independent dense brute force (tests/test_oracle_*.py).
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXP 32

/* threads the OpenMP loops of this file use */
int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* sets the threads of the OpenMP loops that follow (k >= 1; for timing:
   every result of this file is independent of the thread count, the dot
   sums fixed blocks of 512 terms) */
void or_set_num_threads(int k)
{
#ifdef _OPENMP
    if (k >= 1) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

/* ------------------------------------------------------------------ */
/* O1. GLL points and weights (Sec. 3, Eq. 3): xi_0 = -1, xi_N = 1, the
 * interior points are the roots of L_N', the weights are
 * 2 / (N (N+1) L_N(xi)^2).                                            */

/* Legendre L_N(x) and its first two derivatives by the three-term
 * recurrence (k+1) L_{k+1} = (2k+1) x L_k - k L_{k-1}. */
static void legendre(int N, double x, double *L, double *dL, double *d2L)
{
    double p0 = 1.0, p1 = x;      /* L_0, L_1 */
    double d0 = 0.0, d1 = 1.0;    /* L_0', L_1' */
    double s0 = 0.0, s1 = 0.0;    /* L_0'', L_1'' */
    if (N == 0) { *L = 1.0; *dL = 0.0; *d2L = 0.0; return; }
    for (int k = 1; k < N; ++k) {
        double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
        double d2 = ((2 * k + 1) * (p1 + x * d1) - k * d0) / (k + 1);
        double s2 = ((2 * k + 1) * (2 * d1 + x * s1) - k * s0) / (k + 1);
        p0 = p1; p1 = p2; d0 = d1; d1 = d2; s0 = s1; s1 = s2;
    }
    *L = p1; *dL = d1; *d2L = s1;
}

int or_gll(int N, double *xi, double *w)
{
    if (N < 1 || N + 1 > OR_MAXP) return -1;
    xi[0] = -1.0;
    xi[N] = 1.0;
    for (int j = 1; j < N; ++j) {
        double x = -cos(M_PI * j / N);   /* Chebyshev-Gauss-Lobatto guess */
        for (int it = 0; it < 100; ++it) {
            double L, dL, d2L;
            legendre(N, x, &L, &dL, &d2L);
            double dx = dL / d2L;        /* Newton on L_N' */
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        xi[j] = x;
    }
    for (int j = 0; j <= N; ++j) {
        double L, dL, d2L;
        legendre(N, xi[j], &L, &dL, &d2L);
        w[j] = 2.0 / (N * (N + 1.0) * L * L);
    }
    return 0;
}

/* O2. Derivative matrix D_ij = l_j'(xi_i) (Sec. 3, Eq. 4), textbook
 * closed form for Lagrange interpolants through the GLL points. */
int or_deriv(int N, const double *xi, double *D)
{
    int P = N + 1;
    if (N < 1 || P > OR_MAXP) return -1;
    double Lv[OR_MAXP];
    for (int i = 0; i < P; ++i) {
        double dL, d2L;
        legendre(N, xi[i], &Lv[i], &dL, &d2L);
    }
    for (int i = 0; i < P; ++i)
        for (int j = 0; j < P; ++j) {
            double v;
            if (i != j) v = Lv[i] / (Lv[j] * (xi[i] - xi[j]));
            else if (i == 0) v = -N * (N + 1.0) / 4.0;
            else if (i == N) v = N * (N + 1.0) / 4.0;
            else v = 0.0;
            D[i * P + j] = v;
        }
    return 0;
}

/* ------------------------------------------------------------------ */
/* O4. Geometry of linearly deformed hexahedra (Sec. 5.1: trilinear map
 * from the eight vertices).  X(xi) = sum_abc v_abc phi_a(xi) phi_b(eta)
 * phi_c(gamma), phi_0(s) = (1-s)/2, phi_1(s) = (1+s)/2.               */

static double phi(int a, double s) { return a ? 0.5 * (1.0 + s) : 0.5 * (1.0 - s); }
static double dphi(int a) { return a ? 0.5 : -0.5; }

/* Jacobian J[d][r] = dX_d / dxi_r at reference point (x, y, z). */
static void jacobian(const double *v, double x, double y, double z, double J[3][3])
{
    for (int d = 0; d < 3; ++d)
        for (int r = 0; r < 3; ++r) J[d][r] = 0.0;
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                const double *p = v + 3 * (a + 2 * b + 4 * c);
                double gx = dphi(a) * phi(b, y) * phi(c, z);
                double gy = phi(a, x) * dphi(b) * phi(c, z);
                double gz = phi(a, x) * phi(b, y) * dphi(c);
                for (int d = 0; d < 3; ++d) {
                    J[d][0] += p[d] * gx;
                    J[d][1] += p[d] * gy;
                    J[d][2] += p[d] * gz;
                }
            }
}

static double det3(double J[3][3])
{
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
         - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
         + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

/* inverse by the adjugate: Ji = adj(J) / det(J) */
static void inv3(double J[3][3], double det, double Ji[3][3])
{
    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
}

/* G[e][6][P^3] = w_q |J| J^-1 J^-T (components 11,12,13,22,23,33) and the
 * diagonal mass B[e][P^3] = w_q |J|.  Returns -1, or the first element
 * whose Jacobian determinant is not positive at some GLL point. */
long or_geom(long E, int N, const double *vert, const double *xi, const double *w,
             double *G, double *B)
{
    int P = N + 1;
    long P3 = (long)P * P * P;
    long bad = -1;
    for (long e = 0; e < E; ++e) {
        const double *v = vert + 24 * e;
        for (int k = 0; k < P; ++k)
            for (int j = 0; j < P; ++j)
                for (int i = 0; i < P; ++i) {
                    long q = i + P * (j + (long)P * k);
                    double J[3][3], Ji[3][3];
                    jacobian(v, xi[i], xi[j], xi[k], J);
                    double det = det3(J);
                    if (!(det > 0.0)) {
                        if (bad < 0) bad = e;
                        det = 1.0;
                    }
                    inv3(J, det, Ji);
                    double s = w[i] * w[j] * w[k] * det;
                    double g[3][3];
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) {
                            double t = 0.0;
                            for (int d = 0; d < 3; ++d) t += Ji[a][d] * Ji[b][d];
                            g[a][b] = s * t;
                        }
                    double *Ge = G + 6 * P3 * e;
                    Ge[0 * P3 + q] = g[0][0];
                    Ge[1 * P3 + q] = g[0][1];
                    Ge[2 * P3 + q] = g[0][2];
                    Ge[3 * P3 + q] = g[1][1];
                    Ge[4 * P3 + q] = g[1][2];
                    Ge[5 * P3 + q] = g[2][2];
                    if (B) B[P3 * e + q] = s;
                }
    }
    return bad;
}

/* physical coordinates of every local GLL point: xyz[3][n] */
void or_coords(long E, int N, const double *vert, const double *xi, double *xyz)
{
    int P = N + 1;
    long P3 = (long)P * P * P, n = E * P3;
    for (long e = 0; e < E; ++e) {
        const double *v = vert + 24 * e;
        for (int k = 0; k < P; ++k)
            for (int j = 0; j < P; ++j)
                for (int i = 0; i < P; ++i) {
                    long l = e * P3 + i + P * (j + (long)P * k);
                    for (int d = 0; d < 3; ++d) {
                        double s = 0.0;
                        for (int c = 0; c < 2; ++c)
                            for (int b = 0; b < 2; ++b)
                                for (int a = 0; a < 2; ++a)
                                    s += v[3 * (a + 2 * b + 4 * c) + d]
                                         * phi(a, xi[i]) * phi(b, xi[j]) * phi(c, xi[k]);
                        xyz[d * n + l] = s;
                    }
                }
    }
}

/* ------------------------------------------------------------------ */
/* O5. Local operator w_e = D^T G^e D u_e for every element (Eq. 4-5):
 * u_r = sum_l D_il u_ljk, u_s = sum_l D_jl u_ilk, u_t = sum_l D_kl u_ijl,
 * (v_r, v_s, v_t) = G (u_r, u_s, u_t),
 * w_ijk = sum_l D_li v_r,ljk + D_lj v_s,ilk + D_lk v_t,ijl.            */
void or_ax_local(long E, int N, const double *D, const double *G,
                 const double *u, double *w)
{
    int P = N + 1;
    long P3 = (long)P * P * P;
#pragma omp parallel for schedule(static)
    for (long e = 0; e < E; ++e) {
        double *vr = (double *)malloc(sizeof(double) * 3 * P3);
        double *vs = vr + P3, *vt = vs + P3;
        const double *ue = u + e * P3;
        const double *Ge = G + 6 * P3 * e;
        double *we = w + e * P3;
        for (int k = 0; k < P; ++k)
            for (int j = 0; j < P; ++j)
                for (int i = 0; i < P; ++i) {
                    long q = i + P * (j + (long)P * k);
                    double ur = 0.0, us = 0.0, ut = 0.0;
                    for (int l = 0; l < P; ++l) {
                        ur += D[i * P + l] * ue[l + P * (j + P * k)];
                        us += D[j * P + l] * ue[i + P * (l + P * k)];
                        ut += D[k * P + l] * ue[i + P * (j + P * l)];
                    }
                    double g11 = Ge[q], g12 = Ge[P3 + q], g13 = Ge[2 * P3 + q];
                    double g22 = Ge[3 * P3 + q], g23 = Ge[4 * P3 + q], g33 = Ge[5 * P3 + q];
                    vr[q] = g11 * ur + g12 * us + g13 * ut;
                    vs[q] = g12 * ur + g22 * us + g23 * ut;
                    vt[q] = g13 * ur + g23 * us + g33 * ut;
                }
        for (int k = 0; k < P; ++k)
            for (int j = 0; j < P; ++j)
                for (int i = 0; i < P; ++i) {
                    double s = 0.0;
                    for (int l = 0; l < P; ++l) {
                        s += D[l * P + i] * vr[l + P * (j + P * k)];
                        s += D[l * P + j] * vs[i + P * (l + P * k)];
                        s += D[l * P + k] * vt[i + P * (j + P * l)];
                    }
                    we[i + P * (j + P * k)] = s;
                }
        free(vr);
    }
}

/* ------------------------------------------------------------------ */
/* O6. Gather-scatter QQ^T (Sec. 3.1 and 4.3): every local copy of a
 * global point receives the sum of all copies, summed in ascending local
 * index.  sum is caller scratch of n_glob doubles.                    */
void or_gs(long n, const int64_t *glob_id, long n_glob, double *w, double *sum)
{
    memset(sum, 0, sizeof(double) * n_glob);
    for (long l = 0; l < n; ++l) sum[glob_id[l]] += w[l];
    for (long l = 0; l < n; ++l) w[l] = sum[glob_id[l]];
}

/* Dirichlet mask (Algorithm 1, mask step): zero every boundary copy. */
void or_mask(long n, const uint8_t *dirichlet, double *w)
{
    for (long l = 0; l < n; ++l)
        if (dirichlet[l]) w[l] = 0.0;
}

/* multiplicity m_l = number of local copies of the global point of l */
void or_multiplicity(long n, const int64_t *glob_id, long n_glob, double *m)
{
    double *cnt = (double *)calloc(n_glob, sizeof(double));
    for (long l = 0; l < n; ++l) cnt[glob_id[l]] += 1.0;
    for (long l = 0; l < n; ++l) m[l] = cnt[glob_id[l]];
    free(cnt);
}

/* O7. Weighted inner product <a, b, c> = sum_l a_l b_l c_l with c = 1/m
 * (Algorithm 1).  Sums in blocks of `blk` points, then the block sums
 * pairwise, so rounding stays small at large n. */
static double pairwise(double *s, long cnt)
{
    while (cnt > 1) {
        long h = (cnt + 1) / 2;
        for (long t = 0; t + h < cnt; ++t) s[t] += s[t + h];
        cnt = h;
    }
    return cnt ? s[0] : 0.0;
}

double or_dot(long n, const double *a, const double *b, const double *m)
{
    const long blk = 512;
    long nb = (n + blk - 1) / blk;
    double *s = (double *)malloc(sizeof(double) * (nb > 0 ? nb : 1));
#pragma omp parallel for schedule(static)
    for (long t = 0; t < nb; ++t) {
        double acc = 0.0;
        long hi = (t + 1) * blk < n ? (t + 1) * blk : n;
        for (long l = t * blk; l < hi; ++l) acc += a[l] * b[l] / m[l];
        s[t] = acc;
    }
    double r = pairwise(s, nb);
    free(s);
    return r;
}

/* ------------------------------------------------------------------ */
/* The full operator of Algorithm 1, mask(QQ^T A_L u).                 */
typedef struct {
    long E; int N; long n; long n_glob;
    const double *D, *G; const int64_t *glob_id; const uint8_t *dirichlet;
    double *sum;
} or_op;

static void apply_A(const or_op *op, const double *u, double *w)
{
    or_ax_local(op->E, op->N, op->D, op->G, u, w);
    or_gs(op->n, op->glob_id, op->n_glob, w, op->sum);
    or_mask(op->n, op->dirichlet, w);
}

void or_apply_A(long E, int N, const double *D, const double *G, const int64_t *glob_id,
                long n_glob, const uint8_t *dirichlet, const double *u, double *w)
{
    or_op op = {E, N, E * (long)(N + 1) * (N + 1) * (N + 1), n_glob, D, G, glob_id,
                dirichlet, (double *)malloc(sizeof(double) * n_glob)};
    apply_A(&op, u, w);
    free(op.sum);
}

/* O9. Unpreconditioned CG on SEM, Algorithm 1, steps in the paper's order.
 * x holds x0 on entry (masked by the caller) and the solution on exit.
 * tol > 0: stop when sqrt(rho_i/rho_0) <= tol; fixed > 0: run exactly
 * `fixed` iterations.  Histories (length max_iter+1, may be NULL):
 * rho[i] (rho[0] = rho_0), alpha[i], beta[i] for i >= 1.
 * Returns the number of iterations done. */
int or_cg(long E, int N, const double *D, const double *G, const int64_t *glob_id,
          long n_glob, const uint8_t *dirichlet, const double *m, const double *b,
          double *x, double tol, int max_iter, int fixed,
          double *rho_hist, double *alpha_hist, double *beta_hist)
{
    long n = E * (long)(N + 1) * (N + 1) * (N + 1);
    or_op op = {E, N, n, n_glob, D, G, glob_id, dirichlet,
                (double *)malloc(sizeof(double) * n_glob)};
    double *r = (double *)malloc(sizeof(double) * n);
    double *p = (double *)malloc(sizeof(double) * n);
    double *w = (double *)malloc(sizeof(double) * n);
    apply_A(&op, x, w);
    for (long l = 0; l < n; ++l) r[l] = b[l] - w[l];      /* r0 = b - A x0 */
    double beta = 0.0;                                      /* beta_0 = 0 */
    for (long l = 0; l < n; ++l) p[l] = 0.0;                /* p0 = 0 */
    double rho_prev = or_dot(n, r, r, m);                   /* rho_0 */
    double rho0 = rho_prev;
    if (rho_hist) rho_hist[0] = rho0;
    int it = 0;
    int limit = fixed > 0 ? fixed : max_iter;
    if (fixed <= 0 && rho0 == 0.0) limit = 0;
    for (int i = 1; i <= limit; ++i) {
        for (long l = 0; l < n; ++l) p[l] = r[l] + beta * p[l];
        apply_A(&op, p, w);                                  /* w = QQ^T A_L p, masked */
        double alpha = rho_prev / or_dot(n, p, w, m);
        for (long l = 0; l < n; ++l) x[l] += alpha * p[l];
        for (long l = 0; l < n; ++l) r[l] -= alpha * w[l];
        double rho = or_dot(n, r, r, m);
        beta = rho / rho_prev;
        if (rho_hist) rho_hist[i] = rho;
        if (alpha_hist) alpha_hist[i] = alpha;
        if (beta_hist) beta_hist[i] = beta;
        rho_prev = rho;
        it = i;
        if (fixed <= 0 && sqrt(rho / rho0) <= tol) break;
    }
    free(r); free(p); free(w); free(op.sum);
    return it;
}

/* ------------------------------------------------------------------ */
/* f4. Jacobi preconditioner: the diagonal of the assembled operator
 * A = Q^T A_L Q (Sec. 3, Eq. 4), in local (replicated) form.
 * Element diagonal from the definition A_L = sum_{a,b} D_a^T G_ab D_b:
 * (A_L)_qq = sum_{a,b} sum_q' (D_a)_{q'q} G_ab(q') (D_b)_{q'q}, where
 * (D_r)_{q'q} = D[i'][i] if (j',k') = (j,k) and 0 otherwise (likewise D_s
 * along j, D_t along k).  For a = b, q' runs over the line through q in
 * direction a; for a != b the two lines meet only at q' = q.
 * The element diagonals are then summed over the copies of every global
 * point (gather-scatter).  diag is n doubles. */
void or_diag_A(long E, int N, const double *D, const double *G, const int64_t *glob_id,
               long n_glob, double *diag)
{
    int P = N + 1;
    long P3 = (long)P * P * P;
#pragma omp parallel for schedule(static)
    for (long e = 0; e < E; ++e) {
        const double *Ge = G + 6 * P3 * e;
        for (int k = 0; k < P; ++k)
            for (int j = 0; j < P; ++j)
                for (int i = 0; i < P; ++i) {
                    long q = i + P * (j + (long)P * k);
                    double s = 0.0;
                    for (int l = 0; l < P; ++l) {
                        s += D[l * P + i] * D[l * P + i] * Ge[0 * P3 + l + P * (j + P * k)];
                        s += D[l * P + j] * D[l * P + j] * Ge[3 * P3 + i + P * (l + P * k)];
                        s += D[l * P + k] * D[l * P + k] * Ge[5 * P3 + i + P * (j + P * l)];
                    }
                    s += 2.0 * D[i * P + i] * D[j * P + j] * Ge[1 * P3 + q];
                    s += 2.0 * D[i * P + i] * D[k * P + k] * Ge[2 * P3 + q];
                    s += 2.0 * D[j * P + j] * D[k * P + k] * Ge[4 * P3 + q];
                    diag[e * P3 + q] = s;
                }
    }
    double *sum = (double *)malloc(sizeof(double) * n_glob);
    or_gs(E * P3, glob_id, n_glob, diag, sum);
    free(sum);
}

/* f4. Jacobi-preconditioned CG: Algorithm 1 with z = M^-1 r (M the
 * diagonal of A on the free points; minv = 1/diag there and 0 on the
 * Dirichlet points): p_i = z_{i-1} + beta p_{i-1}, alpha = <r,z>/<p,w>,
 * beta = <r_i,z_i>/<r_{i-1},z_{i-1}>.  The stopping test is the same as
 * or_cg's, on <r, r, c>.  Histories as or_cg, rho_hist holding <r, r, c>.
 * Returns the number of iterations done. */
int or_pcg(long E, int N, const double *D, const double *G, const int64_t *glob_id,
           long n_glob, const uint8_t *dirichlet, const double *m, const double *minv,
           const double *b, double *x, double tol, int max_iter, int fixed,
           double *rho_hist, double *alpha_hist, double *beta_hist)
{
    long n = E * (long)(N + 1) * (N + 1) * (N + 1);
    or_op op = {E, N, n, n_glob, D, G, glob_id, dirichlet,
                (double *)malloc(sizeof(double) * n_glob)};
    double *r = (double *)malloc(sizeof(double) * n);
    double *z = (double *)malloc(sizeof(double) * n);
    double *p = (double *)malloc(sizeof(double) * n);
    double *w = (double *)malloc(sizeof(double) * n);
    apply_A(&op, x, w);
    for (long l = 0; l < n; ++l) r[l] = b[l] - w[l];      /* r0 = b - A x0 */
    for (long l = 0; l < n; ++l) z[l] = minv[l] * r[l];   /* z0 = M^-1 r0 */
    double beta = 0.0;
    for (long l = 0; l < n; ++l) p[l] = 0.0;
    double rz_prev = or_dot(n, r, z, m);
    double rr0 = or_dot(n, r, r, m);
    if (rho_hist) rho_hist[0] = rr0;
    int it = 0;
    int limit = fixed > 0 ? fixed : max_iter;
    if (fixed <= 0 && rr0 == 0.0) limit = 0;
    for (int i = 1; i <= limit; ++i) {
        for (long l = 0; l < n; ++l) p[l] = z[l] + beta * p[l];
        apply_A(&op, p, w);
        double alpha = rz_prev / or_dot(n, p, w, m);
        for (long l = 0; l < n; ++l) x[l] += alpha * p[l];
        for (long l = 0; l < n; ++l) r[l] -= alpha * w[l];
        for (long l = 0; l < n; ++l) z[l] = minv[l] * r[l];
        double rz = or_dot(n, r, z, m);
        double rr = or_dot(n, r, r, m);
        beta = rz / rz_prev;
        if (rho_hist) rho_hist[i] = rr;
        if (alpha_hist) alpha_hist[i] = alpha;
        if (beta_hist) beta_hist[i] = beta;
        rz_prev = rz;
        it = i;
        if (fixed <= 0 && sqrt(rr / rr0) <= tol) break;
    }
    free(r); free(z); free(p); free(w); free(op.sum);
    return it;
}
