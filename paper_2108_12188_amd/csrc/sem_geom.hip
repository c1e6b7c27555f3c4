// sem_geom.hip -- FP64 setup of the geometric factors, mass and coordinates.
//
// Elements are trilinear images of the reference cube (Sec. 5.1: "linearly
// deformed").  At GLL point (xi_i, xi_j, xi_k) the columns of the Jacobian
// are x_xi, x_eta, x_gamma; with the cofactor rows r0 = x_eta x x_gamma,
// r1 = x_gamma x x_xi, r2 = x_xi x x_eta and |J| = x_xi . r0, the inverse
// Jacobian rows are r_a / |J|, so the symmetric factors of Eq. 4 are
//   G_ab = w_q |J| (J^-1 J^-T)_ab = (w_q / |J|) r_a . r_b,
// stored as (G11, G12, G13, G22, G23, G33), and the diagonal mass is
// B_q = w_q |J|.
#include "sem_internal.h"

namespace sem {
namespace {

struct GeomArgs {
    int64_t E;
    int P;
    const double *vert;
    const double *xi;
    const double *w;
    double *G64;
    float *G32;
    double *B64;
    unsigned long long *bad;   // smallest element index with |J| <= 0
};

__device__ __forceinline__ void corner(const double *v, int c, double out[3]) {
    out[0] = v[3 * c];
    out[1] = v[3 * c + 1];
    out[2] = v[3 * c + 2];
}

// Jacobian columns of the trilinear map at reference point (x, y, z).
__device__ void jac_columns(const double *v, double x, double y, double z, double Jx[3],
                            double Jy[3], double Jz[3]) {
    const double fx[2] = {0.5 * (1 - x), 0.5 * (1 + x)};
    const double fy[2] = {0.5 * (1 - y), 0.5 * (1 + y)};
    const double fz[2] = {0.5 * (1 - z), 0.5 * (1 + z)};
    const double dx[2] = {-0.5, 0.5};
    for (int d = 0; d < 3; ++d) {
        Jx[d] = Jy[d] = Jz[d] = 0.0;
    }
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                double p[3];
                corner(v, a + 2 * b + 4 * c, p);
                const double sx = dx[a] * fy[b] * fz[c];
                const double sy = fx[a] * dx[b] * fz[c];
                const double sz = fx[a] * fy[b] * dx[c];
                for (int d = 0; d < 3; ++d) {
                    Jx[d] += sx * p[d];
                    Jy[d] += sy * p[d];
                    Jz[d] += sz * p[d];
                }
            }
}

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ __forceinline__ double dotv(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// The six factors (G11, G12, G13, G22, G23, G33) at GLL point (i, j, k)
// of the element with vertices v; returns |J| (weights w, points xi).
__device__ double gfactors(const double *v, const double *xi, const double *w, int i, int j,
                           int k, double G[6], double *wq_out = nullptr) {
    double Jx[3], Jy[3], Jz[3];
    jac_columns(v, xi[i], xi[j], xi[k], Jx, Jy, Jz);
    double r0[3], r1[3], r2[3];
    cross3(Jy, Jz, r0);
    cross3(Jz, Jx, r1);
    cross3(Jx, Jy, r2);
    const double det = dotv(Jx, r0);
    const double wq = w[i] * w[j] * w[k];
    const double s = wq / det;
    G[0] = s * dotv(r0, r0);
    G[1] = s * dotv(r0, r1);
    G[2] = s * dotv(r0, r2);
    G[3] = s * dotv(r1, r1);
    G[4] = s * dotv(r1, r2);
    G[5] = s * dotv(r2, r2);
    if (wq_out) *wq_out = wq;
    return det;
}

__global__ void geometry_kernel(GeomArgs g) {
    const int P = g.P, P2 = P * P, P3 = P2 * P;
    const int64_t n = g.E * P3;
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n) return;
    const int64_t e = l / P3;
    const int q = (int)(l - e * P3);
    const int i = q % P, j = (q / P) % P, k = q / P2;
    double G[6], wq = 0.0;
    const double det = gfactors(g.vert + 24 * e, g.xi, g.w, i, j, k, G, &wq);
    if (!(det > 0.0)) atomicMin(g.bad, (unsigned long long)e);
    const int64_t gb = e * 6 * P3 + q;
    if (g.G64)
        for (int c = 0; c < 6; ++c) g.G64[gb + (int64_t)c * P3] = G[c];
    if (g.G32)
        for (int c = 0; c < 6; ++c) g.G32[gb + (int64_t)c * P3] = (float)G[c];
    g.B64[l] = wq * det;
}

// Diagonal of the element operator A_L = sum_{a,b} D_a^T G_ab D_b (Eq. 4)
// at local point q = (i, j, k): the unit vector e_q has derivative
// D[l][i] along the i-line through q (likewise j, k), so the diagonal
// blocks contribute sum_l D[l][i]^2 G11(l, j, k) (and the j-, k-lines),
// and the mixed blocks, whose lines meet only at q, 2 D[i][i] D[j][j] G12(q)
// and so on.  The factors come from the vertices (FP64), so the result
// does not depend on which G form the mesh stores.
__global__ void diag_local_kernel(int64_t E, int P, const double *vert, const double *xi,
                                  const double *w, const double *D, double *diag) {
    const int P2 = P * P, P3 = P2 * P;
    const int64_t n = E * P3;
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n) return;
    const int64_t e = l / P3;
    const int q = (int)(l - e * P3);
    const int i = q % P, j = (q / P) % P, k = q / P2;
    const double *v = vert + 24 * e;
    double G[6];
    double s = 0.0;
    for (int t = 0; t < P; ++t) {
        gfactors(v, xi, w, t, j, k, G);
        s += D[t * P + i] * D[t * P + i] * G[0];
        gfactors(v, xi, w, i, t, k, G);
        s += D[t * P + j] * D[t * P + j] * G[3];
        gfactors(v, xi, w, i, j, t, G);
        s += D[t * P + k] * D[t * P + k] * G[5];
    }
    gfactors(v, xi, w, i, j, k, G);
    const double di = D[i * P + i], dj = D[j * P + j], dk = D[k * P + k];
    s += 2.0 * di * dj * G[1];
    s += 2.0 * di * dk * G[2];
    s += 2.0 * dj * dk * G[4];
    diag[l] = s;
}

__global__ void coords_kernel(int64_t E, int P, const double *vert, const double *xi,
                              double *xyz) {
    const int P2 = P * P, P3 = P2 * P;
    const int64_t n = E * P3;
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n) return;
    const int64_t e = l / P3;
    const int q = (int)(l - e * P3);
    const double x = xi[q % P], y = xi[(q / P) % P], z = xi[q / P2];
    const double fx[2] = {0.5 * (1 - x), 0.5 * (1 + x)};
    const double fy[2] = {0.5 * (1 - y), 0.5 * (1 + y)};
    const double fz[2] = {0.5 * (1 - z), 0.5 * (1 + z)};
    const double *v = vert + 24 * e;
    double s[3] = {0, 0, 0};
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                const double f = fx[a] * fy[b] * fz[c];
                for (int d = 0; d < 3; ++d) s[d] += f * v[3 * (a + 2 * b + 4 * c) + d];
            }
    for (int d = 0; d < 3; ++d) xyz[(int64_t)d * n + l] = s[d];
}

}  // namespace

int64_t launch_geometry(Mesh &m, hipStream_t s) {
    unsigned long long *bad = nullptr;
    SEM_HIP(hipMalloc(&bad, sizeof(unsigned long long)));
    SEM_HIP(hipMemsetAsync(bad, 0xFF, sizeof(unsigned long long), s));
    GeomArgs g{m.E, m.P, m.vert64, m.b64.xi, m.b64.w, m.G64, m.G32, m.B64, bad};
    const int64_t nb = (m.n + 255) / 256;
    hipLaunchKernelGGL(geometry_kernel, dim3((unsigned)nb), dim3(256), 0, s, g);
    hipError_t le = hipGetLastError();
    unsigned long long res = 0;
    hipError_t ce = hipMemcpyAsync(&res, bad, sizeof res, hipMemcpyDeviceToHost, s);
    hipError_t se = hipStreamSynchronize(s);
    (void)hipFree(bad);
    check_hip(le, "geometry kernel launch");
    check_hip(ce, "geometry result copy");
    check_hip(se, "geometry kernel");
    return res == ~0ull ? -1 : (int64_t)res;
}

void launch_diag_local(const Mesh &m, double *d, hipStream_t s) {
    const int64_t nb = (m.n + 255) / 256;
    hipLaunchKernelGGL(diag_local_kernel, dim3((unsigned)nb), dim3(256), 0, s, m.E, m.P, m.vert64,
                       m.b64.xi, m.b64.w, m.b64.D, d);
    check_hip(hipGetLastError(), "diagonal kernel launch");
}

void launch_coords(const Mesh &m, double *xyz, hipStream_t s) {
    const int64_t nb = (m.n + 255) / 256;
    hipLaunchKernelGGL(coords_kernel, dim3((unsigned)nb), dim3(256), 0, s, m.E, m.P, m.vert64,
                       m.b64.xi, xyz);
    check_hip(hipGetLastError(), "coords kernel launch");
}

}  // namespace sem
