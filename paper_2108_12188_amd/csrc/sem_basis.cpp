// sem_basis.cpp -- GLL points, weights and the derivative matrix (host, FP64).
//
// The basis of Sec. 3 (Eq. 3): Lagrange interpolants through the N+1
// Gauss-Lobatto-Legendre points.  The interior points are the roots of
// L_N', which is proportional to the Jacobi polynomial P^(1,1)_{N-1}; they
// are found by Newton iteration on that polynomial.  The derivative matrix
// (Eq. 4, "D") uses the barycentric form D_ij = (lam_j/lam_i)/(x_i - x_j)
// with the diagonal set to minus the off-diagonal row sum, so D annihilates
// constants to rounding.
#include <cmath>

#include "sem_internal.h"

namespace sem {

// P^(1,1)_n(x) and its derivative by the three-term recurrence
//   n(n+2) P_n = (2n+1)(n+1) x P_{n-1} - n(n+1) P_{n-2},  P_0 = 1, P_1 = 2x.
static void jacobi11(int n, double x, double &p, double &dp) {
    double pm2 = 0.0, pm1 = 1.0, dm2 = 0.0, dm1 = 0.0;
    if (n == 0) {
        p = 1.0;
        dp = 0.0;
        return;
    }
    for (int k = 1; k <= n; ++k) {
        const double a = (2.0 * k + 1.0) * (k + 1.0), b = k * (k + 1.0), c = k * (k + 2.0);
        const double pk = (a * x * pm1 - b * pm2) / c;
        const double dk = (a * (pm1 + x * dm1) - b * dm2) / c;
        pm2 = pm1;
        pm1 = pk;
        dm2 = dm1;
        dm1 = dk;
    }
    p = pm1;
    dp = dm1;
}

static double legendre_value(int n, double x) {
    double a = 1.0, b = x;
    if (n == 0) return 1.0;
    for (int k = 1; k < n; ++k) {
        const double c = ((2.0 * k + 1.0) * x * b - k * a) / (k + 1.0);
        a = b;
        b = c;
    }
    return b;
}

void gll_points(int N, std::vector<double> &xi, std::vector<double> &w) {
    const int P = N + 1;
    xi.assign(P, 0.0);
    w.assign(P, 0.0);
    xi[0] = -1.0;
    xi[N] = 1.0;
    for (int j = 1; j < N; ++j) {
        double x = -std::cos(M_PI * j / N);
        for (int it = 0; it < 60; ++it) {
            double p, dp;
            jacobi11(N - 1, x, p, dp);
            const double step = p / dp;
            x -= step;
            if (std::fabs(step) <= 1e-17) break;
        }
        xi[j] = x;
    }
    // symmetrise (the point set is symmetric about 0)
    for (int j = 0; j < P / 2; ++j) {
        const double s = 0.5 * (xi[N - j] - xi[j]);
        xi[j] = -s;
        xi[N - j] = s;
    }
    if (P % 2 == 1) xi[N / 2] = 0.0;
    for (int j = 0; j < P; ++j) {
        const double L = legendre_value(N, xi[j]);
        w[j] = 2.0 / (N * (N + 1.0) * L * L);
    }
}

void derivative_matrix(const std::vector<double> &xi, std::vector<double> &D) {
    const int P = (int)xi.size();
    std::vector<double> lam(P, 1.0);
    for (int j = 0; j < P; ++j) {
        double prod = 1.0;
        for (int k = 0; k < P; ++k)
            if (k != j) prod *= (xi[j] - xi[k]);
        lam[j] = 1.0 / prod;
    }
    D.assign((size_t)P * P, 0.0);
    for (int i = 0; i < P; ++i) {
        double row = 0.0;
        for (int j = 0; j < P; ++j) {
            if (j == i) continue;
            const double v = (lam[j] / lam[i]) / (xi[i] - xi[j]);
            D[(size_t)i * P + j] = v;
            row += v;
        }
        D[(size_t)i * P + i] = -row;
    }
}

}  // namespace sem
