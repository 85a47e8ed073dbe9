// Eigen-decomposition of a real symmetric tridiagonal matrix (host only):
// implicit QL iteration with Wilkinson shifts, accumulating the eigenvectors
// (Golub & Van Loan, "Matrix Computations", the symmetric tridiagonal QR/QL
// step).  Used to evaluate a function of a Lanczos matrix T_k.
#pragma once

#include <cmath>
#include <vector>

namespace ovl {

// d[0..n-1] diagonal, e[0..n-2] off-diagonal (destroyed).  On return d holds
// the eigenvalues and Z (nrow x n, row-major, Z[r*n + j] = component row0 + r
// of eigenvector j) the requested rows of the orthonormal eigenvectors: all
// of them by default, or e.g. only the last (nrow 1, row0 n-1), which costs
// O(n^2) instead of O(n^3).  Returns false if an eigenvalue fails to
// converge in 60 sweeps.
// One plane rotation of the eigenvector accumulation: columns i, i+1 of Z
// become (c z_i - s z_{i+1}, s z_i + c z_{i+1}).
struct PlaneRot {
    int i;
    double c, s;
};

inline bool tridiag_eig(int n, std::vector<double> &d, std::vector<double> e, std::vector<double> &Z, int nrow = -1,
                        int row0 = 0, std::vector<PlaneRot> *rots = nullptr)
{
    if (nrow < 0) nrow = n, row0 = 0;
    Z.assign((size_t)nrow * n, 0.0);
    for (int r = 0; r < nrow; r++) Z[(size_t)r * n + row0 + r] = 1.0;
    if (n == 1) return true;
    e.resize(n);
    e[n - 1] = 0.0;
    for (int l = 0; l < n; l++) {
        int iter = 0;
        for (;;) {
            // the first negligible off-diagonal at or after l splits the matrix
            int m = l;
            for (; m < n - 1; m++) {
                const double s = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= 1e-16 * s) break;
            }
            if (m == l) break;
            if (++iter > 60) return false;
            // Wilkinson shift from the leading 2x2 block of rows l, l+1
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
            double s = 1.0, c = 1.0, p = 0.0;
            int i = m - 1;
            for (; i >= l; i--) {
                double f = s * e[i];
                const double b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {
                    // an exact zero appeared: deflate and restart the sweep
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                // the rotation acts on eigenvector columns i and i+1
                if (rots) rots->push_back({i, c, s});
                for (int k = 0; k < nrow; k++) {
                    const double zi = Z[(size_t)k * n + i], zi1 = Z[(size_t)k * n + i + 1];
                    Z[(size_t)k * n + i + 1] = s * zi + c * zi1;
                    Z[(size_t)k * n + i] = c * zi - s * zi1;
                }
            }
            if (r == 0.0 && i >= l) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    return true;
}

// c = |b| sign(T) e_1 for the Lanczos matrix T (diagonal a, off-diagonal
// bt): the coefficients of the Lanczos approximation of sign(A) b in the
// Lanczos basis.  With T = Z diag(theta) Z^T, c = |b| Z (sign(theta) .* Z^T e_1):
// the first row of Z is accumulated alongside the QL sweeps (Z^T e_1), and Z
// times the weighted vector is formed by applying the logged rotations
// (Z = G_1 G_2 ... G_N) in reverse order, so the cost is O(n^2), not the O(n^3)
// of forming Z.  A zero Ritz value counts as +1.  Returns false if the
// eigen-decomposition fails.
inline bool tridiag_sign_e1(int n, const double *a, const double *bt, double bnorm, std::vector<double> &c)
{
    std::vector<double> d(a, a + n), e(bt, bt + (n > 1 ? n - 1 : 0)), z0;
    std::vector<PlaneRot> rots;
    if (!tridiag_eig(n, d, e, z0, 1, 0, &rots)) return false;
    c.assign(n, 0.0);
    for (int j = 0; j < n; j++) c[j] = (d[j] >= 0.0 ? 1.0 : -1.0) * z0[j] * bnorm;   // sign(theta_j) z_j(0) |b|
    for (size_t r = rots.size(); r-- > 0;) {
        const PlaneRot &g = rots[r];
        const double x = c[g.i], y = c[g.i + 1];
        c[g.i] = g.c * x + g.s * y;
        c[g.i + 1] = -g.s * x + g.c * y;
    }
    return true;
}

}  // namespace ovl
