// Eigen-decomposition of a small complex Hermitian matrix (host only): cyclic
// Jacobi.  Each rotation first removes the phase of the pivot a_pq with a
// diagonal unitary on index q, then zeroes the (now real) pivot with a real
// plane rotation (Golub & Van Loan, "Matrix Computations", the symmetric
// Jacobi method; the phase step extends it to Hermitian matrices).  Used for
// the Rayleigh-Ritz step of the low-mode computation.
#pragma once

#include <cmath>
#include <complex>
#include <vector>

namespace ovl {

// A: n x n Hermitian, row-major (destroyed).  On return w[j] holds the
// eigenvalues and V (n x n, row-major, V[i*n + j] = component i of
// eigenvector j) the orthonormal eigenvectors, unsorted.  Returns false if the
// off-diagonal mass is not below 1e-15 of the matrix norm after 60 sweeps.
inline bool herm_jacobi(int n, std::vector<std::complex<double>> &A, std::vector<double> &w,
                        std::vector<std::complex<double>> &V)
{
    using cd = std::complex<double>;
    V.assign((size_t)n * n, cd(0.0));
    for (int i = 0; i < n; i++) V[(size_t)i * n + i] = 1.0;
    auto a = [&](int i, int j) -> cd & { return A[(size_t)i * n + j]; };
    double fro = 0.0;
    for (const cd &x : A) fro += std::norm(x);
    fro = std::sqrt(fro);
    bool ok = n <= 1 || fro == 0.0;
    for (int sweep = 0; sweep < 60 && !ok; sweep++) {
        double off = 0.0;
        for (int p = 0; p < n; p++)
            for (int q = p + 1; q < n; q++) off += std::norm(a(p, q));
        if (std::sqrt(2.0 * off) <= 1e-15 * fro) {
            ok = true;
            break;
        }
        for (int p = 0; p < n - 1; p++) {
            for (int q = p + 1; q < n; q++) {
                const double r = std::abs(a(p, q));
                if (r == 0.0) continue;
                // phase: column q times d, row q times conj(d), d = conj(a_pq)/|a_pq|
                const cd d = std::conj(a(p, q)) / r;
                for (int k = 0; k < n; k++) {
                    if (k != q) {
                        a(k, q) *= d;
                        a(q, k) *= std::conj(d);
                    }
                    V[(size_t)k * n + q] *= d;
                }
                // real rotation zeroing a_pq = r
                const double app = a(p, p).real(), aqq = a(q, q).real();
                const double th = (aqq - app) / (2.0 * r);
                const double t = (th >= 0.0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; k++) {
                    // columns p, q
                    const cd kp = a(k, p), kq = a(k, q);
                    a(k, p) = c * kp - s * kq;
                    a(k, q) = s * kp + c * kq;
                }
                for (int k = 0; k < n; k++) {
                    // rows p, q
                    const cd pk = a(p, k), qk = a(q, k);
                    a(p, k) = c * pk - s * qk;
                    a(q, k) = s * pk + c * qk;
                }
                a(p, q) = 0.0;
                a(q, p) = 0.0;
                a(p, p) = app - t * r;
                a(q, q) = aqq + t * r;
                for (int k = 0; k < n; k++) {
                    const cd vp = V[(size_t)k * n + p], vq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vp - s * vq;
                    V[(size_t)k * n + q] = s * vp + c * vq;
                }
            }
        }
    }
    w.resize(n);
    for (int i = 0; i < n; i++) w[i] = a(i, i).real();
    return ok;
}

}  // namespace ovl
