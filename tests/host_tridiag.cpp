// Host-logic test shim: exposes the library's small dense eigensolvers
// (paper_1410_7170_amd/csrc/tridiag.h, hermeig.h) with a C ABI so that a CPU
// test can compare them with LAPACK.  Built by tests/test_host_logic.py with g++.
#include "../paper_1410_7170_amd/csrc/hermeig.h"
#include "../paper_1410_7170_amd/csrc/tridiag.h"

extern "C" int tri_eig(int n, const double *d, const double *e, double *w, double *z)
{
    std::vector<double> dd(d, d + n), ee(e, e + (n > 1 ? n - 1 : 0)), Z;
    if (!ovl::tridiag_eig(n, dd, ee, Z)) return 1;
    for (int i = 0; i < n; i++) w[i] = dd[i];
    for (size_t k = 0; k < Z.size(); k++) z[k] = Z[k];
    return 0;
}

extern "C" int tri_sign_e1(int n, const double *a, const double *b, double bnorm, double *c)
{
    std::vector<double> cv;
    if (!ovl::tridiag_sign_e1(n, a, b, bnorm, cv)) return 1;
    for (int i = 0; i < n; i++) c[i] = cv[i];
    return 0;
}

// a: n x n complex Hermitian (interleaved re, im, row-major); w: eigenvalues,
// v: eigenvectors (interleaved, v[i*n + j] component i of vector j)
extern "C" int herm_eig(int n, const double *a, double *w, double *v)
{
    std::vector<std::complex<double>> A((size_t)n * n), V;
    for (size_t k = 0; k < A.size(); k++) A[k] = {a[2 * k], a[2 * k + 1]};
    std::vector<double> ww;
    if (!ovl::herm_jacobi(n, A, ww, V)) return 1;
    for (int i = 0; i < n; i++) w[i] = ww[i];
    for (size_t k = 0; k < V.size(); k++) {
        v[2 * k] = V[k].real();
        v[2 * k + 1] = V[k].imag();
    }
    return 0;
}
