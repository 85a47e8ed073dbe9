// Host-logic test shim: exposes the library's tridiagonal eigensolver
// (paper_1410_7170_amd/csrc/tridiag.h) with a C ABI so that a CPU test can
// compare it with LAPACK.  Built by tests/test_host_logic.py with g++.
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
