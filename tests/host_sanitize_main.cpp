// Host-code sanitizer driver: runs the library's host-only numerics (the
// tridiagonal QL eigensolver and its sign(T) e_1 form, the Hermitian Jacobi
// eigensolver, the Zolotarev coefficients) on many sizes and edge cases, with
// their own residual checks, so that a build with AddressSanitizer and
// UndefinedBehaviorSanitizer sees every code path.  Built and run by
// tests/test_host_sanitizers.py with g++; exit status 0 and a final "ok" line
// mean every check passed and no sanitizer reported.
#include <cmath>
#include <complex>
#include <cstdio>
#include <random>
#include <vector>

#include "../include/ovl.h"
#include "../paper_1410_7170_amd/csrc/hermeig.h"
#include "../paper_1410_7170_amd/csrc/tridiag.h"

static int failures = 0;

static void check(bool ok, const char *what, int n)
{
    if (!ok) {
        std::printf("FAIL %s (n = %d)\n", what, n);
        failures++;
    }
}

// T Z = Z diag(d) and Z^T Z = I for the full decomposition; the one-row form
// reproduces the first row of Z; sign(T) e_1 agrees with Z sign(d) Z^T e_1.
static void tridiag_case(int n, std::mt19937_64 &g, bool split, bool repeated)
{
    std::normal_distribution<double> nd;
    std::vector<double> a(n), b(n > 1 ? n - 1 : 0);
    for (double &x : a) x = repeated ? 1.0 : nd(g);
    for (double &x : b) x = nd(g);
    if (split && n > 4) b[n / 2] = 0.0;
    std::vector<double> d(a), Z;
    check(ovl::tridiag_eig(n, d, b, Z), "tridiag_eig converged", n);
    double scale = 1.0;
    for (double x : d) scale = std::fmax(scale, std::fabs(x));
    double res = 0.0, orth = 0.0;
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            double tz = a[i] * Z[(size_t)i * n + j];
            if (i > 0) tz += b[i - 1] * Z[(size_t)(i - 1) * n + j];
            if (i + 1 < n) tz += b[i] * Z[(size_t)(i + 1) * n + j];
            res = std::fmax(res, std::fabs(tz - d[j] * Z[(size_t)i * n + j]));
            double o = 0.0;
            for (int k = 0; k < n; k++) o += Z[(size_t)k * n + i] * Z[(size_t)k * n + j];
            orth = std::fmax(orth, std::fabs(o - (i == j ? 1.0 : 0.0)));
        }
    check(res <= 1e-11 * scale, "tridiag_eig residual", n);
    check(orth <= 1e-12 * n, "tridiag_eig orthonormality", n);

    std::vector<double> d1(a), Z1;
    check(ovl::tridiag_eig(n, d1, b, Z1, 1, 0), "tridiag_eig first row converged", n);
    double row = 0.0;
    for (int j = 0; j < n; j++) row = std::fmax(row, std::fabs(Z1[j] - Z[j]) + std::fabs(d1[j] - d[j]));
    check(row <= 1e-13 * scale, "tridiag_eig first row", n);

    std::vector<double> c;
    const double bnorm = 2.5;
    check(ovl::tridiag_sign_e1(n, a.data(), b.data(), bnorm, c), "tridiag_sign_e1 converged", n);
    double sg = 0.0;
    for (int i = 0; i < n; i++) {
        double ref = 0.0;
        for (int j = 0; j < n; j++) ref += Z[(size_t)i * n + j] * (d[j] >= 0.0 ? 1.0 : -1.0) * Z[j] * bnorm;
        sg = std::fmax(sg, std::fabs(ref - c[i]));
    }
    check(sg <= 1e-11 * bnorm, "tridiag_sign_e1 vs Z sign(d) Z^T e_1", n);
}

// A V = V diag(w) and V^H V = I.
static void herm_case(int n, std::mt19937_64 &g, bool zero)
{
    using cd = std::complex<double>;
    std::normal_distribution<double> nd;
    std::vector<cd> A((size_t)n * n), A0, V;
    for (int i = 0; i < n; i++)
        for (int j = i; j < n; j++) {
            cd x = zero ? cd(0.0) : (i == j ? cd(nd(g)) : cd(nd(g), nd(g)));
            A[(size_t)i * n + j] = x;
            A[(size_t)j * n + i] = std::conj(x);
        }
    A0 = A;
    std::vector<double> w;
    check(ovl::herm_jacobi(n, A, w, V), "herm_jacobi converged", n);
    double scale = 1.0;
    for (double x : w) scale = std::fmax(scale, std::fabs(x));
    double res = 0.0, orth = 0.0;
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            cd av = 0.0, o = 0.0;
            for (int k = 0; k < n; k++) {
                av += A0[(size_t)i * n + k] * V[(size_t)k * n + j];
                o += std::conj(V[(size_t)k * n + i]) * V[(size_t)k * n + j];
            }
            res = std::fmax(res, std::abs(av - w[j] * V[(size_t)i * n + j]));
            orth = std::fmax(orth, std::abs(o - (i == j ? 1.0 : 0.0)));
        }
    check(res <= 1e-12 * scale * n, "herm_jacobi residual", n);
    check(orth <= 1e-12 * n, "herm_jacobi orthonormality", n);
}

// Valid inputs: positive increasing shifts, positive weights, and the
// relative error of x R(x) within delta on [lambda_min, lambda_max].
static void zolo_case(double lmin, double lmax, int n)
{
    std::vector<double> s(n), w(n);
    double delta = -1.0;
    check(ovl_zolotarev(lmin, lmax, n, s.data(), w.data(), &delta) == OVL_OK, "ovl_zolotarev valid call", n);
    check(delta > 0.0 && delta < 1.0, "ovl_zolotarev delta in (0, 1)", n);
    for (int j = 0; j < n; j++) {
        check(s[j] > 0.0 && w[j] > 0.0, "ovl_zolotarev positive shifts and weights", n);
        if (j) check(s[j] > s[j - 1], "ovl_zolotarev increasing shifts", n);
    }
    double err = 0.0;
    for (int k = 0; k <= 2000; k++) {
        const double x = lmin * std::pow(lmax / lmin, k / 2000.0);
        double r = 0.0;
        for (int j = 0; j < n; j++) r += w[j] / (x * x + s[j]);
        err = std::fmax(err, std::fabs(x * r - 1.0));
    }
    check(err <= delta * (1.0 + 1e-6) + 1e-15, "ovl_zolotarev error within delta", n);
}

int main()
{
    std::mt19937_64 g(20241017);
    for (int n : {1, 2, 3, 5, 17, 64, 150}) {
        tridiag_case(n, g, false, false);
        tridiag_case(n, g, true, false);
        tridiag_case(n, g, false, true);
    }
    for (int n : {1, 2, 3, 8, 24}) {
        herm_case(n, g, false);
        herm_case(n, g, true);
    }
    for (int n : {1, 2, 8, 20, 24, OVL_MAX_SHIFTS}) {
        zolo_case(0.05, 6.0, n);
        zolo_case(1e-3, 7.5, n);
        zolo_case(0.5, 0.5000001 + 0.5, n);
    }
    // invalid arguments are rejected without touching the outputs
    double s[4] = {7, 7, 7, 7}, w[4] = {7, 7, 7, 7}, delta = 7;
    check(ovl_zolotarev(0.1, 5.0, 0, s, w, &delta) == OVL_ERR_INVALID, "npoles 0 rejected", 0);
    check(ovl_zolotarev(0.1, 5.0, OVL_MAX_SHIFTS + 1, s, w, &delta) == OVL_ERR_INVALID, "npoles too large", 0);
    check(ovl_zolotarev(0.0, 5.0, 4, s, w, &delta) == OVL_ERR_INVALID, "lambda_min 0 rejected", 4);
    check(ovl_zolotarev(5.0, 5.0, 4, s, w, &delta) == OVL_ERR_INVALID, "empty interval rejected", 4);
    check(ovl_zolotarev(NAN, 5.0, 4, s, w, &delta) == OVL_ERR_INVALID, "NaN rejected", 4);
    check(ovl_zolotarev(0.1, INFINITY, 4, s, w, &delta) == OVL_ERR_INVALID, "infinite bound rejected", 4);
    check(ovl_zolotarev(0.1, 5.0, 4, nullptr, w, &delta) == OVL_ERR_INVALID, "null shifts rejected", 4);
    check(ovl_zolotarev(0.1, 5.0, 4, s, nullptr, &delta) == OVL_ERR_INVALID, "null weights rejected", 4);
    check(s[0] == 7 && w[0] == 7 && delta == 7, "outputs untouched on rejection", 4);
    // the delta output is optional
    check(ovl_zolotarev(0.1, 5.0, 4, s, w, nullptr) == OVL_OK, "null delta accepted", 4);
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
