// Zolotarev coefficients for sign(x) on lambda_min <= |x| <= lambda_max.
//
// With k = lambda_min/lambda_max and the unit-interval form
//   sign(x) ~ D x sum_j a_j / (x^2 + sigma_j),   k <= |x| <= 1,
// the optimal (2n-1, 2n) rational function has poles -sigma_j = -c_{2j-1} and
// numerator roots -c_{2j}, c_l = k^2 sn^2(l K'/(2n); k') / cn^2(l K'/(2n); k'),
// k' = sqrt(1 - k^2), K' = K(k').  Here sn/cn comes from Jacobi theta
// functions (Abramowitz & Stegun 16.36): with the nome q of modulus k',
//   sn/cn (u; k') = (theta3(0)/theta4(0)) theta1(z)/theta2(z),  z = pi u / (2 K(k')),
// and theta4(0)^2/theta3(0)^2 is the complementary modulus k, so
// c_l = k (theta1/theta2)^2
// at z = pi l / (4n).  The normalisation D centres the relative error
// D R(x) - 1 between -delta and +delta, found from the extremes of R on [k,1].
#include <cmath>
#include <vector>

#include "../../include/ovl.h"

namespace {

double agm(double a, double b)
{
    for (int k = 0; k < 80; k++) {
        double m = 0.5 * (a + b), g = std::sqrt(a * b);
        a = m;
        b = g;
        if (std::fabs(a - b) <= 1e-17 * a) break;
    }
    return a;
}

// theta1(z)/theta2(z) for nome q (the common factor 2 q^{1/4} cancels)
double theta_ratio(double z, double q)
{
    double num = 0.0, den = 0.0;
    for (int n = 0; n < 60; n++) {
        double w = std::pow(q, (double)n * (n + 1));
        if (w < 1e-300) break;
        num += (n % 2 ? -w : w) * std::sin((2 * n + 1) * z);
        den += w * std::cos((2 * n + 1) * z);
        if (w < 1e-20) break;
    }
    return num / den;
}

double unit_R(double x, int n, const double *sig, const double *a)
{
    double s = 0.0;
    for (int j = 0; j < n; j++) s += a[j] / (x * x + sig[j]);
    return x * s;
}

// maximum of R over [lo, hi] by ternary search in log x (R is unimodal there)
double local_max(double lo, double hi, int n, const double *sig, const double *a)
{
    double u = std::log(lo), v = std::log(hi);
    for (int it = 0; it < 200 && v - u > 1e-15; it++) {
        double m1 = u + (v - u) / 3, m2 = v - (v - u) / 3;
        if (unit_R(std::exp(m1), n, sig, a) < unit_R(std::exp(m2), n, sig, a)) u = m1; else v = m2;
    }
    return unit_R(std::exp(0.5 * (u + v)), n, sig, a);
}

}  // namespace

extern "C" int ovl_zolotarev(double lambda_min, double lambda_max, int32_t npoles, double *shifts, double *weights,
                             double *delta)
{
    if (!shifts || !weights || npoles < 1 || npoles > OVL_MAX_SHIFTS) return OVL_ERR_INVALID;
    if (!(lambda_min > 0.0) || !(lambda_max > lambda_min) || !std::isfinite(lambda_max)) return OVL_ERR_INVALID;
    const int n = npoles;
    const double k = lambda_min / lambda_max;
    const double kp = std::sqrt((1.0 - k) * (1.0 + k));
    // nome of modulus k': q = exp(-pi K(k)/K(k')), K(m) = pi / (2 AGM(1, sqrt(1-m^2)))
    const double q = std::exp(-M_PI * agm(1.0, k) / agm(1.0, kp));
    std::vector<double> c(2 * n + 1);
    for (int l = 1; l <= 2 * n - 1; l++) {
        double t = theta_ratio(M_PI * l / (4.0 * n), q);
        c[l] = k * t * t;
    }
    std::vector<double> sig(n), a(n);
    for (int j = 0; j < n; j++) sig[j] = c[2 * j + 1];
    for (int j = 0; j < n; j++) {
        double num = 1.0, den = 1.0;
        for (int i = 1; i < n; i++) num *= (c[2 * i] - sig[j]);
        for (int i = 0; i < n; i++)
            if (i != j) den *= (sig[i] - sig[j]);
        a[j] = num / den;
    }
    // R equals its minimum at both ends of [k,1]; between consecutive sample
    // points bracket every local maximum and refine it
    double rmin = std::min(unit_R(k, n, sig.data(), a.data()), unit_R(1.0, n, sig.data(), a.data()));
    double rmax = rmin;
    const int G = 64 * n + 256;
    std::vector<double> xs(G + 1), rs(G + 1);
    for (int g = 0; g <= G; g++) {
        xs[g] = k * std::pow(1.0 / k, (double)g / G);
        rs[g] = unit_R(xs[g], n, sig.data(), a.data());
        rmin = std::min(rmin, rs[g]);
    }
    for (int g = 1; g < G; g++)
        if (rs[g] >= rs[g - 1] && rs[g] >= rs[g + 1])
            rmax = std::max(rmax, local_max(xs[g - 1], xs[g + 1], n, sig.data(), a.data()));
    const double D = 2.0 / (rmax + rmin);
    for (int j = 0; j < n; j++) {
        shifts[j] = sig[j] * lambda_max * lambda_max;
        weights[j] = D * a[j] * lambda_max;
    }
    if (delta) *delta = (rmax - rmin) / (rmax + rmin);
    return OVL_OK;
}
