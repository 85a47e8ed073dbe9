// Low-mode deflation of sign(Q), Q = Gamma_5 D_W(m0) (Section 5.2).
//
// With the k eigenpairs (lambda_i, xi_i) of Q smallest in |lambda|,
// Xi = [xi_1 .. xi_k] and the projector Pi = I - Xi Xi^H,
//     sign(Q) chi = sum_i sign(lambda_i) (xi_i^H chi) xi_i + sign(Q) Pi chi;
// the first term is exact and the second is left to the rational (or Lanczos)
// approximation, whose lower spectral bound rises from |lambda_1| to the
// smallest |lambda| outside the deflated set.
//
// The eigenpairs come from ovl_low_modes: a Lanczos run on Q^2 seeds a block
// of nev + extra vectors and the interval of a Chebyshev filter p(Q^2) that
// stays within [-1, 1] above a lower edge theta_cut and grows steeply below
// it; then subspace iteration with that filter (X <- p(Q^2) X, orthonormalised)
// and Rayleigh-Ritz with Q itself on span X, which separates the +-lambda
// pairs that are nearly degenerate in Q^2.  Plain Lanczos on Q^2 converges
// slowly here: its low end is dense.  The edge moves down every iteration to
// an upper bound of the block's last eigenvalue of Q^2.  Memory: steps + 1
// basis fields plus 5 (nev + extra) + 1 work fields, FP64.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <numeric>
#include <vector>

#include "hermeig.h"
#include "mscg.h"
#include "tridiag.h"

namespace ovl {

namespace {

using cd = std::complex<double>;

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

Fld field(Fld f, const Lat &L, int i) { return sub(f, L.V, i, 1); }

// |f_r| for every field of f, to the host (partials: nrhs * nblk doubles)
int field_norms(const Lat &L, Fld f, double *partials, double *red, double *out, hipStream_t st)
{
    OVL_HIP(launch_norm2(L, f, partials, st));
    OVL_HIP(launch_reduce(partials, 1, f.nrhs, site_blocks(L), red, st));
    std::vector<double> h(f.nrhs);
    OVL_HIP(hipMemcpyAsync(h.data(), red, sizeof(double) * f.nrhs, hipMemcpyDeviceToHost, st));
    OVL_HIP(hipStreamSynchronize(st));
    for (int q = 0; q < f.nrhs; q++) out[q] = std::sqrt(h[q]);
    return OVL_OK;
}

// c[f] = <V_f, w> for the nv fields of V, to the host; the device copy stays in
// coef ([re..., im...])
int mdot(const Lat &L, Fld V, int nv, Fld w, double *partials, double *coef, cd *c, hipStream_t st)
{
    dim3 grid(site_blocks(L), nv);
    k_mdot<<<grid, kBlock, 0, st>>>(L.g, L.nb, nv, (const double2 *)V.d, (const double2 *)w.d, partials);
    OVL_HIP(hipGetLastError());
    OVL_HIP(launch_reduce(partials, 2, nv, site_blocks(L), coef, st));
    std::vector<double> h(2 * nv);
    OVL_HIP(hipMemcpyAsync(h.data(), coef, sizeof(double) * 2 * nv, hipMemcpyDeviceToHost, st));
    OVL_HIP(hipStreamSynchronize(st));
    for (int f = 0; f < nv; f++) c[f] = cd(h[f], h[nv + f]);
    return OVL_OK;
}

// w += sum_f c[f] V_f (c from the host, staged through the device buffer coef)
int mcaxpy(const Lat &L, Fld V, int nv, const cd *c, Fld w, double *coef, hipStream_t st)
{
    std::vector<double> h(2 * nv);
    for (int f = 0; f < nv; f++) {
        h[f] = c[f].real();
        h[nv + f] = c[f].imag();
    }
    OVL_HIP(hipMemcpyAsync(coef, h.data(), sizeof(double) * 2 * nv, hipMemcpyHostToDevice, st));
    k_mcaxpy<<<site_blocks(L), kBlock, 0, st>>>(L.g, L.nb, nv, coef, 1.0, (const double2 *)V.d, (double2 *)w.d);
    OVL_HIP(hipGetLastError());
    // the host vector h must outlive the copy
    OVL_HIP(hipStreamSynchronize(st));
    return OVL_OK;
}

hipError_t q_apply(const Lat &L, const void *U64, double m0, Fld in, Fld out, hipStream_t st)
{
    WArgs a{};
    a.U = U64;
    a.diag = m0 + 4.0;
    a.nrhs = in.nrhs;
    a.in = in.d;
    a.out = out.d;
    return launch_wilson(L, P_F64, W_PLAIN, true, a, st);
}

// T = tridiag(alpha, beta): ascending eigenvalues theta and the matching
// eigenvector columns, all rows (Z[i*n + j] component i of eigenvector j) or
// only the last (last_only: Z[j] = component n-1 of eigenvector j)
bool tridiag_sorted(int n, const std::vector<double> &alpha, const std::vector<double> &beta,
                    std::vector<double> &theta, std::vector<double> &Z, bool last_only = false)
{
    std::vector<double> d(alpha.begin(), alpha.begin() + n), e(beta.begin(), beta.begin() + (n - 1)), Zu;
    const int nrow = last_only ? 1 : n;
    if (!tridiag_eig(n, d, e, Zu, nrow, n - nrow)) return false;
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] < d[b]; });
    theta.resize(n);
    Z.assign((size_t)nrow * n, 0.0);
    for (int j = 0; j < n; j++) {
        theta[j] = d[idx[j]];
        for (int i = 0; i < nrow; i++) Z[(size_t)i * n + j] = Zu[(size_t)i * n + idx[j]];
    }
    return true;
}

}  // namespace

namespace {

struct EigDims {
    int k, kp, m;   // wanted, block size, steps of the seeding Lanczos run
};

EigDims eig_dims(const ovl_eig_params *p)
{
    EigDims d;
    d.k = p->nev;
    d.kp = p->nev + (p->extra > 0 ? p->extra : p->nev / 2 + 4);
    d.m = p->steps > 0 ? p->steps : std::max(40, d.kp + 8);
    return d;
}

}  // namespace

size_t low_modes_ws_bytes(const Lat &L, const ovl_eig_params *p)
{
    const EigDims d = eig_dims(p);
    WsCarve c{nullptr, 0, 0};
    const size_t F = field_bytes(P_F64, L.V);
    const int nv = std::max(d.m + 1, 2 * d.kp);
    c.take(F * (d.m + 1));                                   // Lanczos basis of the seeding run
    c.take(F * 2 * d.kp);                                    // Y, then Q Y (Chebyshev: y_j and (Q^2+s) y_j)
    c.take(F * d.kp);                                        // X
    c.take(F * d.kp);                                        // Q y inside (Q^2 + s) y
    c.take(F);                                               // w
    c.take(sizeof(double) * 2 * nv * site_blocks(L));        // partials
    c.take(sizeof(double) * 2 * nv);                         // reduced sums / coefficients
    return c.off + 256;
}

// Low modes of Q: a Lanczos run on Q^2 seeds a block of kp = nev + extra
// vectors and the filter interval; then Chebyshev-filtered subspace
// iteration: X <- T_deg(a Q^2 + b) X, orthonormalised, Rayleigh-Ritz with Q;
// see include/ovl.h
int low_modes(const Lat &L, const void *U64, double m0, Fld start, const ovl_eig_params *p, Fld evecs, double *evals,
              double *resid, ovl_eig_stats *S, char *ws, size_t ws_bytes, hipStream_t st)
{
    const double t0 = now_s();
    const EigDims dm = eig_dims(p);
    const int k = dm.k, kp = dm.kp, m = dm.m;
    WsCarve c{ws, 0, ws_bytes};
    const size_t F = field_bytes(P_F64, L.V);
    const int nv = std::max(m + 1, 2 * kp);
    Fld V{c.take(F * (m + 1)), nullptr, P_F64, m + 1};
    Fld YQ{c.take(F * 2 * kp), nullptr, P_F64, 2 * kp};   // Y_0..Y_kp-1, then Q Y_0..
    Fld Y = sub(YQ, L.V, 0, kp), QY = sub(YQ, L.V, kp, kp);
    Fld X{c.take(F * kp), nullptr, P_F64, kp};
    Fld T{c.take(F * kp), nullptr, P_F64, kp};
    Fld w{c.take(F), nullptr, P_F64, 1};
    double *partials = (double *)c.take(sizeof(double) * 2 * nv * site_blocks(L));
    double *coef = (double *)c.take(sizeof(double) * 2 * nv);
    if (c.off > ws_bytes) return OVL_ERR_WORKSPACE;
    int64_t q2n = 0;
    int e;

    // out = (Q^2 + s) in for a field set: the second stencil adds s * in in
    // its epilogue
    auto q2s = [&](Fld in, Fld out, double s) -> hipError_t {
        Fld t = sub(T, L.V, 0, in.nrhs);
        hipError_t h = q_apply(L, U64, m0, in, t, st);
        if (h != hipSuccess) return h;
        WArgs a{};
        a.U = U64;
        a.diag = m0 + 4.0;
        a.nrhs = in.nrhs;
        a.in = t.d;
        a.out = out.d;
        a.p = in.d;
        a.shift = s;
        q2n += in.nrhs;
        return launch_wilson(L, P_F64, W_SHIFT, true, a, st);
    };

    // ---- seeding run: Lanczos on Q^2 with full reorthogonalisation
    double bn;
    e = field_norms(L, start, partials, coef, &bn, st);
    if (e) return e;
    if (!(bn > 0.0) || !std::isfinite(bn)) return bn == 0.0 ? OVL_ERR_INVALID : OVL_ERR_NONFINITE;
    OVL_HIP(launch_axpby(L, 1.0 / bn, start, 0.0, field(V, L, 0), st));
    std::vector<double> alpha, beta;
    std::vector<cd> h(nv);
    int n0 = 0;
    for (int j = 0; j < m; j++) {
        OVL_HIP(q2s(field(V, L, j), w, 0.0));
        double a = 0.0;
        for (int pass = 0; pass < 2; pass++) {
            e = mdot(L, V, j + 1, w, partials, coef, h.data(), st);
            if (e) return e;
            k_mcaxpy<<<site_blocks(L), kBlock, 0, st>>>(L.g, L.nb, j + 1, coef, -1.0, (const double2 *)V.d,
                                                        (double2 *)w.d);
            OVL_HIP(hipGetLastError());
            a += h[j].real();
        }
        double b;
        e = field_norms(L, w, partials, coef, &b, st);
        if (e) return e;
        if (!std::isfinite(a) || !std::isfinite(b)) return OVL_ERR_NONFINITE;
        alpha.push_back(a);
        n0 = j + 1;
        if (b <= 1e-14 * std::max(1.0, std::fabs(a)) || n0 == m) break;   // invariant subspace or done
        beta.push_back(b);
        OVL_HIP(launch_axpby(L, 1.0 / b, w, 0.0, field(V, L, j + 1), st));
    }
    if (n0 < k) return OVL_ERR_INVALID;   // the Krylov space is smaller than nev
    const int q = std::min(kp, n0);       // block size
    std::vector<double> theta, Z;
    if (!tridiag_sorted(n0, alpha, beta, theta, Z)) return OVL_ERR_NONFINITE;
    // filter interval: the largest Ritz value converges from below within a
    // few steps (1% above it bounds the spectrum; an eigenvalue just outside
    // is only mildly amplified); the q-th smallest Ritz value is >= theta_q
    // (interlacing), so the first edge keeps the q lowest modes amplified
    const double tmax = 1.01 * theta[n0 - 1] + 1e-12;
    double tcut = theta[std::min(q, n0 - 1)];
    if (!(tcut < tmax)) tcut = 0.5 * tmax;
    // the block starts as the q lowest Ritz vectors of Q^2
    {
        std::vector<cd> cz(n0);
        for (int i = 0; i < q; i++) {
            for (int j = 0; j < n0; j++) cz[j] = Z[(size_t)j * n0 + i];
            OVL_HIP(launch_zero(L, field(X, L, i), st));
            e = mcaxpy(L, V, n0, cz.data(), field(X, L, i), coef, st);
            if (e) return e;
        }
    }
    const Fld Xq = sub(X, L.V, 0, q), Yq = sub(Y, L.V, 0, q), QYq = sub(QY, L.V, 0, q);

    double tlow = theta[0];   // >= theta_1 (interlacing)
    int64_t degs = 0;
    std::vector<double> lam, sig, rn(q);
    std::vector<cd> H, H2, Cm, C2, col(2 * kp), cc(2 * kp);
    std::vector<int> order(q);
    bool ok = false;
    int iters = 0;
    for (int it = 0; it < p->stages && !ok; it++) {
        iters++;
        // Y = T_deg(a Q^2 + b) X by the three-term recurrence, y_0 = X,
        // y_1 = (a Q^2 + b) X, y_{j+1} = 2 (a Q^2 + b) y_j - y_{j-1}, in the
        // buffers X and Y (the Q Y half holds (Q^2 + b/a) y_j)
        const double ca = 2.0 / (tmax - tcut), cbb = -(tmax + tcut) / (tmax - tcut);
        // degree: at most p->degree, and low enough that the filter's gain at
        // the lowest eigenvalue estimate stays below 1e5 (T_d(x) =
        // cosh(d acosh|x|)); a larger spread would leave the block's weaker
        // directions below the rounding of its dominant ones
        const double xlow = std::fabs(ca * tlow + cbb);
        int deg = p->degree;
        if (xlow > 1.0) deg = std::max(1, std::min(deg, (int)std::ceil(std::acosh(1e5) / std::acosh(xlow))));
        Fld y0 = Xq, y1 = Yq;
        OVL_HIP(q2s(y0, QYq, cbb / ca));
        OVL_HIP(launch_axpby(L, ca, QYq, 0.0, y1, st));
        for (int j = 2; j <= deg; j++) {
            OVL_HIP(q2s(y1, QYq, cbb / ca));
            OVL_HIP(launch_axpby(L, 2.0 * ca, QYq, -1.0, y0, st));
            std::swap(y0, y1);
        }
        if (y1.d != Yq.d) OVL_HIP(hipMemcpyAsync(Yq.d, y1.d, F * q, hipMemcpyDeviceToDevice, st));
        // orthonormalise the block (classical Gram-Schmidt, twice)
        for (int i = 0; i < q; i++) {
            Fld yi = field(Y, L, i);
            for (int pass = 0; pass < 2 && i > 0; pass++) {
                e = mdot(L, Y, i, yi, partials, coef, h.data(), st);
                if (e) return e;
                k_mcaxpy<<<site_blocks(L), kBlock, 0, st>>>(L.g, L.nb, i, coef, -1.0, (const double2 *)Y.d,
                                                            (double2 *)yi.d);
                OVL_HIP(hipGetLastError());
            }
            double nn;
            e = field_norms(L, yi, partials, coef, &nn, st);
            if (e) return e;
            if (!(nn > 0.0) || !std::isfinite(nn)) return OVL_ERR_NONFINITE;
            OVL_HIP(launch_axpby(L, 1.0 / nn, yi, 0.0, yi, st));
        }
        // Rayleigh-Ritz with Q (H) and Q^2 (H2 = (QY)^H QY) on span Y
        OVL_HIP(q_apply(L, U64, m0, Yq, QYq, st));
        H.assign((size_t)q * q, 0.0);
        H2.assign((size_t)q * q, 0.0);
        for (int b = 0; b < q; b++) {
            e = mdot(L, Yq, q, field(QY, L, b), partials, coef, col.data(), st);
            if (e) return e;
            for (int a = 0; a < q; a++) H[(size_t)a * q + b] = col[a];
            e = mdot(L, QYq, q, field(QY, L, b), partials, coef, col.data(), st);
            if (e) return e;
            for (int a = 0; a < q; a++) H2[(size_t)a * q + b] = col[a];
        }
        for (auto *M : {&H, &H2})
            for (int a = 0; a < q; a++)
                for (int b = a; b < q; b++) {
                    const cd sv = 0.5 * ((*M)[(size_t)a * q + b] + std::conj((*M)[(size_t)b * q + a]));
                    (*M)[(size_t)a * q + b] = sv;
                    (*M)[(size_t)b * q + a] = std::conj(sv);
                }
        if (!herm_jacobi(q, H, lam, Cm) || !herm_jacobi(q, H2, sig, C2)) return OVL_ERR_NONFINITE;
        std::sort(sig.begin(), sig.end());
        // residual of pair i: R_i = sum_a C_ai (Q Y_a - lam_i Y_a) into X_i for
        // its norm, then X_i = sum_a C_ai Y_a
        for (int i = 0; i < q; i++) {
            std::fill(cc.begin(), cc.end(), cd(0.0));
            for (int a = 0; a < q; a++) {
                cc[a] = -lam[i] * Cm[(size_t)a * q + i];
                cc[kp + a] = Cm[(size_t)a * q + i];
            }
            OVL_HIP(launch_zero(L, field(X, L, i), st));
            e = mcaxpy(L, YQ, 2 * kp, cc.data(), field(X, L, i), coef, st);
            if (e) return e;
        }
        e = field_norms(L, Xq, partials, coef, rn.data(), st);
        if (e) return e;
        for (int i = 0; i < q; i++) {
            for (int a = 0; a < q; a++) col[a] = Cm[(size_t)a * q + i];
            OVL_HIP(launch_zero(L, field(X, L, i), st));
            e = mcaxpy(L, Yq, q, col.data(), field(X, L, i), coef, st);
            if (e) return e;
        }
        std::iota(order.begin(), order.end(), 0);
        std::sort(order.begin(), order.end(), [&](int a, int b) {
            return lam[a] * lam[a] + rn[a] * rn[a] < lam[b] * lam[b] + rn[b] * rn[b];
        });
        double mx = 0.0;
        for (int i = 0; i < k; i++) mx = std::max(mx, rn[order[i]]);
        ok = mx <= p->tol;
        // the q-th Rayleigh-Ritz value of Q^2 bounds theta_q from above
        tcut = std::min(tcut, 1.05 * sig[q - 1]);
        tlow = sig[0];
        degs += deg;
    }

    // the k pairs with the smallest |Q x|, ascending |lambda|, to evecs
    std::vector<int> best(order.begin(), order.begin() + k);
    std::sort(best.begin(), best.end(), [&](int a, int b) { return std::fabs(lam[a]) < std::fabs(lam[b]); });
    for (int i = 0; i < k; i++) {
        OVL_HIP(hipMemcpyAsync(field(evecs, L, i).d, field(X, L, best[i]).d, F, hipMemcpyDeviceToDevice, st));
        evals[i] = lam[best[i]];
    }
    // exact residuals |Q xi - lambda xi| / |xi|
    Fld R = sub(Y, L.V, 0, k);
    OVL_HIP(q_apply(L, U64, m0, evecs, R, st));
    for (int i = 0; i < k; i++) OVL_HIP(launch_axpby(L, -evals[i], field(evecs, L, i), 1.0, field(R, L, i), st));
    std::vector<double> rr(k), xn(k);
    e = field_norms(L, R, partials, coef, rr.data(), st);
    if (e) return e;
    e = field_norms(L, evecs, partials, coef, xn.data(), st);
    if (e) return e;
    double mx = 0.0;
    ok = true;
    for (int i = 0; i < k; i++) {
        resid[i] = rr[i] / xn[i];
        if (!std::isfinite(resid[i]) || !std::isfinite(evals[i])) return OVL_ERR_NONFINITE;
        mx = std::max(mx, resid[i]);
        ok = ok && resid[i] <= p->tol;
    }
    if (S) {
        S->steps = n0;
        S->stages = iters;
        S->q2_applies = q2n;
        S->converged = ok ? 1 : 0;
        S->max_residual = mx;
        double nxt = 0.0;
        for (int i = k; i < q; i++) {
            const double v = std::fabs(lam[order[i]]);
            if (nxt == 0.0 || v < nxt) nxt = v;
        }
        S->lambda_next = nxt;
        S->theta_cut = tcut;
        S->mean_degree = iters > 0 ? (double)degs / iters : 0.0;
        S->seconds = now_s() - t0;
    }
    return ok ? OVL_OK : OVL_NOT_CONVERGED;
}

// ---------------------------------------------------------------- deflated apply
size_t deflation_ws_bytes(const Lat &L, int nrhs, int k)
{
    WsCarve c{nullptr, 0, 0};
    c.take(field_bytes(P_F64, L.V) * nrhs);              // Pi b
    c.take(field_bytes(P_F64, L.V));                     // the Gamma_5 correction
    c.take(sizeof(double) * 2 * k * site_blocks(L));     // partials
    c.take(sizeof(double) * 2 * k);                      // coefficients
    return c.off;
}

// Stage 1: coefficients c[r][i] = xi_i^H b_r and the projected sources
// proj_r = b_r - sum_i c[r][i] xi_i
int deflate_project(const Lat &L, const ovl_deflation *D, Fld b, Fld proj, std::vector<cd> &cr, char *ws,
                    hipStream_t st)
{
    const int k = D->evecs.nrhs, R = b.nrhs;
    WsCarve c{ws, 0, deflation_ws_bytes(L, R, k)};
    c.take(field_bytes(P_F64, L.V) * R);
    c.take(field_bytes(P_F64, L.V));
    double *partials = (double *)c.take(sizeof(double) * 2 * k * site_blocks(L));
    double *coef = (double *)c.take(sizeof(double) * 2 * k);
    const Fld X = fld(&D->evecs);
    cr.assign((size_t)R * k, cd(0.0));
    OVL_HIP(hipMemcpyAsync(proj.d, b.d, field_bytes(P_F64, L.V) * R, hipMemcpyDeviceToDevice, st));
    for (int r = 0; r < R; r++) {
        int e = mdot(L, X, k, field(b, L, r), partials, coef, &cr[(size_t)r * k], st);
        if (e) return e;
        k_mcaxpy<<<site_blocks(L), kBlock, 0, st>>>(L.g, L.nb, k, coef, -1.0, (const double2 *)X.d,
                                                    (double2 *)field(proj, L, r).d);
        OVL_HIP(hipGetLastError());
    }
    return OVL_OK;
}

// Stage 2: add the deflated modes back exactly.  sign form:
//     out_r += sum_i sign(lambda_i) c_ri xi_i;
// overlap form (out_r = rho (Pi b_r + Gamma_5 sign(Q) Pi b_r) on entry):
//     out_r += rho sum_i c_ri xi_i + Gamma_5 (rho sum_i sign(lambda_i) c_ri xi_i)
int deflate_restore(const Lat &L, const ovl_deflation *D, const std::vector<cd> &cr, double rho, bool overlap,
                    Fld out, char *ws, hipStream_t st)
{
    const int k = D->evecs.nrhs, R = out.nrhs;
    WsCarve c{ws, 0, deflation_ws_bytes(L, R, k)};
    c.take(field_bytes(P_F64, L.V) * R);
    Fld tmp{c.take(field_bytes(P_F64, L.V)), nullptr, P_F64, 1};
    c.take(sizeof(double) * 2 * k * site_blocks(L));
    double *coef = (double *)c.take(sizeof(double) * 2 * k);
    const Fld X = fld(&D->evecs);
    std::vector<cd> d(k);
    for (int r = 0; r < R; r++) {
        const Fld o = field(out, L, r);
        const double f = overlap ? rho : 1.0;
        for (int i = 0; i < k; i++) d[i] = f * (D->evals[i] >= 0.0 ? 1.0 : -1.0) * cr[(size_t)r * k + i];
        if (!overlap) {
            int e = mcaxpy(L, X, k, d.data(), o, coef, st);
            if (e) return e;
            continue;
        }
        OVL_HIP(launch_zero(L, tmp, st));
        int e = mcaxpy(L, X, k, d.data(), tmp, coef, st);
        if (e) return e;
        dim3 grid(site_blocks(L), 1);
        k_gamma5<<<grid, kBlock, 0, st>>>(L.g, L.nb, (const double2 *)tmp.d, (double2 *)tmp.d);
        OVL_HIP(hipGetLastError());
        OVL_HIP(launch_axpby(L, 1.0, tmp, 1.0, o, st));
        for (int i = 0; i < k; i++) d[i] = rho * cr[(size_t)r * k + i];
        e = mcaxpy(L, X, k, d.data(), o, coef, st);
        if (e) return e;
    }
    return OVL_OK;
}

}  // namespace ovl
