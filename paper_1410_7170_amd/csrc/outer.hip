// Outer solver for D_ov psi = eta (the paper's eq. (linsys)) and the Wilson
// solve that serves as its preconditioner.
//
// ovl_overlap_solve: restarted flexible GMRES, FGMRES(m_restart), in FP64.
// Every Krylov step applies D_ov once (ovl_overlap_apply), with the multishift
// CG's tolerance relaxed as the residual falls: at step k the sign function
// needs a relative accuracy of order eps_outer / (|r_k|/|eta|) only, taken
// here as eps_outer * relax_factor / (|r_k|/|eta|), capped (the paper's
// relaxation, Table (allparms1): eps_sign = eps_outer / |r_k| * 1e-2).
// Optionally each step is right-preconditioned by D_W(m0^prec)^{-1} applied to
// a relative accuracy eps_prec (Section 3: D_W(m0^prec) shares its
// eigenvectors with D_N for normal D_W, and eq. (default_m) gives the paper's
// default m0^prec), computed by one of ovl_wilson_solve's two methods.
// Orthogonalisation: classical Gram-Schmidt applied twice, each pass one
// batched dot kernel and one batched update kernel; the Hessenberg least-squares
// problem is solved on the host with complex Givens rotations.
//
// ovl_wilson_solve: D_W(m0) x = b through the normal equations
// D_W^H D_W x = D_W^H b, D_W^H = Gamma_5 D_W Gamma_5 (eq. (gamma_5_symmetry)), so
// D_W^H D_W = Q^2 and D_W^H b = Q (Gamma_5 b): the FP32 blocked CG with FP64
// residual replacement on (Q^2 + 0) x = Q Gamma_5 b, then the FP64 true
// residual |b - D_W x| / |b|.
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "mscg.h"

namespace ovl {

// ---------------------------------------------------------------- kernels
// <V_f, w> for the nv fields V_f of a field set and one field w: partials
// [2][nv][nblk] (real parts, then imaginary parts)
__global__ __launch_bounds__(kBlock) void k_mdot(Geom g, int nb, int nv, const double2 *V, const double2 *w,
                                                  double *partials)
{
    __shared__ double lds[8];
    const int f = blockIdx.y, b = blockIdx.x;
    const int p = b / nb, i = (b % nb) * kBlock + threadIdx.x;
    double re = 0.0, im = 0.0;
    if (i < g.Vh) {
        cplx<double> s[4][3], t[4][3];
        spinor_ref<P_F64>(V, nullptr, g.S, f).load(p, i, s);
        spinor_ref<P_F64>(w, nullptr, g.S, 0).load(p, i, t);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            const cplx<double> c = cmc(s[k / 3][k % 3], t[k / 3][k % 3]);
            re += c.x;
            im += c.y;
        }
    }
    const double t0 = block_sum(re, lds);
    const double t1 = block_sum(im, lds + 4);
    if (threadIdx.x == 0) {
        partials[(size_t)f * gridDim.x + b] = t0;
        partials[(size_t)(nv + f) * gridDim.x + b] = t1;
    }
}

// w += sgn * sum_f c_f V_f, c_f = coef[f] + i coef[nv + f] (device)
__global__ __launch_bounds__(kBlock) void k_mcaxpy(Geom g, int nb, int nv, const double *coef, double sgn,
                                                    const double2 *V, double2 *w)
{
    const int b = blockIdx.x;
    const int p = b / nb, i = (b % nb) * kBlock + threadIdx.x;
    if (i >= g.Vh) return;
    const auto W = spinor_ref<P_F64>(w, nullptr, g.S, 0);
    cplx<double> acc[4][3];
    W.load(p, i, acc);
    for (int f = 0; f < nv; f++) {
        const cplx<double> c = {sgn * coef[f], sgn * coef[nv + f]};
        cplx<double> s[4][3];
        spinor_ref<P_F64>(V, nullptr, g.S, f).load(p, i, s);
#pragma unroll
        for (int k = 0; k < 12; k++) acc[k / 3][k % 3] = cmac(acc[k / 3][k % 3], c, s[k / 3][k % 3]);
    }
    W.store(p, i, acc);
}

// out = Gamma_5 in = diag(-1, -1, 1, 1) in spin (FP64, nrhs fields)
__global__ __launch_bounds__(kBlock) void k_gamma5(Geom g, int nb, const double2 *in, double2 *out)
{
    const int r = blockIdx.y, b = blockIdx.x;
    const int p = b / nb, i = (b % nb) * kBlock + threadIdx.x;
    if (i >= g.Vh) return;
    cplx<double> s[4][3];
    spinor_ref<P_F64>(in, nullptr, g.S, r).load(p, i, s);
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int c = 0; c < 3; c++) s[a][c] = {-s[a][c].x, -s[a][c].y};
    spinor_ref<P_F64>(out, nullptr, g.S, r).store(p, i, s);
}

namespace {

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// |f_r| per RHS of an FP64 field set, to the host
int norms(const Lat &L, Fld f, double *partials, double *red, double *out, hipStream_t st)
{
    OVL_HIP(launch_norm2(L, f, partials, st));
    OVL_HIP(launch_reduce(partials, 1, f.nrhs, site_blocks(L), red, st));
    std::vector<double> h(f.nrhs);
    OVL_HIP(hipMemcpyAsync(h.data(), red, sizeof(double) * f.nrhs, hipMemcpyDeviceToHost, st));
    OVL_HIP(hipStreamSynchronize(st));
    for (int q = 0; q < f.nrhs; q++) out[q] = std::sqrt(h[q]);
    return OVL_OK;
}

}  // namespace

// ---------------------------------------------------------------- Wilson solve
size_t wilson_solve_ws_bytes(const Lat &L, int nrhs, int m)
{
    WsCarve c{nullptr, 0, 0};
    const size_t F = field_bytes(P_F64, L.V);
    c.take(F * nrhs);   // Gamma_5 b, then the residual
    c.take(F * nrhs);   // Q Gamma_5 b
    c.take(sizeof(double) * 2 * NR * site_blocks(L));
    c.take(sizeof(double) * 4 * NR);
    c.take(blocked_ws_bytes(L, nrhs, 1, m, true, P_F32, true));
    return c.off + 256;
}

// D_W(m0) x = b (FP64 fields, nrhs each); true_res[q] = |b - D_W x| / |b|,
// iters[q] the CG iterations.  Returns OVL_OK, OVL_NOT_CONVERGED (maxiter)
// or an error.
int wilson_solve(const Lat &L, const ovl_gauge *U, double m0, Fld b, Fld x, double tol, int maxiter, int m,
                 double *true_res, int *iters, char *ws, size_t ws_bytes, hipStream_t st)
{
    const int R = b.nrhs;
    if (!U->f64 || !U->f32 || R > NR || m < 1 || m > MB) return OVL_ERR_INVALID;
    if (ws_bytes < wilson_solve_ws_bytes(L, R, m)) return OVL_ERR_WORKSPACE;
    WsCarve c{ws, 0, ws_bytes};
    const size_t F = field_bytes(P_F64, L.V);
    Fld t{c.take(F * R), nullptr, P_F64, R};
    Fld rhs{c.take(F * R), nullptr, P_F64, R};
    double *partials = (double *)c.take(sizeof(double) * 2 * NR * site_blocks(L));
    double *red = (double *)c.take(sizeof(double) * 4 * NR);
    char *bws = ws + c.off;
    const size_t bws_bytes = ws_bytes - c.off;
    dim3 grid(site_blocks(L), R);
    // rhs = Q Gamma_5 b = D_W^H b
    k_gamma5<<<grid, kBlock, 0, st>>>(L.g, L.nb, (const double2 *)b.d, (double2 *)t.d);
    OVL_HIP(hipGetLastError());
    WArgs a{};
    a.U = U->f64;
    a.diag = m0 + 4.0;
    a.nrhs = R;
    a.in = t.d;
    a.out = rhs.d;
    OVL_HIP(launch_wilson(L, P_F64, W_PLAIN, true, a, st));
    // (Q^2 + 0) x = rhs: FP32 blocked CG, FP64 x and residual replacement
    ovl_solver_params p;
    ovl_default_params(&p);
    p.tol = tol;
    p.maxiter = maxiter;
    p.block = m;
    BlkOpts o;
    o.m = m;
    o.keep_x = true;
    o.reliable = true;
    o.quiet = true;
    o.x_ext = x;
    o.iters_out = iters;
    const double zero = 0.0;
    int rc = mscg_blocked_t<P_F32>(L, U, m0, 1, &zero, nullptr, rhs, Fld{}, o, &p, nullptr, bws, bws_bytes, st,
                                   nullptr);
    if (rc < 0) return rc;
    // true residual b - D_W x, in t
    a.in = x.d;
    a.out = t.d;
    OVL_HIP(launch_wilson(L, P_F64, W_PLAIN, false, a, st));
    OVL_HIP(launch_axpby(L, 1.0, b, -1.0, t, st));
    std::vector<double> nr(R), nb(R);
    int e = norms(L, t, partials, red, nr.data(), st);
    if (e) return e;
    e = norms(L, b, partials, red, nb.data(), st);
    if (e) return e;
    for (int q = 0; q < R; q++) {
        true_res[q] = nb[q] > 0 ? nr[q] / nb[q] : 0.0;
        if (!std::isfinite(true_res[q])) return OVL_ERR_NONFINITE;
    }
    return rc;
}

// ---------------------------------------------------------------- FGMRES
size_t outer_ws_bytes(const Lat &L, int npoles, const ovl_outer_params *p, const ovl_lattice *lat)
{
    WsCarve c{nullptr, 0, 0};
    const size_t F = field_bytes(P_F64, L.V);
    const int m = p->restart;
    c.take(F * (m + 1));                                  // V
    if (p->precondition) c.take(F * m);                   // Z
    c.take(F);                                            // w
    c.take(F);                                            // residual
    c.take(sizeof(double) * 2 * (m + 1) * site_blocks(L));
    c.take(sizeof(double) * 2 * (m + 1));                 // reductions
    c.take(sizeof(double) * 2 * (m + 1));                 // coefficients
    size_t inner = ovl_workspace_bytes(lat, OVL_OP_MSCG, OVL_F64, 1, npoles, &p->inner);
    if (p->precondition)
        inner = std::max(inner, p->prec_even_odd ? wilson_solve_eo_ws_bytes(L) : wilson_solve_ws_bytes(L, 1, p->prec_block));
    c.take(inner);
    return c.off + 256;
}

int overlap_solve(const ovl_lattice *lat, const ovl_gauge *U, double rho, const ovl_zolo *z, Fld eta, Fld psi,
                  const ovl_outer_params *prm, ovl_outer_stats *stats, char *ws, size_t ws_bytes, hipStream_t st)
{
    const double t_start = now_s();
    const Lat L = make_lat(lat);
    const size_t F = field_bytes(P_F64, L.V);
    const int m = prm->restart;
    const int nblk = site_blocks(L);
    if (ws_bytes < outer_ws_bytes(L, z->npoles, prm, lat)) return OVL_ERR_WORKSPACE;
    WsCarve c{ws, 0, ws_bytes};
    Fld V{c.take(F * (m + 1)), nullptr, P_F64, m + 1};
    Fld Z = prm->precondition ? Fld{c.take(F * m), nullptr, P_F64, m} : V;
    Fld w{c.take(F), nullptr, P_F64, 1};
    Fld r{c.take(F), nullptr, P_F64, 1};
    double *partials = (double *)c.take(sizeof(double) * 2 * (m + 1) * nblk);
    double *red = (double *)c.take(sizeof(double) * 2 * (m + 1));
    double *coef = (double *)c.take(sizeof(double) * 2 * (m + 1));
    char *iws = ws + c.off;
    const size_t iws_bytes = ws_bytes - c.off;
    ovl_outer_stats S{};
    using cd = std::complex<double>;
    auto field = [&](Fld f, int k) { return sub(f, L.V, k, 1); };
    auto spin = [&](Fld f) {
        ovl_spinor s{f.d, nullptr, OVL_F64, 1};
        return s;
    };
    // D_ov applied to src into dst with the multishift tolerance tol_sign
    auto apply = [&](Fld src, Fld dst, double tol_sign) -> int {
        ovl_solver_params ip = prm->inner;
        ip.tol = tol_sign;
        if (ip.mode == OVL_SOLVE_MIXED && prm->inner.tol > 0) {
            // keep the FP64 phase's hand-over at the same distance above the
            // relaxed tolerance as above the configured one
            ip.sloppy_below = std::min(0.5, prm->inner.sloppy_below * tol_sign / prm->inner.tol);
        }
        ovl_spinor a = spin(src), o = spin(dst);
        ovl_solver_stats is;
        int e = ovl_overlap_apply(lat, U, rho, z, &a, &o, &ip, &is, iws, iws_bytes, st);
        S.overlap_applies++;
        S.mscg_iterations += is.iterations[0];
        return e < 0 ? e : OVL_OK;   // a relaxed apply that misses its tolerance still serves
    };
    // residual r = eta - D_ov psi with a tight sign tolerance; returns |r|
    auto true_residual = [&](double tol_sign, double *rn) -> int {
        int e = apply(psi, r, tol_sign);
        if (e) return e;
        OVL_HIP(launch_axpby(L, 1.0, eta, -1.0, r, st));
        return norms(L, r, partials, red, rn, st);
    };
    double beta0;
    int e = norms(L, eta, partials, red, &beta0, st);
    if (e) return e;
    OVL_HIP(launch_zero(L, psi, st));
    if (!(beta0 > 0.0)) {
        S.seconds = now_s() - t_start;
        if (stats) *stats = S;
        return std::isfinite(beta0) ? OVL_OK : OVL_ERR_NONFINITE;
    }
    const double check_tol = prm->tol * prm->relax_factor;   // sign accuracy of the residual checks
    OVL_HIP(hipMemcpyAsync(r.d, eta.d, F, hipMemcpyDeviceToDevice, st));
    double beta = beta0;
    bool converged = false;
    std::vector<cd> H((size_t)(m + 1) * m), g(m + 1), sn(m);
    std::vector<double> cs(m);
    std::vector<double> hd(2 * (m + 1));
    while (!converged && S.iterations < prm->maxiter) {
        // v_0 = r / beta
        OVL_HIP(launch_axpby(L, 1.0 / beta, r, 0.0, field(V, 0), st));
        std::fill(g.begin(), g.end(), cd(0.0));
        g[0] = beta;
        int j = 0, jn = 0;
        for (; j < m && S.iterations < prm->maxiter; j++) {
            Fld zj = field(Z, j);
            if (prm->precondition) {
                double tr;
                int it = 0;
                e = prm->prec_even_odd
                        ? wilson_solve_eo(L, U, prm->prec_m0, field(V, j), zj, prm->prec_tol, prm->prec_maxiter, &tr,
                                          &it, iws, iws_bytes, st)
                        : wilson_solve(L, U, prm->prec_m0, field(V, j), zj, prm->prec_tol, prm->prec_maxiter,
                                       prm->prec_block, &tr, &it, iws, iws_bytes, st);
                if (e < 0) return e;
                S.prec_iterations += it;
            }
            const double rel = std::abs(g[j]) / beta0;
            double ts = prm->tol * prm->relax_factor;
            if (prm->relax) ts = std::min(prm->sign_tol_max, ts / std::max(rel, 1e-300));
            e = apply(zj, w, ts);
            if (e) return e;
            S.iterations++;
            // classical Gram-Schmidt, twice: h = V^H w, w -= V h
            std::vector<cd> h(j + 2, cd(0.0));
            for (int pass = 0; pass < 2; pass++) {
                dim3 grid(nblk, j + 1);
                k_mdot<<<grid, kBlock, 0, st>>>(L.g, L.nb, j + 1, (const double2 *)V.d, (const double2 *)w.d,
                                               partials);
                OVL_HIP(hipGetLastError());
                OVL_HIP(launch_reduce(partials, 2, j + 1, nblk, coef, st));
                k_mcaxpy<<<nblk, kBlock, 0, st>>>(L.g, L.nb, j + 1, coef, -1.0, (const double2 *)V.d,
                                                  (double2 *)w.d);
                OVL_HIP(hipGetLastError());
                OVL_HIP(hipMemcpyAsync(hd.data(), coef, sizeof(double) * 2 * (j + 1), hipMemcpyDeviceToHost, st));
                OVL_HIP(hipStreamSynchronize(st));
                for (int i = 0; i <= j; i++) h[i] += cd(hd[i], hd[j + 1 + i]);
            }
            double hn;
            e = norms(L, w, partials, red, &hn, st);
            if (e) return e;
            if (!std::isfinite(hn)) return OVL_ERR_NONFINITE;
            h[j + 1] = hn;
            if (hn > 0.0) OVL_HIP(launch_axpby(L, 1.0 / hn, w, 0.0, field(V, j + 1), st));
            // earlier rotations, then a new one that zeroes h[j+1]
            for (int i = 0; i < j; i++) {
                const cd a = h[i], bb = h[i + 1];
                h[i] = cs[i] * a + sn[i] * bb;
                h[i + 1] = -std::conj(sn[i]) * a + cs[i] * bb;
            }
            const cd a = h[j];
            const double bmag = std::abs(h[j + 1]), amag = std::abs(a);
            const double nrm = std::hypot(amag, bmag);
            if (amag == 0.0) {
                cs[j] = 0.0;
                sn[j] = 1.0;
                h[j] = h[j + 1];
            } else {
                cs[j] = amag / nrm;
                sn[j] = (a / amag) * std::conj(h[j + 1]) / nrm;
                h[j] = (a / amag) * nrm;
            }
            h[j + 1] = 0.0;
            g[j + 1] = -std::conj(sn[j]) * g[j];
            g[j] = cs[j] * g[j];
            for (int i = 0; i <= j; i++) H[(size_t)i * m + j] = h[i];
            jn = j + 1;
            S.estimated_residual = std::abs(g[j + 1]) / beta0;
            if (std::abs(g[j + 1]) <= prm->tol * beta0 || hn == 0.0) break;
        }
        // y = H^{-1} g (upper triangular, jn x jn); psi += sum_k y_k z_k
        std::vector<cd> y(jn);
        for (int i = jn - 1; i >= 0; i--) {
            cd s = g[i];
            for (int k = i + 1; k < jn; k++) s -= H[(size_t)i * m + k] * y[k];
            y[i] = s / H[(size_t)i * m + i];
        }
        for (int k = 0; k < jn; k++) {
            hd[k] = y[k].real();
            hd[jn + k] = y[k].imag();
        }
        OVL_HIP(hipMemcpyAsync(coef, hd.data(), sizeof(double) * 2 * jn, hipMemcpyHostToDevice, st));
        k_mcaxpy<<<nblk, kBlock, 0, st>>>(L.g, L.nb, jn, coef, 1.0, (const double2 *)Z.d, (double2 *)psi.d);
        OVL_HIP(hipGetLastError());
        // true residual of the new iterate: the restart vector and the test
        e = true_residual(check_tol, &beta);
        if (e) return e;
        S.residual = beta / beta0;
        converged = beta <= prm->tol * beta0;
        if (!converged && S.iterations < prm->maxiter) S.restarts++;
    }
    S.seconds = now_s() - t_start;
    if (stats) *stats = S;
    return converged ? OVL_OK : OVL_NOT_CONVERGED;
}

}  // namespace ovl
