// Mixed-precision multishift CG for (Q^2 + s_j) x_j = b.
//
// 0. FP64 phase (when sloppy_below > 0): the blocked multishift CG in FP64,
//    with FP64 x_j, until the base residual |r|/|b| falls below sloppy_below.
//    The rounding errors of a sloppy phase enter every shifted residual in
//    proportion to the size of the residuals at the time they are made, so
//    starting it only here keeps them of order eps_32 * sloppy_below.
// 1. Sloppy phase: the same recurrences continue with FP32 links, stencil
//    and Krylov vectors (ring, p0, t, p_j); the solutions x_j accumulate in
//    FP64; the base residual is replaced by the FP64 true residual
//    b - (Q^2 + s0) x_0 whenever |r| has dropped by reliable_delta since the
//    last replacement.
// 2. Verification: every shifted system's FP64 true residual
//    |b - (Q^2 + s_j) x_j| / |b|.
// 3. Refinement: each system above tol solves (Q^2 + s_j) e = r_j with the
//    FP32 solver (batched over systems, one shift per batch entry) to the
//    relative accuracy that brings it below tol, and x_j += e in FP64;
//    repeated (at most 3 rounds) until every system verifies.
// The caller then forms y = sum_j w_j x_j in FP64.
#include <cmath>
#include <cstring>
#include <vector>

#include "mscg.h"

namespace ovl {

hipError_t launch_combine(const Lat &L, const double *w, int nshift, Fld x, Fld y, hipStream_t st);

size_t mixed_ws_bytes(const Lat &L, int nrhs, int nshift, int m, bool f64_phase)
{
    const size_t F = field_bytes(P_F64, L.V);
    WsCarve c{nullptr, 0, 0};
    c.take(F * nrhs * nshift);                        // x_j
    c.take(F * NR);                                   // batch right-hand sides
    c.take(F * NR);                                   // batch corrections
    c.take(F * nrhs);                                 // residual scratch
    c.take(F * nrhs);
    c.take(sizeof(double) * 2 * NR * site_blocks(L));
    c.take(sizeof(double) * 4 * NR);
    c.take(sizeof(double) * NR * NS);                 // shift of each (shift, RHS) field
    // the FP64 phase's workspace stays alive while the FP32 phase takes over
    size_t a = blocked_ws_bytes(L, nrhs, nshift, m, true, P_F32, true);
    if (f64_phase) a += blocked_ws_bytes(L, nrhs, nshift, m, true, P_F64, true);
    size_t b = blocked_ws_bytes(L, NR, 1, m, true, P_F32);
    return c.off + std::max(a, b) + 256;
}

// FP64 residuals res = b - (Q^2 + s) x for the nrhs fields of x; norms of
// res and b per RHS to host (nres, nb)
static int residual_f64(const Lat &L, const void *U64, double m0, double s, Fld b, Fld x, Fld t, Fld res,
                        double *partials, double *red, double *nres, double *nb, hipStream_t st)
{
    const int R = b.nrhs;
    const int nblk = site_blocks(L);
    WArgs A{};
    A.U = U64;
    A.diag = m0 + 4.0;
    A.nrhs = R;
    A.in = x.d;
    A.out = t.d;
    OVL_HIP(launch_wilson(L, P_F64, W_PLAIN, true, A, st));
    WArgs B = A;
    B.in = t.d;
    B.p = x.d;
    B.shift = s;
    B.out = res.d;
    OVL_HIP(launch_wilson(L, P_F64, W_SHIFT, true, B, st));
    OVL_HIP(launch_axpby(L, 1.0, b, -1.0, res, st));
    OVL_HIP(launch_norm2(L, res, partials, st));
    OVL_HIP(launch_reduce(partials, 1, R, nblk, red, st));
    OVL_HIP(launch_norm2(L, b, partials, st));
    OVL_HIP(launch_reduce(partials, 1, R, nblk, red + R, st));
    double h[2 * NR];
    OVL_HIP(hipMemcpyAsync(h, red, sizeof(double) * 2 * R, hipMemcpyDeviceToHost, st));
    OVL_HIP(hipStreamSynchronize(st));
    for (int q = 0; q < R; q++) {
        nres[q] = std::sqrt(h[q]);
        nb[q] = std::sqrt(h[R + q]);
    }
    return OVL_OK;
}

int mscg_mixed(const Lat &L, const ovl_gauge *U, double m0, int nshift, const double *shifts, const double *weights,
               Fld b, Fld y, const ovl_solver_params *prm, ovl_solver_stats *stats, char *ws, size_t ws_bytes,
               hipStream_t st)
{
    const int R = b.nrhs;
    const int m = prm->block > 0 ? prm->block : 16;
    const size_t F = field_bytes(P_F64, L.V);
    const bool f64_phase = prm->sloppy_below > 0.0;
    if (ws_bytes < mixed_ws_bytes(L, R, nshift, m, f64_phase)) return OVL_ERR_WORKSPACE;
    WsCarve c{ws, 0, ws_bytes};
    Fld X{c.take(F * R * nshift), nullptr, P_F64, R * nshift};
    Fld Eb{c.take(F * NR), nullptr, P_F64, NR};
    Fld Ex{c.take(F * NR), nullptr, P_F64, NR};
    Fld T{c.take(F * R), nullptr, P_F64, R};
    Fld Res{c.take(F * R), nullptr, P_F64, R};
    double *partials = (double *)c.take(sizeof(double) * 2 * NR * site_blocks(L));
    double *red = (double *)c.take(sizeof(double) * 4 * NR);
    double *fsh = (double *)c.take(sizeof(double) * NR * NS);
    char *sws = ws + c.off;
    size_t sws_bytes = ws_bytes - c.off;

    // 0. FP64 phase, 1. sloppy phase
    BlkOpts o;
    o.m = m;
    o.keep_x = true;
    o.reliable = true;
    o.x_ext = X;
    int rc;
    MsScratch h64{};
    if (f64_phase) {
        const size_t w64 = blocked_ws_bytes(L, R, nshift, m, true, P_F64, true);
        BlkOpts o64 = o;
        o64.reliable = false;
        o64.switch_rel = prm->sloppy_below;
        rc = mscg_blocked_t<P_F64>(L, U, m0, nshift, shifts, nullptr, b, Fld{}, o64, prm, stats, sws, w64, st, &h64);
        if (rc < 0) return rc;
        if (rc == kSwitched) {
            o.resume = &h64;
            rc = mscg_blocked_t<P_F32>(L, U, m0, nshift, shifts, nullptr, b, Fld{}, o, prm, stats, sws + w64,
                                       sws_bytes - w64, st, nullptr);
            if (rc < 0) return rc;
        }
    } else {
        rc = mscg_blocked_t<P_F32>(L, U, m0, nshift, shifts, nullptr, b, Fld{}, o, prm, stats, sws, sws_bytes, st,
                                   nullptr);
        if (rc < 0) return rc;
    }

    // 2./3. verification and refinement
    const int nblk = site_blocks(L);
    std::vector<double> res((size_t)R * nshift), bn(R), hsh((size_t)R * nshift);
    for (int f = 0; f < R * nshift; f++) hsh[f] = shifts[f / R];
    OVL_HIP(hipMemcpyAsync(fsh, hsh.data(), sizeof(double) * R * nshift, hipMemcpyHostToDevice, st));
    {
        double h[NR];
        OVL_HIP(launch_norm2(L, b, partials, st));
        OVL_HIP(launch_reduce(partials, 1, R, nblk, red, st));
        OVL_HIP(hipMemcpyAsync(h, red, sizeof(double) * R, hipMemcpyDeviceToHost, st));
        OVL_HIP(hipStreamSynchronize(st));
        for (int q = 0; q < R; q++) bn[q] = std::sqrt(h[q]);
    }
    // FP64 true residuals |b - (Q^2 + s_j) x_j| / |b| of the fields f0 .. f0+n-1
    // of X (field f = j*R + q), up to NR fields per pair of batched stencils:
    // t = Q x, then the norm of b - (Q t + s x) without storing it
    auto verify = [&](int f0, int n) -> int {
        for (int c0 = f0; c0 < f0 + n; c0 += NR) {
            const int nc = std::min(NR, f0 + n - c0);
            WArgs A{};
            A.U = U->f64;
            A.diag = m0 + 4.0;
            A.nrhs = nc;
            A.in = sub(X, L.V, c0, nc).d;
            A.out = Eb.d;
            OVL_HIP(launch_wilson(L, P_F64, W_PLAIN, true, A, st));
            WArgs B = A;
            B.in = Eb.d;
            B.out = nullptr;
            B.p = A.in;
            B.shiftv = fsh + c0;
            B.rin = b.d;
            B.rin_first = c0 % R;
            B.rin_count = R;
            B.partials = partials;
            OVL_HIP(launch_wilson(L, P_F64, W_RESNORM, true, B, st));
            OVL_HIP(launch_reduce(partials, 1, nc, nblk, red, st));
            double h[NR];
            OVL_HIP(hipMemcpyAsync(h, red, sizeof(double) * nc, hipMemcpyDeviceToHost, st));
            OVL_HIP(hipStreamSynchronize(st));
            for (int k = 0; k < nc; k++) {
                const int f = c0 + k;
                res[f] = bn[f % R] > 0 ? std::sqrt(h[k]) / bn[f % R] : 0.0;
            }
            if (stats) stats->stencil_applies += 2;
        }
        return OVL_OK;
    };
    {
        int e = verify(0, R * nshift);
        if (e) return e;
    }
    int refine_iters = 0;
    for (int round = 0; round < 3 && prm->refine; round++) {
        std::vector<std::pair<int, int>> bad;   // (shift, rhs)
        for (int j = 0; j < nshift; j++)
            for (int q = 0; q < R; q++)
                if (res[(size_t)j * R + q] > prm->tol) bad.push_back({j, q});
        if (bad.empty()) break;
        for (size_t b0 = 0; b0 < bad.size(); b0 += NR) {
            const int nbat = (int)std::min<size_t>(NR, bad.size() - b0);
            double bshift[NR], btol[NR];
            for (int k = 0; k < nbat; k++) {
                const int j = bad[b0 + k].first, q = bad[b0 + k].second;
                // right-hand side r_j = b - (Q^2 + s_j) x_j for this RHS
                double nr[NR], nb[NR];
                int e = residual_f64(L, U->f64, m0, shifts[j], b, sub(X, L.V, j * R, R), T, Res, partials, red, nr,
                                     nb, st);
                if (e) return e;
                OVL_HIP(hipMemcpyAsync((char *)Eb.d + F * k, (char *)Res.d + F * q, F, hipMemcpyDeviceToDevice, st));
                bshift[k] = shifts[j];
                const double rel = nb[q] > 0 ? nr[q] / nb[q] : 0.0;
                btol[k] = std::min(0.5, std::max(1e-7, 0.25 * prm->tol / std::max(rel, 1e-300)));
                if (stats) stats->stencil_applies += 2;
            }
            Fld eb = sub(Eb, L.V, 0, nbat), ex = sub(Ex, L.V, 0, nbat);
            BlkOpts oc;
            oc.m = m;
            oc.keep_x = true;
            oc.reliable = true;
            oc.quiet = true;
            oc.rhs_shift = bshift;
            oc.rhs_tol = btol;
            oc.x_ext = ex;
            int its[NR] = {0};
            oc.iters_out = its;
            const double zero = 0.0;
            int e = mscg_blocked_t<P_F32>(L, U, m0, 1, &zero, nullptr, eb, Fld{}, oc, prm, stats, sws, sws_bytes, st,
                                          nullptr);
            if (e < 0) return e;
            int mx = 0;
            for (int k = 0; k < nbat; k++) mx = std::max(mx, its[k]);
            refine_iters += mx;
            for (int k = 0; k < nbat; k++) {
                const int j = bad[b0 + k].first, q = bad[b0 + k].second;
                OVL_HIP(launch_axpby(L, 1.0, sub(ex, L.V, k, 1), 1.0, sub(X, L.V, j * R + q, 1), st));
            }
        }
        for (int j = 0; j < nshift; j++) {
            bool any = false;
            for (auto &pr : bad) any = any || pr.first == j;
            if (!any) continue;
            int e = verify(j * R, R);
            if (e) return e;
        }
    }
    int status = rc;
    for (int j = 0; j < nshift; j++)
        for (int q = 0; q < R; q++) {
            if (stats) stats->true_residual[q][j] = res[(size_t)j * R + q];
            if (!(res[(size_t)j * R + q] <= prm->tol)) status = OVL_NOT_CONVERGED;
        }
    if (stats) stats->refine_iterations += refine_iters;
    OVL_HIP(launch_combine(L, weights, nshift, X, y, st));
    return status;
}

}  // namespace ovl
