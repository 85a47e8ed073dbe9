// Mixed-precision multishift CG for (Q^2 + s_j) x_j = b, combined into
// y = sum_j w_j x_j.
//
// 0. FP64 phase (when sloppy_below > 0): the blocked multishift CG in FP64,
//    accumulating y directly, until the base residual |r|/|b| falls below
//    sloppy_below.  The rounding errors of a sloppy phase enter every shifted
//    residual in proportion to the size of the residuals at the time they are
//    made, so starting it only here keeps them of order eps_32 * sloppy_below.
// 1. Sloppy phase: the same recurrences continue with FP32 links, stencil and
//    Krylov vectors (ring, p0, t, p_j); the increments dx_j of the solutions
//    accumulate in FP64.  At the hand-over the residual of shift j is
//    zeta_j r0 (r0 the FP64 base residual then, exact up to FP64 rounding),
//    so the true residual of x_j is zeta_j r0 - (Q^2 + s_j) dx_j; for the base
//    shift (zeta = 1) it replaces the recursive residual whenever |r| has
//    dropped by reliable_delta since the last replacement.
// 2. Verification: every shifted system's FP64 true relative residual.  A
//    shift frozen in the FP64 phase has no sloppy part; its residual is the
//    FP64 recursive one at the iteration it froze.
// 3. Refinement: each system above tol solves (Q^2 + s_j) e = r_j with the
//    FP32 solver (batched over systems, one shift per batch entry) to the
//    relative accuracy that brings it below tol, and dx_j += e in FP64;
//    repeated (at most 3 rounds) until every system verifies.
// Finally y += sum_j w_j dx_j in FP64.
// Without an FP64 phase (sloppy_below = 0) the sloppy phase starts from
// x_j = 0 with r0 = b and zeta_j = 1.
//
// Base system.  When every shift is positive (and one more fits), the
// recurrences run with an extra shift 0 of weight 0 as their base: the
// unshifted system Q^2 x = b shares the Krylov space of all the others, so
// every shifted iterate is the same, while its residual update needs no s0 p0
// term and its stencil does not read p0 (one field less per iteration).  The
// extra system is neither verified, refined nor combined, and the caller's
// per-shift statistics exclude it.  It converges last, as the smallest shift
// did, a small fraction of an iteration later.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "mscg.h"

namespace ovl {

hipError_t launch_combine(const Lat &L, const double *w, int nshift, Fld x, Fld y, hipStream_t st,
                          bool accumulate = false);

// Systems per refinement batch: as many as RHS (at most NR), so that the
// workspace grows with nrhs only; refinement is rare and small.
static int refine_batch(int nrhs) { return std::max(1, std::min(NR, nrhs)); }

// Workspace: [fixed part][region A: the FP64 phase][region B].  Region B
// holds, one after another, the FP32 phase, the verification's Q x fields and
// the refinement.  With an FP64 phase the increments dx_j take over that
// phase's FP64 p_j fields (same count, same layout): the FP32 phase's first
// pass reads p_j and writes dx_j at the same element in the same thread, and
// nothing reads p_j afterwards.  At 48^3x96 with 24 poles that saves 24 FP64
// fields (49 GB) per RHS.
static size_t region_b_bytes(const Lat &L, int nrhs, int nshift, int m)
{
    const size_t F = field_bytes(P_F64, L.V);
    size_t a = blocked_ws_bytes(L, nrhs, nshift, m, true, P_F32, true);
    size_t b = blocked_ws_bytes(L, refine_batch(nrhs), 1, m, true, P_F32);
    return std::max(std::max(a, b), F);
}

// systems the recurrences carry for nshift caller shifts (room for the extra
// unshifted base)
static int mixed_systems(int nshift) { return nshift < NS ? nshift + 1 : nshift; }

// Workspace of the FP64 phase: FP64 storage, or room for either form with
// 48-bit storage (which falls back to FP64 storage without an unshifted base)
static size_t phase64_ws_bytes(const Lat &L, int nrhs, int nshift, int m64, bool s48)
{
    const size_t w = blocked_ws_bytes(L, nrhs, nshift, m64, false, P_F64);
    return s48 ? std::max(w, blocked_ws_bytes(L, nrhs, nshift, m64, false, P_F48)) : w;
}

size_t mixed_ws_bytes(const Lat &L, int nrhs, int nshift_caller, int m, int m64, bool f64_phase, bool f16_store,
                      bool s48)
{
    const size_t F = field_bytes(P_F64, L.V);
    const int nshift = mixed_systems(nshift_caller);
    WsCarve c{nullptr, 0, 0};
    if (f16_store) {
        c.take(field_bytes(P_F16S, L.V) * nrhs);      // FP16 storage of the sloppy vectors
        c.take(scale_bytes(L.V) * nrhs);
    }
    const int nbat = refine_batch(nrhs);
    if (!f64_phase) c.take(F * nrhs * nshift);        // x_j (no FP64 phase to lend its p_j)
    c.take(F * nbat);                                 // refinement batch right-hand sides
    c.take(F * nbat);                                 // refinement batch corrections
    c.take(F * nrhs);                                 // residual scratch
    c.take(F * nrhs);
    c.take(F * nrhs);                                 // base residual at the hand-over
    c.take(sizeof(double) * 2 * NR * site_blocks(L));
    c.take(sizeof(double) * 4 * NR);
    c.take(sizeof(double) * NR * NS);                 // shift of each (shift, RHS) field
    c.take(sizeof(double) * NR * NS);                 // zeta at the hand-over of each field
    if (f64_phase) c.take(align256(phase64_ws_bytes(L, nrhs, nshift, m64, s48)));
    c.take(region_b_bytes(L, nrhs, nshift, m));
    return c.off + 256;
}

// FP64 residuals res = bscale*b - (Q^2 + s) x for the nrhs fields of x (b has
// one field per RHS); their norms per RHS to host
static int residual_f64(const Lat &L, const void *U64, double m0, double s, Fld b, double bscale, Fld x, Fld t,
                        Fld res, double *partials, double *red, double *nres, hipStream_t st)
{
    const int R = x.nrhs;
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
    OVL_HIP(launch_axpby(L, bscale, b, -1.0, res, st));
    OVL_HIP(launch_norm2(L, res, partials, st));
    OVL_HIP(launch_reduce(partials, 1, R, nblk, red, st));
    double h[NR];
    OVL_HIP(hipMemcpyAsync(h, red, sizeof(double) * R, hipMemcpyDeviceToHost, st));
    OVL_HIP(hipStreamSynchronize(st));
    for (int q = 0; q < R; q++) nres[q] = std::sqrt(h[q]);
    return OVL_OK;
}

// The solve on nshift systems; base0: system 0 is the extra unshifted base
// (weight 0), which is not verified, refined or combined.
static int mixed_solve(const Lat &L, const ovl_gauge *U, double m0, int nshift, const double *shifts,
                       const double *weights, bool base0, Fld b, Fld y, const ovl_solver_params *prm,
                       ovl_solver_stats *stats, char *ws, size_t ws_bytes, hipStream_t st)
{
    const int R = b.nrhs;
    const int m = mixed_block(prm), m64 = mixed_block_f64(prm);
    const size_t F = field_bytes(P_F64, L.V);
    const bool f64_phase = prm->sloppy_below > 0.0;
    const bool f16 = prm->sloppy_f16 != 0;
    const int j1 = base0 ? 1 : 0;   // first caller shift
    WsCarve c{ws, 0, ws_bytes};
    Fld F16{};
    if (f16) {
        F16.d = c.take(field_bytes(P_F16S, L.V) * R);
        F16.sc = (float *)c.take(scale_bytes(L.V) * R);
        F16.prec = P_F16S;
        F16.nrhs = R;
    }
    const int NB = refine_batch(R);
    // the increments dx_j (field j*R + q): their own fields without an FP64
    // phase, else that phase's p_j (set after it)
    Fld X{f64_phase ? nullptr : c.take(F * R * nshift), nullptr, P_F64, R * nshift};
    Fld Eb{c.take(F * NB), nullptr, P_F64, NB};
    Fld Ex{c.take(F * NB), nullptr, P_F64, NB};
    Fld T{c.take(F * R), nullptr, P_F64, R};
    Fld Res{c.take(F * R), nullptr, P_F64, R};
    Fld R0{c.take(F * R), nullptr, P_F64, R};
    double *partials = (double *)c.take(sizeof(double) * 2 * NR * site_blocks(L));
    double *red = (double *)c.take(sizeof(double) * 4 * NR);
    double *fsh = (double *)c.take(sizeof(double) * NR * NS);
    double *fze = (double *)c.take(sizeof(double) * NR * NS);
    // region A (FP64 phase), then region B
    // 48-bit storage of the FP64 phase's vectors needs the unshifted base
    const bool s48 = f64_phase && prm->store48 && *std::min_element(shifts, shifts + nshift) == 0.0;
    const size_t w64 = f64_phase ? align256(phase64_ws_bytes(L, R, nshift, m64, prm->store48 != 0)) : 0;
    // The 48-bit rounding of the FP64 phase (2^-37 relative, made while |r| is
    // still of the order of |b|) opens a gap between the recursive and the true
    // residuals, about 1e-12 |b| in a CPU simulation of the format on an 8^4
    // field, that neither the residuals recorded for shifts frozen in that phase
    // nor the verification of the others (which starts from the hand-over
    // residual) sees.  The solve then aims at 0.9 tol, so that the true
    // residuals stay within tol with a tenth of it to spare.
    ovl_solver_params p48;
    if (s48) {
        p48 = *prm;
        p48.tol = 0.9 * prm->tol;
        prm = &p48;
    }
    char *sws = ws + c.off;
    char *swb = sws + w64;
    const size_t swb_bytes = ws_bytes - c.off - w64;
    const int nblk = site_blocks(L);

    // |b| per RHS
    std::vector<double> bn(R);
    {
        double h[NR];
        OVL_HIP(launch_norm2(L, b, partials, st));
        OVL_HIP(launch_reduce(partials, 1, R, nblk, red, st));
        OVL_HIP(hipMemcpyAsync(h, red, sizeof(double) * R, hipMemcpyDeviceToHost, st));
        OVL_HIP(hipStreamSynchronize(st));
        for (int q = 0; q < R; q++) bn[q] = std::sqrt(h[q]);
    }

    // 0. FP64 phase (y mode), 1. sloppy phase (x mode: x_j, or dx_j after a hand-over)
    BlkOpts o;
    o.m = m;
    o.keep_x = true;
    o.reliable = true;
    o.f16 = F16;   // the bulk only: the refinement keeps FP32 storage
    int rc;
    bool switched = false;
    Fld r0 = b;                                                    // residual at the hand-over
    std::vector<double> zeta((size_t)R * nshift, 1.0);             // zeta_j at the hand-over
    std::vector<double> frozen_res((size_t)R * nshift, -1.0);      // shifts frozen in the FP64 phase
    // shifts j >= nz froze in the FP64 phase for every RHS (shifts ascend, and
    // the largest converge first): their increments stay zero, so nothing
    // writes, verifies, refines or combines them
    int nz = nshift;
    if (f64_phase) {
        BlkOpts o64;
        o64.m = m64;
        o64.switch_rel = prm->sloppy_below;
        MsScratch h64{};
        rc = s48 ? mscg_blocked_t<P_F48>(L, U, m0, nshift, shifts, weights, b, y, o64, prm, stats, sws, w64, st, &h64)
                 : mscg_blocked_t<P_F64>(L, U, m0, nshift, shifts, weights, b, y, o64, prm, stats, sws, w64, st, &h64);
        if (rc < 0) return rc;
        if (rc != kSwitched) return rc;   // converged (or stopped) within the FP64 phase: y is complete
        switched = true;
        static thread_local MState hs;
        OVL_HIP(hipMemcpyAsync(&hs, h64.S, sizeof(MState), hipMemcpyDeviceToHost, st));
        OVL_HIP(hipStreamSynchronize(st));
        for (int j = 0; j < nshift; j++)
            for (int q = 0; q < R; q++) {
                zeta[(size_t)j * R + q] = hs.zeta[q][j];
                if (!hs.act[q][j] && bn[q] > 0)
                    frozen_res[(size_t)j * R + q] = std::sqrt(hs.frozen_rr[q][j]) / bn[q];
            }
        nz = 0;
        for (int j = 0; j < nshift; j++)
            for (int q = 0; q < R; q++)
                if (frozen_res[(size_t)j * R + q] < 0.0) nz = j + 1;
        // keep r0 outside the solver workspace, which the refinement reuses
        if (h64.r.prec == P_F64) OVL_HIP(hipMemcpyAsync(R0.d, h64.r.d, F * R, hipMemcpyDeviceToDevice, st));
        else OVL_HIP(launch_convert(L, h64.r, R0, st));
        r0 = R0;
        h64.host = &hs;
        o.resume = &h64;
        o.x_zero_shifts = nz;   // the increments dx_j (j < nz) start at zero
        // dx_j take over the FP64 p_j, which the first pass reads in place;
        // with 48-bit storage they go over the phase's dead ring, p0 and t
        // (xlend), and the first pass reads the 48-bit p_j from their fields
        if (h64.pj.nrhs != R * nshift) return OVL_ERR_INVALID;
        if (h64.pj.prec == P_F64) X.d = h64.pj.d;
        else if (h64.pj.prec == P_F48 && h64.xlend) X.d = h64.xlend;
        else return OVL_ERR_INVALID;
        o.x_ext = X;
        // the base system's true residual during the sloppy phase is r0 - (Q^2 + s0) dx_0
        rc = mscg_blocked_t<P_F32>(L, U, m0, nshift, shifts, nullptr, r0, Fld{}, o, prm, stats, swb, swb_bytes, st,
                                   nullptr);
        if (rc < 0) return rc;
    } else {
        o.x_ext = X;
        rc = mscg_blocked_t<P_F32>(L, U, m0, nshift, shifts, nullptr, b, Fld{}, o, prm, stats, swb, swb_bytes, st,
                                   nullptr);
        if (rc < 0) return rc;
    }

    // 2./3. verification and refinement
    std::vector<double> res((size_t)R * nshift), hsh((size_t)R * nshift);
    for (int f = 0; f < R * nshift; f++) hsh[f] = shifts[f / R];
    OVL_HIP(hipMemcpyAsync(fsh, hsh.data(), sizeof(double) * R * nshift, hipMemcpyHostToDevice, st));
    OVL_HIP(hipMemcpyAsync(fze, zeta.data(), sizeof(double) * R * nshift, hipMemcpyHostToDevice, st));
    // FP64 true residuals |zeta_j r0 - (Q^2 + s_j) x_j| / |b| of the fields
    // f0 .. f0+n-1 of X (field f = j*R + q), up to NV fields per pair of
    // batched stencils: t = Q x (into the solver workspace, free between
    // solves), then the norm without storing the residual
    const int NV = (int)std::min<size_t>(NR, std::max<size_t>(1, swb_bytes / F));
    Fld Tv{swb, nullptr, P_F64, NV};
    auto verify = [&](int f0, int n) -> int {
        for (int c0 = f0; c0 < f0 + n; c0 += NV) {
            const int nc = std::min(NV, f0 + n - c0);
            WArgs A{};
            A.U = U->f64;
            A.diag = m0 + 4.0;
            A.nrhs = nc;
            A.in = sub(X, L.V, c0, nc).d;
            A.out = Tv.d;
            OVL_HIP(launch_wilson(L, P_F64, W_PLAIN, true, A, st));
            WArgs B = A;
            B.in = Tv.d;
            B.out = nullptr;
            B.p = A.in;
            B.shiftv = fsh + c0;
            B.rin = r0.d;
            B.rin_first = c0 % R;
            B.rin_count = R;
            B.rin_scale = fze + c0;
            B.partials = partials;
            OVL_HIP(launch_wilson(L, P_F64, W_RESNORM, true, B, st));
            OVL_HIP(launch_reduce(partials, 1, nc, nblk, red, st));
            double h[NR];
            OVL_HIP(hipMemcpyAsync(h, red, sizeof(double) * nc, hipMemcpyDeviceToHost, st));
            OVL_HIP(hipStreamSynchronize(st));
            for (int k = 0; k < nc; k++) {
                const int f = c0 + k;
                res[f] = frozen_res[f] >= 0.0 ? frozen_res[f] : bn[f % R] > 0 ? std::sqrt(h[k]) / bn[f % R] : 0.0;
            }
            if (stats) stats->stencil_applies += 2;
        }
        return OVL_OK;
    };
    {
        // shifts frozen for every RHS in the FP64 phase need no stencils
        for (int f = nz * R; f < R * nshift; f++) res[f] = frozen_res[f];
        for (int f = 0; f < j1 * R; f++) res[f] = 0.0;   // the extra base: not verified
        if (nz > j1) {
            int e = verify(j1 * R, (nz - j1) * R);
            if (e) return e;
        }
    }
    int ncomb = nz;   // shifts whose increments enter y
    int refine_iters = 0;
    for (int round = 0; round < 3 && prm->refine; round++) {
        // A system frozen in the FP64 phase froze because its FP64 recursive
        // residual met tol (the freeze test is its convergence criterion), and
        // its solution lives in y only: it is never refined.  Every other
        // system (j, q) has j < nz = ncomb, so its increment field was written
        // by the first FP32 pass.
        std::vector<std::pair<int, int>> bad;   // (shift, rhs)
        for (int j = j1; j < nshift; j++)
            for (int q = 0; q < R; q++) {
                const size_t f = (size_t)j * R + q;
                if (frozen_res[f] < 0.0 && res[f] > prm->tol) bad.push_back({j, q});
            }
        if (bad.empty()) break;
        for (size_t b0 = 0; b0 < bad.size(); b0 += NB) {
            const int nbat = (int)std::min<size_t>(NB, bad.size() - b0);
            double bshift[NR], btol[NR];
            for (int k = 0; k < nbat; k++) {
                const int j = bad[b0 + k].first, q = bad[b0 + k].second;
                // right-hand side r_j = zeta_j r0 - (Q^2 + s_j) x_j of this RHS
                double nr[NR];
                int e = residual_f64(L, U->f64, m0, shifts[j], sub(r0, L.V, q, 1), zeta[(size_t)j * R + q],
                                     sub(X, L.V, j * R + q, 1), T, Res, partials, red, nr, st);
                if (e) return e;
                OVL_HIP(hipMemcpyAsync((char *)Eb.d + F * k, Res.d, F, hipMemcpyDeviceToDevice, st));
                bshift[k] = shifts[j];
                const double rel = bn[q] > 0 ? nr[0] / bn[q] : 0.0;
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
            int e = mscg_blocked_t<P_F32>(L, U, m0, 1, &zero, nullptr, eb, Fld{}, oc, prm, stats, swb, swb_bytes, st,
                                          nullptr);
            if (e < 0) return e;
            int mx = 0;
            for (int k = 0; k < nbat; k++) mx = std::max(mx, its[k]);
            refine_iters += mx;
            for (int k = 0; k < nbat; k++) {
                const int j = bad[b0 + k].first, q = bad[b0 + k].second;
                OVL_HIP(launch_axpby(L, 1.0, sub(ex, L.V, k, 1), 1.0, sub(X, L.V, j * R + q, 1), st));
                // a refined shift now has a sloppy part: verify it like the others
                frozen_res[(size_t)j * R + q] = -1.0;
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
    int status = rc == kSwitched ? OVL_OK : rc;
    for (int j = j1; j < nshift; j++)
        for (int q = 0; q < R; q++) {
            if (stats) stats->true_residual[q][j] = res[(size_t)j * R + q];
            // a system frozen in the FP64 phase met the freeze test; its
            // reported residual may round one ulp above tol
            if (frozen_res[(size_t)j * R + q] < 0.0 && !(res[(size_t)j * R + q] <= prm->tol))
                status = OVL_NOT_CONVERGED;
        }
    if (stats) stats->refine_iterations += refine_iters;
    if (ncomb > j1)
        OVL_HIP(launch_combine(L, weights + j1, ncomb - j1, sub(X, L.V, j1 * R, (ncomb - j1) * R), y, st, switched));
    else if (!switched)
        OVL_HIP(launch_zero(L, y, st));
    return status;
}

int mscg_mixed(const Lat &L, const ovl_gauge *U, double m0, int nshift, const double *shifts, const double *weights,
               Fld b, Fld y, const ovl_solver_params *prm, ovl_solver_stats *stats, char *ws, size_t ws_bytes,
               hipStream_t st)
{
    if (!weights) return OVL_ERR_INVALID;
    if (ws_bytes < mixed_ws_bytes(L, b.nrhs, nshift, mixed_block(prm), mixed_block_f64(prm), prm->sloppy_below > 0.0,
                                  prm->sloppy_f16 != 0, prm->store48 != 0))
        return OVL_ERR_WORKSPACE;
    bool base0 = mixed_systems(nshift) > nshift;
    for (int j = 0; j < nshift; j++) base0 = base0 && shifts[j] > 0.0;
    if (!base0) return mixed_solve(L, U, m0, nshift, shifts, weights, false, b, y, prm, stats, ws, ws_bytes, st);
    double sh[NS], w[NS];
    sh[0] = 0.0;
    w[0] = 0.0;
    for (int j = 0; j < nshift; j++) {
        sh[j + 1] = shifts[j];
        w[j + 1] = weights[j];
    }
    const int rc = mixed_solve(L, U, m0, nshift + 1, sh, w, true, b, y, prm, stats, ws, ws_bytes, st);
    if (stats) {
        // the caller's shifts are systems 1..nshift
        for (int q = 0; q < NR; q++) {
            for (int j = 0; j < nshift; j++) {
                stats->shift_iters[q][j] = stats->shift_iters[q][j + 1];
                stats->true_residual[q][j] = stats->true_residual[q][j + 1];
            }
            stats->shift_iters[q][nshift] = 0;
            stats->true_residual[q][nshift] = -1.0;
        }
    }
    return rc;
}

}  // namespace ovl
