// Multishift CG for (Q^2 + s_j) x_j = b on gfx950, Q = Gamma_5 D_W(m0).
//
// Shifted systems share one Krylov space (Jegerlehner's shifted CG
// recurrences).  One iteration is five launches, all on the caller's stream,
// with every scalar kept in device memory:
//   K_A  t = Q p0                        stencil; partials |t|^2, |p0|^2
//   K_a  alpha = rr / (|t|^2 + s0 |p0|^2), zeta_j', alpha_j  (one block per RHS)
//   K_B  r -= alpha (Q t + s0 p0)        stencil; partial |r|^2
//   K_b  beta, beta_j, convergence and freezing of shifts
//   K_C  x_j += alpha_j p_j, p_j = zeta_j' r + beta_j p_j for the active shifts
// (p0 is the smallest shift's direction; (p0, (Q^2+s0) p0) = |Q p0|^2 + s0|p0|^2.)
// The host only polls the per-RHS "finished" flags every check_every iterations.
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "mscg.h"

namespace ovl {

__global__ void k_ms_init(MState *st, const double *bb, int nrhs, int nshift, int j0)
{
    int t = threadIdx.x;
    if (t < nrhs) {
        st->bb[t] = bb[t];
        st->rr[t] = bb[t];
        st->rr_ref[t] = bb[t];
        st->alpha[t] = 0.0;
        st->alpha_old[t] = 1.0;
        st->beta[t] = 0.0;
        st->iter[t] = 0;
        st->skip[t] = !(bb[t] > 0.0);
        st->nonfinite[t] = !isfinite(bb[t]);
        st->want_update[t] = 0;
        for (int j = 0; j < nshift; j++) {
            st->zeta[t][j] = st->zeta_old[t][j] = st->zeta_new[t][j] = 1.0;
            st->aj[t][j] = st->bj[t][j] = 0.0;
            st->act[t][j] = st->skip[t] ? 0 : 1;
            st->act_cur[t][j] = 0;
            st->frozen_at[t][j] = st->skip[t] ? 0 : -1;
        }
    }
}

// alpha and the shifted zeta_j', alpha_j for RHS blockIdx.x; the partials
// have row stride nblk, of which the first cnt slots can be nonzero
__global__ __launch_bounds__(kBlock) void k_ms_alpha(MState *st, const double *partials, int nblk, int cnt)
{
    __shared__ double lds[8];
    const int r = blockIdx.x;
    const int nr = st->nrhs;
    const int j = threadIdx.x;   // shift j is thread j (NS <= 64: all in wave 0)
    // the previous iteration's p0 update has run (stream order)
    if (j == 0) st->run_c[r] = 0;
    if (st->skip[r]) {
        if (j < NS) st->act_cur[r][j] = 0;
        return;
    }
    // |t|^2 + s0 |p|^2; an unshifted base needs no |p|^2 (its t stencil writes
    // only the first set of partials)
    const double s0 = st->s0r[r];
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < cnt; k += kBlock) {
        a += partials[(size_t)r * nblk + k];
        if (s0 != 0.0) b += partials[(size_t)(nr + r) * nblk + k];
    }
    const double tt = block_sum_all(a, lds);
    const double pp = block_sum_all(b, lds + 4);
    const double pq = tt + s0 * pp;
    const double alpha = st->rr[r] / pq;
    if (!isfinite(alpha) || !(pq > 0.0)) {
        if (j < st->nshift) st->act_cur[r][j] = 0;
        if (j == 0) {
            st->nonfinite[r] = 1;
            st->skip[r] = 1;
        }
        return;
    }
    if (j == 0) st->alpha[r] = alpha;
    if (j < st->nshift) {
        const int on = st->act[r][j];
        st->act_cur[r][j] = on;
        if (on) {
            const double ao = st->alpha_old[r], be = st->beta[r];
            const double z = st->zeta[r][j], zo = st->zeta_old[r][j];
            const double zn = z * zo * ao / (alpha * be * (zo - z) + zo * ao * (1.0 + alpha * st->delta[j]));
            st->zeta_new[r][j] = zn;
            st->aj[r][j] = alpha * zn / z;
        }
    }
}

// beta, beta_j, freezing; RHS blockIdx.x, shift j in thread j
__global__ __launch_bounds__(kBlock) void k_ms_beta(MState *st, const double *partials, int nblk, int cnt)
{
    __shared__ double lds[4];
    const int r = blockIdx.x;
    const int j = threadIdx.x;
    if (st->skip[r]) return;
    double a = 0.0;
    for (int k = threadIdx.x; k < cnt; k += kBlock) a += partials[(size_t)r * nblk + k];
    const double rr_new = block_sum_all(a, lds);
    const int it = st->iter[r] + 1;
    if (!isfinite(rr_new)) {
        if (j == 0) {
            st->iter[r] = it;
            st->nonfinite[r] = 1;
            st->skip[r] = 1;
        }
        return;
    }
    const double beta = rr_new / st->rr[r];
    const double thr = st->tol2r[r] * st->bb[r];
    int live = 0;
    if (j < st->nshift && st->act_cur[r][j]) {
        const double z = st->zeta[r][j], zn = st->zeta_new[r][j];
        const double q = zn / z;
        st->bj[r][j] = beta * q * q;
        st->zeta_old[r][j] = z;
        st->zeta[r][j] = zn;
        if (zn * zn * rr_new <= thr) {
            st->act[r][j] = 0;
            st->frozen_at[r][j] = it;
            st->frozen_rr[r][j] = zn * zn * rr_new;
        } else {
            live = 1;
        }
    }
    // also the barrier between every thread's reads of rr and iter and
    // thread 0's writes below
    const int left = __syncthreads_count(live);
    if (j == 0) {
        st->iter[r] = it;
        st->beta[r] = beta;
        st->rr[r] = rr_new;
        st->alpha_old[r] = st->alpha[r];
        if (!left) st->skip[r] = 1;
    }
}

// Shift update, FP64 fields.  Fields: r [nrhs], p and x [nshift][nrhs].
template <int PREC>
__global__ __launch_bounds__(kBlock) void k_ms_update(Geom g, int nb, const MState *st, const void *rf, const float *rsc,
                                                      void *pf, float *psc, void *xf, float *xsc, int nrhs)
{
    using T = typename Real<PREC>::T;
    const int r = blockIdx.y;
    const int ns = st->nshift;
    int any = 0;
    for (int j = 0; j < ns; j++) any |= st->act_cur[r][j];
    if (!any) return;
    const int b = blockIdx.x;
    const int p = b / nb, i = (b % nb) * kBlock + threadIdx.x;
    if (i >= g.Vh) return;
    cplx<T> rv[4][3];
    spinor_ref<PREC>(rf, rsc, g.S, r).load(p, i, rv);
    for (int j = 0; j < ns; j++) {
        if (!st->act_cur[r][j]) continue;
        const T aj = (T)st->aj[r][j], bj = (T)st->bj[r][j], zn = (T)st->zeta_new[r][j];
        auto P = spinor_ref<PREC>(pf, psc, g.S, j * nrhs + r);
        auto X = spinor_ref<PREC>(xf, xsc, g.S, j * nrhs + r);
        cplx<T> pv[4][3], xv[4][3];
        P.load(p, i, pv);
        X.load(p, i, xv);
#pragma unroll
        for (int s = 0; s < 4; s++)
#pragma unroll
            for (int c = 0; c < 3; c++) {
                xv[s][c] = {fma(aj, pv[s][c].x, xv[s][c].x), fma(aj, pv[s][c].y, xv[s][c].y)};
                pv[s][c] = {fma(zn, rv[s][c].x, bj * pv[s][c].x), fma(zn, rv[s][c].y, bj * pv[s][c].y)};
            }
        X.store(p, i, xv);
        P.store(p, i, pv);
    }
}

// r = b, p_j = b, x_j = 0 (FP64 solver start)
__global__ __launch_bounds__(kBlock) void k_ms_start(Geom g, int nb, const double2 *b, double2 *r, double2 *pf, double2 *xf,
                                                     int nrhs, int nshift)
{
    const int rr = blockIdx.y;
    const int bl = blockIdx.x;
    const int p = bl / nb, i = (bl % nb) * kBlock + threadIdx.x;
    if (i >= g.Vh) return;
    cplx<double> v[4][3], z[4][3];
    spinor_ref<P_F64>(b, nullptr, g.S, rr).load(p, i, v);
    spinor_ref<P_F64>(r, nullptr, g.S, rr).store(p, i, v);
#pragma unroll
    for (int k = 0; k < 12; k++) z[k / 3][k % 3] = {0.0, 0.0};
    for (int j = 0; j < nshift; j++) {
        spinor_ref<P_F64>(pf, nullptr, g.S, j * nrhs + rr).store(p, i, v);
        spinor_ref<P_F64>(xf, nullptr, g.S, j * nrhs + rr).store(p, i, z);
    }
}

// y_r = sum_j w_j x_{j,r} (FP64)
// y = sum_j w_j x_j, or y += sum_j w_j x_j with accumulate
__global__ __launch_bounds__(kBlock) void k_combine(Geom g, int nb, ShiftWeights w, const double2 *xf, double2 *y,
                                                    int nrhs, int nshift, int accumulate)
{
    const int rr = blockIdx.y;
    const int bl = blockIdx.x;
    const int p = bl / nb, i = (bl % nb) * kBlock + threadIdx.x;
    if (i >= g.Vh) return;
    cplx<double> acc[4][3], v[4][3];
    if (accumulate) {
        spinor_ref<P_F64>(y, nullptr, g.S, rr).load(p, i, acc);
    } else {
#pragma unroll
        for (int k = 0; k < 12; k++) acc[k / 3][k % 3] = {0.0, 0.0};
    }
    for (int j = 0; j < nshift; j++) {
        spinor_ref<P_F64>(xf, nullptr, g.S, j * nrhs + rr).load(p, i, v);
        const double wj = w.w[j];
#pragma unroll
        for (int k = 0; k < 12; k++)
            acc[k / 3][k % 3] = {fma(wj, v[k / 3][k % 3].x, acc[k / 3][k % 3].x), fma(wj, v[k / 3][k % 3].y, acc[k / 3][k % 3].y)};
    }
    spinor_ref<P_F64>(y, nullptr, g.S, rr).store(p, i, acc);
}

// ------------------------------------------------------------------ host

// Workspace of the FP64 multishift CG: state, partial sums, r, t, p_j, x_j
// and two scratch fields.
size_t mscg_ws_bytes(const Lat &L, int nrhs, int nshift)
{
    WsCarve c{nullptr, 0, 0};
    size_t F = field_bytes(P_F64, L.V);
    c.take(sizeof(MState));
    c.take(sizeof(double) * 2 * nrhs * site_blocks(L));
    c.take(sizeof(double) * 4 * NR);
    c.take(F * nrhs);            // r
    c.take(F * nrhs);            // t
    c.take(F * nrhs * nshift);   // p
    c.take(F * nrhs * nshift);   // x
    c.take(F * nrhs);            // scratch 1
    c.take(F * nrhs);            // scratch 2
    return c.off + 256;
}

static int read_state(MState &h, const MState *d, hipStream_t st)
{
    OVL_HIP(hipMemcpyAsync(&h, d, sizeof(MState), hipMemcpyDeviceToHost, st));
    OVL_HIP(hipStreamSynchronize(st));
    return OVL_OK;
}

// Upload the constant part of the scalar state, |b|^2 per RHS and the
// initial recurrence values.  *j0_out: index of the smallest (base) shift.
int mscg_init_state(const Lat &L, MState *S, double *partials, double *red, Fld b, int nshift, const double *shifts,
                    const ovl_solver_params *prm, int *j0_out, hipStream_t st, const double *rhs_shift,
                    const double *rhs_tol)
{
    const int R = b.nrhs;
    int j0 = 0;
    for (int j = 1; j < nshift; j++)
        if (shifts[j] < shifts[j0]) j0 = j;
    static thread_local MState h;
    std::memset(&h, 0, sizeof h);
    for (int r = 0; r < R; r++) {
        h.s0r[r] = rhs_shift ? rhs_shift[r] : shifts[j0];
        double t = rhs_tol ? rhs_tol[r] : prm->tol;
        h.tol2r[r] = t * t;
        h.one[r] = 1.0;
    }
    h.nrhs = R;
    h.nshift = nshift;
    for (int j = 0; j < nshift; j++) h.delta[j] = shifts[j] - shifts[j0];
    OVL_HIP(hipMemcpyAsync(S, &h, sizeof(MState), hipMemcpyHostToDevice, st));
    OVL_HIP(launch_norm2(L, b, partials, st));
    OVL_HIP(launch_reduce(partials, 1, R, site_blocks(L), red, st));
    k_ms_init<<<1, 64, 0, st>>>(S, red, R, nshift, j0);
    OVL_HIP(hipGetLastError());
    *j0_out = j0;
    return OVL_OK;
}

// FP64 multishift CG.  The solutions x_j (field j*nrhs + r) stay in the
// workspace and are returned through scr->x.  Leaves per-shift iterations in
// stats.  Returns status.
int mscg_f64(const Lat &L, const void *U64, double m0, int nshift, const double *shifts, Fld b,
             const ovl_solver_params *prm, ovl_solver_stats *stats, char *ws, size_t ws_bytes, hipStream_t st,
             MsScratch *scr)
{
    const int R = b.nrhs;
    const int nblk = site_blocks(L);
    const int npart = stencil_partials(L, P_F64, R);   // slots the iteration stencils fill
    WsCarve c{ws, 0, ws_bytes};
    size_t F = field_bytes(P_F64, L.V);
    MState *S = (MState *)c.take(sizeof(MState));
    double *partials = (double *)c.take(sizeof(double) * 2 * R * nblk);
    double *red = (double *)c.take(sizeof(double) * 4 * NR);
    Fld r{c.take(F * R), nullptr, P_F64, R};
    Fld t{c.take(F * R), nullptr, P_F64, R};
    Fld pfl{c.take(F * R * nshift), nullptr, P_F64, R * nshift};
    Fld x{c.take(F * R * nshift), nullptr, P_F64, R * nshift};
    Fld y{c.take(F * R), nullptr, P_F64, R};
    Fld y2{c.take(F * R), nullptr, P_F64, R};
    if (c.off > ws_bytes) return OVL_ERR_WORKSPACE;
    scr->partials = partials;
    scr->red = red;
    scr->x = x;
    scr->s1 = y;
    scr->s2 = y2;

    int j0 = 0;
    int rc0 = mscg_init_state(L, S, partials, red, b, nshift, shifts, prm, &j0, st, nullptr, nullptr);
    if (rc0) return rc0;
    const double s0 = shifts[j0];
    MState h;
    dim3 sgrid(nblk, R);
    k_ms_start<<<sgrid, kBlock, 0, st>>>(L.g, L.nb, (const double2 *)b.d, (double2 *)r.d, (double2 *)pfl.d,
                                         (double2 *)x.d, R, nshift);
    OVL_HIP(hipGetLastError());

    Fld p0 = sub(pfl, L.V, j0 * R, R);
    WArgs A{};
    A.U = U64;
    A.diag = m0 + 4.0;
    A.partials = partials;
    A.skip = S->skip;
    A.nrhs = R;
    WArgs B = A;
    A.in = p0.d;
    A.out = t.d;
    B.in = t.d;
    B.p = p0.d;
    B.rin = r.d;   // r is updated in place
    B.out = r.d;
    B.shift = s0;
    B.alpha = S->alpha;

    const int check = prm->check_every > 0 ? prm->check_every : 10;
    int it = 0;
    int stencils = 0;
    bool done = false;
    Prof prof;
    prof.on = prm->profile != 0 && stats;
    prof.stencil_only = prm->profile == 2;
    prof.st = st;
    while (it < prm->maxiter && !done) {
        int batch = std::min(check, prm->maxiter - it);
        // each timed kernel records its own start and end (prof.pair)
        hipEvent_t v0, v1;
        for (int k = 0; k < batch; k++) {
            prof.pair(OVL_K_STENCIL, &v0, &v1);
            OVL_HIP(launch_wilson(L, P_F64, W_NORM, true, A, st, v0, v1));
            prof.pair(OVL_K_SCALAR, &v0, &v1);
            launch_k(k_ms_alpha, dim3(R), dim3(kBlock), st, v0, v1, S, (const double *)partials, nblk, npart);
            prof.pair(OVL_K_STENCIL, &v0, &v1);
            OVL_HIP(launch_wilson(L, P_F64, W_RUPDATE, true, B, st, v0, v1));
            prof.pair(OVL_K_SCALAR, &v0, &v1);
            launch_k(k_ms_beta, dim3(R), dim3(kBlock), st, v0, v1, S, (const double *)partials, nblk, npart);
            prof.pair(OVL_K_UPDATE, &v0, &v1);
            launch_k(k_ms_update<P_F64>, sgrid, dim3(kBlock), st, v0, v1, L.g, L.nb, (const MState *)S,
                     (const void *)r.d, (const float *)nullptr, pfl.d, (float *)nullptr, x.d, (float *)nullptr, R);
            OVL_HIP(hipGetLastError());
            stencils += 2;
        }
        int prc = prof.flush(stats);
        if (prc) return prc;
        it += batch;
        int one[NR];
        OVL_HIP(hipMemcpyAsync(one, S->skip, sizeof(int) * NR, hipMemcpyDeviceToHost, st));
        OVL_HIP(hipStreamSynchronize(st));
        done = true;
        for (int q = 0; q < R; q++) done = done && one[q];
    }
    int rc = read_state(h, S, st);
    if (rc) return rc;
    int status = OVL_OK;
    for (int q = 0; q < R; q++) {
        if (h.nonfinite[q]) return OVL_ERR_NONFINITE;
        if (stats) stats->iterations[q] = h.iter[q];
        for (int j = 0; j < nshift; j++) {
            if (stats) stats->shift_iters[q][j] = h.frozen_at[q][j] >= 0 ? h.frozen_at[q][j] : h.iter[q];
            if (h.frozen_at[q][j] < 0) status = OVL_NOT_CONVERGED;
        }
    }
    if (stats) {
        stats->stencil_applies += stencils;
        // compulsory bytes per iteration: K_A reads p0 and the links and writes
        // t; K_B reads t, the links, p0 and r and writes r; K_C reads r once and
        // reads and writes p_j, x_j of every active shift.  (Launches on an RHS
        // whose blocks exit early move nothing and are not counted.)
        double Fb = (double)F, G = (double)L.V * 4 * 96.0;
        double sten = 0, upd = 0;
        for (int q = 0; q < R; q++) {
            long act_iters = 0;
            for (int j = 0; j < nshift; j++) act_iters += stats->shift_iters[q][j];
            sten += h.iter[q] * (6 * Fb + 2 * G);
            upd += h.iter[q] * Fb + act_iters * 4 * Fb;
        }
        stats->kernel_bytes[OVL_K_STENCIL] += sten;
        stats->kernel_bytes[OVL_K_UPDATE] += upd;
        stats->algorithmic_bytes += sten + upd;
    }
    return status;
}

// ||b - (Q^2 + s) x|| / ||b|| per RHS for FP64 fields; q, t scratch (nrhs fields)
int true_residuals_f64(const Lat &L, const void *U64, double m0, double s, Fld b, Fld x, Fld q, Fld t,
                       double *partials, double *red, double *out, hipStream_t st)
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
    B.out = q.d;
    OVL_HIP(launch_wilson(L, P_F64, W_SHIFT, true, B, st));
    OVL_HIP(launch_diff_norm2(L, b, q, partials, st));
    OVL_HIP(launch_reduce(partials, 1, R, nblk, red, st));
    OVL_HIP(launch_norm2(L, b, partials, st));
    OVL_HIP(launch_reduce(partials, 1, R, nblk, red + R, st));
    double h[2 * NR];
    OVL_HIP(hipMemcpyAsync(h, red, sizeof(double) * 2 * R, hipMemcpyDeviceToHost, st));
    OVL_HIP(hipStreamSynchronize(st));
    for (int q2 = 0; q2 < R; q2++) out[q2] = h[R + q2] > 0 ? std::sqrt(h[q2] / h[R + q2]) : 0.0;
    return OVL_OK;
}

hipError_t launch_combine(const Lat &L, const double *w, int nshift, Fld x, Fld y, hipStream_t st, bool accumulate)
{
    ShiftWeights sw;
    for (int j = 0; j < NS; j++) sw.w[j] = j < nshift ? w[j] : 0.0;
    dim3 grid(site_blocks(L), y.nrhs);
    k_combine<<<grid, kBlock, 0, st>>>(L.g, L.nb, sw, (const double2 *)x.d, (double2 *)y.d, y.nrhs, nshift,
                                       accumulate ? 1 : 0);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Lanczos
// Extreme eigenvalues of a symmetric tridiagonal matrix (diagonal a[0..m-1],
// off-diagonal e[0..m-2]) by bisection on the inertia of T - x I.
static int count_below(int m, const double *a, const double *e, double x)
{
    int neg = 0;
    double q = a[0] - x;
    neg += q < 0;
    for (int k = 1; k < m; k++) {
        double piv = (q != 0.0) ? q : 1e-300;
        q = (a[k] - x) - e[k - 1] * e[k - 1] / piv;
        neg += q < 0;
    }
    return neg;
}

static double kth_eig(int m, const double *a, const double *e, int k, double lo, double hi)
{
    while (hi - lo > 1e-15 * std::max(std::fabs(lo), std::fabs(hi)) && hi - lo > 1e-300) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (count_below(m, a, e, mid) > k) hi = mid; else lo = mid;
    }
    return 0.5 * (lo + hi);
}

size_t lanczos_ws_bytes(const Lat &L)
{
    size_t F = field_bytes(P_F64, L.V);
    return align256(sizeof(double) * 2 * site_blocks(L)) + align256(sizeof(double) * 8) + 4 * align256(F) + 256;
}

int lanczos_bounds(const Lat &L, const void *U64, double m0, int iters, Fld start, double *tmin, double *tmax,
                   char *ws, size_t ws_bytes, hipStream_t st)
{
    const int nblk = site_blocks(L);
    size_t F = field_bytes(P_F64, L.V);
    WsCarve c{ws, 0, ws_bytes};
    double *partials = (double *)c.take(sizeof(double) * 2 * nblk);
    double *red = (double *)c.take(sizeof(double) * 8);
    Fld v{c.take(F), nullptr, P_F64, 1}, vp{c.take(F), nullptr, P_F64, 1};
    Fld w{c.take(F), nullptr, P_F64, 1}, t{c.take(F), nullptr, P_F64, 1};
    if (c.off > ws_bytes) return OVL_ERR_WORKSPACE;
    std::vector<double> al, be;
    double h[2];
    OVL_HIP(launch_norm2(L, start, partials, st));
    OVL_HIP(launch_reduce(partials, 1, 1, nblk, red, st));
    OVL_HIP(hipMemcpyAsync(h, red, sizeof(double), hipMemcpyDeviceToHost, st));
    OVL_HIP(hipStreamSynchronize(st));
    if (!(h[0] > 0) || !std::isfinite(h[0])) return OVL_ERR_INVALID;
    OVL_HIP(launch_axpby(L, 1.0 / std::sqrt(h[0]), start, 0.0, v, st));
    OVL_HIP(launch_zero(L, vp, st));
    double bprev = 0.0;
    for (int k = 0; k < iters; k++) {
        WArgs A{};
        A.U = U64;
        A.diag = m0 + 4.0;
        A.nrhs = 1;
        A.in = v.d;
        A.out = t.d;
        OVL_HIP(launch_wilson(L, P_F64, W_PLAIN, true, A, st));
        A.in = t.d;
        A.out = w.d;
        OVL_HIP(launch_wilson(L, P_F64, W_PLAIN, true, A, st));
        OVL_HIP(launch_dot(L, v, w, partials, st));
        OVL_HIP(launch_reduce(partials, 1, 1, nblk, red, st));
        OVL_HIP(hipMemcpyAsync(h, red, sizeof(double), hipMemcpyDeviceToHost, st));
        OVL_HIP(hipStreamSynchronize(st));
        double a = h[0];
        al.push_back(a);
        // w -= a v + bprev vp
        OVL_HIP(launch_axpby(L, -a, v, 1.0, w, st));
        OVL_HIP(launch_axpby(L, -bprev, vp, 1.0, w, st));
        OVL_HIP(launch_norm2(L, w, partials, st));
        OVL_HIP(launch_reduce(partials, 1, 1, nblk, red, st));
        OVL_HIP(hipMemcpyAsync(h, red, sizeof(double), hipMemcpyDeviceToHost, st));
        OVL_HIP(hipStreamSynchronize(st));
        double bn = std::sqrt(h[0]);
        if (!std::isfinite(a) || !std::isfinite(bn)) return OVL_ERR_NONFINITE;
        if (bn < 1e-14 || k == iters - 1) break;
        be.push_back(bn);
        // vp = v; v = w / bn
        std::swap(vp, v);
        OVL_HIP(launch_axpby(L, 1.0 / bn, w, 0.0, v, st));
        bprev = bn;
    }
    int m = (int)al.size();
    double lo = al[0], hi = al[0];
    for (int k = 0; k < m; k++) {
        double rad = (k > 0 ? std::fabs(be[k - 1]) : 0.0) + (k < m - 1 ? std::fabs(be[k]) : 0.0);
        lo = std::min(lo, al[k] - rad);
        hi = std::max(hi, al[k] + rad);
    }
    *tmin = kth_eig(m, al.data(), be.data(), 0, lo, hi);
    *tmax = kth_eig(m, al.data(), be.data(), m - 1, lo, hi);
    return OVL_OK;
}

}  // namespace ovl
