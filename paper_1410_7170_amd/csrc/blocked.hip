// Multishift CG with blocked shift updates (FP64 throughout).
//
// The iterates are those of the standard multishift CG (Jegerlehner's shifted
// recurrences), but the shifted vectors are not touched every iteration.
// Each iteration runs only the base CG on the smallest shift s0:
//   K_A  t = Q p0                       (stencil; partials |t|^2, |p0|^2)
//   K_a  alpha, zeta_j', alpha_j        (one block per RHS)
//   K_B  r^{k+1} = r^k - alpha (Q t + s0 p0)   (stencil; partial |r|^2), into a ring slot
//   K_b  beta, beta_j, freezing, and the block coefficients of every shift
//   K_C  p0 = r^{k+1} + beta p0
// The ring keeps the last m residuals.  Because the shift recurrences are
// linear, after m iterations (or when the RHS finishes) one pass applies
//   x_j += XP p_j + sum_i X_i r^{k0+i},   p_j = P p_j + sum_i C_i r^{k0+i}
// (or y += sum_j w_j (...) directly), so each shifted vector is read and
// written once per block instead of once per iteration.
#include <cmath>
#include <cstring>

#include "mscg.h"

namespace ovl {

__global__ void k_blk_reset(Blk *bk, const MState *st, int nrhs, int nshift)
{
    int r = blockIdx.x, j = threadIdx.x;
    if (r < nrhs && j < NS) {
        bk->P[r][j] = 1.0;
        bk->XP[r][j] = 0.0;
        for (int i = 0; i <= MB; i++) bk->C[r][j][i] = bk->X[r][j][i] = 0.0;
        bk->inblk[r][j] = (j < nshift) ? st->act[r][j] : 0;
        if (j == 0) bk->t[r] = 0;
    }
}

// beta, beta_j, freezing, and the block coefficients; RHS blockIdx.x
__global__ __launch_bounds__(kBlock) void k_blk_beta(MState *st, Blk *bk, const double *partials, int nblk)
{
    __shared__ double lds[4];
    const int r = blockIdx.x;
    if (st->skip[r]) return;
    double a = 0.0;
    for (int k = threadIdx.x; k < nblk; k += kBlock) a += partials[(size_t)r * nblk + k];
    double rr_new = block_sum(a, lds);
    if (threadIdx.x == 0) {
        int it = ++st->iter[r];
        if (!isfinite(rr_new)) {
            st->nonfinite[r] = 1;
            st->skip[r] = 1;
            return;
        }
        double beta = rr_new / st->rr[r];
        st->beta[r] = beta;
        const double thr = st->tol2 * st->bb[r];
        const int t = bk->t[r];
        int left = 0;
        for (int j = 0; j < st->nshift; j++) {
            if (!st->act_cur[r][j]) continue;
            double z = st->zeta[r][j], zn = st->zeta_new[r][j];
            double q = zn / z;
            double bj = beta * q * q;
            double aj = st->aj[r][j];
            // x += a p^{(t)};  p^{(t+1)} = zn r^{(t+1)} + bj p^{(t)}
            double P = bk->P[r][j];
            bk->XP[r][j] += aj * P;
            bk->P[r][j] = bj * P;
            for (int i = 1; i <= t; i++) {
                double c = bk->C[r][j][i];
                bk->X[r][j][i] += aj * c;
                bk->C[r][j][i] = bj * c;
            }
            bk->C[r][j][t + 1] = zn;
            st->bj[r][j] = bj;
            st->zeta_old[r][j] = z;
            st->zeta[r][j] = zn;
            if (zn * zn * rr_new <= thr) {
                st->act[r][j] = 0;
                st->frozen_at[r][j] = it;
            } else {
                left++;
            }
        }
        bk->t[r] = t + 1;
        st->rr[r] = rr_new;
        st->alpha_old[r] = st->alpha[r];
        if (!left) st->skip[r] = 1;
    }
}

// p0 = r_new + beta p0 on RHS that are still iterating
__global__ __launch_bounds__(kBlock) void k_base_p(Geom g, int nb, const MState *st, const double2 *rn, double2 *p0)
{
    const int r = blockIdx.y;
    if (st->skip[r]) return;
    const int b = blockIdx.x;
    const int p = b / nb, i = (b % nb) * kBlock + threadIdx.x;
    if (i >= g.Vh) return;
    const double be = st->beta[r];
    const size_t off = (size_t)r * 24 * g.S + (size_t)p * 12 * g.S + i;
#pragma unroll
    for (int c = 0; c < 12; c++) {
        double2 a = rn[off + (size_t)c * g.S];
        double2 q = p0[off + (size_t)c * g.S];
        p0[off + (size_t)c * g.S] = make_double2(fma(be, q.x, a.x), fma(be, q.y, a.y));
    }
}

struct RingPtrs {
    const double2 *slot[MB + 1];   // fields r^{k0+1..k0+T} of all RHS, slot[i] for r^{k0+i}
};

// The block pass.  y mode (xf == null): y_r += sum_j w_j dx_j; x mode: x_j += dx_j.
__global__ __launch_bounds__(kBlock) void k_blk_pass(Geom g, int nb, const MState *st, const Blk *bk, RingPtrs ring,
                                                     ShiftWeights w, double2 *pf, double2 *xf, double2 *y, int nrhs)
{
    __shared__ double sP[NS], sXP[NS], sW[NS];
    __shared__ double sC[NS][MB + 1], sX[NS][MB + 1];
    __shared__ int sj[NS], sact[NS];
    __shared__ int sn;
    const int r = blockIdx.y;
    const int T = bk->t[r];
    if (T == 0) return;
    if (threadIdx.x == 0) {
        int n = 0;
        for (int j = 0; j < st->nshift; j++)
            if (bk->inblk[r][j]) {
                sj[n] = j;
                sact[n] = st->act[r][j];
                sP[n] = bk->P[r][j];
                sXP[n] = bk->XP[r][j];
                sW[n] = w.w[j];
                n++;
            }
        sn = n;
    }
    __syncthreads();
    const int n = sn;
    for (int k = threadIdx.x; k < n * (MB + 1); k += kBlock) {
        int q = k / (MB + 1), i = k % (MB + 1);
        sC[q][i] = bk->C[r][sj[q]][i];
        sX[q][i] = bk->X[r][sj[q]][i];
    }
    __syncthreads();
    if (n == 0) return;
    const int b = blockIdx.x;
    const int p = b / nb, i = (b % nb) * kBlock + threadIdx.x;
    if (i >= g.Vh) return;
    const size_t site = (size_t)p * 12 * g.S + i;
    const size_t F = (size_t)24 * g.S;
    for (int c = 0; c < 12; c++) {
        const size_t off = site + (size_t)c * g.S;
        double2 rv[MB];
#pragma unroll
        for (int q = 0; q < MB; q++)
            if (q < T) rv[q] = ring.slot[q + 1][(size_t)r * F + off];
        double2 ya = make_double2(0.0, 0.0);
        for (int q = 0; q < n; q++) {
            const int j = sj[q];
            double2 *pp = pf + ((size_t)j * nrhs + r) * F + off;
            double2 pv = *pp;
            double2 dx = make_double2(sXP[q] * pv.x, sXP[q] * pv.y);
            double2 pn = make_double2(sP[q] * pv.x, sP[q] * pv.y);
#pragma unroll
            for (int t = 0; t < MB; t++)
                if (t < T) {
                    const double xc = sX[q][t + 1], cc = sC[q][t + 1];
                    dx.x = fma(xc, rv[t].x, dx.x);
                    dx.y = fma(xc, rv[t].y, dx.y);
                    pn.x = fma(cc, rv[t].x, pn.x);
                    pn.y = fma(cc, rv[t].y, pn.y);
                }
            if (sact[q]) *pp = pn;
            if (xf) {
                double2 *xp = xf + ((size_t)j * nrhs + r) * F + off;
                double2 xv = *xp;
                *xp = make_double2(xv.x + dx.x, xv.y + dx.y);
            } else {
                ya.x = fma(sW[q], dx.x, ya.x);
                ya.y = fma(sW[q], dx.y, ya.y);
            }
        }
        if (!xf) {
            double2 *yp = y + (size_t)r * F + off;
            double2 yv = *yp;
            *yp = make_double2(yv.x + ya.x, yv.y + ya.y);
        }
    }
}

// ring slot 0 = b, p0 = b, p_j = b, and y = 0 or x_j = 0
__global__ __launch_bounds__(kBlock) void k_blk_start(Geom g, int nb, const double2 *b, double2 *r0, double2 *p0, double2 *pf,
                                                      double2 *xf, double2 *y, int nrhs, int nshift)
{
    const int rr = blockIdx.y;
    const int bl = blockIdx.x;
    const int p = bl / nb, i = (bl % nb) * kBlock + threadIdx.x;
    if (i >= g.Vh) return;
    const size_t F = (size_t)24 * g.S;
    const size_t off = (size_t)rr * F + (size_t)p * 12 * g.S + i;
    const double2 z = make_double2(0.0, 0.0);
    for (int c = 0; c < 12; c++) {
        const size_t o = off + (size_t)c * g.S;
        double2 v = b[o];
        r0[o] = v;
        p0[o] = v;
        for (int j = 0; j < nshift; j++) {
            size_t oj = (size_t)j * nrhs * F + o;
            pf[oj] = v;
            if (xf) xf[oj] = z;
        }
        if (!xf) y[o] = z;
    }
}

int mscg_init_state(const Lat &L, MState *S, double *partials, double *red, Fld b, int nshift, const double *shifts,
                    const ovl_solver_params *prm, int *j0_out, hipStream_t st);

size_t blocked_ws_bytes(const Lat &L, int nrhs, int nshift, int m, bool keep_x)
{
    WsCarve c{nullptr, 0, 0};
    size_t F = field_bytes(P_F64, L.V);
    c.take(sizeof(MState));
    c.take(sizeof(Blk));
    c.take(sizeof(double) * 2 * nrhs * site_blocks(L));
    c.take(sizeof(double) * 4 * NR);
    c.take(F * nrhs * (m + 1));          // ring
    c.take(F * nrhs);                    // p0
    c.take(F * nrhs);                    // t
    c.take(F * nrhs * nshift);           // p_j
    if (keep_x) {
        c.take(F * nrhs * nshift);       // x_j
        c.take(F * nrhs);                // verification scratch
        c.take(F * nrhs);
    }
    return c.off + 256;
}

// Blocked FP64 multishift CG.  y mode (keep_x false): y (nrhs FP64 fields)
// receives sum_j w_j x_j.  x mode: the x_j stay in the workspace and are
// handed back through scr.
int mscg_blocked(const Lat &L, const void *U64, double m0, int nshift, const double *shifts, const double *weights,
                 Fld b, Fld yout, bool keep_x, int m, const ovl_solver_params *prm, ovl_solver_stats *stats,
                 char *ws, size_t ws_bytes, hipStream_t st, MsScratch *scr)
{
    const int R = b.nrhs;
    const int nblk = site_blocks(L);
    if (m < 1 || m > MB) return OVL_ERR_INVALID;
    WsCarve c{ws, 0, ws_bytes};
    const size_t F = field_bytes(P_F64, L.V);
    MState *S = (MState *)c.take(sizeof(MState));
    Blk *BK = (Blk *)c.take(sizeof(Blk));
    double *partials = (double *)c.take(sizeof(double) * 2 * R * nblk);
    double *red = (double *)c.take(sizeof(double) * 4 * NR);
    char *ring = (char *)c.take(F * R * (m + 1));
    Fld p0{c.take(F * R), nullptr, P_F64, R};
    Fld t{c.take(F * R), nullptr, P_F64, R};
    Fld pj{c.take(F * R * nshift), nullptr, P_F64, R * nshift};
    Fld xs{}, s1{}, s2{};
    if (keep_x) {
        xs = {c.take(F * R * nshift), nullptr, P_F64, R * nshift};
        s1 = {c.take(F * R), nullptr, P_F64, R};
        s2 = {c.take(F * R), nullptr, P_F64, R};
    }
    if (c.off > ws_bytes) return OVL_ERR_WORKSPACE;
    if (scr) *scr = MsScratch{partials, red, xs, s1, s2};
    Fld out = keep_x ? xs : yout;
    double2 *xf = keep_x ? (double2 *)out.d : nullptr;
    double2 *y = keep_x ? nullptr : (double2 *)out.d;
    auto slot = [&](long k) { return (double2 *)(ring + F * R * (size_t)(k % (m + 1))); };

    int j0 = 0;
    int rc = mscg_init_state(L, S, partials, red, b, nshift, shifts, prm, &j0, st);
    if (rc) return rc;
    dim3 sgrid(nblk, R);
    k_blk_start<<<sgrid, kBlock, 0, st>>>(L.g, L.nb, (const double2 *)b.d, slot(0), (double2 *)p0.d,
                                          (double2 *)pj.d, xf, y, R, nshift);
    k_blk_reset<<<R, NS, 0, st>>>(BK, S, R, nshift);
    OVL_HIP(hipGetLastError());
    ShiftWeights sw;
    for (int j = 0; j < NS; j++) sw.w[j] = (weights && j < nshift) ? weights[j] : 0.0;
    const double s0 = shifts[j0];

    WArgs A{};
    A.U = U64;
    A.diag = m0 + 4.0;
    A.partials = partials;
    A.skip = S->skip;
    A.nrhs = R;
    A.in = p0.d;
    A.out = t.d;
    WArgs B = A;
    B.in = t.d;
    B.p = p0.d;
    B.shift = s0;
    B.alpha = S->alpha;

    Prof prof;
    prof.on = prm->profile != 0 && stats;
    prof.st = st;
    long k = 0;
    int passes = 0;
    bool done = false;
    while (k < prm->maxiter && !done) {
        int batch = (int)std::min<long>(m, prm->maxiter - k);
        for (int q = 0; q < batch; q++, k++) {
            int e0 = prof.mark();
            OVL_HIP(launch_wilson(L, P_F64, W_NORM, true, A, st));
            int e1 = prof.mark();
            k_ms_alpha<<<R, kBlock, 0, st>>>(S, partials, nblk);
            int e2 = prof.mark();
            B.rin = slot(k);
            B.out = slot(k + 1);
            OVL_HIP(launch_wilson(L, P_F64, W_RUPDATE, true, B, st));
            int e3 = prof.mark();
            k_blk_beta<<<R, kBlock, 0, st>>>(S, BK, partials, nblk);
            int e4 = prof.mark();
            k_base_p<<<sgrid, kBlock, 0, st>>>(L.g, L.nb, S, slot(k + 1), (double2 *)p0.d);
            int e5 = prof.mark();
            OVL_HIP(hipGetLastError());
            prof.span(e0, e1, OVL_K_STENCIL);
            prof.span(e2, e3, OVL_K_STENCIL);
            prof.span(e1, e2, OVL_K_SCALAR);
            prof.span(e3, e4, OVL_K_SCALAR);
            prof.span(e4, e5, OVL_K_UPDATE);
        }
        // block pass over the residuals r^{k0+1..k0+T} (slots k0+1 .. k0+batch)
        RingPtrs rp;
        for (int i = 0; i <= MB; i++) rp.slot[i] = slot((k - batch + i + (m + 1)) % (m + 1));
        int e6 = prof.mark();
        k_blk_pass<<<sgrid, kBlock, 0, st>>>(L.g, L.nb, S, BK, rp, sw, (double2 *)pj.d, xf, y, R);
        int e7 = prof.mark();
        k_blk_reset<<<R, NS, 0, st>>>(BK, S, R, nshift);
        OVL_HIP(hipGetLastError());
        prof.span(e6, e7, OVL_K_UPDATE);
        passes++;
        int prc = prof.flush(stats);
        if (prc) return prc;
        int one[NR];
        OVL_HIP(hipMemcpyAsync(one, S->skip, sizeof(int) * NR, hipMemcpyDeviceToHost, st));
        OVL_HIP(hipStreamSynchronize(st));
        done = true;
        for (int q = 0; q < R; q++) done = done && one[q];
    }
    MState h;
    OVL_HIP(hipMemcpyAsync(&h, S, sizeof(MState), hipMemcpyDeviceToHost, st));
    OVL_HIP(hipStreamSynchronize(st));
    int status = OVL_OK;
    long iters_all = 0;
    for (int q = 0; q < R; q++) {
        if (h.nonfinite[q]) return OVL_ERR_NONFINITE;
        if (stats) stats->iterations[q] = h.iter[q];
        iters_all += h.iter[q];
        for (int j = 0; j < nshift; j++) {
            int fj = h.frozen_at[q][j] >= 0 ? h.frozen_at[q][j] : h.iter[q];
            if (stats) stats->shift_iters[q][j] = fj;
            if (h.frozen_at[q][j] < 0) status = OVL_NOT_CONVERGED;
        }
    }
    if (stats) {
        stats->stencil_applies += 2 * (int)k;
        // compulsory bytes: K_A 2F + links and K_B 4F + links per iteration,
        // K_C 3F; each pass reads the block's residuals once, and a shift
        // active up to iteration f takes part in ceil(f/m) passes, reading p_j
        // in each and writing it in all but the last (x mode also reads and
        // writes x_j each time); y mode reads and writes y once per pass.
        const double Fb = (double)F, G = (double)L.V * 4 * 96.0;
        double sten = iters_all * (6 * Fb + 2 * G);
        double upd = iters_all * 3 * Fb;
        double pass = iters_all * Fb + (keep_x ? 0.0 : 2.0 * passes * R * Fb);
        for (int q = 0; q < R; q++)
            for (int j = 0; j < nshift; j++) {
                int f = stats->shift_iters[q][j];
                int np = (f + m - 1) / m;
                if (np > 0) pass += (2.0 * np - 1.0) * Fb + (keep_x ? 2.0 * np * Fb : 0.0);
            }
        stats->kernel_bytes[OVL_K_STENCIL] += sten;
        stats->kernel_bytes[OVL_K_UPDATE] += upd + pass;
        stats->algorithmic_bytes += sten + upd + pass;
    }
    return status;
}

}  // namespace ovl
