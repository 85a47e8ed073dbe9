// sign(Q) b by a Krylov subspace method instead of a rational function: the
// Lanczos approximation |b| V_k sign(T_k) e_1 on the Krylov space of the
// Hermitian Q = Gamma_5 D_W (the paper's "sign function iteration" approximates
// sign(Gamma_5 D_W) chi by a Krylov method, Section 5; it restarts with thick
// restarts to bound memory).  Here memory is bounded by two passes instead:
//   pass 1: Lanczos on Q from v_1 = b/|b|, keeping only the coefficients
//           alpha_k, beta_k (on the device); every kCheck steps the host forms
//           c_k = |b| sign(T_k) e_1 from an eigen-decomposition of T_k and an
//           RHS stops once |c_k - c_{k-kCheck}| <= tol |b|;
//   pass 2: the same recurrence regenerates v_1..v_m from the stored
//           coefficients (one fused update-and-scale kernel per step),
//           accumulating y = sum_k c_k v_k.
// Four FP64 fields per RHS, twice the stencils of one pass.  Each RHS of a
// batch has its own coefficients; the passes run in step for all of them.
#include <cmath>
#include <cstddef>
#include <cstring>
#include <vector>

#include "mscg.h"
#include "tridiag.h"

namespace ovl {

constexpr int kLzMax = 4096;   // longest Lanczos sequence
constexpr int kCheck = 32;     // steps between convergence checks

// per-RHS Lanczos coefficients on the device: a[k][r], b[k][r] (b the norm
// of the unnormalised next vector), and the pass-2 weights c[k][r]
struct LzCoef {
    double a[kLzMax][NR], b[kLzMax][NR];
};

// w = t - a_k v_k - b_{k-1} v_{k-1} into v_prev's field, partial |w|^2 per
// RHS; in pass 2 (c != null) also y += c_k v_k, and w is stored already
// divided by the known b_k (the next basis vector; no separate scaling
// pass).  a_k comes from the reduced dot ar (pass 1) or the stored
// coefficients (pass 2).
__global__ __launch_bounds__(kBlock) void k_lz_update(Geom g, int nb, int nrhs, const double2 *t, const double2 *vk,
                                                       double2 *vprev, const LzCoef *cf, int k, const double *ar,
                                                       const double *c, double2 *y, double *partials)
{
    __shared__ double lds[8];
    const int r = blockIdx.y, bl = blockIdx.x;
    const int p = bl / nb, i = (bl % nb) * kBlock + threadIdx.x;
    const double a = ar ? ar[r] : cf->a[k][r];
    const double bprev = k > 0 ? cf->b[k - 1][r] : 0.0;
    double n2 = 0.0;
    if (i < g.Vh) {
        cplx<double> tv[4][3], v[4][3], u[4][3];
        spinor_ref<P_F64>(t, nullptr, g.S, r).load(p, i, tv);
        spinor_ref<P_F64>(vk, nullptr, g.S, r).load(p, i, v);
        const auto VP = spinor_ref<P_F64>(vprev, nullptr, g.S, r);
        VP.load(p, i, u);
        const double bk = c ? cf->b[k][r] : 1.0;
        const double inv = bk > 0.0 ? 1.0 / bk : 0.0;
#pragma unroll
        for (int q = 0; q < 12; q++) {
            cplx<double> &w = tv[q / 3][q % 3];
            w = fmac(fmac(w, -a, v[q / 3][q % 3]), -bprev, u[q / 3][q % 3]);
            n2 += norm2(w);
            if (c) w = inv * w;
        }
        VP.store(p, i, tv);
        if (c) {
            const double ck = c[(size_t)k * NR + r];
            const auto Y = spinor_ref<P_F64>(y, nullptr, g.S, r);
            cplx<double> yv[4][3];
            Y.load(p, i, yv);
#pragma unroll
            for (int q = 0; q < 12; q++) yv[q / 3][q % 3] = fmac(yv[q / 3][q % 3], ck, v[q / 3][q % 3]);
            Y.store(p, i, yv);
        }
    }
    const double s = block_sum(n2, lds);
    if (threadIdx.x == 0 && partials) partials[(size_t)r * gridDim.x + bl] = s;
}

// pass 1: v_next = w / b_k (0 when b_k is 0) written over w's field, with
// b_k = |w| from the reduced norm; the first block also records a[k] (the
// reduced dot, real part) and b[k].  An RHS whose new vector vanishes (an
// invariant subspace) keeps b = 0.
__global__ __launch_bounds__(kBlock) void k_lz_scale(Geom g, int nb, double2 *w, LzCoef *cf, int k,
                                                      const double *dot, const double *nrm2)
{
    const int r = blockIdx.y, bl = blockIdx.x;
    const int p = bl / nb, i = (bl % nb) * kBlock + threadIdx.x;
    const double bk = sqrt(fmax(nrm2[r], 0.0));
    if (bl == 0 && threadIdx.x == 0) {
        cf->a[k][r] = dot[r];
        cf->b[k][r] = bk;
    }
    if (i >= g.Vh) return;
    const double inv = bk > 0.0 ? 1.0 / bk : 0.0;
    const auto W = spinor_ref<P_F64>(w, nullptr, g.S, r);
    cplx<double> v[4][3];
    W.load(p, i, v);
#pragma unroll
    for (int q = 0; q < 12; q++) v[q / 3][q % 3] = inv * v[q / 3][q % 3];
    W.store(p, i, v);
}

size_t lanczos_sign_ws_bytes(const Lat &L, int nrhs)
{
    WsCarve c{nullptr, 0, 0};
    const size_t F = field_bytes(P_F64, L.V);
    c.take(3 * F * nrhs);                                  // v_prev, v_k, t
    c.take(sizeof(LzCoef));
    c.take(sizeof(double) * (size_t)kLzMax * NR);          // pass-2 weights
    c.take(sizeof(double) * 2 * NR * site_blocks(L));
    c.take(sizeof(double) * 4 * NR);
    return c.off + 256;
}

// y = sign(Q) b for the nrhs fields of b (FP64); iters[q] the Lanczos steps
// of RHS q.  tol: relative change of the coefficient vector between checks.
int lanczos_sign(const Lat &L, const void *U64, double m0, Fld b, Fld y, double tol, int maxiter, int *iters,
                 char *ws, size_t ws_bytes, hipStream_t st)
{
    const int R = b.nrhs;
    if (ws_bytes < lanczos_sign_ws_bytes(L, R)) return OVL_ERR_WORKSPACE;
    const int kmax = std::min(maxiter, kLzMax - 1);
    WsCarve c{ws, 0, ws_bytes};
    const size_t F = field_bytes(P_F64, L.V);
    char *f3 = (char *)c.take(3 * F * R);
    Fld va{f3, nullptr, P_F64, R}, vb{f3 + F * R, nullptr, P_F64, R}, t{f3 + 2 * F * R, nullptr, P_F64, R};
    LzCoef *cf = (LzCoef *)c.take(sizeof(LzCoef));
    double *cw = (double *)c.take(sizeof(double) * (size_t)kLzMax * NR);
    double *partials = (double *)c.take(sizeof(double) * 2 * NR * site_blocks(L));
    double *red = (double *)c.take(sizeof(double) * 4 * NR);
    const int nblk = site_blocks(L);
    dim3 grid(nblk, R);
    // |b| per RHS
    std::vector<double> bn(R);
    {
        OVL_HIP(launch_norm2(L, b, partials, st));
        OVL_HIP(launch_reduce(partials, 1, R, nblk, red, st));
        OVL_HIP(hipMemcpyAsync(bn.data(), red, sizeof(double) * R, hipMemcpyDeviceToHost, st));
        OVL_HIP(hipStreamSynchronize(st));
        for (int q = 0; q < R; q++) {
            if (!std::isfinite(bn[q])) return OVL_ERR_NONFINITE;
            bn[q] = std::sqrt(bn[q]);
        }
    }
    WArgs A{};
    A.U = U64;
    A.diag = m0 + 4.0;
    A.nrhs = R;
    // start: v_prev = 0, v_1 = b / |b| (an all-zero b gives y = 0)
    auto start = [&]() -> int {
        OVL_HIP(launch_zero(L, va, st));
        for (int q = 0; q < R; q++)
            OVL_HIP(launch_axpby(L, bn[q] > 0 ? 1.0 / bn[q] : 0.0, sub(b, L.V, q, 1), 0.0, sub(vb, L.V, q, 1), st));
        return OVL_OK;
    };
    // one step: t = Q v_k, w = t - a_k v_k - b_{k-1} v_{k-1} into v_prev's
    // field, then v_{k+1} = w / b_k; the roles of the two fields swap
    Fld vprev = va, vk = vb;
    std::vector<int> mq(R, 0);          // steps of each RHS (0: not converged yet)
    std::vector<std::vector<double>> cprev(R), cbest(R);
    std::vector<double> ha((size_t)(kmax + 1) * NR), hb((size_t)(kmax + 1) * NR);
    int rc = start();
    if (rc) return rc;
    int k = 0;
    bool all = false;
    for (int q = 0; q < R; q++)
        if (!(bn[q] > 0)) mq[q] = -1;   // nothing to do
    while (!all && k < kmax) {
        A.in = vk.d;
        A.out = t.d;
        OVL_HIP(launch_wilson(L, P_F64, W_PLAIN, true, A, st));
        OVL_HIP(launch_dot(L, vk, t, partials, st));
        OVL_HIP(launch_reduce(partials, 1, R, nblk, red, st));   // real parts
        k_lz_update<<<grid, kBlock, 0, st>>>(L.g, L.nb, R, (const double2 *)t.d, (const double2 *)vk.d,
                                             (double2 *)vprev.d, cf, k, red, nullptr, nullptr, partials);
        OVL_HIP(hipGetLastError());
        OVL_HIP(launch_reduce(partials, 1, R, nblk, red + NR, st));
        k_lz_scale<<<grid, kBlock, 0, st>>>(L.g, L.nb, (double2 *)vprev.d, cf, k, red, red + NR);
        OVL_HIP(hipGetLastError());
        std::swap(vprev, vk);
        k++;
        if (k % kCheck == 0 || k == kmax) {
            // device addresses of the coefficient arrays (no host access to cf)
            const double *da = (const double *)((const char *)cf + offsetof(LzCoef, a));
            const double *db = (const double *)((const char *)cf + offsetof(LzCoef, b));
            OVL_HIP(hipMemcpyAsync(ha.data(), da, sizeof(double) * NR * k, hipMemcpyDeviceToHost, st));
            OVL_HIP(hipMemcpyAsync(hb.data(), db, sizeof(double) * NR * k, hipMemcpyDeviceToHost, st));
            OVL_HIP(hipStreamSynchronize(st));
            all = true;
            for (int q = 0; q < R; q++) {
                if (mq[q] != 0) continue;
                std::vector<double> a(k), bt(k);
                bool brk = false;
                int kk = k;
                for (int j = 0; j < k; j++) {
                    a[j] = ha[(size_t)j * NR + q];
                    bt[j] = hb[(size_t)j * NR + q];
                    if (!std::isfinite(a[j]) || !std::isfinite(bt[j])) return OVL_ERR_NONFINITE;
                    if (bt[j] <= 1e-14 * std::fabs(a[j]) + 1e-300) {   // invariant subspace: exact
                        kk = j + 1;
                        brk = true;
                        break;
                    }
                }
                std::vector<double> cq;
                if (!tridiag_sign_e1(kk, a.data(), bt.data(), bn[q], cq)) return OVL_ERR_NONFINITE;
                double diff = 0.0;
                for (int j = 0; j < kk; j++) {
                    const double o = j < (int)cprev[q].size() ? cprev[q][j] : 0.0;
                    diff += (cq[j] - o) * (cq[j] - o);
                }
                if (brk || std::sqrt(diff) <= tol * bn[q]) {
                    mq[q] = kk;
                    cbest[q] = cq;
                } else {
                    all = false;
                    cprev[q] = cq;
                }
            }
        }
    }
    int status = OVL_OK;
    int kmx = 0;
    for (int q = 0; q < R; q++) {
        if (mq[q] == 0) {   // maxiter: use the last coefficients
            status = OVL_NOT_CONVERGED;
            mq[q] = (int)cprev[q].size();
            cbest[q] = cprev[q];
        }
        if (mq[q] < 0) mq[q] = 0;
        kmx = std::max(kmx, mq[q]);
        if (iters) iters[q] = mq[q];
    }
    // pass 2: the weights c_k per RHS (0 beyond its own steps), then the same
    // recurrence from the stored coefficients with y += c_k v_k
    std::vector<double> hc((size_t)std::max(kmx, 1) * NR, 0.0);
    for (int q = 0; q < R; q++)
        for (int j = 0; j < mq[q]; j++) hc[(size_t)j * NR + q] = cbest[q][j];
    OVL_HIP(hipMemcpyAsync(cw, hc.data(), sizeof(double) * hc.size(), hipMemcpyHostToDevice, st));
    OVL_HIP(launch_zero(L, y, st));
    rc = start();
    if (rc) return rc;
    vprev = va;
    vk = vb;
    for (int j = 0; j < kmx; j++) {
        A.in = vk.d;
        A.out = t.d;
        OVL_HIP(launch_wilson(L, P_F64, W_PLAIN, true, A, st));
        k_lz_update<<<grid, kBlock, 0, st>>>(L.g, L.nb, R, (const double2 *)t.d, (const double2 *)vk.d,
                                             (double2 *)vprev.d, cf, j, nullptr, cw, (double2 *)y.d, nullptr);
        OVL_HIP(hipGetLastError());
        std::swap(vprev, vk);
    }
    OVL_HIP(hipStreamSynchronize(st));
    return status;
}

}  // namespace ovl
