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
#include <algorithm>
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

// beta, beta_j, freezing, and the block coefficients; RHS blockIdx.x, shift
// j in thread j.  sw2 > 0: an RHS with |r|^2 <= sw2 |b|^2 pauses (hand-over).
__global__ __launch_bounds__(kBlock) void k_blk_beta(MState *st, Blk *bk, const double *partials, int nblk,
                                                     int cnt, double sw2)
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
    const int t = bk->t[r];
    int live = 0;
    if (j < st->nshift && st->act_cur[r][j]) {
        const double z = st->zeta[r][j], zn = st->zeta_new[r][j];
        const double q = zn / z;
        const double bj = beta * q * q;
        const double aj = st->aj[r][j];
        // x += a p^{(t)};  p^{(t+1)} = zn r^{(t+1)} + bj p^{(t)}
        const double P = bk->P[r][j];
        bk->XP[r][j] += aj * P;
        bk->P[r][j] = bj * P;
        for (int i = 1; i <= t; i++) {
            const double c = bk->C[r][j][i];
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
            st->frozen_rr[r][j] = zn * zn * rr_new;
        } else {
            live = 1;
        }
    }
    // also the barrier between every thread's reads of rr, iter and t and
    // thread 0's writes below
    const int left = __syncthreads_count(live);
    if (j == 0) {
        st->iter[r] = it;
        st->beta[r] = beta;
        bk->t[r] = t + 1;
        st->rr[r] = rr_new;
        st->alpha_old[r] = st->alpha[r];
        st->run_c[r] = left ? 1 : 0;
        if (!left) {
            st->skip[r] = 1;
        } else if (sw2 > 0.0 && rr_new <= sw2 * st->bb[r]) {
            st->paused[r] = 1;
            st->skip[r] = 1;
        }
    }
}

// Element traits of the solver's vector fields: FP64 fields are arrays of
// complex128 (12 per site and parity), FP32 fields of float4 (two complex,
// 6 per site and parity), 48-bit fields hold two complex per element in two
// places (the top 32 bits of each real in one 16-byte array, the low 16 bits
// in half of another; see SpinorRef<P_F48>).  ld/st address element e of
// site (p, i) of a field set at field offset k (in 16-byte units); W is a
// field's size in 16-byte units per stride S, so field k of a set starts at element k*W*S; off gives the
// offset of element e of site (p, i) within a field.
template <int PS>
struct El;
template <>
struct El<P_F64> {
    using V = double2;
    static constexpr int N = 12;   // elements per site and parity
    static constexpr int C = 1;    // complex numbers per element
    static constexpr int W = 24;
    __device__ static void get(const V &v, double *re, double *im) { re[0] = v.x; im[0] = v.y; }
    __device__ static V put(const double *re, const double *im) { return make_double2(re[0], im[0]); }
    __device__ static V fresh(const V &v) { return v; }
    using O = size_t;
    __device__ static O off(int S, int p, int i, int e) { return (size_t)(p * N + e) * S + i; }
    __device__ static V ld(const void *f, size_t k, O o) { return ((const V *)f)[k + o]; }
    __device__ static void st(void *f, size_t k, O o, const V &v) { ((V *)f)[k + o] = v; }
    __device__ static V ldnt(const void *f, size_t k, O o)
    {
        nt_d2 t = __builtin_nontemporal_load((const nt_d2 *)f + k + o);
        return make_double2(t.x, t.y);
    }
};
struct V48 {
    uint4 h;   // top 32 bits: re, im of complex 2e, then of 2e+1
    uint2 l;   // low 16 bits: (re | im << 16) of complex 2e, 2e+1
};
typedef unsigned int nt_u2 __attribute__((ext_vector_type(2)));
template <>
struct El<P_F48> {
    using V = V48;
    static constexpr int N = 6;
    static constexpr int C = 2;
    static constexpr int W = 18;
    __device__ static void get(const V &v, double *re, double *im)
    {
        re[0] = f48_value(v.h.x, v.l.x & 0xffffu);
        im[0] = f48_value(v.h.y, v.l.x >> 16);
        re[1] = f48_value(v.h.z, v.l.y & 0xffffu);
        im[1] = f48_value(v.h.w, v.l.y >> 16);
    }
    __device__ static V put(const double *re, const double *im)
    {
        unsigned long long b[4] = {f48_bits(re[0]), f48_bits(im[0]), f48_bits(re[1]), f48_bits(im[1])};
        V v;
        v.h = make_uint4(f48_hi(b[0]), f48_hi(b[1]), f48_hi(b[2]), f48_hi(b[3]));
        v.l = make_uint2(f48_lo(b[0]) | (f48_lo(b[1]) << 16), f48_lo(b[2]) | (f48_lo(b[3]) << 16));
        return v;
    }
    // as El<P_F32>::fresh: the decoding of a value held across a loop stays
    // inside the loop
    __device__ static V fresh(const V &v)
    {
        V c = v;
        asm volatile("" : "+v"(c.h.x), "+v"(c.h.y), "+v"(c.h.z), "+v"(c.h.w), "+v"(c.l.x), "+v"(c.l.y));
        return c;
    }
    // 16-byte index of the top words, 8-byte index of the low words
    struct O {
        size_t h, l;
    };
    __device__ static O off(int S, int p, int i, int e)
    {
        return {(size_t)(p * 9 + e) * S + i, 2 * ((size_t)(p * 9 + 6 + e / 2) * S + i) + (e & 1)};
    }
    __device__ static V ld(const void *f, size_t k, O o)
    {
        V v;
        v.h = ((const uint4 *)f)[k + o.h];
        v.l = ((const uint2 *)f)[2 * k + o.l];
        return v;
    }
    __device__ static void st(void *f, size_t k, O o, const V &v)
    {
        ((uint4 *)f)[k + o.h] = v.h;
        ((uint2 *)f)[2 * k + o.l] = v.l;
    }
    __device__ static V ldnt(const void *f, size_t k, O o)
    {
        nt_u4 h = __builtin_nontemporal_load((const nt_u4 *)f + k + o.h);
        nt_u2 l = __builtin_nontemporal_load((const nt_u2 *)f + 2 * k + o.l);
        V v;
        v.h = make_uint4(h.x, h.y, h.z, h.w);
        v.l = make_uint2(l.x, l.y);
        return v;
    }
};
template <>
struct El<P_F32> {
    using V = float4;
    static constexpr int N = 6;
    static constexpr int C = 2;
    static constexpr int W = 12;
    __device__ static void get(const V &v, double *re, double *im)
    {
        re[0] = v.x; im[0] = v.y; re[1] = v.z; im[1] = v.w;
    }
    __device__ static V put(const double *re, const double *im)
    {
        return make_float4((float)re[0], (float)im[0], (float)re[1], (float)im[1]);
    }
    // A copy the compiler cannot see through (an empty asm statement), so
    // the widening of a value held across a loop stays inside the loop instead
    // of being hoisted, which would hold the value twice as wide in registers.
    __device__ static V fresh(const V &v)
    {
        V c = v;
        asm volatile("" : "+v"(c.x), "+v"(c.y), "+v"(c.z), "+v"(c.w));
        return c;
    }
    using O = size_t;
    __device__ static O off(int S, int p, int i, int e) { return (size_t)(p * N + e) * S + i; }
    __device__ static V ld(const void *f, size_t k, O o) { return ((const V *)f)[k + o]; }
    __device__ static void st(void *f, size_t k, O o, const V &v) { ((V *)f)[k + o] = v; }
    __device__ static V ldnt(const void *f, size_t k, O o)
    {
        nt_f4 t = __builtin_nontemporal_load((const nt_f4 *)f + k + o);
        return make_float4(t.x, t.y, t.z, t.w);
    }
};

// p0 = r_new + beta p0 on RHS that are still iterating or paused in this
// iteration (run_c).  Non-temporal loads: FP64 214 -> 194 us, FP32 89 -> 86 us
// at 32^3x64 (a non-temporal store as well made it slower).
template <int PS>
__global__ __launch_bounds__(kBlock) void k_base_p(Geom g, int nb, const MState *st, const void *rnv, void *p0v)
{
    using E = El<PS>;
    const int r = blockIdx.y;
    if (!st->run_c[r]) return;
    const int b = blockIdx.x;
    const int p = b / nb, i = (b % nb) * kBlock + threadIdx.x;
    if (i >= g.Vh) return;
    const double be = st->beta[r];
#pragma unroll
    for (int e = 0; e < E::N; e++) {
        double ar[E::C], ai[E::C], qr[E::C], qi[E::C];
        const typename E::O o = E::off(g.S, p, i, e);
        const size_t k = (size_t)r * E::W * g.S;
        E::get(E::ldnt(rnv, k, o), ar, ai);
        E::get(E::ldnt(p0v, k, o), qr, qi);
#pragma unroll
        for (int c = 0; c < E::C; c++) {
            qr[c] = fma(be, qr[c], ar[c]);
            qi[c] = fma(be, qi[c], ai[c]);
        }
        E::st(p0v, k, o, E::put(qr, qi));
    }
}

struct RingPtrs {
    const void *slot[MB + 1];   // fields r^{k0+1..k0+T} of all RHS, slot[i] for r^{k0+i}
};

// The block pass.  Sloppy fields (ring, p_j) in precision PS; x_j and y are
// FP64.  y mode (xf == null): y_r += sum_j w_j dx_j; x mode: x_j += dx_j.
// first: the first pass of a fresh solve, where every p_j still equals b
// (ring slot 0): it is read from there, and written for every shift of the
// block.  pin (FP32 passes): the first pass of a solve that continues FP64
// recurrences reads the p_j from the FP64 solve's fields (stored in FP64 or,
// PIN48, in 48 bits), rounded to FP32 as a conversion would round them.  xzero (x mode): the x_j of shifts
// j < xzero start at zero; the pass writes x_j = dx_j for the block's shifts
// and zeros for the others below xzero (for every one of an RHS with no
// iteration in the block).  The block's shifts all lie below xzero.
// The 48-bit 16-slot build is held to three waves per SIMD (its residuals
// take 6 registers a slot; left alone it takes 173 and two waves, 3.25 ms a
// pass at 32^3x64 against 2.94-3.02 ms at three waves with a 28-byte spill;
// the low words of the residuals kept in LDS instead fit 149 registers
// without spilling but took 3.11 ms).
template <int PS, int MBT, bool PIN48 = false>
__global__ __launch_bounds__(kBlock, PS == P_F48 && MBT <= 16 ? 3 : 1) void k_blk_pass(Geom g, int nb, const MState *st, const Blk *bk, RingPtrs ring,
                                                     ShiftWeights w, void *pfv, double2 *xf, double2 *y, int nrhs,
                                                     int first, const void *pin, int xzero)
{
    using E = El<PS>;
    using V = typename E::V;
    __shared__ double sP[NS], sXP[NS], sW[NS];
    __shared__ double sC[NS][MBT + 1], sX[NS][MBT + 1];
    __shared__ int sj[NS], sact[NS];
    __shared__ int sn;
    const int r = blockIdx.y;
    const int T = bk->t[r];
    const size_t F64 = (size_t)24 * g.S;               // FP64 field, in double2
    const int b = blockIdx.x;
    const int p = b / nb, i = (b % nb) * kBlock + threadIdx.x;
    const size_t site64 = (size_t)p * 12 * g.S + i;
    auto zero_x = [&](int j) {
        double2 *xp = xf + ((size_t)j * nrhs + r) * F64 + site64;
#pragma unroll
        for (int c = 0; c < 12; c++) xp[(size_t)c * g.S] = make_double2(0.0, 0.0);
    };
    const bool xz = xzero > 0 && xf;
    const int nzs = xzero < st->nshift ? xzero : st->nshift;
    if (T == 0) {
        if (xz && i < g.Vh)
            for (int j = 0; j < nzs; j++) zero_x(j);
        return;
    }
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
    for (int k = threadIdx.x; k < n * (MBT + 1); k += kBlock) {
        int q = k / (MBT + 1), i = k % (MBT + 1);
        sC[q][i] = bk->C[r][sj[q]][i];
        sX[q][i] = bk->X[r][sj[q]][i];
    }
    __syncthreads();
    if (i >= g.Vh) return;
    if (xz)
        for (int j = 0; j < nzs; j++)
            if (!bk->inblk[r][j]) zero_x(j);
    if (n == 0) return;
    const size_t FS = (size_t)E::W * g.S;   // sloppy field, in 16-byte units
    for (int e = 0; e < E::N; e++) {
        const typename E::O off = E::off(g.S, p, i, e);
        // the block's residuals stay in their storage precision in registers
        // (4 VGPRs per slot, 6 for 48-bit fields) and are widened where they
        // are used
        V rv[MBT];
#pragma unroll
        for (int q = 0; q < MBT; q++)
            if (q < T) rv[q] = E::ld(ring.slot[q + 1], (size_t)r * FS, off);
        V pb{};
        if (first) pb = E::ld(ring.slot[0], (size_t)r * FS, off);
        double yre[E::C], yim[E::C];
#pragma unroll
        for (int c = 0; c < E::C; c++) yre[c] = yim[c] = 0.0;
        // software pipeline over the shifts: the next shift's p_j (and x_j)
        // are loaded before this shift's results are stored, so a load is
        // always in flight while the previous shift computes
        auto pfield = [&](int q) { return ((size_t)sj[q] * nrhs + r) * FS; };
        auto xptr = [&](int q) {
            return xf + ((size_t)sj[q] * nrhs + r) * F64 + site64 + (size_t)(e * E::C) * g.S;
        };
        auto pload = [&](int q) -> V {
            if (PS == P_F32 && PIN48 && pin) {
                using E48 = El<P_F48>;
                double re[2], im[2];
                E48::get(E48::ld(pin, ((size_t)sj[q] * nrhs + r) * E48::W * g.S, E48::off(g.S, p, i, e)), re, im);
                return E::put(re, im);
            }
            if (PS == P_F32 && !PIN48 && pin) {
                const double2 *b64 = (const double2 *)pin + ((size_t)sj[q] * nrhs + r) * F64 + site64 + (size_t)(e * E::C) * g.S;
                double re[E::C], im[E::C];
#pragma unroll
                for (int c = 0; c < E::C; c++) {
                    const double2 v = b64[(size_t)c * g.S];
                    re[c] = v.x;
                    im[c] = v.y;
                }
                return E::put(re, im);
            }
            return E::ld(pfv, pfield(q), off);
        };
        V pcur = first ? pb : pload(0);
        double2 xcur[E::C];
        if (xf) {
#pragma unroll
            for (int c = 0; c < E::C; c++) xcur[c] = xz ? make_double2(0.0, 0.0) : xptr(0)[(size_t)c * g.S];
        }
        for (int q = 0; q < n; q++) {
            V pnext = pcur;
            double2 xnext[E::C];
            if (q + 1 < n) {
                if (!first) pnext = pload(q + 1);
                if (xf) {
#pragma unroll
                    for (int c = 0; c < E::C; c++)
                        xnext[c] = xz ? make_double2(0.0, 0.0) : xptr(q + 1)[(size_t)c * g.S];
                }
            }
            double pre[E::C], pim[E::C];
            E::get(pcur, pre, pim);
            double dxr[E::C], dxi[E::C], pnr[E::C], pni[E::C];
#pragma unroll
            for (int c = 0; c < E::C; c++) {
                dxr[c] = sXP[q] * pre[c];
                dxi[c] = sXP[q] * pim[c];
                pnr[c] = sP[q] * pre[c];
                pni[c] = sP[q] * pim[c];
            }
#pragma unroll
            for (int t = 0; t < MBT; t++)
                if (t < T) {
                    const double xc = sX[q][t + 1], cc = sC[q][t + 1];
                    double rre[E::C], rim[E::C];
                    E::get(E::fresh(rv[t]), rre, rim);
#pragma unroll
                    for (int c = 0; c < E::C; c++) {
                        dxr[c] = fma(xc, rre[c], dxr[c]);
                        dxi[c] = fma(xc, rim[c], dxi[c]);
                        pnr[c] = fma(cc, rre[c], pnr[c]);
                        pni[c] = fma(cc, rim[c], pni[c]);
                    }
                }
            if (sact[q] || first) E::st(pfv, pfield(q), off, E::put(pnr, pni));
            if (xf) {
                double2 *xp = xptr(q);
#pragma unroll
                for (int c = 0; c < E::C; c++)
                    xp[(size_t)c * g.S] = make_double2(xcur[c].x + dxr[c], xcur[c].y + dxi[c]);
#pragma unroll
                for (int c = 0; c < E::C; c++) xcur[c] = xnext[c];
            } else {
#pragma unroll
                for (int c = 0; c < E::C; c++) {
                    yre[c] = fma(sW[q], dxr[c], yre[c]);
                    yim[c] = fma(sW[q], dxi[c], yim[c]);
                }
            }
            pcur = pnext;
        }
        if (!xf) {
            double2 *yp = y + (size_t)r * F64 + site64 + (size_t)(e * E::C) * g.S;
#pragma unroll
            for (int c = 0; c < E::C; c++) {
                double2 yv = yp[(size_t)c * g.S];
                yp[(size_t)c * g.S] = make_double2(yv.x + yre[c], yv.y + yim[c]);
            }
        }
    }
}

// The block pass build for the block length (16 residuals in registers, or
// MB) and, in FP32, for the precision of the p_j of a continued FP64 solve.
template <int PS, typename... A>
static void launch_blk_pass(int m, bool pin48, dim3 grid, hipStream_t st, hipEvent_t e0, hipEvent_t e1, A... a)
{
    const dim3 b(kBlock);
    if constexpr (PS == P_F32) {
        if (pin48) {
            if (m <= 16) launch_k(k_blk_pass<PS, 16, true>, grid, b, st, e0, e1, a...);
            else launch_k(k_blk_pass<PS, MB, true>, grid, b, st, e0, e1, a...);
            return;
        }
    }
    if (m <= 16) launch_k(k_blk_pass<PS, 16>, grid, b, st, e0, e1, a...);
    else launch_k(k_blk_pass<PS, MB>, grid, b, st, e0, e1, a...);
}

// ring slot 0 = b, p0 = b (precision PS), and y = 0 or x_j = 0 (FP64).  The
// p_j (= b) are left to the first block pass, which reads b from slot 0;
// only an RHS that is finished from the start (b = 0) gets them here.
template <int PS>
__global__ __launch_bounds__(kBlock) void k_blk_start(Geom g, int nb, const MState *st, const double2 *b, void *r0v,
                                                      void *p0v, void *pfv, double2 *xf, double2 *y, int nrhs,
                                                      int nshift)
{
    using E = El<PS>;
    using V = typename E::V;
    const int rr = blockIdx.y;
    const int bl = blockIdx.x;
    const int p = bl / nb, i = (bl % nb) * kBlock + threadIdx.x;
    if (i >= g.Vh) return;
    const size_t F64 = (size_t)24 * g.S;
    const size_t off64 = (size_t)rr * F64 + (size_t)p * 12 * g.S + i;
    const double2 z = make_double2(0.0, 0.0);
    for (int e = 0; e < E::N; e++) {
        double re[E::C], im[E::C];
#pragma unroll
        for (int c = 0; c < E::C; c++) {
            double2 v = b[off64 + (size_t)(e * E::C + c) * g.S];
            re[c] = v.x;
            im[c] = v.y;
        }
        V v = E::put(re, im);
        const typename E::O o = E::off(g.S, p, i, e);
        const size_t FS = (size_t)E::W * g.S;
        E::st(r0v, rr * FS, o, v);
        E::st(p0v, rr * FS, o, v);
        if (st->skip[rr])
            for (int j = 0; j < nshift; j++) E::st(pfv, ((size_t)j * nrhs + rr) * FS, o, v);
    }
    for (int c = 0; c < 12; c++) {
        const size_t o64 = off64 + (size_t)c * g.S;
        for (int j = 0; j < nshift; j++)
            if (xf) xf[(size_t)j * nrhs * F64 + o64] = z;
        if (!xf) y[o64] = z;
    }
}

// continuing switched recurrences: the next replacement is due once |r| has
// fallen by reliable_delta from the hand-over
__global__ void k_resume(MState *st, int nrhs)
{
    int r = threadIdx.x;
    if (r < nrhs) {
        st->rr_ref[r] = st->rr[r];
        if (st->paused[r]) {
            st->paused[r] = 0;
            st->skip[r] = 0;
        }
    }
}

// after a residual replacement: rr = rr_ref = |r_hi|^2 for RHS still iterating
__global__ void k_set_rr(MState *st, const double *rr, int nrhs)
{
    int r = threadIdx.x;
    if (r < nrhs && !st->skip[r]) {
        st->rr[r] = rr[r];
        st->rr_ref[r] = rr[r];
    }
}

size_t blocked_ws_bytes(const Lat &L, int nrhs, int nshift, int m, bool keep_x, int ps, bool ext_x)
{
    WsCarve c{nullptr, 0, 0};
    const size_t F = field_bytes(P_F64, L.V), FS = field_bytes(ps, L.V);
    c.take(sizeof(MState));
    c.take(sizeof(Blk));
    c.take(sizeof(double) * 2 * nrhs * site_blocks(L));
    c.take(sizeof(double) * 4 * NR);
    if (ps == P_F48) {
        // p_j first, then the ring, p0 and t, spanning at least nrhs*nshift
        // FP64 fields (MsScratch::xlend)
        c.take(FS * nrhs * nshift);
        c.take(std::max(FS * nrhs * (m + 3), F * nrhs * nshift));
    } else {
        c.take(FS * nrhs * (m + 1));     // ring
        c.take(FS * nrhs);               // p0
        c.take(FS * nrhs);               // t
        c.take(FS * nrhs * nshift);      // p_j
    }
    if (keep_x && !ext_x) c.take(F * nrhs * nshift);   // x_j
    if (keep_x || ps == P_F32) {
        c.take(F * nrhs);                // FP64 scratch (verification, residual replacement)
        c.take(F * nrhs);
    }
    return c.off + 256;
}

// Blocked multishift CG with sloppy vectors of precision PS (FP64 or FP32)
// and FP64 x_j / y.  y mode (!o.keep_x): y (nrhs FP64 fields) receives
// sum_j w_j x_j.  x mode: x_j go to o.x_ext if given, else to the workspace,
// and are handed back through scr.  With o.reliable the base residual is
// replaced by the FP64 true residual b - (Q^2 + s0) x_0 at block ends once
// |r| has dropped by prm->reliable_delta (needs x mode).
template <int PS>
int mscg_blocked_t(const Lat &L, const ovl_gauge *U, double m0, int nshift, const double *shifts,
                   const double *weights, Fld b, Fld yout, const BlkOpts &o, const ovl_solver_params *prm,
                   ovl_solver_stats *stats, char *ws, size_t ws_bytes, hipStream_t st, MsScratch *scr)
{
    const int R = b.nrhs;
    const int nblk = site_blocks(L);
    const int npart = stencil_partials(L, PS, R);   // slots the iteration stencils fill
    const int m = o.m;
    if (m < 1 || m > MB || R > NR) return OVL_ERR_INVALID;
    if (o.reliable && !o.keep_x) return OVL_ERR_INVALID;
    // 48-bit storage: y mode of a fresh solve on an unshifted base (the t
    // recurrence; neither p0 nor the base-direction update is needed)
    if (PS == P_F48 && (o.keep_x || o.resume || o.rhs_shift || *std::min_element(shifts, shifts + nshift) != 0.0))
        return OVL_ERR_INVALID;
    const void *Us = PS == P_F32 ? U->f32 : U->f64;
    if (!Us || !U->f64) return OVL_ERR_INVALID;
    WsCarve c{ws, 0, ws_bytes};
    const size_t F = field_bytes(P_F64, L.V), FS = field_bytes(PS, L.V);
    MState *S = (MState *)c.take(sizeof(MState));
    Blk *BK = (Blk *)c.take(sizeof(Blk));
    double *partials = (double *)c.take(sizeof(double) * 2 * R * nblk);
    double *red = (double *)c.take(sizeof(double) * 4 * NR);
    char *ring;
    Fld p0{nullptr, nullptr, PS, R}, t{nullptr, nullptr, PS, R}, pj{nullptr, nullptr, PS, R * nshift};
    void *xlend = nullptr;
    if (PS == P_F48) {
        pj.d = c.take(FS * R * nshift);
        xlend = c.take(std::max(FS * R * (m + 3), F * R * nshift));
        ring = (char *)xlend;
        p0.d = ring + FS * R * (m + 1);
        t.d = ring + FS * R * (m + 2);
    } else {
        ring = (char *)c.take(FS * R * (m + 1));
        p0.d = c.take(FS * R);
        t.d = c.take(FS * R);
        pj.d = c.take(FS * R * nshift);
    }
    Fld xs{}, s1{}, s2{};
    if (o.keep_x) xs = {o.x_ext.d ? o.x_ext.d : c.take(F * R * nshift), nullptr, P_F64, R * nshift};
    if (o.keep_x || PS == P_F32) {
        s1 = {c.take(F * R), nullptr, P_F64, R};
        s2 = {c.take(F * R), nullptr, P_F64, R};
    }
    if (c.off > ws_bytes) return OVL_ERR_WORKSPACE;
    if (scr) *scr = MsScratch{partials, red, xs, s1, s2};
    double2 *xf = o.keep_x ? (double2 *)xs.d : nullptr;
    double2 *y = o.keep_x ? nullptr : (double2 *)yout.d;
    auto slot = [&](long k) { return (void *)(ring + FS * R * (size_t)(k % (m + 1))); };

    int j0 = 0;
    int it0[NR] = {0};   // iterations done before this solve (a resumed solve)
    dim3 sgrid(nblk, R);
    static thread_local MState h;
    if (o.resume) {
        // continue the recurrences of a switched solve: same scalars, the
        // vectors r, p0 and p_j rounded to this precision, x_j kept
        const MsScratch &rs = *o.resume;
        if (!o.keep_x || rs.r.nrhs != R || rs.pj.nrhs != R * nshift || (rs.pj.prec != P_F64 && rs.pj.prec != P_F48))
            return OVL_ERR_INVALID;
        j0 = rs.j0;
        OVL_HIP(hipMemcpyAsync(S, rs.S, sizeof(MState), hipMemcpyDeviceToDevice, st));
        OVL_HIP(launch_convert(L, rs.r, Fld{slot(0), nullptr, PS, R}, st));
        OVL_HIP(launch_convert(L, rs.p0, p0, st));
        // an FP32 solve's first pass reads the p_j from rs.pj
        if (PS != P_F32) OVL_HIP(launch_convert(L, rs.pj, pj, st));
        k_resume<<<1, 64, 0, st>>>(S, R);
        OVL_HIP(hipGetLastError());
        if (rs.host) {
            // the caller's copy has what the host needs (no wait for the GPU)
            h = *rs.host;
        } else {
            OVL_HIP(hipMemcpyAsync(&h, S, sizeof(MState), hipMemcpyDeviceToHost, st));
            OVL_HIP(hipStreamSynchronize(st));
        }
        for (int q = 0; q < R; q++) it0[q] = h.iter[q];
    } else {
        int rc = mscg_init_state(L, S, partials, red, b, nshift, shifts, prm, &j0, st, o.rhs_shift, o.rhs_tol);
        if (rc) return rc;
        k_blk_start<PS><<<sgrid, kBlock, 0, st>>>(L.g, L.nb, S, (const double2 *)b.d, slot(0), p0.d, pj.d, xf, y, R,
                                                  nshift);
    }
    k_blk_reset<<<R, NS, 0, st>>>(BK, S, R, nshift);
    OVL_HIP(hipGetLastError());
    // an unshifted base system (every RHS's base shift exactly 0) needs no
    // s0 p0 term in the residual update, so that stencil does not read p0
    const int rmode = !o.rhs_shift && shifts[j0] == 0.0 ? W_RUPDATE0 : W_RUPDATE;
    // With that base in FP64, p0 is read by nothing but the next t = Q p0, so
    // t follows its own recurrence t_k = Q r_k + beta_{k-1} t_{k-1} (Q is
    // linear) from the stored residual, in place, and p0 is never formed: the
    // base system's own shift vector p_j0, which the block passes keep and
    // which equals p0 (zeta = 1, the same alpha and beta), serves whoever needs
    // p0 afterwards (the hand-over to the FP32 phase).  The recurrence adds
    // rounding at each step, of the order of the steps since t was last formed
    // directly times eps relative to t: FP64 forms t directly once, FP32 at
    // every block start from p_j0, which the block pass has just brought to
    // the current iteration.
    // (not in the FP16-storage measurement mode, whose subject is the stored p0
    // and Q p0)
    const bool trec = rmode == W_RUPDATE0 && (PS == P_F64 || PS == P_F48 || (PS == P_F32 && !o.f16.d));
    const Fld pj0 = sub(pj, L.V, j0 * R, R);
    ShiftWeights sw;
    for (int j = 0; j < NS; j++) sw.w[j] = (weights && j < nshift) ? weights[j] : 0.0;

    WArgs A{};
    A.U = Us;
    A.diag = m0 + 4.0;
    A.partials = partials;
    A.skip = S->skip;
    A.nrhs = R;
    A.in = p0.d;
    A.out = t.d;
    WArgs B = A;
    B.in = t.d;
    B.p = p0.d;
    B.shiftv = S->s0r;
    B.alpha = S->alpha;

    Prof prof;
    prof.on = prm->profile != 0 && stats;
    prof.stencil_only = prm->profile == 2;
    prof.st = st;
    long k = 0;
    int passes = 0, replacements = 0;
    bool done = false, switched = false;
    const double rd2 = prm->reliable_delta * prm->reliable_delta;
    const double sw2 = o.switch_rel * o.switch_rel;
    long it_left = prm->maxiter;
    for (int q = 0; q < R; q++) it_left = std::min<long>(it_left, prm->maxiter - it0[q]);
    // the next block's length (below); |r|^2 at the last block end
    int next_batch = m;
    double rr_prev[NR];
    bool rr_known = false;
    if (o.resume) {
        for (int q = 0; q < R; q++) rr_prev[q] = h.rr[q];
        rr_known = true;
    }
    while (k < it_left && !done && !switched) {
        int batch = (int)std::min<long>(next_batch, it_left - k);
        // FP16 storage of the Krylov vectors (measurement mode): each new
        // vector is rounded through the FP16S set and back after its kernel
        const bool f16 = PS == P_F32 && o.f16.d;
        auto round16 = [&](void *d) -> hipError_t {
            const Fld f{d, nullptr, P_F32, R};
            hipError_t h = launch_convert(L, f, o.f16, st);
            return h == hipSuccess ? launch_convert(L, o.f16, f, st) : h;
        };
        // each timed kernel records its own start and end (prof.pair)
        hipEvent_t v0, v1;
        for (int q = 0; q < batch; q++, k++) {
            prof.pair(OVL_K_STENCIL, &v0, &v1);
            if (trec && k > 0 && !(PS == P_F32 && q == 0)) {
                // t = Q r_k + beta t (in place; beta of the previous iteration)
                WArgs At = A;
                At.in = slot(k);
                At.p = t.d;
                At.shiftv = S->beta;
                OVL_HIP(launch_wilson(L, PS, W_SNORM, true, At, st, v0, v1));
            } else if (trec) {
                // t = Q p0 directly: p0 = r0 at the start of a fresh solve, the
                // handed-over p0 at the start of a resumed one, p_j0 at a block start
                WArgs At = A;
                if (k > 0) At.in = pj0.d;
                else if (!o.resume) At.in = slot(0);
                OVL_HIP(launch_wilson(L, PS, W_NORM, true, At, st, v0, v1));
            } else {
                OVL_HIP(launch_wilson(L, PS, W_NORM, true, A, st, v0, v1));
            }
            if (f16) OVL_HIP(round16(t.d));
            prof.pair(OVL_K_SCALAR, &v0, &v1);
            launch_k(k_ms_alpha, dim3(R), dim3(kBlock), st, v0, v1, S, (const double *)partials, nblk, npart);
            B.rin = slot(k);
            B.out = slot(k + 1);
            prof.pair(OVL_K_STENCIL, &v0, &v1);
            OVL_HIP(launch_wilson(L, PS, rmode, true, B, st, v0, v1));
            if (f16) OVL_HIP(round16(slot(k + 1)));
            prof.pair(OVL_K_SCALAR, &v0, &v1);
            launch_k(k_blk_beta, dim3(R), dim3(kBlock), st, v0, v1, S, BK, (const double *)partials, nblk, npart, sw2);
            if (!trec) {
                prof.pair(OVL_K_UPDATE, &v0, &v1);
                launch_k(k_base_p<PS>, sgrid, dim3(kBlock), st, v0, v1, L.g, L.nb, (const MState *)S,
                         (const void *)slot(k + 1), p0.d);
            }
            if (f16) OVL_HIP(round16(p0.d));
            OVL_HIP(hipGetLastError());
            // the previous block's times, read while this iteration runs
            if (q == 0) {
                int prc = prof.collect(stats);
                if (prc) return prc;
            }
        }
        // block pass over the residuals r^{k0+1..k0+T} (slots k0+1 .. k0+batch)
        RingPtrs rp;
        for (int i = 0; i <= MB; i++) rp.slot[i] = slot((k - batch + i + (m + 1)) % (m + 1));
        // blocks of up to 16 take the build that holds 16 residuals in
        // registers (more waves per SIMD)
        const int first = !o.resume && passes == 0;
        const void *pin = PS == P_F32 && o.resume && passes == 0 ? o.resume->pj.d : nullptr;
        const bool pin48 = pin && o.resume->pj.prec == P_F48;
        const int xzero = passes == 0 ? o.x_zero_shifts : 0;
        prof.pair(OVL_K_UPDATE, &v0, &v1);
        launch_blk_pass<PS>(m, pin48, sgrid, st, v0, v1, L.g, L.nb, (const MState *)S, (const Blk *)BK, rp, sw, pj.d,
                            xf, y, R, first, pin, xzero);
        k_blk_reset<<<R, NS, 0, st>>>(BK, S, R, nshift);
        OVL_HIP(hipGetLastError());
        passes++;
        OVL_HIP(hipMemcpyAsync(&h, S, sizeof(MState), hipMemcpyDeviceToHost, st));
        OVL_HIP(hipStreamSynchronize(st));
        // an RHS is finished (skip without pause), paused at the hand-over
        // level (k_blk_beta stops it at the iteration it gets there) or open;
        // the hand-over comes once no RHS is open
        done = true;
        bool want = false;
        switched = sw2 > 0.0;
        for (int q = 0; q < R; q++) {
            const bool fin = h.skip[q] && !h.paused[q];
            done = done && fin;
            if (!h.skip[q] && h.rr[q] < rd2 * h.rr_ref[q]) want = true;
            if (!fin && !h.paused[q]) switched = false;
        }
        switched = switched && !done;
        // The next block's length: the iterations the slowest system still
        // needs (the base, which freezes last, or the hand-over level),
        // predicted from the fall of |r| over this block with a quarter and
        // two iterations to spare.  Launches past an RHS's end exit at once
        // but still cost a launch and a gap each; a block cut short costs
        // one more block pass.
        next_batch = m;
        if (rr_known) {
            int need = 0;
            bool ok = true;
            for (int q = 0; q < R && ok; q++) {
                if (h.skip[q]) continue;
                const double target = std::max(h.tol2r[q], sw2) * h.bb[q];
                const double r0 = rr_prev[q], r1 = h.rr[q];
                if (!(r1 > target)) {
                    need = std::max(need, 2);
                    continue;
                }
                if (!(r1 > 0.0 && r0 > r1)) {
                    ok = false;
                    break;
                }
                const double per = std::log(r1 / r0) / batch;
                need = std::max(need, (int)std::ceil(1.25 * std::log(target / r1) / per) + 2);
            }
            if (ok && need > 0) next_batch = std::min(m, need);
        }
        for (int q = 0; q < R; q++) rr_prev[q] = h.rr[q];
        rr_known = true;
        if (o.reliable && want && !done && !switched) {
            // residual replacement: r = b - (Q^2 + s0) x_0 in FP64: s1 = Q x0,
            // then the residual-update stencil r = b - 1 * (Q s1 + s0 x0) with
            // its partials of |r|^2 (the unshifted base reads no x0)
            int e8 = prof.mark();
            Fld x0 = sub(xs, L.V, j0 * R, R);
            WArgs Q1{};
            Q1.U = U->f64;
            Q1.diag = m0 + 4.0;
            Q1.nrhs = R;
            Q1.in = x0.d;
            Q1.out = s1.d;
            Q1.skip = S->skip;
            OVL_HIP(launch_wilson(L, P_F64, W_PLAIN, true, Q1, st));
            WArgs Q2 = Q1;
            Q2.in = s1.d;
            Q2.p = x0.d;
            Q2.shiftv = S->s0r;
            Q2.rin = b.d;
            Q2.out = s2.d;
            Q2.alpha = S->one;
            Q2.partials = partials;
            OVL_HIP(launch_wilson(L, P_F64, rmode, true, Q2, st));
            OVL_HIP(launch_reduce(partials, 1, R, nblk, red, st));
            Fld cur{slot(k), nullptr, PS, R};
            OVL_HIP(launch_convert(L, s2, cur, st));
            k_set_rr<<<1, 64, 0, st>>>(S, red, R);
            OVL_HIP(hipGetLastError());
            int e9 = prof.mark();
            prof.span(e8, e9, OVL_K_OTHER);
            replacements++;
        }
        int prc = prof.rotate(stats);
        if (prc) return prc;
    }
    {
        int prc = prof.flush(stats);
        if (prc) return prc;
    }
    OVL_HIP(hipMemcpyAsync(&h, S, sizeof(MState), hipMemcpyDeviceToHost, st));
    OVL_HIP(hipStreamSynchronize(st));
    int status = switched ? kSwitched : OVL_OK;
    long iters_all = 0;
    int fz[NR][NS];   // iterations of this solve in which shift j took part
    for (int q = 0; q < R; q++) {
        if (h.nonfinite[q]) return OVL_ERR_NONFINITE;
        if (stats && !o.quiet) stats->iterations[q] = h.iter[q];
        iters_all += h.iter[q] - it0[q];
        for (int j = 0; j < nshift; j++) {
            const int f = h.frozen_at[q][j] >= 0 ? h.frozen_at[q][j] : h.iter[q];
            fz[q][j] = std::max(0, f - it0[q]);
            if (stats && !o.quiet) stats->shift_iters[q][j] = f;
            if (h.frozen_at[q][j] < 0 && !switched) status = OVL_NOT_CONVERGED;
        }
    }
    if (o.iters_out)
        for (int q = 0; q < R; q++) o.iters_out[q] = h.iter[q] - it0[q];
    if (scr && switched) {
        // RHS q stopped after it_q iterations of this solve, so its residual
        // is in ring slot it_q; gather every RHS's residual into slot k
        for (int q = 0; q < R; q++) {
            const long kq = h.iter[q] - it0[q];
            if (kq >= 0 && kq % (m + 1) != k % (m + 1))
                OVL_HIP(hipMemcpyAsync((char *)slot(k) + FS * q, (const char *)slot(kq) + FS * q, FS,
                                       hipMemcpyDeviceToDevice, st));
        }
        scr->S = S;
        scr->r = Fld{slot(k), nullptr, PS, R};
        // with the t recurrence p0 was never formed: p_j0 equals it
        scr->p0 = trec ? pj0 : p0;
        scr->pj = pj;
        scr->j0 = j0;
        scr->xlend = xlend;
    }
    if (stats) {
        stats->stencil_applies += 2 * (int)k + 2 * replacements;
        stats->reliable_updates += replacements;
        // compulsory bytes: K_A 2F + links and K_B 4F + links per iteration
        // (3F + links with an unshifted base, which does not read p0), K_C 3F;
        // each pass reads the block's residuals once, and a shift
        // active up to iteration f takes part in ceil(f/m) passes, reading p_j
        // in each and writing it in all but the last (x mode also reads and
        // writes the FP64 x_j each time); y mode reads and writes y once per pass.
        // A fresh solve's first pass reads b once per RHS in place of the p_j
        // and writes every p_j.
        const double Fs = (double)FS, F8 = (double)F;
        const double G = (double)L.V * 4 * (PS == P_F32 ? 48.0 : 96.0);
        const bool fresh = !o.resume;
        // (with the t recurrence: K_A 3F + links, K_B 3F + links, no K_C)
        double sten = iters_all * ((rmode == W_RUPDATE0 && !trec ? 5 : 6) * Fs + 2 * G);
        double upd = trec ? 0.0 : iters_all * 3 * Fs;
        double pass = iters_all * Fs + (o.keep_x ? 0.0 : 2.0 * passes * R * F8) + (fresh && passes ? R * Fs : 0.0);
        for (int q = 0; q < R; q++)
            for (int j = 0; j < nshift; j++) {
                int np = (fz[q][j] + m - 1) / m;
                double pj_io = fresh ? (np >= 2 ? 2.0 * np - 2.0 : 1.0) : 2.0 * np - 1.0;
                // an FP32 solve's first pass reads the FP64 (or 48-bit) p_j it continues
                const double wide =
                    !fresh && PS == P_F32 ? (double)field_bytes(o.resume->pj.prec, L.V) - Fs : 0.0;
                if (np > 0) pass += pj_io * Fs + wide + (o.keep_x ? 2.0 * np * F8 : 0.0);
            }
        // replacement: Q x0 (768 B per site), the update stencil, the rounding into the ring
        double other = replacements * R * ((768.0 + (rmode == W_RUPDATE0 ? 960.0 : 1152.0)) * L.V + F8 + Fs);
        stats->kernel_bytes[OVL_K_STENCIL] += sten;
        stats->kernel_bytes[OVL_K_UPDATE] += upd + pass;
        stats->kernel_bytes[OVL_K_OTHER] += other;
        stats->algorithmic_bytes += sten + upd + pass + other;
    }
    return status;
}

template int mscg_blocked_t<P_F64>(const Lat &, const ovl_gauge *, double, int, const double *, const double *, Fld,
                                   Fld, const BlkOpts &, const ovl_solver_params *, ovl_solver_stats *, char *, size_t,
                                   hipStream_t, MsScratch *);
template int mscg_blocked_t<P_F48>(const Lat &, const ovl_gauge *, double, int, const double *, const double *, Fld,
                                   Fld, const BlkOpts &, const ovl_solver_params *, ovl_solver_stats *, char *, size_t,
                                   hipStream_t, MsScratch *);
template int mscg_blocked_t<P_F32>(const Lat &, const ovl_gauge *, double, int, const double *, const double *, Fld,
                                   Fld, const BlkOpts &, const ovl_solver_params *, ovl_solver_stats *, char *, size_t,
                                   hipStream_t, MsScratch *);

}  // namespace ovl
