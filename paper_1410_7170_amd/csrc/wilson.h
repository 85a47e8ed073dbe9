// Wilson-Dirac hopping stencil on the even-odd layout (gfx950).
//
// Implements eq. (Wilson-Dirac) of Brannick et al. (arXiv:1410.7170), a = 1:
//   (D psi)(x) = (m0+4) psi(x) - 1/2 sum_mu (I - gamma_mu) U_mu(x) psi(x+mu)
//                              - 1/2 sum_mu (I + gamma_mu) U_mu(x-mu)^H psi(x-mu)
// in the chiral basis gamma_5 = diag(-1,-1,1,1).  (I -+ gamma_mu) has rank 2,
// so each hop projects the neighbour to a two-spin "half spinor" h, applies
// the 3x3 link to h only and rebuilds the lower two spins from the product.
#pragma once

#include "device.h"

namespace ovl {

enum WMode {
    W_PLAIN = 0,     // out = D in            (or Gamma_5 D in)
    W_NORM = 1,      // out = Gamma_5 D in;  partials |out|^2, |in(x)|^2
    W_SHIFT = 2,     // out = Gamma_5 D in + shift * p
    W_RUPDATE = 3,   // r  -= alpha_r (Gamma_5 D in + shift * p); partial |r|^2
    W_RESNORM = 4,   // partial |rin - (Gamma_5 D in + shift * p)|^2, nothing stored
    W_RUPDATE0 = 5,  // r  -= alpha_r Gamma_5 D in (an unshifted system: p is not read);
                     // partial |r|^2
    W_SNORM = 6,     // out = Gamma_5 D in + shift * p; partial |out|^2 (t = Q r + beta t of an
                     // unshifted base, whose alpha needs no |p|^2)
};

struct WArgs {
    Geom g;
    const void *in;
    const float *in_sc;
    void *out;
    float *out_sc;
    const void *U;
    const void *p;          // W_SHIFT / W_RUPDATE second field
    const float *p_sc;
    const void *rin;        // W_RUPDATE(0): read r from here (may equal out)
    const float *rin_sc;
    int rin_first;          // W_RESNORM: RHS r reads field (rin_first + r) % rin_count of rin
    int rin_count;
    const double *rin_scale;  // W_RESNORM: rin of RHS r taken times rin_scale[r] (null: 1)
    double diag;            // m0 + 4
    double shift;
    const double *shiftv;   // per-RHS shift (device), overrides shift when set
    const double *alpha;    // W_RUPDATE(0): alpha per RHS (device)
    double *partials;       // [quantity][nrhs][nblk]
    const int *skip;        // per-RHS flag: block exits if skip[r] != 0 (may be null)
    int nblk;               // partial-sum slots per RHS and quantity (2 * blocks per parity)
    int nrhs;
    int kr;                 // streaming form: K = 2^kr consecutive lanes hold K RHS of one
                            // site (set by launch_wilson)
};

template <int PREC>
__device__ __forceinline__ SpinorRef<PREC> spinor_ref(const void *base, const float *sc, int S, int r);

template <>
__device__ __forceinline__ SpinorRef<P_F64> spinor_ref<P_F64>(const void *base, const float *, int S, int r)
{
    return {(double2 *)base + (size_t)r * 24 * S, S};
}

template <>
__device__ __forceinline__ SpinorRef<P_F32> spinor_ref<P_F32>(const void *base, const float *, int S, int r)
{
    return {(float4 *)base + (size_t)r * 12 * S, S};
}

template <>
__device__ __forceinline__ SpinorRef<P_F48> spinor_ref<P_F48>(const void *base, const float *, int S, int r)
{
    return {(uint4 *)base + (size_t)r * 18 * S, S};
}

template <>
__device__ __forceinline__ SpinorRef<P_F16S> spinor_ref<P_F16S>(const void *base, const float *sc, int S, int r)
{
    return {(uint4 *)base + (size_t)r * 6 * S, (float *)sc + (size_t)r * 2 * S, S};
}

// Accumulate the hop in direction mu (FWD: from x+mu with U_mu(x);
// !FWD: from x-mu with U_mu(x-mu)^H) into acc, with boundary phase ph.
template <typename T, int MU, bool FWD>
__device__ __forceinline__ void hop(cplx<T> acc[4][3], const cplx<T> s[4][3], const cplx<T> u[3][3], T ph)
{
    cplx<T> h[2][3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        if (MU == 0) {
            h[0][c] = FWD ? s[0][c] - s[2][c] : s[0][c] + s[2][c];
            h[1][c] = FWD ? s[1][c] - s[3][c] : s[1][c] + s[3][c];
        } else if (MU == 1) {
            h[0][c] = FWD ? s[0][c] + ti(s[3][c]) : s[0][c] + tmi(s[3][c]);
            h[1][c] = FWD ? s[1][c] + ti(s[2][c]) : s[1][c] + tmi(s[2][c]);
        } else if (MU == 2) {
            h[0][c] = FWD ? s[0][c] + s[3][c] : s[0][c] - s[3][c];
            h[1][c] = FWD ? s[1][c] - s[2][c] : s[1][c] + s[2][c];
        } else {
            h[0][c] = FWD ? s[0][c] + ti(s[2][c]) : s[0][c] + tmi(s[2][c]);
            h[1][c] = FWD ? s[1][c] + tmi(s[3][c]) : s[1][c] + ti(s[3][c]);
        }
    }
    cplx<T> w[2][3];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            cplx<T> t;
            if (FWD) {
                t = cm(u[c][0], h[a][0]);
                t = cmac(t, u[c][1], h[a][1]);
                t = cmac(t, u[c][2], h[a][2]);
            } else {
                t = cmc(u[0][c], h[a][0]);
                t = cmacc(t, u[1][c], h[a][1]);
                t = cmacc(t, u[2][c], h[a][2]);
            }
            w[a][c] = t;
        }
    // the phase enters as the factor of each accumulation (a fused
    // multiply-add in place of an add, no separate scaling of w)
    const T mh = -ph;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        acc[0][c] = fmac(acc[0][c], ph, w[0][c]);
        acc[1][c] = fmac(acc[1][c], ph, w[1][c]);
        if (MU == 0) {
            acc[2][c] = fmac(acc[2][c], FWD ? mh : ph, w[0][c]);
            acc[3][c] = fmac(acc[3][c], FWD ? mh : ph, w[1][c]);
        } else if (MU == 1) {
            acc[2][c] = fmac(acc[2][c], ph, FWD ? tmi(w[1][c]) : ti(w[1][c]));
            acc[3][c] = fmac(acc[3][c], ph, FWD ? tmi(w[0][c]) : ti(w[0][c]));
        } else if (MU == 2) {
            acc[2][c] = fmac(acc[2][c], FWD ? mh : ph, w[1][c]);
            acc[3][c] = fmac(acc[3][c], FWD ? ph : mh, w[0][c]);
        } else {
            acc[2][c] = fmac(acc[2][c], ph, FWD ? tmi(w[0][c]) : ti(w[0][c]));
            acc[3][c] = fmac(acc[3][c], ph, FWD ? ti(w[1][c]) : tmi(w[1][c]));
        }
    }
}

// lo: element offset of the thread's RHS field from in's field (RHS tiles of
// the streaming form, else 0); links are shared by every RHS.
template <int PREC, int MU>
__device__ __forceinline__ void hops_mu(const Geom &g, const SpinorRef<PREC> &in, const GaugeRef<PREC> &U,
                                        int p, int i, const int x[4], cplx<typename Real<PREC>::T> acc[4][3],
                                        int lo = 0)
{
    using T = typename Real<PREC>::T;
    cplx<T> s[4][3], u[3][3];
    int y[4] = {x[0], x[1], x[2], x[3]};
    // forward neighbour x+mu, link U_mu(x) stored at (p, i)
    T ph = (T)1;
    y[MU] = x[MU] + 1;
    if (y[MU] == g.L[MU]) { y[MU] = 0; ph = (T)g.bc[MU]; }
    int j = cb_index(g, y);
    in.load(1 - p, j + lo, s);
    U.load(p, MU, i, u);
    hop<T, MU, true>(acc, s, u, ph);
    // backward neighbour x-mu, link U_mu(x-mu) stored at (1-p, j)
    ph = (T)1;
    y[MU] = x[MU] - 1;
    if (y[MU] < 0) { y[MU] = g.L[MU] - 1; ph = (T)g.bc[MU]; }
    j = cb_index(g, y);
    in.load(1 - p, j + lo, s);
    U.load(1 - p, MU, j, u);
    hop<T, MU, false>(acc, s, u, ph);
}

// LDS copy of one time slice of a streaming block: the centres of its NT
// sites as component arrays indexed by the thread's local site index
// (double2 per complex in FP64, float4 per complex pair otherwise).
template <int PREC, int NT = kBlock>
struct LdsPsi {
    using E = float4;
    static constexpr int NC = 6;
    E (*d)[NT];
    __device__ __forceinline__ void store(int l, const cplx<float> s[4][3]) const
    {
#pragma unroll
        for (int k = 0; k < 6; k++) {
            cplx<float> a = s[(2 * k) / 3][(2 * k) % 3], c = s[(2 * k + 1) / 3][(2 * k + 1) % 3];
            d[k][l] = make_float4(a.x, a.y, c.x, c.y);
        }
    }
    __device__ __forceinline__ void load(int l, cplx<float> s[4][3]) const
    {
#pragma unroll
        for (int k = 0; k < 6; k++) {
            float4 v = d[k][l];
            s[(2 * k) / 3][(2 * k) % 3] = {v.x, v.y};
            s[(2 * k + 1) / 3][(2 * k + 1) % 3] = {v.z, v.w};
        }
    }
};
template <int NT>
struct LdsPsi<P_F64, NT> {
    using E = double2;
    static constexpr int NC = 12;
    E (*d)[NT];
    __device__ __forceinline__ void store(int l, const cplx<double> s[4][3]) const
    {
#pragma unroll
        for (int k = 0; k < 12; k++) d[k][l] = make_double2(s[k / 3][k % 3].x, s[k / 3][k % 3].y);
    }
    __device__ __forceinline__ void load(int l, cplx<double> s[4][3]) const
    {
#pragma unroll
        for (int k = 0; k < 12; k++) {
            double2 v = d[k][l];
            s[k / 3][k % 3] = {v.x, v.y};
        }
    }
};

// 48-bit fields keep their encoding in LDS (36 KB per 256 sites): the
// streaming kernel stores the words it loaded for the next slice's centres
// (store_raw), so a slice costs no encode.
template <int NT>
struct LdsPsi<P_F48, NT> {
    using E = uint4;
    static constexpr int NC = 9;
    E (*d)[NT];
    __device__ __forceinline__ void store(int l, const cplx<double> s[4][3]) const
    {
        F48Code c;
        f48_encode(s, c);
        store_raw(l, c);
    }
    __device__ __forceinline__ void store_raw(int l, const F48Code &c) const
    {
#pragma unroll
        for (int k = 0; k < 6; k++) d[k][l] = c.h[k];
#pragma unroll
        for (int k = 0; k < 3; k++) d[6 + k][l] = c.l[k];
    }
    __device__ __forceinline__ void load(int l, cplx<double> s[4][3]) const
    {
        F48Code c;
#pragma unroll
        for (int k = 0; k < 6; k++) c.h[k] = d[k][l];
#pragma unroll
        for (int k = 0; k < 3; k++) c.l[k] = d[6 + k][l];
        f48_decode(c, s);
    }
};

// Neighbour spinor from the slice's LDS copy (local index ln) when inside,
// else from memory (parity pn, index jn): one generic-pointer load path for
// both, so the compiler need not carry both versions.  The LDS and memory
// layouts share their element type; FP16 (never staged) keeps a branch.
template <int PREC, int NT>
__device__ __forceinline__ void load_either(const LdsPsi<PREC, NT> &lp, const SpinorRef<PREC> &in, bool inside,
                                            int ln, int pn, int jn, int S, cplx<typename Real<PREC>::T> s[4][3])
{
    if constexpr (PREC == P_F16S) {
        if (inside) lp.load(ln, s);
        else in.load(pn, jn, s);
    } else {
        using E = typename LdsPsi<PREC, NT>::E;
        constexpr int NC = LdsPsi<PREC, NT>::NC;
        const E *b = inside ? (const E *)&lp.d[0][ln] : (const E *)in.d + (size_t)pn * NC * S + jn;
        const size_t stride = inside ? (size_t)NT : (size_t)S;
        E v[NC];
#pragma unroll
        for (int k = 0; k < NC; k++) v[k] = b[k * stride];
        if constexpr (PREC == P_F64) {
#pragma unroll
            for (int k = 0; k < 12; k++) s[k / 3][k % 3] = {v[k].x, v[k].y};
        } else if constexpr (PREC == P_F48) {
            F48Code c;
#pragma unroll
            for (int k = 0; k < 6; k++) c.h[k] = v[k];
#pragma unroll
            for (int k = 0; k < 3; k++) c.l[k] = v[6 + k];
            f48_decode(c, s);
        } else {
#pragma unroll
            for (int k = 0; k < 6; k++) {
                s[(2 * k) / 3][(2 * k) % 3] = {v[k].x, v[k].y};
                s[(2 * k + 1) / 3][(2 * k + 1) % 3] = {v[k].z, v[k].w};
            }
        }
    }
}

// Hops in direction MU = 2 or 3 of the LDS-staged streaming form: a
// neighbour inside the block (every x3 neighbour; x2 neighbours except from
// the block's first and last rows) comes from the slice's LDS copy, others
// from memory.  l: the thread's LDS slot, sl = l >> kr its local site (the K
// lanes of a site hold K RHS, so a site's slot is l with the site index
// shifted by kr); rows of L3 sites.
template <int PREC, int MU, int NT>
__device__ __forceinline__ void hops_mu_lds(const Geom &g, const SpinorRef<PREC> &in, const GaugeRef<PREC> &U,
                                            const LdsPsi<PREC, NT> &lp, int p, int i, const int x[4], int l, int kr,
                                            int lo, cplx<typename Real<PREC>::T> acc[4][3])
{
    using T = typename Real<PREC>::T;
    const int L3 = g.L[3];
    const int row = (l >> kr) / L3, rows = (NT >> kr) / L3;
    const int drow = L3 << kr;   // slot distance of one x2 row
    cplx<T> s[4][3], u[3][3];
    int y[4] = {x[0], x[1], x[2], x[3]};
    T ph = (T)1;
    y[MU] = x[MU] + 1;
    if (y[MU] == g.L[MU]) { y[MU] = 0; ph = (T)g.bc[MU]; }
    int j = cb_index(g, y);
    if (MU == 3) lp.load(l + ((y[3] - x[3]) << kr), s);
    else load_either(lp, in, row + 1 < rows, l + drow, 1 - p, j + lo, g.S, s);
    U.load(p, MU, i, u);
    hop<T, MU, true>(acc, s, u, ph);
    ph = (T)1;
    y[MU] = x[MU] - 1;
    if (y[MU] < 0) { y[MU] = g.L[MU] - 1; ph = (T)g.bc[MU]; }
    j = cb_index(g, y);
    if (MU == 3) lp.load(l + ((y[3] - x[3]) << kr), s);
    else load_either(lp, in, row > 0, l - drow, 1 - p, j + lo, g.S, s);
    U.load(1 - p, MU, j, u);
    hop<T, MU, false>(acc, s, u, ph);
}

// Output of one site from v = (m0+4) d - acc/2 (the Wilson operator on the
// site before Gamma_5) and |d|^2 of its centre d: applies Gamma_5, then the
// mode's shift term, residual update or residual norm; stores the result and
// adds the site's norms to q0, q1.
// r: the RHS; its fields are field rb of a.p, a.rin, a.out at element offset
// lo (RHS tiles: rb the tile's first RHS, lo the lane's offset; else rb = r,
// lo = 0).  A lane with live false (an idle or finished RHS of a tile)
// computes like the others, adds no norms and stores into the padding
// element Vh of its component arrays, which no kernel reads (every array has
// at least 24 padding elements): a select of the address, not a branch, since
// a branch around the stores makes the compiler keep far more values live
// and spill.
template <int PREC, int MODE, bool G5>
__device__ __forceinline__ void site_out(const WArgs &a, int r, int rb, int lo, int p, int i, double shift_r,
                                         double rin_s, cplx<typename Real<PREC>::T> o[4][3],
                                         typename Real<PREC>::T dn2, double &q0, double &q1, bool live = true)
{
    using T = typename Real<PREC>::T;
    constexpr bool kShift = MODE == W_SHIFT || MODE == W_RUPDATE || MODE == W_RESNORM || MODE == W_SNORM;
    const Geom &g = a.g;
    const int ist = live ? i : g.Vh;   // store index
    if (G5) {
#pragma unroll
        for (int s = 0; s < 2; s++)
#pragma unroll
            for (int c = 0; c < 3; c++) o[s][c] = {-o[s][c].x, -o[s][c].y};
    }
    if (MODE == W_NORM) {
        T n0 = 0;
#pragma unroll
        for (int s = 0; s < 4; s++)
#pragma unroll
            for (int c = 0; c < 3; c++) n0 += norm2(o[s][c]);
        q0 += live ? (double)n0 : 0.0;
        q1 += live ? (double)dn2 : 0.0;
    }
    if (kShift) {
        const SpinorRef<PREC> pf = spinor_ref<PREC>(a.p, a.p_sc, g.S, rb);
        cplx<T> pv[4][3];
        pf.load_nt(p, i + lo, pv);
        const T sh = (T)shift_r;
#pragma unroll
        for (int s = 0; s < 4; s++)
#pragma unroll
            for (int c = 0; c < 3; c++) o[s][c] = {fma(sh, pv[s][c].x, o[s][c].x), fma(sh, pv[s][c].y, o[s][c].y)};
    }
    if (MODE == W_SNORM) {
        T n0 = 0;
#pragma unroll
        for (int s = 0; s < 4; s++)
#pragma unroll
            for (int c = 0; c < 3; c++) n0 += norm2(o[s][c]);
        q0 += live ? (double)n0 : 0.0;
    }
    if (MODE == W_RUPDATE || MODE == W_RUPDATE0) {
        cplx<T> rv[4][3];
        spinor_ref<PREC>(a.rin, a.rin_sc, g.S, rb).load_nt(p, i + lo, rv);
        const T al = (T)a.alpha[r];
        T n0 = 0;
#pragma unroll
        for (int s = 0; s < 4; s++)
#pragma unroll
            for (int c = 0; c < 3; c++) {
                rv[s][c] = {fma(-al, o[s][c].x, rv[s][c].x), fma(-al, o[s][c].y, rv[s][c].y)};
                n0 += norm2(rv[s][c]);
            }
        spinor_ref<PREC>(a.out, a.out_sc, g.S, rb).store_nt(p, ist + lo, rv);
        q0 += live ? (double)n0 : 0.0;
    } else if (MODE == W_RESNORM) {
        cplx<T> rv[4][3];
        const int f = (a.rin_first + r) % a.rin_count;
        if (lo == 0) {
            spinor_ref<PREC>(a.rin, a.rin_sc, g.S, f).load_nt(p, i, rv);
        } else {
            // field f at an element offset from field 0 (RHS tiles)
            spinor_ref<PREC>(a.rin, a.rin_sc, g.S, 0).load_nt(p, i + f * (int)spinor_elems(PREC, g.S), rv);
        }
        const T rs = (T)rin_s;
        T n0 = 0;
#pragma unroll
        for (int s = 0; s < 4; s++)
#pragma unroll
            for (int c = 0; c < 3; c++) n0 += norm2(rs * rv[s][c] - o[s][c]);
        q0 += live ? (double)n0 : 0.0;
    } else {
        spinor_ref<PREC>(a.out, a.out_sc, g.S, rb).store_nt(p, ist + lo, o);
    }
}

// v = (m0+4) d - acc/2 in place of acc; returns |d|^2
template <typename T>
__device__ __forceinline__ T diag_minus_half(cplx<T> acc[4][3], const cplx<T> d[4][3], T diag)
{
    T dn2 = 0;
#pragma unroll
    for (int s = 0; s < 4; s++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            acc[s][c] = {fma(diag, d[s][c].x, (T)-0.5 * acc[s][c].x), fma(diag, d[s][c].y, (T)-0.5 * acc[s][c].y)};
            dn2 += norm2(d[s][c]);
        }
    return dn2;
}

template <int PREC, int MODE, bool G5>
__global__ __launch_bounds__(kBlock) void k_wilson(WArgs a)
{
    using T = typename Real<PREC>::T;
    __shared__ double lds[8];
    // Blocks are ordered (site block, RHS) with the RHS fastest, so the nrhs
    // blocks covering the same sites run back to back on one XCD and share
    // each link through its L2.
    const int lbr = xcd_remap(blockIdx.x, gridDim.x);
    const int r = lbr % a.nrhs;
    const int lb = lbr / a.nrhs;
    const int nb = gridDim.x / a.nrhs;   // site blocks (both parities)
    if (a.skip && a.skip[r]) return;
    // the epilogue's shift, read once up front (a uniform scalar)
    constexpr bool kShift = MODE == W_SHIFT || MODE == W_RUPDATE || MODE == W_RESNORM || MODE == W_SNORM;
    const double shift_r = kShift ? (a.shiftv ? a.shiftv[r] : a.shift) : 0.0;
    // the residual norm's scale of rin, likewise read once up front (a load
    // left inside the epilogue behind the null test made the compiler keep far
    // more values live across the hops and spill)
    const double rin_s = MODE == W_RESNORM && a.rin_scale ? a.rin_scale[r] : 1.0;
    const int p = lb & 1;
    const int jl = (lb >> 1) * kBlock + threadIdx.x;
    const Geom &g = a.g;
    const bool valid = jl < g.Vh;
    const SpinorRef<PREC> in = spinor_ref<PREC>(a.in, a.in_sc, g.S, r);
    const GaugeRef<PREC> U = gauge_ref<PREC>(a.U, g.S);
    double q0 = 0.0, q1 = 0.0;
    if (valid) {
        int x[4];
        tiled_coords(g, p, jl, x);
        const int i = cb_index(g, x);
        cplx<T> acc[4][3];
#pragma unroll
        for (int s = 0; s < 4; s++)
#pragma unroll
            for (int c = 0; c < 3; c++) acc[s][c] = {(T)0, (T)0};
        hops_mu<PREC, 0>(g, in, U, p, i, x, acc);
        hops_mu<PREC, 1>(g, in, U, p, i, x, acc);
        hops_mu<PREC, 2>(g, in, U, p, i, x, acc);
        hops_mu<PREC, 3>(g, in, U, p, i, x, acc);
        cplx<T> d[4][3];
        in.load(p, i, d);
        const T dn2 = diag_minus_half(acc, d, (T)a.diag);
        site_out<PREC, MODE, G5>(a, r, r, 0, p, i, shift_r, rin_s, acc, dn2, q0, q1);
    }
    if (MODE == W_NORM || MODE == W_SNORM || MODE == W_RUPDATE || MODE == W_RUPDATE0 || MODE == W_RESNORM) {
        double t0 = block_sum(q0, lds);
        if (threadIdx.x == 0) a.partials[(size_t)r * nb + lb] = t0;
        if (MODE == W_NORM) {
            double t1 = block_sum(q1, lds + 4);
            if (threadIdx.x == 0) a.partials[(size_t)(a.nrhs + r) * nb + lb] = t1;
        }
    }
}

// Backward time hop split in two: w = U_0(x-0)^H (1 + gamma_0) psi(x-0) on the
// two independent spins, and its reconstruction into the four spins of acc.
template <typename T>
__device__ __forceinline__ void tback_half(cplx<T> w[2][3], const cplx<T> s[4][3], const cplx<T> u[3][3])
{
    cplx<T> h[2][3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        h[0][c] = s[0][c] + s[2][c];
        h[1][c] = s[1][c] + s[3][c];
    }
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int c = 0; c < 3; c++) w[a][c] = cmacc(cmacc(cmc(u[0][c], h[a][0]), u[1][c], h[a][1]), u[2][c], h[a][2]);
}

template <typename T>
__device__ __forceinline__ void tback_add(cplx<T> acc[4][3], const cplx<T> w[2][3], T ph)
{
#pragma unroll
    for (int c = 0; c < 3; c++) {
        acc[0][c] = fmac(acc[0][c], ph, w[0][c]);
        acc[1][c] = fmac(acc[1][c], ph, w[1][c]);
        acc[2][c] = fmac(acc[2][c], ph, w[0][c]);
        acc[3][c] = fmac(acc[3][c], ph, w[1][c]);
    }
}

// Time-streaming form of the stencil.  A thread owns one spatial site
// (x1, x2, x3) of one RHS and walks Ts consecutive time slices (g.Ts64 for
// FP64 when set, else g.Ts).  K = 2^a.kr consecutive lanes hold the K RHS of
// a tile of one site, so every link load serves K RHS within one wave
// instruction (and a wave reads K runs of consecutive sites, one per RHS
// field).  Block lb covers the NS = NT/K consecutive spatial sites of spatial
// block lb % nsb (x3 fastest, so a wave reads whole x3 rows of both
// parities) in time chunk lb / nsb, for RHS tile rt.  The time hops need no
// neighbour loads after the first slice: psi(t+1), loaded for the forward
// hop, is the centre of the next slice, and the backward hop's
// U_0(t)^H (1 + gamma_0) psi(t) is formed while slice t holds U_0(t) and
// psi(t) in registers.  Requires L1*L2*L3 % NS == 0 and Ts | L0.
// WPE is the minimum number of waves per SIMD the build allows for (1 or 2);
// the one-wave build overlaps pairs of time slices.  STAGE (blocks of whole
// x3 rows of consecutive x2 at one x1: NS % L3 == 0 and L2*L3 % NS == 0)
// keeps each slice's centres in LDS, where the next slice reads its x3 and
// in-block x2 neighbours.  NT = 256, or 192 for x3 extents such as 24 and 48
// whose rows do not tile 256 sites (stream_threads).
// Lanes of an RHS beyond nrhs (last tile) or of a finished RHS (skip) take
// part in the walk and the barriers but store nothing and add no norms.
// Partial sums: for each RHS q of the tile, slot lb holds the block's sum and
// the block zeroes the slots lb + m*nbt (m >= 1) below a.nblk, so all 2*nb
// slots per RHS are valid.
// TILED builds take the RHS tile from a.kr; the others have K = 1 at compile
// time, so the RHS index and everything derived from it stay block-uniform
// (scalar registers).
template <int PREC, int MODE, bool G5, int WPE, bool STAGE, int NT = kBlock, bool TILED = false>
__global__ __launch_bounds__(NT, WPE) void k_wilson_ts(WArgs a)
{
    using T = typename Real<PREC>::T;
    __shared__ double lds[2 * (NT / 64) * 8];
    __shared__ typename LdsPsi<PREC, NT>::E lds_psi[STAGE ? LdsPsi<PREC, NT>::NC : 1][NT];
    const LdsPsi<PREC, NT> lp{lds_psi};
    const Geom &g = a.g;
    const int kr = TILED ? a.kr : 0;
    const int K = 1 << kr;
    const int ntile = (a.nrhs + K - 1) >> kr;
    const int lbr = xcd_remap(blockIdx.x, gridDim.x);
    const int rt = lbr % ntile;
    const int lb = lbr / ntile;
    const int nbt = gridDim.x / ntile;   // blocks per RHS tile
    const int rq = rt * K + (threadIdx.x & (K - 1));
    const int r = rq < a.nrhs ? rq : a.nrhs - 1;   // idle lanes walk the tile's last RHS
    const bool live = rq < a.nrhs && !(a.skip && a.skip[rq]);
    if (!TILED) {
        if (!live) return;
    } else if (!__syncthreads_or(live)) {
        return;   // every RHS of the tile is finished (block-uniform)
    }
    constexpr bool kShift = MODE == W_SHIFT || MODE == W_RUPDATE || MODE == W_RESNORM || MODE == W_SNORM;
    const double shift_r = kShift ? (a.shiftv ? a.shiftv[r] : a.shift) : 0.0;
    // the residual norm's scale of rin, likewise read once up front (a load
    // left inside the epilogue behind the null test made the compiler keep far
    // more values live across the hops and spill)
    const double rin_s = MODE == W_RESNORM && a.rin_scale ? a.rin_scale[r] : 1.0;
    const int L0 = g.L[0], L1 = g.L[1], L2 = g.L[2], L3 = g.L[3];
    const int NS = NT >> kr;
    const int nsb = L1 * L2 * L3 / NS;
    const int sb = lb % nsb, tc = lb / nsb;
    const int sidx = sb * NS + (threadIdx.x >> kr);
    int x[4];
    x[3] = sidx % L3;
    x[2] = (sidx / L3) % L2;
    x[1] = sidx / (L3 * L2);
    const int Ts = (PREC == P_F64 || PREC == P_F48) && g.Ts64 > 0 ? g.Ts64 : g.Ts;
    const int t0 = tc * Ts;
    // tiles: field pointers at the tile's first RHS (uniform), the lane's RHS
    // as an element offset of the site index (32-bit, in vector registers)
    const int rb = TILED ? rt * K : r;
    const int lo = TILED ? (r - rb) * (int)spinor_elems(PREC, g.S) : 0;
    const SpinorRef<PREC> in = spinor_ref<PREC>(a.in, a.in_sc, g.S, rb);
    const GaugeRef<PREC> U = gauge_ref<PREC>(a.U, g.S);
    const int sp = x[1] + x[2] + x[3];   // parity of the spatial part
    cplx<T> cen[4][3], w[2][3];   // centre of the current slice, backward-hop carry
    {
        // centre of the first slice and the backward-hop carry from t0 - 1
        x[0] = t0;
        in.load((t0 + sp) & 1, cb_index(g, x) + lo, cen);
        int y[4] = {t0 == 0 ? L0 - 1 : t0 - 1, x[1], x[2], x[3]};
        const int py = (y[0] + sp) & 1, iy = cb_index(g, y);
        cplx<T> sv[4][3], u[3][3];
        in.load(py, iy + lo, sv);
        U.load_nt(py, 0, iy, u);
        tback_half(w, sv, u);
    }
    if (STAGE) {
        lp.store(threadIdx.x, cen);
        __syncthreads();
    }
    double q0 = 0.0, q1 = 0.0;
#pragma unroll(WPE == 1 ? 2 : 1)
    for (int k = 0; k < Ts; k++) {
        const int t = t0 + k;
        x[0] = t;
        const int p = (t + sp) & 1;
        const int i = cb_index(g, x);
        cplx<T> acc[4][3];
#pragma unroll
        for (int s = 0; s < 4; s++)
#pragma unroll
            for (int c = 0; c < 3; c++) acc[s][c] = {(T)0, (T)0};
        tback_add(acc, w, t == 0 ? (T)g.bc[0] : (T)1);
        hops_mu<PREC, 1>(g, in, U, p, i, x, acc, lo);
        if (STAGE) {
            hops_mu_lds<PREC, 2>(g, in, U, lp, p, i, x, threadIdx.x, kr, lo, acc);
            hops_mu_lds<PREC, 3>(g, in, U, lp, p, i, x, threadIdx.x, kr, lo, acc);
        } else {
            hops_mu<PREC, 2>(g, in, U, p, i, x, acc, lo);
            hops_mu<PREC, 3>(g, in, U, p, i, x, acc, lo);
        }
        // U_0(t): the next slice's carry from this centre, then the centre's
        // diagonal term; the centre is then dead before psi(t+1) arrives
        cplx<T> u[3][3];
        U.load_nt(p, 0, i, u);   // U_0(t) is read by the K lanes of this site only
        tback_half(w, cen, u);
        const T dn2 = diag_minus_half(acc, cen, (T)a.diag);
        // 48-bit staged builds keep the next centre's words as loaded, store
        // them to LDS unchanged and decode the centre back from there, so the
        // decoded centre is not held across the epilogue
        constexpr bool kRaw = PREC == P_F48 && STAGE;
        F48Code raw;
        {
            // forward time hop, subtracted with its factor -1/2 straight into v
            int y[4] = {t + 1 == L0 ? 0 : t + 1, x[1], x[2], x[3]};
            if constexpr (kRaw) {
                in.load_raw(1 - p, cb_index(g, y) + lo, raw);
                f48_decode(raw, cen);
            } else {
                in.load(1 - p, cb_index(g, y) + lo, cen);
            }
            cplx<T> f[4][3];
#pragma unroll
            for (int s = 0; s < 4; s++)
#pragma unroll
                for (int c = 0; c < 3; c++) f[s][c] = {(T)0, (T)0};
            hop<T, 0, true>(f, cen, u, t + 1 == L0 ? (T)(-0.5 * g.bc[0]) : (T)-0.5);
#pragma unroll
            for (int s = 0; s < 4; s++)
#pragma unroll
                for (int c = 0; c < 3; c++) acc[s][c] = acc[s][c] + f[s][c];
        }
        site_out<PREC, MODE, G5>(a, r, rb, lo, p, i, shift_r, rin_s, acc, dn2, q0, q1, !TILED || live);
        if (STAGE) {
            // every thread has read this slice's copy: replace it by the next slice
            __syncthreads();
            if constexpr (kRaw) lp.store_raw(threadIdx.x, raw);
            else lp.store(threadIdx.x, cen);
            __syncthreads();
            if constexpr (kRaw) lp.load(threadIdx.x, cen);
        }
    }
    if (MODE == W_NORM || MODE == W_SNORM || MODE == W_RUPDATE || MODE == W_RUPDATE0 || MODE == W_RESNORM) {
        constexpr int nq = MODE == W_NORM ? 2 : 1;
        double t0s = block_sum_k<NT / 64>(q0, lds, kr);
        double t1s = nq == 2 ? block_sum_k<NT / 64>(q1, lds + (NT / 64) * 8, kr) : 0.0;
        // thread q of the first K holds RHS rt*K + q's sums; the zeroed slots
        // of the tile's RHS are spread over the block's threads
        __shared__ double sums[2][8];
        if (threadIdx.x < K) {
            sums[0][threadIdx.x] = t0s;
            sums[1][threadIdx.x] = t1s;
        }
        __syncthreads();
        const int nz = (a.nblk - 1 - lb) / nbt + 1;   // slots lb + m*nbt below nblk
        for (int idx = threadIdx.x; idx < K * nz; idx += NT) {
            const int q = idx % K, m = idx / K;
            const int rr = rt * K + q;
            if (rr >= a.nrhs || (a.skip && a.skip[rr])) continue;
            const size_t slot = (size_t)lb + (size_t)m * nbt;
            a.partials[(size_t)rr * a.nblk + slot] = m == 0 ? sums[0][q] : 0.0;
            if (nq == 2) a.partials[(size_t)(a.nrhs + rr) * a.nblk + slot] = m == 0 ? sums[1][q] : 0.0;
        }
    }
}

}  // namespace ovl
