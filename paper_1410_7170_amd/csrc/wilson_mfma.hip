// The Wilson-Dirac stencil on several RHS with matrix-core (MFMA)
// instructions, for comparison with the VALU stencils (FP32, D_W or
// Gamma_5 D_W only).
//
// eq. (Wilson-Dirac): (D psi)(x) = (m0+4) psi(x)
//     - 1/2 sum_mu [ U_mu(x) (I - gamma_mu) psi(x+mu) + U_mu(x-mu)^H (I + gamma_mu) psi(x-mu) ].
// For one hop, the link acts on colour and the projector on spin, so with the
// spins and RHS of a site as columns the hop is a 3 x 3 by 3 x (4 nrhs)
// complex product.  In real form (6 x 6 times 6 x N) two sites share one
// v_mfma_f32_16x16x4f32 as a block-diagonal A (rows 6s..6s+5 the real and
// imaginary parts of site s's link rows, K = 12 in three steps of 4), with
// B the projected neighbour spinors (I -+ gamma_mu) psi(x+-mu) of both sites
// (rows 6s + colour / + 3 for the imaginary part) and N = 16 columns = 4
// spins x 4 RHS.  All 8 hops accumulate into the same 16 x 16 accumulator;
// an LDS transpose then gives each lane whole complex outputs for the
// epilogue.  The A operand is half zeros and the projector's rank-2 structure
// is not used, so the matrix cores do about four times the useful work;
// the comparison is of the whole kernel, memory traffic included.
//
// Lane layout of v_mfma_f32_16x16x4f32 (one block): lane l holds A[l % 16][l / 16],
// B[l / 16][l % 16] and the accumulator rows 4 (l / 16) + v, v = 0..3, of
// column l % 16.
#include "internal.h"

namespace ovl {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

// (gamma_mu psi)[a] = g * psi[b]: partner spin b and coefficient g in the
// chiral basis (gamma_0 = [[0,I],[I,0]], gamma_k = [[0,-i sigma_k],[i sigma_k,0]])
__device__ __forceinline__ void gamma_row(int mu, int a, int &b, cplx<float> &g)
{
    switch (mu) {
    case 0: b = a ^ 2; g = {1.f, 0.f}; break;
    case 1: b = 3 - a; g = a < 2 ? cplx<float>{0.f, -1.f} : cplx<float>{0.f, 1.f}; break;
    case 2: b = 3 - a; g = (a == 0 || a == 3) ? cplx<float>{-1.f, 0.f} : cplx<float>{1.f, 0.f}; break;
    default: b = a ^ 2; g = (a == 0 || a == 3) ? cplx<float>{0.f, -1.f} : cplx<float>{0.f, 1.f}; break;
    }
}

// e[k] for a lane-dependent k in 0..2 as an arithmetic blend: a select
// between array elements would be turned into an indexed (scratch) access
__device__ __forceinline__ cplx<float> pick3(int k, cplx<float> e0, cplx<float> e1, cplx<float> e2)
{
    const float m0 = k == 0 ? 1.f : 0.f, m1 = k == 1 ? 1.f : 0.f, m2 = k == 2 ? 1.f : 0.f;
    return {m0 * e0.x + m1 * e1.x + m2 * e2.x, m0 * e0.y + m1 * e1.y + m2 * e2.y};
}

// component (spin, colour) of RHS rhs at (parity p, site i) of an FP32 field
// (float4 = two consecutive components)
__device__ __forceinline__ cplx<float> comp_f32(const float4 *d, int S, int rhs, int p, int i, int comp)
{
    const float2 *e = (const float2 *)(d + (size_t)rhs * 12 * S + (size_t)(p * 6 + comp / 2) * S + i);
    const float2 v = e[comp & 1];
    return {v.x, v.y};
}

}  // namespace

// One wave: two sites of one parity, one tile of 4 RHS.  Block: 4 waves.
template <bool G5>
__global__ __launch_bounds__(kBlock) void k_wilson_mfma(WArgs a)
{
    __shared__ float tile[4][16][17];
    const Geom &g = a.g;
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int npairs = (g.Vh + 1) / 2;
    const int P = blockIdx.x * 4 + wave;
    const int p = P / npairs, pr = P % npairs;
    const bool wave_ok = p < 2;
    const int q0 = blockIdx.y * 4;
    const float4 *in = (const float4 *)a.in;
    const GaugeRef<P_F32> U{(const float4 *)a.U, g.S};
    int site[2], xs[2][4];
    bool sv[2];
#pragma unroll
    for (int s = 0; s < 2; s++) {
        site[s] = 2 * pr + s;
        sv[s] = wave_ok && site[s] < g.Vh;
        if (sv[s]) site_coords(g, p, site[s], xs[s]);
    }
    // A rows (link rows) of this lane
    const int ia = l & 15, ka = l >> 4;
    const int sa = ia / 6, r6 = ia % 6, rr = r6 % 3, pra = r6 / 3;
    // B columns (spin, RHS) of this lane
    const int jb = l & 15, spin = jb >> 2, qb = jb & 3;
    const int rhs = q0 + qb;
    // RHS flagged in a.skip are neither read nor written
    const bool col_ok = rhs < a.nrhs && !(a.skip && a.skip[rhs]);
    // per-lane values of site sa (A rows) written as selects, so that no
    // private array is indexed by a lane-dependent value
    const int site_a = sa ? site[1] : site[0];
    const bool sv_a = sa ? sv[1] : sv[0];
    v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int mu = 0; mu < 4; mu++) {
#pragma unroll
        for (int dir = 1; dir >= -1; dir -= 2) {
            // neighbours of both sites and their boundary phases
            int nb[2] = {0, 0};
            float ph[2] = {1.f, 1.f};
#pragma unroll
            for (int s = 0; s < 2; s++) {
                if (!sv[s]) continue;
                int y[4] = {xs[s][0], xs[s][1], xs[s][2], xs[s][3]};
                y[mu] += dir;
                if (y[mu] == g.L[mu]) { y[mu] = 0; ph[s] = (float)g.bc[mu]; }
                if (y[mu] < 0) { y[mu] = g.L[mu] - 1; ph[s] = (float)g.bc[mu]; }
                nb[s] = cb_index(g, y);
            }
            // row rr of the link of site sa: U_mu(x) forward, U_mu(x-mu)^H
            // backward
            cplx<float> wr[3] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
            const bool arow = ia < 12 && sv_a;
            if (arow) {
                cplx<float> u[3][3];
                if (dir > 0) U.load(p, mu, site_a, u);
                else U.load(1 - p, mu, sa ? nb[1] : nb[0], u);
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    if (dir > 0) {
                        wr[c] = pick3(rr, u[0][c], u[1][c], u[2][c]);
                    } else {
                        const cplx<float> e = pick3(rr, u[c][0], u[c][1], u[c][2]);
                        wr[c] = {e.x, -e.y};
                    }
                }
            }
            int bs;
            cplx<float> gc;
            gamma_row(mu, spin, bs, gc);
#pragma unroll
            for (int st = 0; st < 3; st++) {
                const int k = 4 * st + ka;   // this lane's A column and B row
                const int sk = k / 6, c6 = k % 6, cc = c6 % 3, pc = c6 / 3;
                float av = 0.f;
                if (arow && sk == sa) {
                    const cplx<float> e = pick3(cc, wr[0], wr[1], wr[2]);
                    av = pra == 0 ? (pc == 0 ? e.x : -e.y) : (pc == 0 ? e.y : e.x);
                }
                // B[k][j]: (I - dir gamma_mu) psi at the neighbour of site sk,
                // times the boundary phase
                float bv = 0.f;
                const bool sv_k = sk ? sv[1] : sv[0];
                if (col_ok && sv_k) {
                    const int nb_k = sk ? nb[1] : nb[0];
                    const float ph_k = sk ? ph[1] : ph[0];
                    const cplx<float> x1 = comp_f32(in, g.S, rhs, 1 - p, nb_k, 3 * spin + cc);
                    const cplx<float> x2 = comp_f32(in, g.S, rhs, 1 - p, nb_k, 3 * bs + cc);
                    const cplx<float> gx = cm(gc, x2);
                    const cplx<float> h = {ph_k * (x1.x - dir * gx.x), ph_k * (x1.y - dir * gx.y)};
                    bv = pc == 0 ? h.x : h.y;
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
            }
        }
    }
    // accumulator rows 4 (l/16) + v of column l % 16 to LDS, then lanes
    // 0..31 each take one (site, spin, RHS): out = (m0+4) psi - acc/2
#pragma unroll
    for (int v = 0; v < 4; v++) tile[wave][4 * ka + v][jb] = acc[v];
    __syncthreads();
    if (l < 32) {
        const int s = l >> 4, j = l & 15, sp = j >> 2, q = j & 3;
        const int r = q0 + q;
        const int site_s = s ? site[1] : site[0];
        if ((s ? sv[1] : sv[0]) && r < a.nrhs && !(a.skip && a.skip[r])) {
            float2 *out = (float2 *)a.out;
            for (int c = 0; c < 3; c++) {
                const int comp = 3 * sp + c;
                const cplx<float> d = comp_f32(in, g.S, r, p, site_s, comp);
                float re = (float)a.diag * d.x - 0.5f * tile[wave][6 * s + c][j];
                float im = (float)a.diag * d.y - 0.5f * tile[wave][6 * s + 3 + c][j];
                if (G5 && sp < 2) {
                    re = -re;
                    im = -im;
                }
                float2 *e = (float2 *)((float4 *)out + (size_t)r * 12 * g.S + (size_t)(p * 6 + comp / 2) * g.S +
                                       site_s);
                e[comp & 1] = make_float2(re, im);
            }
        }
    }
}

hipError_t launch_wilson_mfma(const Lat &L, bool g5, const WArgs &a, hipStream_t st)
{
    const int npairs = (L.Vh + 1) / 2;
    dim3 grid((unsigned)((2 * npairs + 3) / 4), (unsigned)((a.nrhs + 3) / 4));
    if (g5) k_wilson_mfma<true><<<grid, kBlock, 0, st>>>(a);
    else k_wilson_mfma<false><<<grid, kBlock, 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace ovl
