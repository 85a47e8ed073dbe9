// Layout conversion and BLAS-1 kernels on packed even-odd fields.
//
// All kernels here are site parallel: block b of a launch covers parity
// b / nb, checkerboard sites (b % nb)*256 .. +255, and blockIdx.y selects the
// RHS.  Per-block partial sums go to partials[rhs][block] and are combined by
// k_reduce in a fixed order, so every reduction is bitwise reproducible.
#include "internal.h"

namespace ovl {

Lat make_lat(const ovl_lattice *lat)
{
    Lat L;
    for (int m = 0; m < 4; m++) {
        L.g.L[m] = lat->dims[m];
        L.g.bc[m] = lat->bc[m];
    }
    L.V = (int64_t)lat->dims[0] * lat->dims[1] * lat->dims[2] * lat->dims[3];
    L.Vh = (int)(L.V / 2);
    L.g.Vh = L.Vh;
    L.g.S = padded_stride(L.Vh);
    L.g.T = lat->tile_t;
    L.g.Ts = lat->stream_t;
    L.g.Ts64 = lat->stream_t64;
    L.g.Kr = lat->rhs_tile >= 8 ? 3 : lat->rhs_tile >= 4 ? 2 : lat->rhs_tile >= 2 ? 1 : 0;
    L.g.Mfma = lat->mfma;
    L.nb = (L.Vh + kBlock - 1) / kBlock;
    return L;
}

static thread_local int g_last_hip = 0;
int hip_fail(hipError_t e)
{
    g_last_hip = (int)e;
    return OVL_ERR_HIP;
}
int last_hip_error() { return g_last_hip; }

int site_blocks(const Lat &L) { return 2 * L.nb; }

// The time-streaming stencil (FP64, FP32 with a stream length) runs
// blocks_per_tile blocks per RHS tile, one partial slot each; the one-site
// form fills all 2 nb slots.
int stencil_partials(const Lat &L, int prec, int nrhs)
{
    const StencilShape sh = stencil_shape(L, prec, nrhs);
    return sh.ts > 0 ? sh.blocks_per_tile : 2 * L.nb;
}

// ---------------------------------------------------------------- pack
template <int PREC>
__global__ __launch_bounds__(kBlock) void k_pack_spinor(Geom g, int64_t V, const double2 *canon, void *d, float *sc)
{
    using T = typename Real<PREC>::T;
    int64_t lex = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int r = blockIdx.y;
    if (lex >= V) return;
    int x3 = (int)(lex % g.L[3]);
    int64_t t = lex / g.L[3];
    int x2 = (int)(t % g.L[2]);
    t /= g.L[2];
    int x1 = (int)(t % g.L[1]);
    int x0 = (int)(t / g.L[1]);
    int p = (x0 + x1 + x2 + x3) & 1;
    int i = (int)(lex >> 1);
    const double2 *src = canon + ((size_t)r * V + lex) * 12;
    cplx<T> s[4][3];
#pragma unroll
    for (int k = 0; k < 12; k++) {
        double2 v = src[k];
        s[k / 3][k % 3] = {(T)v.x, (T)v.y};
    }
    spinor_ref<PREC>(d, sc, g.S, r).store(p, i, s);
}

template <int PREC>
__global__ __launch_bounds__(kBlock) void k_unpack_spinor(Geom g, int64_t V, const void *d, const float *sc, double2 *canon)
{
    using T = typename Real<PREC>::T;
    int64_t lex = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int r = blockIdx.y;
    if (lex >= V) return;
    int x3 = (int)(lex % g.L[3]);
    int64_t t = lex / g.L[3];
    int x2 = (int)(t % g.L[2]);
    t /= g.L[2];
    int x1 = (int)(t % g.L[1]);
    int x0 = (int)(t / g.L[1]);
    int p = (x0 + x1 + x2 + x3) & 1;
    int i = (int)(lex >> 1);
    cplx<T> s[4][3];
    spinor_ref<PREC>(d, sc, g.S, r).load(p, i, s);
    double2 *dst = canon + ((size_t)r * V + lex) * 12;
#pragma unroll
    for (int k = 0; k < 12; k++) dst[k] = make_double2((double)s[k / 3][k % 3].x, (double)s[k / 3][k % 3].y);
}

__global__ __launch_bounds__(kBlock) void k_pack_gauge(Geom g, int64_t V, const double2 *canon, int prec, void *out)
{
    int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (id >= 4 * V) return;
    int64_t lex = id >> 2;
    int mu = (int)(id & 3);
    int x3 = (int)(lex % g.L[3]);
    int64_t t = lex / g.L[3];
    int x2 = (int)(t % g.L[2]);
    t /= g.L[2];
    int x1 = (int)(t % g.L[1]);
    int x0 = (int)(t / g.L[1]);
    int p = (x0 + x1 + x2 + x3) & 1;
    size_t i = (size_t)(lex >> 1);
    size_t Vh = (size_t)g.S;   // component stride
    const double2 *u = canon + (size_t)id * 9;
    if (prec == P_F64) {
        double2 *o = (double2 *)out + (size_t)(p * 4 + mu) * 6 * Vh + i;
        for (int e = 0; e < 6; e++) o[e * Vh] = u[e];
    } else if (prec == P_F32) {
        float4 *o = (float4 *)out + (size_t)(p * 4 + mu) * 3 * Vh + i;
        for (int k = 0; k < 3; k++)
            o[k * Vh] = make_float4((float)u[2 * k].x, (float)u[2 * k].y, (float)u[2 * k + 1].x, (float)u[2 * k + 1].y);
    } else {
        uint2 *o = (uint2 *)out + (size_t)(p * 4 + mu) * 3 * Vh + i;
        for (int k = 0; k < 3; k++) {
            unsigned a = (unsigned)f2h((float)u[2 * k].x) | ((unsigned)f2h((float)u[2 * k].y) << 16);
            unsigned b = (unsigned)f2h((float)u[2 * k + 1].x) | ((unsigned)f2h((float)u[2 * k + 1].y) << 16);
            o[k * Vh] = make_uint2(a, b);
        }
    }
}

hipError_t launch_pack_spinor(const Lat &L, const void *canon, Fld out, hipStream_t st)
{
    dim3 grid((unsigned)((L.V + kBlock - 1) / kBlock), out.nrhs);
    if (out.prec == P_F64)
        k_pack_spinor<P_F64><<<grid, kBlock, 0, st>>>(L.g, L.V, (const double2 *)canon, out.d, out.sc);
    else if (out.prec == P_F48)
        k_pack_spinor<P_F48><<<grid, kBlock, 0, st>>>(L.g, L.V, (const double2 *)canon, out.d, out.sc);
    else if (out.prec == P_F32)
        k_pack_spinor<P_F32><<<grid, kBlock, 0, st>>>(L.g, L.V, (const double2 *)canon, out.d, out.sc);
    else
        k_pack_spinor<P_F16S><<<grid, kBlock, 0, st>>>(L.g, L.V, (const double2 *)canon, out.d, out.sc);
    return hipGetLastError();
}

hipError_t launch_unpack_spinor(const Lat &L, Fld in, void *canon, hipStream_t st)
{
    dim3 grid((unsigned)((L.V + kBlock - 1) / kBlock), in.nrhs);
    if (in.prec == P_F64)
        k_unpack_spinor<P_F64><<<grid, kBlock, 0, st>>>(L.g, L.V, in.d, in.sc, (double2 *)canon);
    else if (in.prec == P_F48)
        k_unpack_spinor<P_F48><<<grid, kBlock, 0, st>>>(L.g, L.V, in.d, in.sc, (double2 *)canon);
    else if (in.prec == P_F32)
        k_unpack_spinor<P_F32><<<grid, kBlock, 0, st>>>(L.g, L.V, in.d, in.sc, (double2 *)canon);
    else
        k_unpack_spinor<P_F16S><<<grid, kBlock, 0, st>>>(L.g, L.V, in.d, in.sc, (double2 *)canon);
    return hipGetLastError();
}

hipError_t launch_pack_gauge(const Lat &L, const void *canon, int prec, void *out, hipStream_t st)
{
    dim3 grid((unsigned)((4 * L.V + kBlock - 1) / kBlock));
    k_pack_gauge<<<grid, kBlock, 0, st>>>(L.g, L.V, (const double2 *)canon, prec, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- BLAS-1
template <int PREC>
__global__ __launch_bounds__(kBlock) void k_norm2(Geom g, int nb, const void *d, const float *sc, double *partials)
{
    using T = typename Real<PREC>::T;
    __shared__ double lds[4];
    int r = blockIdx.y, b = blockIdx.x;
    int p = b / nb, i = (b % nb) * kBlock + threadIdx.x;
    double v = 0.0;
    if (i < g.Vh) {
        cplx<T> s[4][3];
        spinor_ref<PREC>(d, sc, g.S, r).load(p, i, s);
        T a = 0;
#pragma unroll
        for (int k = 0; k < 12; k++) a += norm2(s[k / 3][k % 3]);
        v = (double)a;
    }
    double t = block_sum(v, lds);
    if (threadIdx.x == 0) partials[(size_t)r * gridDim.x + b] = t;
}

// |a - b|^2 with both fields widened to double
template <int PA, int PB>
__global__ __launch_bounds__(kBlock) void k_diff_norm2(Geom g, int nb, const void *da, const float *sa,
                                                       const void *db, const float *sb, double *partials)
{
    using TA = typename Real<PA>::T;
    using TB = typename Real<PB>::T;
    __shared__ double lds[4];
    int r = blockIdx.y, b = blockIdx.x;
    int p = b / nb, i = (b % nb) * kBlock + threadIdx.x;
    double v = 0.0;
    if (i < g.Vh) {
        cplx<TA> s[4][3];
        cplx<TB> t[4][3];
        spinor_ref<PA>(da, sa, g.S, r).load(p, i, s);
        spinor_ref<PB>(db, sb, g.S, r).load(p, i, t);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            double dx = (double)s[k / 3][k % 3].x - (double)t[k / 3][k % 3].x;
            double dy = (double)s[k / 3][k % 3].y - (double)t[k / 3][k % 3].y;
            v += dx * dx + dy * dy;
        }
    }
    double t = block_sum(v, lds);
    if (threadIdx.x == 0) partials[(size_t)r * gridDim.x + b] = t;
}

// Re and Im of <a, b> (partials [2][nrhs][nblk])
__global__ __launch_bounds__(kBlock) void k_dot_f64(Geom g, int nb, int nrhs, const void *da, const void *db, double *partials)
{
    __shared__ double lds[8];
    int r = blockIdx.y, b = blockIdx.x;
    int p = b / nb, i = (b % nb) * kBlock + threadIdx.x;
    double re = 0.0, im = 0.0;
    if (i < g.Vh) {
        cplx<double> s[4][3], t[4][3];
        spinor_ref<P_F64>(da, nullptr, g.S, r).load(p, i, s);
        spinor_ref<P_F64>(db, nullptr, g.S, r).load(p, i, t);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            cplx<double> c = cmc(s[k / 3][k % 3], t[k / 3][k % 3]);
            re += c.x;
            im += c.y;
        }
    }
    double t0 = block_sum(re, lds);
    double t1 = block_sum(im, lds + 4);
    if (threadIdx.x == 0) {
        partials[(size_t)r * gridDim.x + b] = t0;
        partials[(size_t)(nrhs + r) * gridDim.x + b] = t1;
    }
}

__global__ __launch_bounds__(kBlock) void k_reduce(const double *partials, int nblk, double *out)
{
    __shared__ double lds[4];
    const double *src = partials + (size_t)blockIdx.x * nblk;
    double v = 0.0;
    for (int k = threadIdx.x; k < nblk; k += kBlock) v += src[k];
    double t = block_sum(v, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = t;
}

template <int PS, int PD>
__global__ __launch_bounds__(kBlock) void k_convert(Geom g, int nb, const void *ds, const float *ss, void *dd, float *sd)
{
    using TS = typename Real<PS>::T;
    using TD = typename Real<PD>::T;
    int r = blockIdx.y, b = blockIdx.x;
    int p = b / nb, i = (b % nb) * kBlock + threadIdx.x;
    if (i >= g.Vh) return;
    cplx<TS> s[4][3];
    cplx<TD> t[4][3];
    spinor_ref<PS>(ds, ss, g.S, r).load(p, i, s);
#pragma unroll
    for (int k = 0; k < 12; k++) t[k / 3][k % 3] = {(TD)s[k / 3][k % 3].x, (TD)s[k / 3][k % 3].y};
    spinor_ref<PD>(dd, sd, g.S, r).store(p, i, t);
}

// y = a x + b y computed in the precision of y's arithmetic type
template <int PX, int PY>
__global__ __launch_bounds__(kBlock) void k_axpby(Geom g, int nb, double a, const void *dx, const float *sx, double bcoef,
                                                  void *dy, float *sy)
{
    using TX = typename Real<PX>::T;
    using TY = typename Real<PY>::T;
    int r = blockIdx.y, b = blockIdx.x;
    int p = b / nb, i = (b % nb) * kBlock + threadIdx.x;
    if (i >= g.Vh) return;
    cplx<TX> s[4][3];
    cplx<TY> t[4][3];
    spinor_ref<PX>(dx, sx, g.S, r).load(p, i, s);
    auto yr = spinor_ref<PY>(dy, sy, g.S, r);
    if (bcoef != 0.0) {
        yr.load(p, i, t);
    } else {
#pragma unroll
        for (int k = 0; k < 12; k++) t[k / 3][k % 3] = {(TY)0, (TY)0};
    }
    const TY A = (TY)a, B = (TY)bcoef;
#pragma unroll
    for (int k = 0; k < 12; k++) {
        cplx<TY> &v = t[k / 3][k % 3];
        v = {fma(A, (TY)s[k / 3][k % 3].x, B * v.x), fma(A, (TY)s[k / 3][k % 3].y, B * v.y)};
    }
    yr.store(p, i, t);
}

template <int PREC>
__global__ __launch_bounds__(kBlock) void k_zero(Geom g, int nb, void *d, float *sc)
{
    using T = typename Real<PREC>::T;
    int r = blockIdx.y, b = blockIdx.x;
    int p = b / nb, i = (b % nb) * kBlock + threadIdx.x;
    if (i >= g.Vh) return;
    cplx<T> t[4][3];
#pragma unroll
    for (int k = 0; k < 12; k++) t[k / 3][k % 3] = {(T)0, (T)0};
    spinor_ref<PREC>(d, sc, g.S, r).store(p, i, t);
}

#define DISPATCH1(prec, KERNEL, ...)                                  \
    do {                                                              \
        if ((prec) == P_F64) KERNEL<P_F64><<<__VA_ARGS__>>>;          \
    } while (0)

hipError_t launch_norm2(const Lat &L, Fld f, double *partials, hipStream_t st)
{
    dim3 grid(2 * L.nb, f.nrhs);
    if (f.prec == P_F64) k_norm2<P_F64><<<grid, kBlock, 0, st>>>(L.g, L.nb, f.d, f.sc, partials);
    else if (f.prec == P_F48) k_norm2<P_F48><<<grid, kBlock, 0, st>>>(L.g, L.nb, f.d, f.sc, partials);
    else if (f.prec == P_F32) k_norm2<P_F32><<<grid, kBlock, 0, st>>>(L.g, L.nb, f.d, f.sc, partials);
    else k_norm2<P_F16S><<<grid, kBlock, 0, st>>>(L.g, L.nb, f.d, f.sc, partials);
    return hipGetLastError();
}

hipError_t launch_diff_norm2(const Lat &L, Fld a, Fld b, double *partials, hipStream_t st)
{
    dim3 grid(2 * L.nb, a.nrhs);
    if (a.prec != P_F64 || b.prec == P_F48) return hipErrorInvalidValue;
    if (b.prec == P_F64) k_diff_norm2<P_F64, P_F64><<<grid, kBlock, 0, st>>>(L.g, L.nb, a.d, a.sc, b.d, b.sc, partials);
    else if (b.prec == P_F32) k_diff_norm2<P_F64, P_F32><<<grid, kBlock, 0, st>>>(L.g, L.nb, a.d, a.sc, b.d, b.sc, partials);
    else k_diff_norm2<P_F64, P_F16S><<<grid, kBlock, 0, st>>>(L.g, L.nb, a.d, a.sc, b.d, b.sc, partials);
    return hipGetLastError();
}

hipError_t launch_dot(const Lat &L, Fld a, Fld b, double *partials, hipStream_t st)
{
    if (a.prec != P_F64 || b.prec != P_F64) return hipErrorInvalidValue;
    dim3 grid(2 * L.nb, a.nrhs);
    k_dot_f64<<<grid, kBlock, 0, st>>>(L.g, L.nb, a.nrhs, a.d, b.d, partials);
    return hipGetLastError();
}

hipError_t launch_reduce(const double *partials, int nq, int nrhs, int nblk, double *out, hipStream_t st)
{
    k_reduce<<<nq * nrhs, kBlock, 0, st>>>(partials, nblk, out);
    return hipGetLastError();
}

template <int PS>
static hipError_t convert_to(const Lat &L, Fld s, Fld d, hipStream_t st)
{
    dim3 grid(2 * L.nb, s.nrhs);
    if (d.prec == P_F64) k_convert<PS, P_F64><<<grid, kBlock, 0, st>>>(L.g, L.nb, s.d, s.sc, d.d, d.sc);
    else if (d.prec == P_F48) k_convert<PS, P_F48><<<grid, kBlock, 0, st>>>(L.g, L.nb, s.d, s.sc, d.d, d.sc);
    else if (d.prec == P_F32) k_convert<PS, P_F32><<<grid, kBlock, 0, st>>>(L.g, L.nb, s.d, s.sc, d.d, d.sc);
    else k_convert<PS, P_F16S><<<grid, kBlock, 0, st>>>(L.g, L.nb, s.d, s.sc, d.d, d.sc);
    return hipGetLastError();
}

hipError_t launch_convert(const Lat &L, Fld s, Fld d, hipStream_t st)
{
    if (s.prec == P_F64) return convert_to<P_F64>(L, s, d, st);
    if (s.prec == P_F48) return convert_to<P_F48>(L, s, d, st);
    if (s.prec == P_F32) return convert_to<P_F32>(L, s, d, st);
    return convert_to<P_F16S>(L, s, d, st);
}

template <int PX>
static hipError_t axpby_to(const Lat &L, double a, Fld x, double b, Fld y, hipStream_t st)
{
    dim3 grid(2 * L.nb, x.nrhs);
    if (y.prec == P_F64) k_axpby<PX, P_F64><<<grid, kBlock, 0, st>>>(L.g, L.nb, a, x.d, x.sc, b, y.d, y.sc);
    else if (y.prec == P_F32) k_axpby<PX, P_F32><<<grid, kBlock, 0, st>>>(L.g, L.nb, a, x.d, x.sc, b, y.d, y.sc);
    else k_axpby<PX, P_F16S><<<grid, kBlock, 0, st>>>(L.g, L.nb, a, x.d, x.sc, b, y.d, y.sc);
    return hipGetLastError();
}

hipError_t launch_axpby(const Lat &L, double a, Fld x, double b, Fld y, hipStream_t st)
{
    if (x.prec == P_F48 || y.prec == P_F48) return hipErrorInvalidValue;   // not needed on 48-bit fields
    if (x.prec == P_F64) return axpby_to<P_F64>(L, a, x, b, y, st);
    if (x.prec == P_F32) return axpby_to<P_F32>(L, a, x, b, y, st);
    return axpby_to<P_F16S>(L, a, x, b, y, st);
}

hipError_t launch_zero(const Lat &L, Fld f, hipStream_t st)
{
    dim3 grid(2 * L.nb, f.nrhs);
    if (f.prec == P_F64) k_zero<P_F64><<<grid, kBlock, 0, st>>>(L.g, L.nb, f.d, f.sc);
    else if (f.prec == P_F48) k_zero<P_F48><<<grid, kBlock, 0, st>>>(L.g, L.nb, f.d, f.sc);
    else if (f.prec == P_F32) k_zero<P_F32><<<grid, kBlock, 0, st>>>(L.g, L.nb, f.d, f.sc);
    else k_zero<P_F16S><<<grid, kBlock, 0, st>>>(L.g, L.nb, f.d, f.sc);
    return hipGetLastError();
}

}  // namespace ovl
