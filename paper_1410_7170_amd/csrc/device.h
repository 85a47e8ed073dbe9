// Device-side building blocks for the gfx950 overlap library: complex
// arithmetic, the even-odd field layouts of ovl.h, field loads/stores per
// storage precision, the XCD-aware block mapping and deterministic block
// reductions.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ovl {

constexpr int kBlock = 256;     // threads per block of every site-parallel kernel
constexpr int kNumXcd = 8;      // MI355X: 8 accelerator complex dies, each with its own L2

template <typename T>
struct cplx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> mk(T x, T y) { return {x, y}; }
template <typename T>
__device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> operator*(T s, cplx<T> a) { return {s * a.x, s * a.y}; }
// i*a and -i*a
template <typename T>
__device__ __forceinline__ cplx<T> ti(cplx<T> a) { return {-a.y, a.x}; }
template <typename T>
__device__ __forceinline__ cplx<T> tmi(cplx<T> a) { return {a.y, -a.x}; }
// a*b
template <typename T>
__device__ __forceinline__ cplx<T> cm(cplx<T> a, cplx<T> b)
{
    return {fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x)};
}
// conj(a)*b
template <typename T>
__device__ __forceinline__ cplx<T> cmc(cplx<T> a, cplx<T> b)
{
    return {fma(a.x, b.x, a.y * b.y), fma(a.x, b.y, -a.y * b.x)};
}
// acc + a*b, acc + conj(a)*b and acc - a*b as four fused multiply-adds
// (sums of products chain through the accumulator instead of adding
// separately rounded products)
template <typename T>
__device__ __forceinline__ cplx<T> cmac(cplx<T> acc, cplx<T> a, cplx<T> b)
{
    return {fma(-a.y, b.y, fma(a.x, b.x, acc.x)), fma(a.y, b.x, fma(a.x, b.y, acc.y))};
}
template <typename T>
__device__ __forceinline__ cplx<T> cmacc(cplx<T> acc, cplx<T> a, cplx<T> b)
{
    return {fma(a.y, b.y, fma(a.x, b.x, acc.x)), fma(-a.y, b.x, fma(a.x, b.y, acc.y))};
}
template <typename T>
__device__ __forceinline__ cplx<T> cmsub(cplx<T> acc, cplx<T> a, cplx<T> b)
{
    return {fma(a.y, b.y, fma(-a.x, b.x, acc.x)), fma(-a.y, b.x, fma(-a.x, b.y, acc.y))};
}
// acc + s*a for a real s
template <typename T>
__device__ __forceinline__ cplx<T> fmac(cplx<T> acc, T s, cplx<T> a)
{
    return {fma(s, a.x, acc.x), fma(s, a.y, acc.y)};
}
template <typename T>
__device__ __forceinline__ T norm2(cplx<T> a) { return fma(a.x, a.x, a.y * a.y); }

// ---------------------------------------------------------------- geometry
// Site (parity p, checkerboard index i): lexicographic index 2*i or 2*i+1,
// whichever has parity p; lex = ((x0*L1 + x1)*L2 + x2)*L3 + x3 with L3 even.
struct Geom {
    int L[4];
    int bc[4];
    int Vh;        // V/2 sites per parity
    int S;         // element stride between the component arrays of a field:
                   // V/2 rounded up to 16, plus 24, so that components do not
                   // sit a power of two apart (which maps all of a site's
                   // components to the same L2 set and HBM channel)
    int T;         // time-tile length of the stencil's site order (divides L0)
    int Ts;        // time slices per thread of the time-streaming stencil (0: not used)
    int Ts64;      // time slices per thread of the FP64 streaming stencil (0: Ts)
    int Kr;        // log2 of the RHS tile of the streaming stencil (lanes per site)
    int Mfma;      // FP32 D_W on several RHS by the matrix-core stencil
};

// Threads (sites) per block of the time-streaming stencil with ts slices per
// thread: 256, or 192 when whole x3 rows tile 192 sites but not 256 (x3
// extents such as 24 and 48), so that the LDS-staged build applies.  192 only
// with ts >= 2, which keeps the block count per RHS within the 2*nb
// partial-sum slots.
inline int stream_threads(const Geom &g, int ts)
{
    const int L2 = g.L[2], L3 = g.L[3];
    const long V3 = (long)g.L[1] * L2 * L3;
    const bool rows256 = kBlock % L3 == 0 && (L2 * L3) % kBlock == 0;
    const bool rows192 = 192 % L3 == 0 && (L2 * L3) % 192 == 0 && V3 % 192 == 0;
    return !rows256 && rows192 && ts >= 2 ? 192 : kBlock;
}

__host__ __device__ inline int padded_stride(int Vh) { return ((Vh + 15) / 16) * 16 + 24; }

__device__ __forceinline__ void site_coords(const Geom &g, int p, int i, int x[4])
{
    int lb = 2 * i;
    int x3e = lb % g.L[3];
    int t = lb / g.L[3];
    x[2] = t % g.L[2];
    t /= g.L[2];
    x[1] = t % g.L[1];
    x[0] = t / g.L[1];
    x[3] = x3e + ((p + x[0] + x[1] + x[2]) & 1);
}

// Stencil site order.  Logical index j within a parity walks
// (t-tile, x1, t within the tile, x2, x3): consecutive blocks sweep one
// x2-x3 plane after another through T time slices before moving to the next
// x1, so a site's +-t neighbours are touched again one plane later and its
// +-x1 neighbours one T-plane column later -- short enough reuse distances
// for one XCD's L2.  Threads of a wave stay on consecutive x3 of one plane,
// i.e. on consecutive memory.
__device__ __forceinline__ void tiled_coords(const Geom &g, int p, int j, int x[4])
{
    const int l3h = g.L[3] >> 1;
    int x3h = j % l3h;
    int q = j / l3h;
    x[2] = q % g.L[2];
    q /= g.L[2];
    int tt = q % g.T;
    q /= g.T;
    x[1] = q % g.L[1];
    x[0] = (q / g.L[1]) * g.T + tt;
    x[3] = 2 * x3h + ((p + x[0] + x[1] + x[2]) & 1);
}

__device__ __forceinline__ int cb_index(const Geom &g, const int x[4])
{
    return ((((x[0] * g.L[1] + x[1]) * g.L[2] + x[2]) * g.L[3]) + x[3]) >> 1;
}

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8).  Give every XCD one contiguous range of logical blocks so that the
// neighbours one block row away are in the same L2.
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    int q = nb / kNumXcd, r = nb % kNumXcd;
    int xcd = b % kNumXcd, k = b / kNumXcd;
    return xcd * q + (xcd < r ? xcd : r) + k;
}

// Streaming stores that do not allocate in L2 (outputs of the stencil are
// not read again by the same kernel, and keeping them out of L2 leaves room
// for the neighbour reuse of the inputs).
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef unsigned int nt_u4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void st_nt(double2 *p, double x, double y)
{
    nt_d2 t = {x, y};
    __builtin_nontemporal_store(t, (nt_d2 *)p);
}
__device__ __forceinline__ void st_nt(float4 *p, float a, float b, float c, float d)
{
    nt_f4 t = {a, b, c, d};
    __builtin_nontemporal_store(t, (nt_f4 *)p);
}
__device__ __forceinline__ void st_nt(uint4 *p, unsigned a, unsigned b, unsigned c, unsigned d)
{
    nt_u4 t = {a, b, c, d};
    __builtin_nontemporal_store(t, (nt_u4 *)p);
}

// ---------------------------------------------------------------- fields
// P_F48: FP64 arithmetic on fields stored in 48 bits per real (a double
// rounded to nearest at 36 stored mantissa bits, relative error <= 2^-37);
// its gauge links are the FP64 ones.
enum { P_F64 = 0, P_F32 = 1, P_F16S = 2, P_F48 = 3 };

template <int PREC>
struct Real {
    using T = float;
};
template <>
struct Real<P_F64> {
    using T = double;
};
template <>
struct Real<P_F48> {
    using T = double;
};

// A spinor field of one RHS: pointer to its parity-0 component-0 element.
// The member named Vh is the component stride (Geom::S) of the layout.
template <int PREC>
struct SpinorRef;

template <>
struct SpinorRef<P_F64> {
    double2 *d;
    int Vh;
    __device__ __forceinline__ void load(int p, int i, cplx<double> s[4][3]) const
    {
        const double2 *b = d + (size_t)p * 12 * Vh + i;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            double2 v = b[(size_t)k * Vh];
            s[k / 3][k % 3] = {v.x, v.y};
        }
    }
    // non-temporal: a centre operand read once
    __device__ __forceinline__ void load_nt(int p, int i, cplx<double> s[4][3]) const
    {
        const double2 *b = d + (size_t)p * 12 * Vh + i;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            nt_d2 v = __builtin_nontemporal_load((const nt_d2 *)&b[(size_t)k * Vh]);
            s[k / 3][k % 3] = {v.x, v.y};
        }
    }
    __device__ __forceinline__ void store(int p, int i, const cplx<double> s[4][3]) const
    {
        double2 *b = d + (size_t)p * 12 * Vh + i;
#pragma unroll
        for (int k = 0; k < 12; k++) b[(size_t)k * Vh] = make_double2(s[k / 3][k % 3].x, s[k / 3][k % 3].y);
    }
    __device__ __forceinline__ void store_nt(int p, int i, const cplx<double> s[4][3]) const
    {
        double2 *b = d + (size_t)p * 12 * Vh + i;
#pragma unroll
        for (int k = 0; k < 12; k++) st_nt(&b[(size_t)k * Vh], s[k / 3][k % 3].x, s[k / 3][k % 3].y);
    }
};

template <>
struct SpinorRef<P_F32> {
    float4 *d;
    int Vh;
    __device__ __forceinline__ void load(int p, int i, cplx<float> s[4][3]) const
    {
        const float4 *b = d + (size_t)p * 6 * Vh + i;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            float4 v = b[(size_t)k * Vh];
            s[(2 * k) / 3][(2 * k) % 3] = {v.x, v.y};
            s[(2 * k + 1) / 3][(2 * k + 1) % 3] = {v.z, v.w};
        }
    }
    __device__ __forceinline__ void load_nt(int p, int i, cplx<float> s[4][3]) const
    {
        const float4 *b = d + (size_t)p * 6 * Vh + i;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            nt_f4 v = __builtin_nontemporal_load((const nt_f4 *)&b[(size_t)k * Vh]);
            s[(2 * k) / 3][(2 * k) % 3] = {v.x, v.y};
            s[(2 * k + 1) / 3][(2 * k + 1) % 3] = {v.z, v.w};
        }
    }
    __device__ __forceinline__ void store(int p, int i, const cplx<float> s[4][3]) const
    {
        float4 *b = d + (size_t)p * 6 * Vh + i;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            cplx<float> a = s[(2 * k) / 3][(2 * k) % 3], c = s[(2 * k + 1) / 3][(2 * k + 1) % 3];
            b[(size_t)k * Vh] = make_float4(a.x, a.y, c.x, c.y);
        }
    }
    __device__ __forceinline__ void store_nt(int p, int i, const cplx<float> s[4][3]) const
    {
        float4 *b = d + (size_t)p * 6 * Vh + i;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            cplx<float> a = s[(2 * k) / 3][(2 * k) % 3], c = s[(2 * k + 1) / 3][(2 * k + 1) % 3];
            st_nt(&b[(size_t)k * Vh], a.x, a.y, c.x, c.y);
        }
    }
};

__device__ __forceinline__ float h2f(unsigned short h) { return __half2float(__ushort_as_half(h)); }
__device__ __forceinline__ unsigned short f2h(float f) { return __half_as_ushort(__float2half_rn(f)); }

template <>
struct SpinorRef<P_F16S> {
    uint4 *d;     // 8 halves = 4 complex components per element
    float *sc;    // per-site scale
    int Vh;
    __device__ __forceinline__ void load(int p, int i, cplx<float> s[4][3]) const
    {
        const uint4 *b = d + (size_t)p * 3 * Vh + i;
        float scale = sc[(size_t)p * Vh + i];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            uint4 v = b[(size_t)k * Vh];
            unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int q = 0; q < 4; q++) {
                int c = 4 * k + q;
                s[c / 3][c % 3] = {scale * h2f((unsigned short)(w[q] & 0xffff)),
                                   scale * h2f((unsigned short)(w[q] >> 16))};
            }
        }
    }
    __device__ __forceinline__ void load_nt(int p, int i, cplx<float> s[4][3]) const { load(p, i, s); }
    __device__ __forceinline__ void store_nt(int p, int i, const cplx<float> s[4][3]) const { store(p, i, s); }
    __device__ __forceinline__ void store(int p, int i, const cplx<float> s[4][3]) const
    {
        float m = 0.f;
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int c = 0; c < 3; c++) m = fmaxf(m, fmaxf(fabsf(s[a][c].x), fabsf(s[a][c].y)));
        float scale = m > 0.f ? m : 1.f;
        float inv = 1.f / scale;
        uint4 *b = d + (size_t)p * 3 * Vh + i;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            unsigned w[4];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                int c = 4 * k + q;
                w[q] = (unsigned)f2h(s[c / 3][c % 3].x * inv) | ((unsigned)f2h(s[c / 3][c % 3].y * inv) << 16);
            }
            b[(size_t)k * Vh] = make_uint4(w[0], w[1], w[2], w[3]);
        }
        sc[(size_t)p * Vh + i] = scale;
    }
};

// 48-bit storage of a double: the top 48 bits of its IEEE pattern after
// rounding the dropped 16 bits to nearest (ties away from zero; a carry moves
// into the exponent as it should).  Infinities and NaNs keep their top bits.
__device__ __forceinline__ unsigned long long f48_bits(double x)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    const bool special = (u & 0x7ff0000000000000ull) == 0x7ff0000000000000ull;
    return special ? u : u + 0x8000ull;
}
__device__ __forceinline__ double f48_value(unsigned hi, unsigned lo16)
{
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | ((unsigned long long)lo16 << 16)));
}
__device__ __forceinline__ unsigned f48_hi(unsigned long long b) { return (unsigned)(b >> 32); }
__device__ __forceinline__ unsigned f48_lo(unsigned long long b) { return (unsigned)(b >> 16) & 0xffffu; }

// The 48-bit layout: per site and parity 9 arrays of 16-byte elements (stride
// Vh).  Arrays 0..5 hold the top 32 bits of complex numbers 2k and 2k+1
// (re, im, re, im); arrays 6..8 the low 16 bits of complex numbers 4g..4g+3,
// word q = lo(re) | lo(im) << 16.  Complex number k is spin k/3, colour k%3.
struct F48Code {
    uint4 h[6], l[3];
};
__device__ __forceinline__ void f48_decode(const F48Code &c, cplx<double> s[4][3])
{
#pragma unroll
    for (int k = 0; k < 12; k++) {
        const uint4 &h = c.h[k / 2];
        const uint4 &l = c.l[k / 4];
        const unsigned hr = (k & 1) ? h.z : h.x, hi = (k & 1) ? h.w : h.y;
        const unsigned lw = (k & 3) == 0 ? l.x : (k & 3) == 1 ? l.y : (k & 3) == 2 ? l.z : l.w;
        s[k / 3][k % 3] = {f48_value(hr, lw & 0xffffu), f48_value(hi, lw >> 16)};
    }
}
__device__ __forceinline__ void f48_encode(const cplx<double> s[4][3], F48Code &c)
{
    unsigned hw[24], lw[12];
#pragma unroll
    for (int k = 0; k < 12; k++) {
        const unsigned long long br = f48_bits(s[k / 3][k % 3].x), bi = f48_bits(s[k / 3][k % 3].y);
        hw[2 * k] = f48_hi(br);
        hw[2 * k + 1] = f48_hi(bi);
        lw[k] = f48_lo(br) | (f48_lo(bi) << 16);
    }
#pragma unroll
    for (int k = 0; k < 6; k++) c.h[k] = make_uint4(hw[4 * k], hw[4 * k + 1], hw[4 * k + 2], hw[4 * k + 3]);
#pragma unroll
    for (int g = 0; g < 3; g++) c.l[g] = make_uint4(lw[4 * g], lw[4 * g + 1], lw[4 * g + 2], lw[4 * g + 3]);
}

template <>
struct SpinorRef<P_F48> {
    uint4 *d;
    int Vh;
    __device__ __forceinline__ void load_raw(int p, int i, F48Code &c) const
    {
        const uint4 *b = d + (size_t)p * 9 * Vh + i;
#pragma unroll
        for (int k = 0; k < 6; k++) c.h[k] = b[(size_t)k * Vh];
#pragma unroll
        for (int k = 0; k < 3; k++) c.l[k] = b[(size_t)(6 + k) * Vh];
    }
    __device__ __forceinline__ void load(int p, int i, cplx<double> s[4][3]) const
    {
        F48Code c;
        load_raw(p, i, c);
        f48_decode(c, s);
    }
    __device__ __forceinline__ void load_nt(int p, int i, cplx<double> s[4][3]) const
    {
        const uint4 *b = d + (size_t)p * 9 * Vh + i;
        F48Code c;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            nt_u4 v = __builtin_nontemporal_load((const nt_u4 *)&b[(size_t)k * Vh]);
            c.h[k] = make_uint4(v.x, v.y, v.z, v.w);
        }
#pragma unroll
        for (int k = 0; k < 3; k++) {
            nt_u4 v = __builtin_nontemporal_load((const nt_u4 *)&b[(size_t)(6 + k) * Vh]);
            c.l[k] = make_uint4(v.x, v.y, v.z, v.w);
        }
        f48_decode(c, s);
    }
    __device__ __forceinline__ void store(int p, int i, const cplx<double> s[4][3]) const
    {
        uint4 *b = d + (size_t)p * 9 * Vh + i;
        F48Code c;
        f48_encode(s, c);
#pragma unroll
        for (int k = 0; k < 6; k++) b[(size_t)k * Vh] = c.h[k];
#pragma unroll
        for (int k = 0; k < 3; k++) b[(size_t)(6 + k) * Vh] = c.l[k];
    }
    __device__ __forceinline__ void store_nt(int p, int i, const cplx<double> s[4][3]) const
    {
        uint4 *b = d + (size_t)p * 9 * Vh + i;
        F48Code c;
        f48_encode(s, c);
#pragma unroll
        for (int k = 0; k < 6; k++) st_nt(&b[(size_t)k * Vh], c.h[k].x, c.h[k].y, c.h[k].z, c.h[k].w);
#pragma unroll
        for (int k = 0; k < 3; k++) st_nt(&b[(size_t)(6 + k) * Vh], c.l[k].x, c.l[k].y, c.l[k].z, c.l[k].w);
    }
};

// Elements (in the pointer's own unit) of one RHS in each layout, S = stride.
__host__ __device__ inline size_t spinor_elems(int prec, int S)
{
    return prec == P_F64 ? (size_t)24 * S : prec == P_F32 ? (size_t)12 * S : prec == P_F48 ? (size_t)18 * S
                                                                                            : (size_t)6 * S;
}

// Gauge links.  Every precision keeps rows 0 and 1 and rebuilds
// row 2 = conj(row0 x row1), which holds for every SU(3) matrix.
template <int PREC>
struct GaugeRef;

template <typename T>
__device__ __forceinline__ void rebuild_row2(cplx<T> u[3][3])
{
    cplx<T> a = cmsub(cm(u[0][1], u[1][2]), u[0][2], u[1][1]);
    cplx<T> b = cmsub(cm(u[0][2], u[1][0]), u[0][0], u[1][2]);
    cplx<T> c = cmsub(cm(u[0][0], u[1][1]), u[0][1], u[1][0]);
    u[2][0] = {a.x, -a.y};
    u[2][1] = {b.x, -b.y};
    u[2][2] = {c.x, -c.y};
}

template <>
struct GaugeRef<P_F64> {
    const double2 *d;   // rows 0 and 1 (6 complex entries)
    int Vh;
    __device__ __forceinline__ void load(int p, int mu, int i, cplx<double> u[3][3]) const
    {
        const double2 *b = d + (size_t)(p * 4 + mu) * 6 * Vh + i;
#pragma unroll
        for (int e = 0; e < 6; e++) {
            double2 v = b[(size_t)e * Vh];
            u[e / 3][e % 3] = {v.x, v.y};
        }
        rebuild_row2(u);
    }
    // non-temporal: a link read once per launch (the time links of the
    // streaming stencil)
    __device__ __forceinline__ void load_nt(int p, int mu, int i, cplx<double> u[3][3]) const
    {
        const double2 *b = d + (size_t)(p * 4 + mu) * 6 * Vh + i;
#pragma unroll
        for (int e = 0; e < 6; e++) {
            nt_d2 v = __builtin_nontemporal_load((const nt_d2 *)&b[(size_t)e * Vh]);
            u[e / 3][e % 3] = {v.x, v.y};
        }
        rebuild_row2(u);
    }
};

template <>
struct GaugeRef<P_F32> {
    const float4 *d;
    int Vh;
    __device__ __forceinline__ void load(int p, int mu, int i, cplx<float> u[3][3]) const
    {
        const float4 *b = d + (size_t)(p * 4 + mu) * 3 * Vh + i;
        float4 v0 = b[0], v1 = b[(size_t)Vh], v2 = b[(size_t)2 * Vh];
        u[0][0] = {v0.x, v0.y};
        u[0][1] = {v0.z, v0.w};
        u[0][2] = {v1.x, v1.y};
        u[1][0] = {v1.z, v1.w};
        u[1][1] = {v2.x, v2.y};
        u[1][2] = {v2.z, v2.w};
        rebuild_row2(u);
    }
    __device__ __forceinline__ void load_nt(int p, int mu, int i, cplx<float> u[3][3]) const
    {
        const float4 *b = d + (size_t)(p * 4 + mu) * 3 * Vh + i;
        nt_f4 v0 = __builtin_nontemporal_load((const nt_f4 *)&b[0]);
        nt_f4 v1 = __builtin_nontemporal_load((const nt_f4 *)&b[(size_t)Vh]);
        nt_f4 v2 = __builtin_nontemporal_load((const nt_f4 *)&b[(size_t)2 * Vh]);
        u[0][0] = {v0.x, v0.y};
        u[0][1] = {v0.z, v0.w};
        u[0][2] = {v1.x, v1.y};
        u[1][0] = {v1.z, v1.w};
        u[1][1] = {v2.x, v2.y};
        u[1][2] = {v2.z, v2.w};
        rebuild_row2(u);
    }
};

// 48-bit fields use the FP64 links.
template <>
struct GaugeRef<P_F48> : GaugeRef<P_F64> {
};

template <int PREC>
__device__ __forceinline__ GaugeRef<PREC> gauge_ref(const void *U, int S)
{
    GaugeRef<PREC> g;
    g.d = (decltype(g.d))U;
    g.Vh = S;
    return g;
}

template <>
struct GaugeRef<P_F16S> {
    const uint2 *d;   // 4 halves = 2 complex entries per element
    int Vh;
    __device__ __forceinline__ void load(int p, int mu, int i, cplx<float> u[3][3]) const
    {
        const uint2 *b = d + (size_t)(p * 4 + mu) * 3 * Vh + i;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            uint2 v = b[(size_t)k * Vh];
            int e0 = 2 * k, e1 = 2 * k + 1;
            u[e0 / 3][e0 % 3] = {h2f((unsigned short)(v.x & 0xffff)), h2f((unsigned short)(v.x >> 16))};
            u[e1 / 3][e1 % 3] = {h2f((unsigned short)(v.y & 0xffff)), h2f((unsigned short)(v.y >> 16))};
        }
        rebuild_row2(u);
    }
    __device__ __forceinline__ void load_nt(int p, int mu, int i, cplx<float> u[3][3]) const { load(p, mu, i, u); }
};

// ---------------------------------------------------------------- reductions
// Sum over a 256-thread block, result valid in thread 0.  Fixed shuffle/LDS
// order, so the result is bitwise reproducible for a given launch shape.
__device__ __forceinline__ double block_sum(double v, double *lds /* >= 4 */)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) t = (lds[0] + lds[1]) + (lds[2] + lds[3]);
    __syncthreads();
    return t;
}

// The same over a block of NW waves (block_sum is NW = 4).
template <int NW>
__device__ __forceinline__ double block_sum_w(double v, double *lds /* >= 4 */)
{
    if constexpr (NW == 4) {
        return block_sum(v, lds);
    } else {
        static_assert(NW == 3, "block_sum_w: 3 or 4 waves");
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) lds[w] = v;
        __syncthreads();
        double t = 0.0;
        if (threadIdx.x == 0) t = (lds[0] + lds[1]) + lds[2];
        __syncthreads();
        return t;
    }
}

// Sums over the lanes of a block of NW waves whose RHS is the lane index
// modulo K = 2^kr (K <= 8): the sum for RHS q is valid in thread q < K.  The
// shuffles skip the offsets below K, then thread q adds the NW wave sums in
// the fixed order of block_sum_w, so K = 1 gives block_sum_w's bits.
template <int NW>
__device__ __forceinline__ double block_sum_k(double v, double *lds /* >= NW * 8 */, int kr)
{
    const int K = 1 << kr;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        if (off >= K) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6, ln = threadIdx.x & 63;
    if (ln < K) lds[w * K + ln] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x < K) {
        const int q = threadIdx.x;
        if constexpr (NW == 4) t = (lds[q] + lds[K + q]) + (lds[2 * K + q] + lds[3 * K + q]);
        else t = (lds[q] + lds[K + q]) + lds[2 * K + q];
    }
    __syncthreads();
    return t;
}

// The same sum, valid in every thread (each adds the four wave sums in the
// same order, so all threads hold the same bits as block_sum's thread 0).
__device__ __forceinline__ double block_sum_all(double v, double *lds /* >= 4 */)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double t = (lds[0] + lds[1]) + (lds[2] + lds[3]);
    __syncthreads();
    return t;
}

}  // namespace ovl
