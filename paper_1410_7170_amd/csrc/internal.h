// Host-side declarations shared by the library's translation units.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "../../include/ovl.h"
#include "device.h"
#include "wilson.h"

namespace ovl {

struct Lat {
    Geom g;
    int64_t V;
    int Vh;
    int nb;        // blocks per parity of a site-parallel launch
};

Lat make_lat(const ovl_lattice *lat);

// record a failed HIP call; returns OVL_ERR_HIP
int hip_fail(hipError_t e);
#define OVL_HIP(call)                                   \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return ::ovl::hip_fail(e_); \
    } while (0)

// bytes of one packed field (one RHS) of precision prec, excluding scales:
// 2 parities x (12, 9, 6 or 3) component arrays of 16-byte elements, padded stride
inline size_t field_bytes(int prec, int64_t V)
{
    size_t S = (size_t)padded_stride((int)(V / 2));
    return prec == P_F64 ? 24 * S * 16 : prec == P_F48 ? 18 * S * 16 : prec == P_F32 ? 12 * S * 16 : 6 * S * 16;
}
// per-site scales of one F16S field: 2 parities x S floats
inline size_t scale_bytes(int64_t V) { return (size_t)2 * padded_stride((int)(V / 2)) * 4; }
inline size_t scale_floats(int64_t V) { return (size_t)2 * padded_stride((int)(V / 2)); }
// packed gauge field: 2 parities x 4 directions x (6 F64 | 3 F32 | 3 F16) arrays
inline size_t gauge_field_bytes(int prec, int64_t V)
{
    size_t S = (size_t)padded_stride((int)(V / 2));
    return prec == P_F64 ? 48 * S * 16 : prec == P_F32 ? 24 * S * 16 : 24 * S * 8;
}

// A packed field set of nrhs fields (device pointers).
struct Fld {
    void *d;
    float *sc;
    int prec;
    int nrhs;
};
inline Fld fld(const ovl_spinor *s) { return {s->d, s->scale, s->prec, s->nrhs}; }
// field k of a field set with `per` fields per group, e.g. shift j, rhs r
inline Fld sub(const Fld &f, int64_t V, int first, int count)
{
    Fld o = f;
    o.d = (char *)f.d + field_bytes(f.prec, V) * first;
    o.sc = f.sc ? f.sc + scale_floats(V) * first : nullptr;
    o.nrhs = count;
    return o;
}

// ---- launchers (return hipError_t of the launch)
// e0, e1 (optional): events the launch records at the stencil's start and end
hipError_t launch_wilson(const Lat &L, int prec, int mode, bool g5, WArgs a, hipStream_t st, hipEvent_t e0 = nullptr,
                         hipEvent_t e1 = nullptr);

// A kernel launch that, given events, has its own dispatch record them at the
// kernel's start and end (no marker packets in the queue); args must have the
// kernel's parameter types.
template <typename F, typename... A>
inline void launch_k(F kern, dim3 grid, dim3 block, hipStream_t st, hipEvent_t e0, hipEvent_t e1, A... args)
{
    if (e0) hipExtLaunchKernelGGL(kern, grid, block, 0, st, e0, e1, 0, args...);
    else hipLaunchKernelGGL(kern, grid, block, 0, st, args...);
}
// FP32 D_W (or Gamma_5 D_W) on the matrix cores (wilson_mfma.hip); a.g set
hipError_t launch_wilson_mfma(const Lat &L, bool g5, const WArgs &a, hipStream_t st);
hipError_t launch_pack_spinor(const Lat &L, const void *canon, Fld out, hipStream_t st);
hipError_t launch_unpack_spinor(const Lat &L, Fld in, void *canon, hipStream_t st);
hipError_t launch_pack_gauge(const Lat &L, const void *canon, int prec, void *out, hipStream_t st);
// per-block partial sums of |f_r|^2 (or Re/Im <a_r, b_r> when b != null)
hipError_t launch_norm2(const Lat &L, Fld f, double *partials, hipStream_t st);
hipError_t launch_diff_norm2(const Lat &L, Fld a, Fld b, double *partials, hipStream_t st);
hipError_t launch_dot(const Lat &L, Fld a, Fld b, double *partials, hipStream_t st);
// out[q*nrhs + r] = sum of partials[(q*nrhs + r)*nblk ...]
hipError_t launch_reduce(const double *partials, int nq, int nrhs, int nblk, double *out, hipStream_t st);
// y = a*x + b*y (FP64 or FP32 fields; per-RHS coefficients on device or host)
hipError_t launch_convert(const Lat &L, Fld src, Fld dst, hipStream_t st);
hipError_t launch_axpby(const Lat &L, double a, Fld x, double b, Fld y, hipStream_t st);
hipError_t launch_zero(const Lat &L, Fld f, hipStream_t st);
// FP64 field-set kernels (outer.hip), grids of site_blocks(L) blocks:
// partials[2][nv][nblk] of <V_f, w> for the nv fields V_f (grid.y = nv);
// w += sgn sum_f (coef[f] + i coef[nv+f]) V_f (coef on the device);
// out = Gamma_5 in per field (grid.y = fields; in place allowed)
__global__ void k_mdot(Geom g, int nb, int nv, const double2 *V, const double2 *w, double *partials);
__global__ void k_mcaxpy(Geom g, int nb, int nv, const double *coef, double sgn, const double2 *V, double2 *w);
__global__ void k_gamma5(Geom g, int nb, const double2 *in, double2 *out);

int elems_per_field(int prec, int Vh);   // flat vector elements of one RHS
int site_blocks(const Lat &L);           // blocks of a flat elementwise launch over one field
// Launch shape of a stencil of precision prec on nrhs fields.  ts > 0: the
// time-streaming form with ts slices per thread, blocks of nt threads, K = 2^kr
// lanes per site (RHS tile) and nt >> kr sites per block; ts = 0: one thread
// per site and RHS.  blocks_per_tile: blocks of one RHS tile (each fills one
// partial-sum slot per RHS of the tile).
struct StencilShape {
    int ts, nt, kr, blocks_per_tile, ntile;
};
StencilShape stencil_shape(const Lat &L, int prec, int nrhs);
// Leading per-RHS partial-sum slots a stencil launch of this precision on
// nrhs fields fills; it zeroes the rest of the site_blocks(L) slots, so a
// consumer may sum only these (the same sum bit for bit).
int stencil_partials(const Lat &L, int prec, int nrhs);

// Even-odd reduced Wilson solve (wilson_eo.hip): D_W(m0) x = b per RHS, to
// |b - D_W x| <= tol |b| (true_res) or maxiter CGLS iterations (iters).
size_t wilson_solve_eo_ws_bytes(const Lat &L);
int wilson_solve_eo(const Lat &L, const ovl_gauge *U, double m0, Fld b, Fld x, double tol, int maxiter,
                    double *true_res, int *iters, char *ws, size_t ws_bytes, hipStream_t st);

}  // namespace ovl
