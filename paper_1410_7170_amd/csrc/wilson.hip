// Launch of the Wilson stencil kernels (wilson.h): blocks of 256 sites (192
// for the streaming form on some extents), ordered (site block, RHS) and
// spread over the XCDs by the kernel itself.
#include "internal.h"

namespace ovl {

template <int PREC, int WPE, bool STAGE, int NT = kBlock>
static void wilson_ts_dispatch_s(int mode, bool g5, dim3 grid, const WArgs &a, hipStream_t st)
{
    if (g5) {
        switch (mode) {
        case W_PLAIN: k_wilson_ts<PREC, W_PLAIN, true, WPE, STAGE, NT><<<grid, NT, 0, st>>>(a); break;
        case W_NORM: k_wilson_ts<PREC, W_NORM, true, WPE, STAGE, NT><<<grid, NT, 0, st>>>(a); break;
        case W_SHIFT: k_wilson_ts<PREC, W_SHIFT, true, WPE, STAGE, NT><<<grid, NT, 0, st>>>(a); break;
        case W_RUPDATE: k_wilson_ts<PREC, W_RUPDATE, true, WPE, STAGE, NT><<<grid, NT, 0, st>>>(a); break;
        default: k_wilson_ts<PREC, W_RESNORM, true, WPE, STAGE, NT><<<grid, NT, 0, st>>>(a); break;
        }
    } else {
        k_wilson_ts<PREC, W_PLAIN, false, WPE, STAGE, NT><<<grid, NT, 0, st>>>(a);
    }
}

// Blocks of whole x3 rows of consecutive x2 at one x1 take the one-wave build
// that stages each slice in LDS, at any grid size (at 32^3x64 it beats the
// two-wave build for one field, 411 against 456 us in FP64, and for batches
// of 7 fields, 2.7 against 2.9 ms); blocks of 192 sites (nt, from
// stream_threads) exist only for that build.  Otherwise launches of at most
// 512 blocks take the one-wave build without staging, larger grids the
// two-wave build.
template <int PREC>
static void wilson_ts_dispatch(int mode, bool g5, dim3 grid, int nt, const WArgs &a, hipStream_t st)
{
    if constexpr (PREC != P_F16S) {
        if (nt == 192) {
            wilson_ts_dispatch_s<PREC, 1, true, 192>(mode, g5, grid, a, st);
            return;
        }
    }
    const int L2 = a.g.L[2], L3 = a.g.L[3];
    const bool rows = kBlock % L3 == 0 && (L2 * L3) % kBlock == 0;
    if (rows) {
        wilson_ts_dispatch_s<PREC, 1, true>(mode, g5, grid, a, st);
    } else if (grid.x <= 512) {
        wilson_ts_dispatch_s<PREC, 1, false>(mode, g5, grid, a, st);
    } else {
        wilson_ts_dispatch_s<PREC, 2, false>(mode, g5, grid, a, st);
    }
}

template <int PREC>
static void wilson_dispatch(int mode, bool g5, dim3 grid, const WArgs &a, hipStream_t st)
{
    if (g5) {
        switch (mode) {
        case W_PLAIN: k_wilson<PREC, W_PLAIN, true><<<grid, kBlock, 0, st>>>(a); break;
        case W_NORM: k_wilson<PREC, W_NORM, true><<<grid, kBlock, 0, st>>>(a); break;
        case W_SHIFT: k_wilson<PREC, W_SHIFT, true><<<grid, kBlock, 0, st>>>(a); break;
        case W_RUPDATE: k_wilson<PREC, W_RUPDATE, true><<<grid, kBlock, 0, st>>>(a); break;
        default: k_wilson<PREC, W_RESNORM, true><<<grid, kBlock, 0, st>>>(a); break;
        }
    } else {
        k_wilson<PREC, W_PLAIN, false><<<grid, kBlock, 0, st>>>(a);
    }
}

hipError_t launch_wilson(const Lat &L, int prec, int mode, bool g5, WArgs a, hipStream_t st)
{
    a.g = L.g;
    a.nblk = 2 * L.nb;
    const int ts = prec == P_F64 && L.g.Ts64 > 0 ? L.g.Ts64 : L.g.Ts;
    if (ts > 0 && prec != P_F16S) {
        // time-streaming form (FP64, FP32): V / (NT Ts) blocks per RHS; the
        // FP16 stencil keeps one site per thread, which measured faster
        const int nt = stream_threads(L.g, ts);
        dim3 grid((unsigned)(L.V / ((int64_t)nt * ts)) * a.nrhs);
        if (prec == P_F64) wilson_ts_dispatch<P_F64>(mode, g5, grid, nt, a, st);
        else if (prec == P_F32) wilson_ts_dispatch<P_F32>(mode, g5, grid, nt, a, st);
        else wilson_ts_dispatch<P_F16S>(mode, g5, grid, nt, a, st);
        return hipGetLastError();
    }
    dim3 grid(2 * L.nb * a.nrhs);
    if (prec == P_F64) wilson_dispatch<P_F64>(mode, g5, grid, a, st);
    else if (prec == P_F32) wilson_dispatch<P_F32>(mode, g5, grid, a, st);
    else wilson_dispatch<P_F16S>(mode, g5, grid, a, st);
    return hipGetLastError();
}

}  // namespace ovl
