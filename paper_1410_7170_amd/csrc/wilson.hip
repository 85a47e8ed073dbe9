// Launch of the Wilson stencil kernels (wilson.h): blocks of 256 sites (192
// for the streaming form on some extents), ordered (site block, RHS) and
// spread over the XCDs by the kernel itself.
#include "internal.h"

namespace ovl {

template <int PREC, int WPE, bool STAGE, int NT = kBlock, bool TILED = false>
static void wilson_ts_dispatch_s(int mode, bool g5, dim3 grid, const WArgs &a, hipStream_t st, hipEvent_t e0,
                                 hipEvent_t e1)
{
    const dim3 b(NT);
    if (g5) {
        switch (mode) {
        case W_PLAIN: launch_k(k_wilson_ts<PREC, W_PLAIN, true, WPE, STAGE, NT, TILED>, grid, b, st, e0, e1, a); break;
        case W_NORM: launch_k(k_wilson_ts<PREC, W_NORM, true, WPE, STAGE, NT, TILED>, grid, b, st, e0, e1, a); break;
        case W_SHIFT: launch_k(k_wilson_ts<PREC, W_SHIFT, true, WPE, STAGE, NT, TILED>, grid, b, st, e0, e1, a); break;
        case W_RUPDATE:
            launch_k(k_wilson_ts<PREC, W_RUPDATE, true, WPE, STAGE, NT, TILED>, grid, b, st, e0, e1, a);
            break;
        case W_RUPDATE0:
            launch_k(k_wilson_ts<PREC, W_RUPDATE0, true, WPE, STAGE, NT, TILED>, grid, b, st, e0, e1, a);
            break;
        case W_SNORM: launch_k(k_wilson_ts<PREC, W_SNORM, true, WPE, STAGE, NT, TILED>, grid, b, st, e0, e1, a); break;
        default: launch_k(k_wilson_ts<PREC, W_RESNORM, true, WPE, STAGE, NT, TILED>, grid, b, st, e0, e1, a); break;
        }
    } else {
        launch_k(k_wilson_ts<PREC, W_PLAIN, false, WPE, STAGE, NT, TILED>, grid, b, st, e0, e1, a);
    }
}

// Blocks of whole x3 rows of consecutive x2 at one x1 take the one-wave build
// that stages each slice in LDS, at any grid size (at 32^3x64 it beats the
// two-wave build for one field, 411 against 456 us in FP64, and for batches
// of 7 fields, 2.7 against 2.9 ms); 48-bit fields, whose loaded words need
// fewer registers, take the staged two-wave build on grids of more than 256
// blocks (stencil_shape sizes them for it); blocks of 192 threads (nt, from
// stream_threads) exist only for that build.  Otherwise launches of at most
// 512 blocks take the one-wave build without staging, larger grids the
// two-wave build.  A block holds nt >> kr sites (K = 2^kr lanes per site).
static bool staged_rows(const Geom &g, int sites)
{
    return sites % g.L[3] == 0 && (g.L[2] * g.L[3]) % sites == 0;
}

template <int PREC>
static void wilson_ts_dispatch(int mode, bool g5, dim3 grid, int nt, const WArgs &a, hipStream_t st, hipEvent_t e0,
                               hipEvent_t e1)
{
    // 192-thread blocks (three waves) in FP64 take the build capped at two
    // waves per SIMD: the one-wave build needs more than 256 registers, so a
    // block holds three of a CU's four SIMDs and the fourth idles (24^3x48,
    // 12 RHS: 1489 -> 1252 us, with a few spilled registers); FP32 measured the
    // same either way
    constexpr int W192 = PREC == P_F64 || PREC == P_F48 ? 2 : 1;
    if (a.kr > 0) {
        // RHS tiles: staged builds only (stencil_shape guarantees whole rows)
        if (nt == 192) wilson_ts_dispatch_s<PREC, W192, true, 192, true>(mode, g5, grid, a, st, e0, e1);
        else wilson_ts_dispatch_s<PREC, 1, true, kBlock, true>(mode, g5, grid, a, st, e0, e1);
        return;
    }
    if (nt == 192) {
        wilson_ts_dispatch_s<PREC, W192, true, 192>(mode, g5, grid, a, st, e0, e1);
        return;
    }
    if (staged_rows(a.g, nt)) {
        if (PREC == P_F48 && grid.x > 256) wilson_ts_dispatch_s<PREC, 2, true>(mode, g5, grid, a, st, e0, e1);
        else wilson_ts_dispatch_s<PREC, 1, true>(mode, g5, grid, a, st, e0, e1);
    } else if (grid.x <= 512) {
        wilson_ts_dispatch_s<PREC, 1, false>(mode, g5, grid, a, st, e0, e1);
    } else {
        wilson_ts_dispatch_s<PREC, 2, false>(mode, g5, grid, a, st, e0, e1);
    }
}

// The streaming form's shape.  The RHS tile K is the lattice's rhs_tile,
// capped at the next power of two of nrhs, and halved until the block's
// sites times the stream length cover at least 256 site-slices (so the
// blocks of one tile fit the 2 nb partial-sum slots per RHS) and the block's
// sites are whole x3 rows (tiles run in the LDS-staged build only).
static StencilShape stencil_shape_ts(const Lat &L, int ts, int nrhs)
{
    StencilShape sh{};
    const int nt = stream_threads(L.g, ts);
    int kr = L.g.Kr;
    while (kr > 0 && (1 << (kr - 1)) >= nrhs) kr--;   // K <= next power of two of nrhs
    while (kr > 0 && ((nt >> kr) * ts < 256 || !staged_rows(L.g, nt >> kr))) kr--;
    sh.ts = ts;
    sh.nt = nt;
    sh.kr = kr;
    sh.blocks_per_tile = (int)(L.V / ((int64_t)(nt >> kr) * ts));
    sh.ntile = (nrhs + (1 << kr) - 1) >> kr;
    return sh;
}

// 48-bit fields take the FP64 length, halved while the launch has fewer than
// 512 blocks: their staged build runs two waves per SIMD (below), which needs
// two blocks per CU (at 32^3x64: 16 slices and 512 blocks, the mixed solver's
// 48-bit stencils 381 -> 367 us (t update) and 382 -> 353 us (residual
// update) against one wave at 32 slices; FP64 itself spills at two waves and
// keeps one)
StencilShape stencil_shape(const Lat &L, int prec, int nrhs)
{
    const int ts = (prec == P_F64 || prec == P_F48) && L.g.Ts64 > 0 ? L.g.Ts64 : L.g.Ts;
    if (ts <= 0 || prec == P_F16S) return StencilShape{};
    StencilShape sh = stencil_shape_ts(L, ts, nrhs);
    while (prec == P_F48 && sh.ts % 2 == 0 && (int64_t)sh.blocks_per_tile * sh.ntile < 512)
        sh = stencil_shape_ts(L, sh.ts / 2, nrhs);
    return sh;
}

template <int PREC>
static void wilson_dispatch(int mode, bool g5, dim3 grid, const WArgs &a, hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    const dim3 b(kBlock);
    if (g5) {
        switch (mode) {
        case W_PLAIN: launch_k(k_wilson<PREC, W_PLAIN, true>, grid, b, st, e0, e1, a); break;
        case W_NORM: launch_k(k_wilson<PREC, W_NORM, true>, grid, b, st, e0, e1, a); break;
        case W_SHIFT: launch_k(k_wilson<PREC, W_SHIFT, true>, grid, b, st, e0, e1, a); break;
        case W_RUPDATE: launch_k(k_wilson<PREC, W_RUPDATE, true>, grid, b, st, e0, e1, a); break;
        case W_RUPDATE0: launch_k(k_wilson<PREC, W_RUPDATE0, true>, grid, b, st, e0, e1, a); break;
        case W_SNORM: launch_k(k_wilson<PREC, W_SNORM, true>, grid, b, st, e0, e1, a); break;
        default: launch_k(k_wilson<PREC, W_RESNORM, true>, grid, b, st, e0, e1, a); break;
        }
    } else {
        launch_k(k_wilson<PREC, W_PLAIN, false>, grid, b, st, e0, e1, a);
    }
}

hipError_t launch_wilson(const Lat &L, int prec, int mode, bool g5, WArgs a, hipStream_t st, hipEvent_t e0,
                         hipEvent_t e1)
{
    a.g = L.g;
    a.nblk = 2 * L.nb;
    a.kr = 0;
    if (prec == P_F32 && mode == W_PLAIN && L.g.Mfma && a.nrhs >= 2) {
        // the matrix-core form: events as markers around its launch
        if (e0) {
            const hipError_t h0 = hipEventRecord(e0, st);
            if (h0 != hipSuccess) return h0;
        }
        const hipError_t h = launch_wilson_mfma(L, g5, a, st);
        if (h == hipSuccess && e1) return hipEventRecord(e1, st);
        return h;
    }
    const StencilShape sh = stencil_shape(L, prec, a.nrhs);
    if (sh.ts > 0) {
        // time-streaming form (FP64, 48-bit, FP32): blocks_per_tile blocks per RHS
        // tile; the FP16 stencil keeps one site per thread, which measured
        // faster
        if (sh.blocks_per_tile > a.nblk) return hipErrorInvalidConfiguration;
        a.kr = sh.kr;
        if (prec == P_F48) a.g.Ts64 = sh.ts;   // the kernel reads its length from there
        dim3 grid((unsigned)sh.blocks_per_tile * sh.ntile);
        if (prec == P_F64) wilson_ts_dispatch<P_F64>(mode, g5, grid, sh.nt, a, st, e0, e1);
        else if (prec == P_F48) wilson_ts_dispatch<P_F48>(mode, g5, grid, sh.nt, a, st, e0, e1);
        else wilson_ts_dispatch<P_F32>(mode, g5, grid, sh.nt, a, st, e0, e1);
        return hipGetLastError();
    }
    dim3 grid(2 * L.nb * a.nrhs);
    if (prec == P_F64) wilson_dispatch<P_F64>(mode, g5, grid, a, st, e0, e1);
    else if (prec == P_F48) wilson_dispatch<P_F48>(mode, g5, grid, a, st, e0, e1);
    else if (prec == P_F32) wilson_dispatch<P_F32>(mode, g5, grid, a, st, e0, e1);
    else wilson_dispatch<P_F16S>(mode, g5, grid, a, st, e0, e1);
    return hipGetLastError();
}

}  // namespace ovl
