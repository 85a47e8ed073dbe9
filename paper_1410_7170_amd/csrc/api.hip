// C ABI entry points (include/ovl.h): argument validation on the host, then
// the stream-ordered launches.  Nothing here throws; every failure is a status.
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "mscg.h"

namespace ovl {
int last_hip_error();
size_t mscg_ws_bytes(const Lat &L, int nrhs, int nshift);
size_t lanczos_ws_bytes(const Lat &L);
int mscg_f64(const Lat &L, const void *U64, double m0, int nshift, const double *shifts, Fld b,
             const ovl_solver_params *prm, ovl_solver_stats *stats, char *ws, size_t ws_bytes, hipStream_t st,
             MsScratch *scr);
int true_residuals_f64(const Lat &L, const void *U64, double m0, double s, Fld b, Fld x, Fld q, Fld t,
                       double *partials, double *red, double *out, hipStream_t st);
hipError_t launch_combine(const Lat &L, const double *w, int nshift, Fld x, Fld y, hipStream_t st,
                          bool accumulate = false);
int lanczos_bounds(const Lat &L, const void *U64, double m0, int iters, Fld start, double *tmin, double *tmax,
                   char *ws, size_t ws_bytes, hipStream_t st);
size_t mixed_ws_bytes(const Lat &L, int nrhs, int nshift, int m, int m64, bool f64_phase, bool f16_store, bool s48);
size_t tune_ws_bytes(const Lat &L, int nrhs);
int autotune_stencil(ovl_lattice *lat, const ovl_gauge *U, int nrhs, char *ws, size_t ws_bytes, hipStream_t st,
                     int32_t *tried, float *times_us, int32_t max_tried);
int autotune_stencil_cached(ovl_lattice *lat, const ovl_gauge *U, int nrhs, char *ws, size_t ws_bytes,
                            hipStream_t st, const char *path, int32_t *tried, float *times_us, int32_t max_tried);
int mscg_mixed(const Lat &L, const ovl_gauge *U, double m0, int nshift, const double *shifts, const double *weights,
               Fld b, Fld y, const ovl_solver_params *prm, ovl_solver_stats *stats, char *ws, size_t ws_bytes,
               hipStream_t st);
size_t wilson_solve_ws_bytes(const Lat &L, int nrhs, int m);
size_t lanczos_sign_ws_bytes(const Lat &L, int nrhs);
int lanczos_sign(const Lat &L, const void *U64, double m0, Fld b, Fld y, double tol, int maxiter, int *iters,
                 char *ws, size_t ws_bytes, hipStream_t st);
int wilson_solve(const Lat &L, const ovl_gauge *U, double m0, Fld b, Fld x, double tol, int maxiter, int m,
                 double *true_res, int *iters, char *ws, size_t ws_bytes, hipStream_t st);
size_t outer_ws_bytes(const Lat &L, int npoles, const ovl_outer_params *p, const ovl_lattice *lat);
int overlap_solve(const ovl_lattice *lat, const ovl_gauge *U, double rho, const ovl_zolo *z, Fld eta, Fld psi,
                  const ovl_outer_params *prm, ovl_outer_stats *stats, char *ws, size_t ws_bytes, hipStream_t st);
size_t low_modes_ws_bytes(const Lat &L, const ovl_eig_params *p);
int low_modes(const Lat &L, const void *U64, double m0, Fld start, const ovl_eig_params *p, Fld evecs, double *evals,
              double *resid, ovl_eig_stats *S, char *ws, size_t ws_bytes, hipStream_t st);
size_t deflation_ws_bytes(const Lat &L, int nrhs, int k);
int deflate_project(const Lat &L, const ovl_deflation *D, Fld b, Fld proj, std::vector<std::complex<double>> &cr,
                    char *ws, hipStream_t st);
int deflate_restore(const Lat &L, const ovl_deflation *D, const std::vector<std::complex<double>> &cr, double rho,
                    bool overlap, Fld out, char *ws, hipStream_t st);
}  // namespace ovl

using namespace ovl;

namespace {

bool lat_ok(const ovl_lattice *lat)
{
    if (!lat) return false;
    int64_t V = 1;
    for (int m = 0; m < 4; m++) {
        if (lat->dims[m] < 2 || (lat->dims[m] & 1)) return false;
        if (lat->bc[m] != 1 && lat->bc[m] != -1) return false;
        V *= lat->dims[m];
    }
    if (lat->tile_t < 1 || lat->dims[0] % lat->tile_t) return false;
    if (lat->stream_t < 0 || lat->stream_t > 256) return false;
    if (lat->stream_t > 0 && (lat->dims[0] % lat->stream_t ||
                              ((int64_t)lat->dims[1] * lat->dims[2] * lat->dims[3]) % 256))
        return false;
    if (lat->stream_t64 < 0 || lat->stream_t64 > 256) return false;
    if (lat->stream_t64 > 0 && (lat->dims[0] % lat->stream_t64 ||
                                ((int64_t)lat->dims[1] * lat->dims[2] * lat->dims[3]) % 256))
        return false;
    if (lat->rhs_tile != 1 && lat->rhs_tile != 2 && lat->rhs_tile != 4 && lat->rhs_tile != 8) return false;
    if (lat->mfma != 0 && lat->mfma != 1) return false;
    return V < ((int64_t)1 << 31) && lat->vol == V;
}

bool spinor_ok(const ovl_spinor *s, int max_fields = OVL_MAX_RHS)
{
    if (!s || !s->d) return false;
    if (s->prec < OVL_F64 || s->prec > OVL_F48) return false;
    if (s->nrhs < 1 || s->nrhs > max_fields) return false;
    if (s->prec == OVL_F16S && !s->scale) return false;
    return true;
}

// pack/unpack convert any field set, e.g. the nshift*nrhs solutions
constexpr int kMaxFields = OVL_MAX_RHS * OVL_MAX_SHIFTS;

const void *gauge_for(const ovl_gauge *U, int prec)
{
    if (!U) return nullptr;
    return prec == OVL_F64 || prec == OVL_F48 ? U->f64 : prec == OVL_F32 ? U->f32 : U->f16;
}

hipStream_t S(void *s) { return (hipStream_t)s; }

bool params_ok(const ovl_solver_params *p)
{
    return p && p->tol > 0.0 && std::isfinite(p->tol) && p->maxiter >= 1 &&
           (p->mode == OVL_SOLVE_F64 || p->mode == OVL_SOLVE_MIXED || p->mode == OVL_SOLVE_LANCZOS) &&
           p->reliable_delta > 0.0 &&
           p->reliable_delta < 1.0 && p->block >= 0 && p->block <= OVL_MAX_BLOCK && p->block_f64 >= 0 && p->block_f64 <= OVL_MAX_BLOCK && p->sloppy_below >= 0.0 &&
           p->sloppy_below < 1.0 && p->rhs_group >= 0 && (p->sloppy_f16 == 0 || p->sloppy_f16 == 1) && (p->store48 == 0 || p->store48 == 1) &&
           (p->even_odd == 0 || p->even_odd == 1) && p->profile >= 0 && p->profile <= 2;
}

bool defl_ok(const ovl_deflation *D)
{
    if (!D || !D->evals || !spinor_ok(&D->evecs, OVL_MAX_NEV) || D->evecs.prec != OVL_F64) return false;
    for (int i = 0; i < D->evecs.nrhs; i++)
        if (!std::isfinite(D->evals[i])) return false;
    return true;
}

bool eig_ok(const ovl_eig_params *p)
{
    return p && p->nev >= 1 && p->nev <= OVL_MAX_NEV && p->extra >= 0 && p->nev + p->extra <= 2 * OVL_MAX_NEV &&
           p->tol > 0.0 && std::isfinite(p->tol) && p->degree >= 1 && p->degree <= 200 && p->steps >= 0 &&
           p->steps <= 4096 && (p->steps == 0 || p->steps >= p->nev + (p->extra > 0 ? p->extra : p->nev / 2 + 4)) &&
           p->stages >= 1 && p->stages <= 200 && p->check_every >= 0;
}

bool zolo_ok(const ovl_zolo *z)
{
    if (!z || !z->shifts || !z->weights || z->npoles < 1 || z->npoles > OVL_MAX_SHIFTS) return false;
    for (int j = 0; j < z->npoles; j++)
        if (!(z->shifts[j] >= 0.0) || !std::isfinite(z->shifts[j]) || !std::isfinite(z->weights[j])) return false;
    return true;
}

double now()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void clear_stats(ovl_solver_stats *st)
{
    if (!st) return;
    std::memset(st, 0, sizeof *st);
    for (int r = 0; r < OVL_MAX_RHS; r++)
        for (int j = 0; j < OVL_MAX_SHIFTS; j++) st->true_residual[r][j] = -1.0;
}

// Add the stats of a group of RHS (its RHS 0..n-1 are the call's g0..g0+n-1).
void merge_stats(ovl_solver_stats *dst, const ovl_solver_stats &src, int g0, int n)
{
    if (!dst) return;
    for (int q = 0; q < n; q++) {
        dst->iterations[g0 + q] = src.iterations[q];
        for (int j = 0; j < OVL_MAX_SHIFTS; j++) {
            dst->shift_iters[g0 + q][j] = src.shift_iters[q][j];
            dst->true_residual[g0 + q][j] = src.true_residual[q][j];
        }
    }
    dst->reliable_updates += src.reliable_updates;
    dst->refine_iterations += src.refine_iterations;
    dst->stencil_applies += src.stencil_applies;
    dst->algorithmic_bytes += src.algorithmic_bytes;
    for (int c = 0; c < 4; c++) {
        dst->kernel_seconds[c] += src.kernel_seconds[c];
        dst->kernel_bytes[c] += src.kernel_bytes[c];
        dst->kernel_launches[c] += src.kernel_launches[c];
    }
}

// RHS per group of a solve returning weighted sums
int group_size(const ovl_solver_params *prm, int R) { return prm->rhs_group > 0 ? std::min(R, prm->rhs_group) : R; }

}  // namespace

namespace ovl {

// (Q^2 + shift) in: Q = Gamma_5 D_W(m0) into the scratch field t (ws), then
// Q t + shift in into out.  Shared by ovl_q2_apply (caller workspace) and the
// entry point without allocation (a library-owned scratch array).
int q2_apply_body(const ovl_lattice *lat, const ovl_gauge *U, double m0, double shift, const ovl_spinor *in,
                  ovl_spinor *out, char *ws, size_t ws_bytes, hipStream_t st)
{
    if (!lat_ok(lat) || !spinor_ok(in) || !spinor_ok(out)) return OVL_ERR_INVALID;
    if (in->prec != out->prec || in->nrhs != out->nrhs || in->d == out->d) return OVL_ERR_INVALID;
    if (!std::isfinite(m0) || !std::isfinite(shift)) return OVL_ERR_INVALID;
    const void *Ud = gauge_for(U, in->prec);
    if (!Ud || !ws) return OVL_ERR_INVALID;
    if (ws_bytes < ovl_workspace_bytes(lat, OVL_OP_Q2, in->prec, in->nrhs, 0, nullptr)) return OVL_ERR_WORKSPACE;
    Lat L = make_lat(lat);
    size_t F = field_bytes(in->prec, L.V) * in->nrhs;
    void *tmp = ws;
    float *tsc = in->prec == OVL_F16S ? (float *)(ws + ((F + 255) & ~(size_t)255)) : nullptr;
    WArgs a{};
    a.in = in->d;
    a.in_sc = in->scale;
    a.out = tmp;
    a.out_sc = tsc;
    a.U = Ud;
    a.diag = m0 + 4.0;
    a.nrhs = in->nrhs;
    OVL_HIP(launch_wilson(L, in->prec, W_PLAIN, true, a, st));
    WArgs b = a;
    b.in = tmp;
    b.in_sc = tsc;
    b.p = in->d;
    b.p_sc = in->scale;
    b.shift = shift;
    b.out = out->d;
    b.out_sc = out->scale;
    OVL_HIP(launch_wilson(L, in->prec, W_SHIFT, true, b, st));
    return OVL_OK;
}

}  // namespace ovl

extern "C" {

int ovl_lattice_init(ovl_lattice *lat, const int32_t dims[4], const int32_t bc[4])
{
    if (!lat || !dims || !bc) return OVL_ERR_INVALID;
    int64_t V = 1;
    for (int m = 0; m < 4; m++) {
        lat->dims[m] = dims[m];
        lat->bc[m] = bc[m];
        if (dims[m] < 2 || (dims[m] & 1) || (bc[m] != 1 && bc[m] != -1)) return OVL_ERR_INVALID;
        V *= dims[m];
    }
    if (V >= ((int64_t)1 << 31)) return OVL_ERR_INVALID;
    lat->vol = V;
    // default time tile: 4 slices when L0 allows it (measured best for the
    // FP64 and FP32 stencils at 32^3x64 on MI355X; 2 or 1 otherwise)
    lat->tile_t = (dims[0] % 4 == 0) ? 4 : (dims[0] % 2 == 0) ? 2 : 1;
    // time-streaming stencil: FP32 takes the longest of 16, 8, 4, 2 slices per
    // thread that divides L0 and still launches >= 512 blocks, FP64 also 32
    // slices when that leaves >= 256 blocks (measured on MI355X at
    // 32^3x64: L2-miss traffic of the FP64 stencil falls from 2.7x to 1.2x of
    // its compulsory reads at 32 slices, of the FP32 one from 2.4x to 1.1x at
    // 16; beyond that too few blocks are left to hide memory latency)
    lat->stream_t = 0;
    lat->stream_t64 = 0;
    lat->rhs_tile = 1;
    lat->mfma = 0;
    const int64_t V3 = (int64_t)dims[1] * dims[2] * dims[3];
    if (V3 % 256 == 0) {
        for (int s : {16, 8, 4, 2})
            if (dims[0] % s == 0 && V / (256 * (int64_t)s) >= 512) {
                lat->stream_t = s;
                break;
            }
        for (int s : {32, 16, 8, 4, 2})
            if (dims[0] % s == 0 && V / (256 * (int64_t)s) >= (s >= 32 ? 256 : 512)) {
                lat->stream_t64 = s;
                break;
            }
    }
    return OVL_OK;
}

size_t ovl_spinor_bytes(const ovl_lattice *lat, int32_t prec)
{
    if (!lat_ok(lat) || prec < 0 || prec > OVL_F48) return 0;
    return field_bytes(prec, lat->vol);
}

size_t ovl_scale_bytes(const ovl_lattice *lat) { return lat_ok(lat) ? scale_bytes(lat->vol) : 0; }

size_t ovl_gauge_bytes(const ovl_lattice *lat, int32_t prec)
{
    if (!lat_ok(lat) || prec < 0 || prec > 2) return 0;
    return gauge_field_bytes(prec, lat->vol);
}

int ovl_pack_spinor(const ovl_lattice *lat, const void *canon, ovl_spinor *out, void *stream)
{
    if (!lat_ok(lat) || !canon || !spinor_ok(out, kMaxFields) || canon == out->d) return OVL_ERR_INVALID;
    Lat L = make_lat(lat);
    OVL_HIP(launch_pack_spinor(L, canon, fld(out), S(stream)));
    return OVL_OK;
}

int ovl_unpack_spinor(const ovl_lattice *lat, const ovl_spinor *in, void *canon, void *stream)
{
    if (!lat_ok(lat) || !canon || !spinor_ok(in, kMaxFields) || canon == in->d) return OVL_ERR_INVALID;
    Lat L = make_lat(lat);
    OVL_HIP(launch_unpack_spinor(L, fld(in), canon, S(stream)));
    return OVL_OK;
}

int ovl_pack_gauge(const ovl_lattice *lat, const void *canon, int32_t prec, void *out, void *stream)
{
    if (!lat_ok(lat) || !canon || !out || canon == out || prec < 0 || prec > 2) return OVL_ERR_INVALID;
    Lat L = make_lat(lat);
    OVL_HIP(launch_pack_gauge(L, canon, prec, out, S(stream)));
    return OVL_OK;
}

static int apply_q_or_w(const ovl_lattice *lat, const ovl_gauge *U, double m0, const ovl_spinor *in,
                        ovl_spinor *out, void *stream, bool g5)
{
    if (!lat_ok(lat) || !spinor_ok(in) || !spinor_ok(out)) return OVL_ERR_INVALID;
    if (in->prec != out->prec || in->nrhs != out->nrhs || in->d == out->d || !std::isfinite(m0)) return OVL_ERR_INVALID;
    const void *Ud = gauge_for(U, in->prec);
    if (!Ud) return OVL_ERR_INVALID;
    Lat L = make_lat(lat);
    WArgs a{};
    a.in = in->d;
    a.in_sc = in->scale;
    a.out = out->d;
    a.out_sc = out->scale;
    a.U = Ud;
    a.diag = m0 + 4.0;
    a.nrhs = in->nrhs;
    OVL_HIP(launch_wilson(L, in->prec, W_PLAIN, g5, a, S(stream)));
    return OVL_OK;
}

int ovl_wilson_apply(const ovl_lattice *lat, const ovl_gauge *U, double m0, const ovl_spinor *in, ovl_spinor *out,
                     void *stream)
{
    return apply_q_or_w(lat, U, m0, in, out, stream, false);
}

int ovl_q_apply(const ovl_lattice *lat, const ovl_gauge *U, double m0, const ovl_spinor *in, ovl_spinor *out,
                void *stream)
{
    return apply_q_or_w(lat, U, m0, in, out, stream, true);
}

int ovl_q2_apply(const ovl_lattice *lat, const ovl_gauge *U, double m0, double shift, const ovl_spinor *in,
                 ovl_spinor *out, void *ws, size_t ws_bytes, void *stream)
{
    if (!ws) return OVL_ERR_INVALID;
    return q2_apply_body(lat, U, m0, shift, in, out, (char *)ws, ws_bytes, S(stream));
}

size_t ovl_workspace_bytes(const ovl_lattice *lat, int32_t op, int32_t prec, int32_t nrhs, int32_t nshift,
                           const ovl_solver_params *prm)
{
    if (!lat_ok(lat) || nrhs < 1 || nrhs > OVL_MAX_RHS) return 0;
    Lat L = make_lat(lat);
    if (op == OVL_OP_Q2) {
        if (prec < 0 || prec > OVL_F48) return 0;
        size_t F = field_bytes(prec, L.V) * nrhs;
        return ((F + 255) & ~(size_t)255) + scale_bytes(L.V) * nrhs + 256;
    }
    if (op == OVL_OP_LANCZOS) return lanczos_ws_bytes(L);
    if (op == OVL_OP_TUNE) return tune_ws_bytes(L, nrhs);
    if (op == OVL_OP_WILSON_SOLVE) {
        if (prm && !params_ok(prm)) return 0;
        if (prm && prm->even_odd) return wilson_solve_eo_ws_bytes(L);
        const int m = prm && prm->block > 0 ? prm->block : 16;
        if (m > OVL_MAX_BLOCK) return 0;
        return wilson_solve_ws_bytes(L, nrhs, m);
    }
    if (op == OVL_OP_MSCG) {
        if (nshift < 1 || nshift > OVL_MAX_SHIFTS || (prm && !params_ok(prm))) return 0;
        // deflation (sign_q_apply, overlap_apply): projected sources of every
        // RHS in front of the solver's own workspace
        size_t yb = 0;
        if (prm && prm->deflation) {
            if (!defl_ok(prm->deflation)) return 0;
            yb = align256(deflation_ws_bytes(L, nrhs, prm->deflation->evecs.nrhs));
        }
        if (prm && prm->rhs_group > 0) nrhs = std::min(nrhs, (int32_t)prm->rhs_group);   // one group
        yb += (field_bytes(P_F64, L.V) * nrhs + 255) & ~(size_t)255;
        if (prm && prm->mode == OVL_SOLVE_LANCZOS) return yb + lanczos_sign_ws_bytes(L, nrhs);
        if (prm && prm->mode == OVL_SOLVE_MIXED)
            return yb + mixed_ws_bytes(L, nrhs, nshift, mixed_block(prm), mixed_block_f64(prm), prm->sloppy_below > 0.0,
                                       prm->sloppy_f16 != 0, prm->store48 != 0);
        if (prm && prm->block > 0)   // x mode, or y mode with the extra unshifted base
            return yb + std::max(blocked_ws_bytes(L, nrhs, nshift, prm->block, true, P_F64),
                                 blocked_ws_bytes(L, nrhs, std::min(nshift + 1, (int32_t)NS), prm->block, false,
                                                  P_F64));
        return yb + mscg_ws_bytes(L, nrhs, nshift);
    }
    return 0;
}

void ovl_default_params(ovl_solver_params *p)
{
    if (!p) return;
    p->tol = 1e-10;
    p->maxiter = 2000;
    p->mode = OVL_SOLVE_F64;
    p->reliable_delta = 0.1;
    p->check_every = 10;
    p->refine = 1;
    p->verify = 0;
    p->profile = 0;
    p->block = 0;
    p->sloppy_below = 3e-5;
    p->block_f64 = 0;
    p->rhs_group = 0;
    p->deflation = nullptr;
    p->sloppy_f16 = 0;
    p->store48 = 1;
    p->even_odd = 0;
}

int ovl_autotune_stencil(ovl_lattice *lat, const ovl_gauge *U, int32_t nrhs, void *ws, size_t ws_bytes,
                         int32_t *tried, float *times_us, int32_t max_tried, void *stream)
{
    if (!lat_ok(lat) || !U || !ws || nrhs < 1 || nrhs > OVL_MAX_RHS || max_tried < 0) return OVL_ERR_INVALID;
    if (!U->f64 && !U->f32 && !U->f16) return OVL_ERR_INVALID;
    return autotune_stencil(lat, U, nrhs, (char *)ws, ws_bytes, (hipStream_t)stream, tried, times_us, max_tried);
}

int ovl_autotune_stencil_cached(ovl_lattice *lat, const ovl_gauge *U, int32_t nrhs, void *ws, size_t ws_bytes,
                                const char *cache_path, int32_t *tried, float *times_us, int32_t max_tried,
                                void *stream)
{
    if (!lat_ok(lat) || !U || !ws || nrhs < 1 || nrhs > OVL_MAX_RHS || max_tried < 0) return OVL_ERR_INVALID;
    if (!U->f64 && !U->f32 && !U->f16) return OVL_ERR_INVALID;
    return autotune_stencil_cached(lat, U, nrhs, (char *)ws, ws_bytes, (hipStream_t)stream, cache_path, tried,
                                   times_us, max_tried);
}

int ovl_spectral_bounds(const ovl_lattice *lat, const ovl_gauge *U, double m0, int32_t iters,
                        const ovl_spinor *start, double lo_margin, double hi_margin, double *lambda_min,
                        double *lambda_max, void *ws, size_t ws_bytes, void *stream)
{
    if (!lat_ok(lat) || !spinor_ok(start) || start->prec != OVL_F64 || start->nrhs != 1) return OVL_ERR_INVALID;
    if (!U || !U->f64 || !lambda_min || !lambda_max || !ws || iters < 2) return OVL_ERR_INVALID;
    if (!(lo_margin > 0.0 && lo_margin <= 1.0 && hi_margin >= 1.0)) return OVL_ERR_INVALID;
    Lat L = make_lat(lat);
    if (ws_bytes < lanczos_ws_bytes(L)) return OVL_ERR_WORKSPACE;
    double t0, t1;
    int rc = lanczos_bounds(L, U->f64, m0, iters, fld(start), &t0, &t1, (char *)ws, ws_bytes, S(stream));
    if (rc) return rc;
    *lambda_min = lo_margin * std::sqrt(std::max(t0, 0.0));
    *lambda_max = hi_margin * std::sqrt(t1);
    return OVL_OK;
}

// Shared body of multishift_cg / sign_q / overlap.  Workspace layout:
// [one nrhs FP64 field set "y"][solver workspace].  If weights != NULL,
// y_r = sum_l w_l x_{l,r} is left in the front field set; the FP64 solver also
// hands back its x_l through *scr.
static int solve_y(const Lat &L, const ovl_gauge *U, double m0, int nshift, const double *shifts,
                   const double *weights, Fld b, const ovl_solver_params *prm, ovl_solver_stats *stats, char *ws,
                   size_t ws_bytes, hipStream_t st, Fld *y_out, MsScratch *scr)
{
    const int R = b.nrhs;
    size_t yb = (field_bytes(P_F64, L.V) * R + 255) & ~(size_t)255;
    Fld y{ws, nullptr, P_F64, R};
    *y_out = y;
    if (prm->mode == OVL_SOLVE_MIXED) {
        // the mixed solver reads FP64 and FP32 links only
        if (!U->f32 || !U->f64 || !weights) return OVL_ERR_INVALID;
        return mscg_mixed(L, U, m0, nshift, shifts, weights, b, y, prm, stats, ws + yb, ws_bytes - yb, st);
    }
    int rc;
    const bool blocked = prm->block > 0;
    const bool keep_x = !weights || prm->verify;
    if (blocked) {
        BlkOpts o;
        o.m = prm->block;
        o.keep_x = keep_x;
        // y mode with positive shifts: the recurrences run on an extra
        // unshifted base of weight 0, as in the mixed solver (no p0 field, t by
        // recurrence, the residual update without the s0 p0 term); the
        // caller's per-shift statistics leave it out
        bool base0 = !keep_x && nshift < NS;
        for (int j = 0; j < nshift; j++) base0 = base0 && shifts[j] > 0.0;
        if (base0) {
            double sh[NS], w[NS];
            sh[0] = w[0] = 0.0;
            for (int j = 0; j < nshift; j++) {
                sh[j + 1] = shifts[j];
                w[j + 1] = weights[j];
            }
            rc = mscg_blocked_t<P_F64>(L, U, m0, nshift + 1, sh, w, b, y, o, prm, stats, ws + yb, ws_bytes - yb, st,
                                       scr);
            if (rc >= 0 && stats)
                for (int q = 0; q < NR; q++) {
                    for (int j = 0; j < nshift; j++) stats->shift_iters[q][j] = stats->shift_iters[q][j + 1];
                    stats->shift_iters[q][nshift] = 0;
                }
        } else {
            rc = mscg_blocked_t<P_F64>(L, U, m0, nshift, shifts, weights, b, y, o, prm, stats, ws + yb,
                                       ws_bytes - yb, st, scr);
        }
    } else
        rc = mscg_f64(L, U->f64, m0, nshift, shifts, b, prm, stats, ws + yb, ws_bytes - yb, st, scr);
    if (rc < 0) return rc;
    if (blocked && !keep_x) return rc;   // y already accumulated
    if (prm->verify && stats) {
        for (int j = 0; j < nshift; j++) {
            double res[NR];
            int rc2 = true_residuals_f64(L, U->f64, m0, shifts[j], b, sub(scr->x, L.V, j * R, R), scr->s1, scr->s2,
                                         scr->partials, scr->red, res, st);
            if (rc2) return rc2;
            for (int q = 0; q < R; q++) stats->true_residual[q][j] = res[q];
            stats->stencil_applies += 2;
        }
    }
    if (weights) OVL_HIP(launch_combine(L, weights, nshift, scr->x, y, st));
    return rc;
}

int ovl_multishift_cg(const ovl_lattice *lat, const ovl_gauge *U, double m0, int32_t nshift, const double *shifts,
                      const double *weights, const ovl_spinor *b, ovl_spinor *x, const ovl_solver_params *prm,
                      ovl_solver_stats *stats, void *ws, size_t ws_bytes, void *stream)
{
    double t0 = now();
    clear_stats(stats);
    if (!lat_ok(lat) || !spinor_ok(b) || !params_ok(prm) || !shifts || !U || !ws) return OVL_ERR_INVALID;
    // x holds nshift*nrhs fields when weights == NULL, so its count may exceed OVL_MAX_RHS
    if (!spinor_ok(x, kMaxFields) || x->prec != OVL_F64) return OVL_ERR_INVALID;
    if (nshift < 1 || nshift > OVL_MAX_SHIFTS || b->prec != OVL_F64 || x->prec != OVL_F64 || b->d == x->d)
        return OVL_ERR_INVALID;
    if (x->nrhs != (weights ? b->nrhs : b->nrhs * nshift)) return OVL_ERR_INVALID;
    if (!U->f64) return OVL_ERR_INVALID;
    for (int j = 0; j < nshift; j++)
        if (!(shifts[j] >= 0.0) || !std::isfinite(shifts[j])) return OVL_ERR_INVALID;
    Lat L = make_lat(lat);
    // the mixed solver returns y only; the Lanczos mode solves no shifted systems
    if ((!weights && prm->mode == OVL_SOLVE_MIXED) || prm->mode == OVL_SOLVE_LANCZOS) return OVL_ERR_INVALID;
    // every x_l at once: no RHS groups
    ovl_solver_params p1 = *prm;
    if (!weights) p1.rhs_group = 0;
    if (ws_bytes < ovl_workspace_bytes(lat, OVL_OP_MSCG, OVL_F64, b->nrhs, nshift, &p1)) return OVL_ERR_WORKSPACE;
    const int R = b->nrhs, G = group_size(&p1, R);
    const size_t F = field_bytes(P_F64, L.V);
    int rc_all = OVL_OK;
    for (int g0 = 0; g0 < R; g0 += G) {
        const int n = std::min(G, R - g0);
        ovl_solver_stats cs;
        clear_stats(&cs);
        Fld y{};
        MsScratch scr{};
        int rc = solve_y(L, U, m0, nshift, shifts, weights, sub(fld(b), L.V, g0, n), &p1, stats ? &cs : nullptr,
                         (char *)ws, ws_bytes, S(stream), &y, &scr);
        if (rc < 0) return rc;
        if (weights)
            OVL_HIP(hipMemcpyAsync((char *)x->d + F * g0, y.d, F * n, hipMemcpyDeviceToDevice, S(stream)));
        else
            OVL_HIP(hipMemcpyAsync(x->d, scr.x.d, F * R * nshift, hipMemcpyDeviceToDevice, S(stream)));
        merge_stats(stats, cs, g0, n);
        if (rc == OVL_NOT_CONVERGED) rc_all = rc;
    }
    OVL_HIP(hipStreamSynchronize(S(stream)));
    if (stats) stats->seconds = now() - t0;
    return rc_all;
}

static int sign_or_overlap_core(const ovl_lattice *lat, const ovl_gauge *U, double m0, double rho,
                                const ovl_zolo *z, const ovl_spinor *b, ovl_spinor *out,
                                const ovl_solver_params *prm, ovl_solver_stats *stats, void *ws, size_t ws_bytes,
                                void *stream, bool overlap)
{
    double t0 = now();
    clear_stats(stats);
    if (!lat_ok(lat) || !spinor_ok(b) || !spinor_ok(out) || !params_ok(prm) || !zolo_ok(z) || !U || !U->f64 || !ws)
        return OVL_ERR_INVALID;
    if (b->prec != OVL_F64 || out->prec != OVL_F64 || b->nrhs != out->nrhs || b->d == out->d) return OVL_ERR_INVALID;
    if (!std::isfinite(m0)) return OVL_ERR_INVALID;
    Lat L = make_lat(lat);
    const int R = b->nrhs, G = group_size(prm, R);
    if (ws_bytes < ovl_workspace_bytes(lat, OVL_OP_MSCG, OVL_F64, R, z->npoles, prm)) return OVL_ERR_WORKSPACE;
    int rc_all = OVL_OK;
    for (int g0 = 0; g0 < R; g0 += G) {
        // RHS g0 .. g0+n-1 in one solve; the workspace is reused by the next group
        const int n = std::min(G, R - g0);
        const Fld bg = sub(fld(b), L.V, g0, n), og = sub(fld(out), L.V, g0, n);
        ovl_solver_stats cs;
        clear_stats(&cs);
        if (prm->mode == OVL_SOLVE_LANCZOS) {
            // s = sign(Q) b in the front field set, then out = s or rho (b + Gamma_5 s)
            const size_t yb = (field_bytes(P_F64, L.V) * G + 255) & ~(size_t)255;
            Fld sg{ws, nullptr, P_F64, n};
            int its[NR] = {0};
            int rc = lanczos_sign(L, U->f64, m0, bg, sg, prm->tol, prm->maxiter, its, (char *)ws + yb,
                                  ws_bytes - yb, S(stream));
            if (rc < 0) return rc;
            if (overlap) {
                dim3 grid(site_blocks(L), n);
                k_gamma5<<<grid, kBlock, 0, S(stream)>>>(L.g, L.nb, (const double2 *)sg.d, (double2 *)og.d);
                OVL_HIP(hipGetLastError());
                OVL_HIP(launch_axpby(L, rho, bg, rho, og, S(stream)));
            } else {
                OVL_HIP(hipMemcpyAsync(og.d, sg.d, field_bytes(P_F64, L.V) * n, hipMemcpyDeviceToDevice,
                                       S(stream)));
            }
            int mx = 0;
            for (int q = 0; q < n; q++) {
                cs.iterations[q] = its[q];
                mx = std::max(mx, its[q]);
            }
            cs.stencil_applies = 2 * mx;
            cs.algorithmic_bytes = 2.0 * mx * (double)L.V * n * 768.0;
            merge_stats(stats, cs, g0, n);
            if (rc == OVL_NOT_CONVERGED) rc_all = rc;
            continue;
        }
        Fld y{};
        MsScratch scr{};
        int rc = solve_y(L, U, m0, z->npoles, z->shifts, z->weights, bg, prm, stats ? &cs : nullptr, (char *)ws,
                         ws_bytes, S(stream), &y, &scr);
        if (rc < 0) return rc;
        WArgs a{};
        a.in = y.d;
        a.out = og.d;
        a.U = U->f64;
        a.diag = m0 + 4.0;
        a.nrhs = n;
        if (overlap) {
            // out = rho (b + D_W(-rho) y)
            OVL_HIP(launch_wilson(L, P_F64, W_PLAIN, false, a, S(stream)));
            OVL_HIP(launch_axpby(L, rho, bg, rho, og, S(stream)));
        } else {
            OVL_HIP(launch_wilson(L, P_F64, W_PLAIN, true, a, S(stream)));
        }
        cs.stencil_applies += 1;
        cs.algorithmic_bytes += (double)L.V * n * 768.0 + (overlap ? (double)field_bytes(P_F64, L.V) * 3 * n : 0.0);
        merge_stats(stats, cs, g0, n);
        if (rc == OVL_NOT_CONVERGED) rc_all = rc;
    }
    OVL_HIP(hipStreamSynchronize(S(stream)));
    if (stats) stats->seconds = now() - t0;
    return rc_all;
}

// With deflation: project the low modes out of b, run the approximation on
// Pi b in the rest of the workspace, then add the modes back exactly
static int sign_or_overlap(const ovl_lattice *lat, const ovl_gauge *U, double m0, double rho, const ovl_zolo *z,
                           const ovl_spinor *b, ovl_spinor *out, const ovl_solver_params *prm,
                           ovl_solver_stats *stats, void *ws, size_t ws_bytes, void *stream, bool overlap)
{
    const ovl_deflation *D = prm ? prm->deflation : nullptr;
    if (!D) return sign_or_overlap_core(lat, U, m0, rho, z, b, out, prm, stats, ws, ws_bytes, stream, overlap);
    const double t0 = now();
    clear_stats(stats);
    if (!lat_ok(lat) || !spinor_ok(b) || !spinor_ok(out) || !params_ok(prm) || !defl_ok(D) || !zolo_ok(z) || !U ||
        !U->f64 || !ws)
        return OVL_ERR_INVALID;
    if (b->prec != OVL_F64 || out->prec != OVL_F64 || b->nrhs != out->nrhs || b->d == out->d) return OVL_ERR_INVALID;
    if (D->evecs.d == b->d || D->evecs.d == out->d) return OVL_ERR_INVALID;
    const int R = b->nrhs;
    if (ws_bytes < ovl_workspace_bytes(lat, OVL_OP_MSCG, OVL_F64, R, z->npoles, prm)) return OVL_ERR_WORKSPACE;
    const Lat L = make_lat(lat);
    const size_t db = align256(deflation_ws_bytes(L, R, D->evecs.nrhs));
    std::vector<std::complex<double>> cr;
    Fld proj{ws, nullptr, P_F64, R};
    int e = deflate_project(L, D, fld(b), proj, cr, (char *)ws, S(stream));
    if (e) return e;
    ovl_solver_params p2 = *prm;
    p2.deflation = nullptr;
    ovl_spinor pb{proj.d, nullptr, OVL_F64, R};
    const int rc = sign_or_overlap_core(lat, U, m0, rho, z, &pb, out, &p2, stats, (char *)ws + db, ws_bytes - db,
                                        stream, overlap);
    if (rc < 0) return rc;
    e = deflate_restore(L, D, cr, rho, overlap, fld(out), (char *)ws, S(stream));
    if (e) return e;
    OVL_HIP(hipStreamSynchronize(S(stream)));
    if (stats) stats->seconds = now() - t0;
    return rc;
}

int ovl_sign_q_apply(const ovl_lattice *lat, const ovl_gauge *U, double m0, const ovl_zolo *z, const ovl_spinor *b,
                     ovl_spinor *out, const ovl_solver_params *prm, ovl_solver_stats *stats, void *ws,
                     size_t ws_bytes, void *stream)
{
    return sign_or_overlap(lat, U, m0, 0.0, z, b, out, prm, stats, ws, ws_bytes, stream, false);
}

int ovl_overlap_apply(const ovl_lattice *lat, const ovl_gauge *U, double rho, const ovl_zolo *z, const ovl_spinor *b,
                      ovl_spinor *out, const ovl_solver_params *prm, ovl_solver_stats *stats, void *ws,
                      size_t ws_bytes, void *stream)
{
    if (!(rho > 0.0) || !std::isfinite(rho)) return OVL_ERR_INVALID;
    return sign_or_overlap(lat, U, -rho, rho, z, b, out, prm, stats, ws, ws_bytes, stream, true);
}

void ovl_default_outer_params(ovl_outer_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->tol = 1e-8;
    p->restart = 100;
    p->maxiter = 1000;
    p->relax = 1;
    p->relax_factor = 1e-2;
    p->sign_tol_max = 1e-2;
    ovl_default_params(&p->inner);
    p->inner.mode = OVL_SOLVE_MIXED;
    p->precondition = 0;
    p->prec_m0 = 0.0;
    p->prec_tol = 1e-1;
    p->prec_maxiter = 200;
    p->prec_block = 16;
    p->prec_even_odd = 1;
}

static bool outer_ok(const ovl_outer_params *p)
{
    return p && p->tol > 0.0 && p->tol < 1.0 && p->restart >= 1 && p->restart <= OVL_MAX_RESTART &&
           p->maxiter >= 1 && (p->relax == 0 || p->relax == 1) && p->relax_factor > 0.0 && p->relax_factor <= 1.0 &&
           p->sign_tol_max > 0.0 && p->sign_tol_max < 1.0 && params_ok(&p->inner) &&
           (p->precondition == 0 || p->precondition == 1) && std::isfinite(p->prec_m0) && p->prec_tol > 0.0 &&
           p->prec_tol < 1.0 && p->prec_maxiter >= 1 && p->prec_block >= 1 && p->prec_block <= OVL_MAX_BLOCK &&
           (p->prec_even_odd == 0 || p->prec_even_odd == 1);
}

size_t ovl_overlap_solve_workspace_bytes(const ovl_lattice *lat, int32_t npoles, const ovl_outer_params *prm)
{
    if (!lat_ok(lat) || !outer_ok(prm) || npoles < 1 || npoles > OVL_MAX_SHIFTS) return 0;
    return outer_ws_bytes(make_lat(lat), npoles, prm, lat);
}

int ovl_overlap_solve(const ovl_lattice *lat, const ovl_gauge *U, double rho, const ovl_zolo *z,
                      const ovl_spinor *eta, ovl_spinor *psi, const ovl_outer_params *prm, ovl_outer_stats *stats,
                      void *ws, size_t ws_bytes, void *stream)
{
    if (stats) std::memset(stats, 0, sizeof *stats);
    if (!lat_ok(lat) || !outer_ok(prm) || !zolo_ok(z) || !U || !U->f64 || !U->f32 || !ws) return OVL_ERR_INVALID;
    if (!spinor_ok(eta) || !spinor_ok(psi) || eta->prec != OVL_F64 || psi->prec != OVL_F64 || eta->nrhs != 1 ||
        psi->nrhs != 1 || eta->d == psi->d)
        return OVL_ERR_INVALID;
    if (!(rho > 0.0) || !std::isfinite(rho)) return OVL_ERR_INVALID;
    const size_t need = ovl_overlap_solve_workspace_bytes(lat, z->npoles, prm);
    if (need == 0) return OVL_ERR_INVALID;
    if (ws_bytes < need) return OVL_ERR_WORKSPACE;
    return overlap_solve(lat, U, rho, z, fld(eta), fld(psi), prm, stats, (char *)ws, ws_bytes, S(stream));
}

int ovl_wilson_solve(const ovl_lattice *lat, const ovl_gauge *U, double m0, const ovl_spinor *b, ovl_spinor *x,
                     const ovl_solver_params *prm, ovl_solver_stats *stats, void *ws, size_t ws_bytes, void *stream)
{
    const double t0 = now();
    clear_stats(stats);
    if (!lat_ok(lat) || !params_ok(prm) || !U || !U->f64 || !U->f32 || !ws || !std::isfinite(m0))
        return OVL_ERR_INVALID;
    if (!spinor_ok(b) || !spinor_ok(x) || b->prec != OVL_F64 || x->prec != OVL_F64 || b->nrhs != x->nrhs ||
        b->d == x->d)
        return OVL_ERR_INVALID;
    const size_t need = ovl_workspace_bytes(lat, OVL_OP_WILSON_SOLVE, OVL_F64, b->nrhs, 0, prm);
    if (need == 0) return OVL_ERR_INVALID;
    if (ws_bytes < need) return OVL_ERR_WORKSPACE;
    const Lat L = make_lat(lat);
    double tr[NR];
    int it[NR] = {0};
    int rc = prm->even_odd ? wilson_solve_eo(L, U, m0, fld(b), fld(x), prm->tol, prm->maxiter, tr, it, (char *)ws,
                                             ws_bytes, S(stream))
                           : wilson_solve(L, U, m0, fld(b), fld(x), prm->tol, prm->maxiter,
                                          prm->block > 0 ? prm->block : 16, tr, it, (char *)ws, ws_bytes, S(stream));
    if (rc >= 0 && stats) {
        for (int q = 0; q < b->nrhs; q++) {
            stats->iterations[q] = it[q];
            stats->true_residual[q][0] = tr[q];
        }
        stats->seconds = now() - t0;
    }
    return rc;
}

void ovl_default_eig_params(ovl_eig_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->nev = 16;
    p->extra = 0;
    p->tol = 1e-10;
    p->degree = 60;
    p->steps = 0;
    p->stages = 40;
    p->check_every = 0;
}

size_t ovl_low_modes_workspace_bytes(const ovl_lattice *lat, const ovl_eig_params *prm)
{
    if (!lat_ok(lat) || !eig_ok(prm)) return 0;
    return low_modes_ws_bytes(make_lat(lat), prm);
}

int ovl_low_modes(const ovl_lattice *lat, const ovl_gauge *U, double m0, const ovl_spinor *start,
                  const ovl_eig_params *prm, ovl_spinor *evecs, double *evals, double *residuals,
                  ovl_eig_stats *stats, void *ws, size_t ws_bytes, void *stream)
{
    if (stats) std::memset(stats, 0, sizeof *stats);
    if (!lat_ok(lat) || !eig_ok(prm) || !U || !U->f64 || !ws || !evals || !residuals || !std::isfinite(m0))
        return OVL_ERR_INVALID;
    if (!spinor_ok(start) || start->prec != OVL_F64 || start->nrhs != 1) return OVL_ERR_INVALID;
    if (!spinor_ok(evecs, OVL_MAX_NEV) || evecs->prec != OVL_F64 || evecs->nrhs != prm->nev ||
        evecs->d == start->d)
        return OVL_ERR_INVALID;
    if (ws_bytes < ovl_low_modes_workspace_bytes(lat, prm)) return OVL_ERR_WORKSPACE;
    return low_modes(make_lat(lat), U->f64, m0, fld(start), prm, fld(evecs), evals, residuals, stats, (char *)ws,
                     ws_bytes, S(stream));
}

const char *ovl_status_string(int s)
{
    switch (s) {
    case OVL_OK: return "ok";
    case OVL_NOT_CONVERGED: return "not converged";
    case OVL_ERR_INVALID: return "invalid argument";
    case OVL_ERR_WORKSPACE: return "workspace too small";
    case OVL_ERR_HIP: return "HIP error";
    case OVL_ERR_NONFINITE: return "non-finite value";
    default: return "unknown status";
    }
}

int ovl_last_hip_error(void) { return last_hip_error(); }

const char *ovl_version(void) { return "ovl 0.1 gfx950"; }

}  // extern "C"
