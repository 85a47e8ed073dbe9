// Multishift CG state and kernels shared by the FP64 and mixed solvers.
#pragma once

#include <map>
#include <vector>

#include "internal.h"

namespace ovl {

constexpr int NR = OVL_MAX_RHS;
constexpr int NS = OVL_MAX_SHIFTS;
constexpr int MB = OVL_MAX_BLOCK;   // longest block of the blocked shift update

inline size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// Block lengths of the mixed solver's phases: FP32 phase (block, default 32)
// and FP64 phase (block_f64, default 16).  The FP32 pass with 32 slots moves
// its bytes about as fast as the 16-slot one, the FP64 one does not.
inline int mixed_block(const ovl_solver_params *p) { return p->block > 0 ? p->block : 32; }
inline int mixed_block_f64(const ovl_solver_params *p) { return p->block_f64 > 0 ? p->block_f64 : 16; }

// Sequential carving of a workspace into 256-byte aligned pieces; with a null
// base it only measures.
struct WsCarve {
    char *base;
    size_t off, cap;
    void *take(size_t n)
    {
        void *p = base ? base + off : nullptr;
        off += align256(n);
        return p;
    }
};

// Coefficients of the blocked shift update.  Over a block of iterations
// k0..k0+T-1 the shift recurrences x_j += a_j p_j, p_j = z_j' r + b_j p_j are
// linear in the block-start p_j and the stored residuals r^{k0+1..k0+T}:
//   p_j^{k0+t} = P p_j^{k0} + sum_{i<=t} C_i r^{k0+i},
//   x_j^{k0+T} = x_j^{k0} + XP p_j^{k0} + sum_i X_i r^{k0+i}.
struct Blk {
    double P[NR][NS], XP[NR][NS];
    double C[NR][NS][MB + 1], X[NR][NS][MB + 1];
    int inblk[NR][NS];   // shift active when the block started
    int t[NR];           // iterations done in the current block
};
// Scalar state of a multishift CG on (Q^2 + s_j) x_j = b, one system per RHS,
// kept in device memory so the iteration runs without host round trips.
struct MState {
    double rr[NR], bb[NR], alpha[NR], alpha_old[NR], beta[NR];
    double zeta[NR][NS], zeta_old[NR][NS], zeta_new[NR][NS], aj[NR][NS], bj[NR][NS];
    double delta[NS];      // s_j - s0 (shift offsets from the base shift)
    double s0r[NR];        // base shift of each RHS system
    double tol2r[NR];      // squared relative tolerance of each RHS system
    int act[NR][NS];       // shift still iterating
    int act_cur[NR][NS];   // shifts updated in the current iteration
    int frozen_at[NR][NS];
    double frozen_rr[NR][NS];   // zeta^2 |r|^2 of a shift at the iteration it froze
    int iter[NR];
    int skip[NR];          // RHS finished (every shift frozen) or failed
    int nonfinite[NR];
    int nrhs, nshift;
    // reliable-update bookkeeping (mixed solver)
    double rr_ref[NR];     // |r|^2 at the last residual replacement
    int want_update[NR];
    // hand-over to another precision: an RHS whose base residual reached the
    // hand-over level stops (skip set, paused set) until the solve that
    // continues its recurrences clears both
    int paused[NR];
    int run_c[NR];         // the iteration's p0 update is due (set by K_b, cleared by K_a)
    double one[NR];        // 1 per RHS: the alpha of a residual replacement's update stencil
};

struct ShiftWeights {
    double w[NS];
};

// Options of the blocked multishift CG.
struct BlkOpts {
    int m = 8;                          // block length
    bool keep_x = false;                // x mode (FP64 x_j) instead of y mode
    bool reliable = false;              // FP64 residual replacement of the base system
    bool quiet = false;                 // do not write iteration counts into stats
    const double *rhs_shift = nullptr;  // per-RHS base shift (host), default the smallest shift
    const double *rhs_tol = nullptr;    // per-RHS tolerance (host), default prm->tol
    Fld x_ext{};                        // x mode: caller's FP64 x_j (field j*nrhs + r)
    int x_zero_shifts = 0;              // x mode: x_j (j < this) start at zero (set by the first pass)
    int *iters_out = nullptr;           // per-RHS iteration counts (host)
    // Each RHS stops at the iteration at which |r| <= switch_rel |b| (the
    // block pass then covers the iterations it did); once no unfinished RHS
    // is still iterating, return kSwitched, leaving the recurrences (scalars,
    // r, p0, p_j; x_j in x mode) in the workspace for a solve in another
    // precision to continue (0: run to convergence).
    double switch_rel = 0.0;
    const struct MsScratch *resume = nullptr;   // continue the recurrences of a switched solve
    // FP32 solves: round r (ring), p0 and t = Q p0 through this FP16S field set
    // (nrhs fields with scales) after every update, as FP16S storage would
    Fld f16{};
};

// Return code of a blocked solve that stopped at switch_rel (internal).
constexpr int kSwitched = 2;

size_t blocked_ws_bytes(const Lat &L, int nrhs, int nshift, int m, bool keep_x, int ps, bool ext_x = false);

// Pieces of a solver workspace that callers reuse after the solve.
struct MsScratch {
    double *partials;
    double *red;
    Fld x;       // solutions, field j*nrhs + r
    Fld s1, s2;  // FP64 scratch fields (nrhs each)
    // state of the recurrences at the end of a switched blocked solve
    MState *S = nullptr;
    Fld r{}, p0{}, pj{};
    int j0 = 0;
    // a host copy of S taken after the switch (optional): a solve continuing
    // these recurrences reads its iteration counts and |r|^2 from there
    const MState *host = nullptr;
    // a switched y-mode solve with 48-bit storage: room for nrhs*nshift FP64
    // fields over its dead ring, p0 and t, where a solve continuing it keeps x_j
    void *xlend = nullptr;
};

// alpha and the shifted zeta_j', alpha_j (one block per RHS); defined in solver.hip
__global__ void k_ms_alpha(MState *st, const double *partials, int nblk, int cnt);

// Upload the constant part of the scalar state (per-RHS base shift and
// tolerance default to the smallest shift and prm->tol), |b|^2 per RHS and
// the initial recurrence values.  *j0_out: index of the smallest shift.
int mscg_init_state(const Lat &L, MState *S, double *partials, double *red, Fld b, int nshift, const double *shifts,
                    const ovl_solver_params *prm, int *j0_out, hipStream_t st, const double *rhs_shift,
                    const double *rhs_tol);

// Events of the profiling spans, kept for reuse across solves (per device:
// an event belongs to the device current at its creation).
inline std::vector<hipEvent_t> &event_cache(int dev)
{
    static thread_local std::map<int, std::vector<hipEvent_t>> c;
    return c[dev];
}

// Optional event timing of the solver's kernels, on the solver's stream.
// pair(cls, &e0, &e1) hands out two events for a launch to record at its
// kernel's start and end and charges that span to a kernel class; mark()
// records an event in stream order and span(a, b, cls) charges the interval
// between two marks.  rotate() ends a block, collect() adds the previous
// block's times to the stats, flush() everything recorded so far.
struct Prof {
    bool on = false;
    bool stencil_only = false;   // time only OVL_K_STENCIL (params.profile 2)
    hipStream_t st = nullptr;
    int dev = -1;
    struct Span {
        int a, b, cls;
    };
    // Two banks of events: a block records into one while the spans of the
    // block before it, in the other, wait to be read (collect) until the new
    // block's first launches are queued, so those event queries overlap GPU
    // work instead of leaving the GPU idle at every block end.
    std::vector<hipEvent_t> ev[2];
    std::vector<Span> spans[2];
    int used[2] = {0, 0};
    int cur = 0, n = 0;
    bool pending = false;
    // the next event of the current bank (from the cache, else new)
    hipEvent_t take()
    {
        std::vector<hipEvent_t> &e = ev[cur];
        if (n == (int)e.size()) {
            if (dev < 0 && hipGetDevice(&dev) != hipSuccess) return nullptr;
            std::vector<hipEvent_t> &c = event_cache(dev);
            hipEvent_t x = nullptr;
            if (!c.empty()) {
                x = c.back();
                c.pop_back();
            } else if (hipEventCreate(&x) != hipSuccess) {
                return nullptr;
            }
            e.push_back(x);
        }
        return e[n++];
    }
    // an event recorded here, in stream order (a span of class OVL_K_OTHER
    // or OVL_K_UPDATE will follow); its index, or -1
    int mark()
    {
        if (!on || stencil_only) return -1;
        hipEvent_t e = take();
        if (!e || hipEventRecord(e, st) != hipSuccess) return -1;
        return n - 1;
    }
    // two events for a launch to record at its kernel's start and end
    // (launch_k, launch_wilson), timed as one span of class cls; null when off
    void pair(int cls, hipEvent_t *e0, hipEvent_t *e1)
    {
        *e0 = *e1 = nullptr;
        if (!on || (stencil_only && cls != OVL_K_STENCIL)) return;
        hipEvent_t a = take(), b = a ? take() : nullptr;
        if (!a || !b) return;
        *e0 = a;
        *e1 = b;
        spans[cur].push_back({n - 2, n - 1, cls});
    }
    void span(int a, int b, int cls)
    {
        if (on && a >= 0 && b >= 0) spans[cur].push_back({a, b, cls});
    }
    // add the times of one bank's spans to the stats
    int read(int bank, ovl_solver_stats *s)
    {
        if (used[bank] > 0) {
            hipError_t e = hipEventSynchronize(ev[bank][used[bank] - 1]);
            if (e != hipSuccess) return hip_fail(e);
        }
        for (auto &sp : spans[bank]) {
            float ms = 0.f;
            hipError_t e = hipEventElapsedTime(&ms, ev[bank][sp.a], ev[bank][sp.b]);
            if (e != hipSuccess) return hip_fail(e);
            if (s) {
                s->kernel_seconds[sp.cls] += 1e-3 * ms;
                s->kernel_launches[sp.cls] += 1;
            }
        }
        spans[bank].clear();
        used[bank] = 0;
        return OVL_OK;
    }
    // read the spans left waiting by rotate
    int collect(ovl_solver_stats *s)
    {
        if (!on || !pending) return OVL_OK;
        pending = false;
        return read(1 - cur, s);
    }
    // end of a block: its spans wait while the next block records into the
    // other bank (read first whatever still waits there)
    int rotate(ovl_solver_stats *s)
    {
        if (!on) return OVL_OK;
        int rc = collect(s);
        if (rc) return rc;
        used[cur] = n;
        pending = true;
        cur = 1 - cur;
        n = 0;
        return OVL_OK;
    }
    // read everything recorded so far
    int flush(ovl_solver_stats *s)
    {
        if (!on) return OVL_OK;
        int rc = collect(s);
        if (rc) return rc;
        used[cur] = n;
        n = 0;
        return read(cur, s);
    }
    ~Prof()
    {
        if (dev < 0) return;
        std::vector<hipEvent_t> &c = event_cache(dev);
        for (auto &b : ev) c.insert(c.end(), b.begin(), b.end());
    }
};

template <int PS>
int mscg_blocked_t(const Lat &L, const ovl_gauge *U, double m0, int nshift, const double *shifts,
                   const double *weights, Fld b, Fld yout, const BlkOpts &o, const ovl_solver_params *prm,
                   ovl_solver_stats *stats, char *ws, size_t ws_bytes, hipStream_t st, MsScratch *scr);

}  // namespace ovl
