// Multishift CG state and kernels shared by the FP64 and mixed solvers.
#pragma once

#include "internal.h"

namespace ovl {

constexpr int NR = OVL_MAX_RHS;
constexpr int NS = OVL_MAX_SHIFTS;

// Scalar state of a multishift CG on (Q^2 + s_j) x_j = b, one system per RHS,
// kept in device memory so the iteration runs without host round trips.
struct MState {
    double rr[NR], bb[NR], alpha[NR], alpha_old[NR], beta[NR];
    double zeta[NR][NS], zeta_old[NR][NS], zeta_new[NR][NS], aj[NR][NS], bj[NR][NS];
    double delta[NS];      // s_j - s0
    double s0, tol2;
    int act[NR][NS];       // shift still iterating
    int act_cur[NR][NS];   // shifts updated in the current iteration
    int frozen_at[NR][NS];
    int iter[NR];
    int skip[NR];          // RHS finished (every shift frozen) or failed
    int nonfinite[NR];
    int nrhs, nshift;
    // reliable-update bookkeeping (mixed solver)
    double rr_ref[NR];     // |r|^2 at the last residual replacement
    int want_update[NR];
};

struct ShiftWeights {
    double w[NS];
};

// Pieces of a solver workspace that callers reuse after the solve.
struct MsScratch {
    double *partials;
    double *red;
    Fld x;       // solutions, field j*nrhs + r
    Fld s1, s2;  // FP64 scratch fields (nrhs each)
};

}  // namespace ovl
