/*
 * ovl.h -- C ABI of an MI355X (gfx950) library that applies the Neuberger
 * overlap operator with a Wilson-Dirac kernel,
 *
 *     D_ov = rho (I + Gamma_5 sign(Q)),   Q = Gamma_5 D_W(-rho),
 *
 * following Brannick, Frommer, Kahl, Leder, Rottmann, Strebel, "Multigrid
 * preconditioning for the overlap operator in lattice QCD" (arXiv:1410.7170):
 * D_W is eq. (Wilson-Dirac), Gamma_5-hermiticity is eq. (gamma_5_symmetry),
 * the overlap operator is eq. (overlap_def) written in the massless
 * normalisation rho (I + Gamma_5 sign(Gamma_5 D_W(-rho))).  sign(Q) is a
 * Zolotarev rational function of Q whose shifted systems
 * (Q^2 + s_l) x_l = b are solved together by multishift CG.
 *
 * Conventions
 * -----------
 * Lattice: extents dims[0..3] = (L0, L1, L2, L3), x0 is time, every extent even
 *   (the device layout is even-odd, as in the red-black ordering of the
 *   proof of Lemma 1).  Hops that cross the boundary in direction mu carry the
 *   phase bc[mu] in {+1,-1}; the usual choice is (-1,+1,+1,+1).
 * Canonical host/device order (complex128):
 *   spinor psi[site][spin][colour], gauge U[site][mu][row][col] with U_mu(x)
 *   the link from x to x+mu, site = ((x0*L1 + x1)*L2 + x2)*L3 + x3.
 * gamma basis: Hermitian chiral basis, gamma_0 = [[0,I],[I,0]],
 *   gamma_k = [[0,-i sigma_k],[i sigma_k,0]], gamma_5 = g0 g1 g2 g3 = diag(-1,-1,1,1).
 * Device layouts (all produced by the pack calls below; treat as opaque).
 * Every array below is indexed [..][S] with S = round_up(V/2, 16) + 24 sites
 * (padding keeps the component arrays of one site off power-of-two strides):
 *   OVL_F64  spinor: complex128 per component, [rhs][parity][12][S]
 *   OVL_F32  spinor: float4 (two components), [rhs][parity][6][S]
 *   OVL_F48  spinor: each real stored in 48 bits (a double rounded to nearest
 *            at 36 stored mantissa bits), [rhs][parity][9][S] of 16-byte
 *            elements: elements 0..5 the top 32 bits of components 2k, 2k+1
 *            (re, im, re, im), elements 6..8 the low 16 bits of components
 *            4g..4g+3 (word q: re | im << 16); its stencils use the F64 links
 *   OVL_F16S spinor: 8 halves (four components), [rhs][parity][3][S], plus
 *            one float scale per site [rhs][parity][S]: stored = value/scale,
 *            scale = largest |real or imaginary part| at that site
 *   gauge F64: rows 0 and 1 as complex128, [parity][mu][6][S]; row 2 is
 *            rebuilt as conj(row0 x row1) (exact for SU(3), which the links
 *            must be)
 *   gauge F32: rows 0 and 1 as 3 float4, [parity][mu][3][S]
 *   gauge F16: rows 0 and 1 as 3 x 4 halves, [parity][mu][3][S]
 *
 * Every call is asynchronous on the caller's HIP stream (`stream`, a
 * hipStream_t; NULL is the null stream) unless it says it synchronises.
 * Device pointers are plain device addresses; the library keeps no pointer
 * after a call returns and allocates no device memory: temporaries live in a
 * caller-provided workspace whose size ovl_workspace_bytes reports.
 * Return values: OVL_OK (0); OVL_NOT_CONVERGED (1) -- outputs and stats hold
 * the last iterate; negative values are errors and leave outputs undefined:
 *   OVL_ERR_INVALID    null pointer, odd extent, mismatched precision or
 *                      RHS count, aliased input/output, out-of-range count
 *   OVL_ERR_WORKSPACE  workspace too small
 *   OVL_ERR_HIP        a HIP call failed (ovl_last_hip_error gives its code)
 *   OVL_ERR_NONFINITE  a norm became NaN or Inf
 * No call throws across this boundary.
 */
#ifndef OVL_H
#define OVL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define OVL_API __attribute__((visibility("default")))
#else
#define OVL_API
#endif

#define OVL_MAX_SHIFTS 32
#define OVL_MAX_RHS 16
#define OVL_MAX_BLOCK 32   /* longest block length of ovl_solver_params.block */

enum ovl_status {
    OVL_OK = 0,
    OVL_NOT_CONVERGED = 1,
    OVL_ERR_INVALID = -1,
    OVL_ERR_WORKSPACE = -2,
    OVL_ERR_HIP = -3,
    OVL_ERR_NONFINITE = -4
};

/* storage precision of a field; arithmetic is FP64 for OVL_F64 and OVL_F48
 * and FP32 (FP64 accumulation of dot products) for OVL_F32 and OVL_F16S.
 * Gauge fields exist in OVL_F64, OVL_F32 and OVL_F16S (as F16 links). */
enum ovl_prec { OVL_F64 = 0, OVL_F32 = 1, OVL_F16S = 2, OVL_F48 = 3 };

/* solver precision modes */
enum ovl_solve_mode {
    OVL_SOLVE_F64 = 0,   /* every vector, link and stencil in FP64 */
    OVL_SOLVE_MIXED = 1, /* sloppy FP32 Krylov bulk, FP64 reliable updates,
                            FP64 per-shift verification and final combination;
                            reads the FP64 and FP32 links (gauge f64, f32) */
    OVL_SOLVE_LANCZOS = 2 /* sign_q_apply / overlap_apply only: sign(Q) b as the
                            Lanczos approximation |b| V_k sign(T_k) e_1 on the
                            Krylov space of Q, in FP64, in two passes (the
                            first keeps only the Lanczos coefficients, the second
                            regenerates the basis), without the Zolotarev
                            function (z is still validated); tol: the relative
                            change of the coefficient vector between checks
                            every 32 steps; maxiter: Lanczos steps (< 4096);
                            stats iterations: the steps of each RHS */
};

typedef struct {
    int32_t dims[4];   /* L0 (time), L1, L2, L3; all even, all >= 2 */
    int32_t bc[4];     /* boundary phase per direction, +1 or -1 */
    int64_t vol;       /* filled by ovl_lattice_init */
    int32_t tile_t;    /* stencil site order: number of time slices swept per
                          x1 column (divides dims[0]); set by ovl_lattice_init,
                          may be changed by an autotuner; results do not
                          depend on it beyond summation order */
    int32_t stream_t;  /* 0: one stencil thread per site, in tile_t order.
                          s > 0: FP64 and FP32 stencils stream in time, each
                          thread walking s consecutive time slices of one
                          spatial site (needs s | dims[0], s <= 256 and
                          dims[1]*dims[2]*dims[3] a multiple of 256); FP16
                          stencils always use one thread per site.  Set by
                          ovl_lattice_init; results do not depend on it
                          beyond summation order */
    int32_t stream_t64;/* time slices per thread of the FP64 stencil in the
                          streaming form (same conditions as stream_t);
                          0: FP64 follows stream_t.  Set by ovl_lattice_init */
    int32_t rhs_tile;  /* 1, 2, 4 or 8: the streaming stencil on several RHS
                          gives each site K consecutive lanes holding K RHS, so
                          one link load serves K RHS; K is this value capped at
                          the next power of two of the RHS count, and halved
                          while a block's sites times the stream length are
                          fewer than 256.  1 (one RHS per block) is set by
                          ovl_lattice_init; results do not depend on it */
    int32_t mfma;      /* 1: FP32 D_W and Gamma_5 D_W (ovl_wilson_apply,
                          ovl_q_apply and the first stencil of ovl_q2_apply) on
                          2 or more RHS run on the matrix cores
                          (v_mfma_f32_16x16x4f32, two sites and four RHS per
                          wave); 0 (set by ovl_lattice_init): vector ALUs.
                          Results agree to FP32 rounding */
} ovl_lattice;

/* A gauge field packed in up to three precisions (device pointers).  An
 * operation uses the copy matching its precision and fails with
 * OVL_ERR_INVALID if that copy is NULL. */
typedef struct {
    const void *f64;
    const void *f32;
    const void *f16;
} ovl_gauge;

/* nrhs packed spinor fields of one precision, stored back to back. */
typedef struct {
    void *d;           /* device data */
    float *scale;      /* OVL_F16S only: per-site scales, else NULL */
    int32_t prec;      /* enum ovl_prec */
    int32_t nrhs;      /* 1 .. OVL_MAX_RHS */
} ovl_spinor;

/* Zolotarev data: sign(x) ~ x sum_l weights[l] / (x^2 + shifts[l]) on
 * lambda_min <= |x| <= lambda_max (host arrays). */
typedef struct {
    int32_t npoles;
    const double *shifts;
    const double *weights;
} ovl_zolo;

/* Low modes of Q for deflation (Section 5.2, deflation of sign(Gamma_5 D_W)):
 * the eigenvectors xi_i of Q = Gamma_5 D_W(m0) with the smallest |lambda_i|,
 * orthonormal, as FP64 fields evecs.d (evecs.nrhs = k of them, field i at
 * i * ovl_spinor_bytes, same layout as any spinor), and the eigenvalues
 * lambda_i (host).  With it, sign(Q) chi = sum_i sign(lambda_i) (xi_i^H chi) xi_i
 * + sign(Q) Pi chi, Pi = I - Xi Xi^H: the Zolotarev/multishift (or Lanczos)
 * approximation acts on Pi chi only, so its lambda_min may be raised to the
 * smallest |lambda| outside the deflated set.  Written by ovl_low_modes or by
 * the caller; read-only to the solvers. */
#define OVL_MAX_NEV 256
typedef struct {
    ovl_spinor evecs;        /* FP64, nrhs = k (1..OVL_MAX_NEV) */
    const double *evals;     /* host, k eigenvalues of Q (signed) */
} ovl_deflation;

typedef struct {
    double tol;              /* target relative residual of every shifted system */
    int32_t maxiter;         /* cap on multishift CG iterations */
    int32_t mode;            /* enum ovl_solve_mode */
    double reliable_delta;   /* mixed: FP64 residual replacement when ||r|| has
                                fallen by this factor since the last one */
    int32_t check_every;     /* iterations between host convergence polls */
    int32_t refine;          /* mixed: verify each shift in FP64 and refine
                                those above tol (1) or only report (0) */
    int32_t verify;          /* FP64 mode: also compute every shift's FP64 true
                                residual into stats (2 FP64 stencils per shift) */
    int32_t profile;         /* time the solver's kernels with HIP events on
                                the call's stream and fill the kernel_* stats:
                                1 every class, 2 the stencils only (each timed
                                kernel costs a little; 2 keeps the cost to the
                                dominant class); 0 (default) none */
    int32_t block;           /* FP64 mode: 0 updates every shifted vector in every
                                iteration; m = 1..OVL_MAX_BLOCK keeps the last m residuals
                                and updates each shifted vector once per m
                                iterations (same iterates, fewer vector passes).
                                Mixed mode: block length of the FP32 phase,
                                0 meaning 32 */
    double sloppy_below;     /* mixed: iterate in FP64 (blocked, accumulating the
                                weighted sum directly) until each RHS's base
                                residual ||r||/||b|| falls below this,
                                then hand the recurrences over to FP32; rounding
                                of the sloppy phase then enters the shifted
                                residuals only at this level.  0: FP32 from the
                                first iteration */
    int32_t block_f64;       /* mixed: block length of the FP64 phase,
                                1..OVL_MAX_BLOCK, 0 meaning 16 */
    int32_t rhs_group;       /* sign_q_apply, overlap_apply and multishift_cg
                                with weights: solve the RHS of a call in
                                consecutive groups of this many, one after
                                another in the same workspace (0: all
                                together); ovl_workspace_bytes sizes the
                                workspace for one group.  Ignored by
                                multishift_cg without weights */
    const ovl_deflation *deflation; /* sign_q_apply, overlap_apply (and through
                                them the outer solver): deflate these low
                                modes of Q (NULL: none, the default).  The
                                Zolotarev interval of the call should then
                                start at the smallest |lambda| not deflated */
    int32_t sloppy_f16;      /* mixed: 1 rounds the FP32 phase's Krylov vectors
                                (residual ring, p0 and Q p0) through FP16
                                storage with per-site scales after every update,
                                as FP16S storage of them would; a measurement
                                mode for that format's residual floor and
                                iteration count (the extra conversions make it
                                slower, not faster).  0 (default): FP32 */
    int32_t even_odd;        /* ovl_wilson_solve only: 1 solves the even-odd
                                reduced system (Schur complement on the even
                                sites) by an FP32 CGLS inside FP64 defect
                                correction and stops on the true residual
                                |b - D_W x| <= tol |b|; maxiter caps its CGLS
                                iterations.  0 (default): CG on the normal
                                equations of the full lattice, as described
                                at ovl_wilson_solve */
    int32_t store48;         /* mixed: 1 (default) stores the FP64 phase's
                                Krylov vectors (residual ring, Q p and the
                                shifted directions p_j) in 48 bits per real
                                (OVL_F48: rounded to nearest at 36 stored
                                mantissa bits, relative error <= 2^-37), with
                                FP64 links and arithmetic.  The rounding opens
                                a gap of about 1e-12 |b| between recursive and
                                true residuals, which the verification does not
                                see, so the solve then aims at 0.9 tol (the
                                reported residuals are then <= 0.9 tol).  It
                                needs the phase's
                                unshifted base system (positive caller shifts,
                                fewer than OVL_MAX_SHIFTS of them) and falls
                                back to FP64 storage without it.  0: FP64 */
} ovl_solver_params;

/* kernel classes of ovl_solver_stats.kernel_* */
enum ovl_kernel_class {
    OVL_K_STENCIL = 0,   /* the two Wilson stencils of each iteration */
    OVL_K_UPDATE = 1,    /* the fused shift update x_l += a_l p_l, p_l = z_l r + b_l p_l */
    OVL_K_SCALAR = 2,    /* block reductions and the FP64 scalar recurrences */
    OVL_K_OTHER = 3      /* reliable updates, refinement, combination */
};

typedef struct {
    int32_t iterations[OVL_MAX_RHS];                  /* multishift CG iterations per RHS */
    int32_t shift_iters[OVL_MAX_RHS][OVL_MAX_SHIFTS]; /* iteration at which each shift froze */
    double true_residual[OVL_MAX_RHS][OVL_MAX_SHIFTS];/* FP64 ||b-(Q^2+s)x||/||b||, or -1 if not computed */
    int32_t reliable_updates;                          /* FP64 residual replacements */
    int32_t refine_iterations;                         /* iterations spent in per-shift refinement */
    int32_t stencil_applies;                           /* Wilson stencils launched (per RHS batch) */
    double algorithmic_bytes;                          /* compulsory HBM bytes of the launches */
    double seconds;                                    /* wall time of the call (it synchronises) */
    /* with params.profile: summed event-timed duration, compulsory bytes and
     * launch count per ovl_kernel_class */
    double kernel_seconds[4];
    double kernel_bytes[4];
    int32_t kernel_launches[4];
} ovl_solver_stats;

/* ---- set-up and layout ------------------------------------------------ */

/* Validates dims (even, >= 2) and bc (+1/-1), fills lat->vol and picks
 * lat->tile_t. */
OVL_API int ovl_lattice_init(ovl_lattice *lat, const int32_t dims[4], const int32_t bc[4]);

/* Bytes of one packed spinor field (per RHS) and of its scale array. */
OVL_API size_t ovl_spinor_bytes(const ovl_lattice *lat, int32_t prec);
OVL_API size_t ovl_scale_bytes(const ovl_lattice *lat);
/* Bytes of a packed gauge field of the given precision. */
OVL_API size_t ovl_gauge_bytes(const ovl_lattice *lat, int32_t prec);

/* Canonical complex128 device spinors ([nrhs][V][4][3]) to and from the
 * packed layout of out->prec / in->prec.  F16S packing picks the per-site
 * scale; unpacking widens exactly.  These two accept field sets of up to
 * OVL_MAX_RHS*OVL_MAX_SHIFTS fields (e.g. the per-shift solutions). */
OVL_API int ovl_pack_spinor(const ovl_lattice *lat, const void *canon, ovl_spinor *out, void *stream);
OVL_API int ovl_unpack_spinor(const ovl_lattice *lat, const ovl_spinor *in, void *canon, void *stream);

/* Canonical complex128 device gauge field ([V][4][3][3]) to the packed layout
 * of precision prec, written to out (ovl_gauge_bytes(lat, prec) bytes). */
OVL_API int ovl_pack_gauge(const ovl_lattice *lat, const void *canon, int32_t prec, void *out, void *stream);

/* ---- operators ---------------------------------------------------------- */

/* out = D_W(m0) in, eq. (Wilson-Dirac) with a = 1:
 *   (D_W psi)(x) = (m0+4) psi(x) - 1/2 sum_mu (I - gamma_mu) U_mu(x) psi(x+mu)
 *                                - 1/2 sum_mu (I + gamma_mu) U_mu(x-mu)^H psi(x-mu).
 * in and out: same precision and RHS count, distinct buffers.  All RHS share
 * each link load. */
OVL_API int ovl_wilson_apply(const ovl_lattice *lat, const ovl_gauge *U, double m0,
                     const ovl_spinor *in, ovl_spinor *out, void *stream);

/* out = Q in = Gamma_5 D_W(m0) in (Hermitian by eq. (gamma_5_symmetry)). */
OVL_API int ovl_q_apply(const ovl_lattice *lat, const ovl_gauge *U, double m0,
                const ovl_spinor *in, ovl_spinor *out, void *stream);

/* out = (Q^2 + shift) in, Q^2 = D_W^H D_W.  ws: device workspace of at least
 * ovl_workspace_bytes(lat, OVL_OP_Q2, in->prec, in->nrhs, 0, NULL) bytes. */
OVL_API int ovl_q2_apply(const ovl_lattice *lat, const ovl_gauge *U, double m0, double shift,
                 const ovl_spinor *in, ovl_spinor *out, void *ws, size_t ws_bytes, void *stream);

/* Bytes of the scratch array of ovl_q2_apply_noalloc, per GPU. */
#define OVL_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)

/* ovl_q2_apply without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops that forbid hipMalloc).  The intermediate field Q in lives in
 * a library-owned device array of OVL_NOALLOC_SCRATCH_BYTES on each GPU,
 * held from the library's load until the process ends.  The call needs
 * ovl_workspace_bytes(lat, OVL_OP_Q2, in->prec, in->nrhs, 0, NULL) to fit it
 * (one FP64 field up to 24^3x48 and two there, one FP32 field at 32^3x64)
 * and returns OVL_ERR_WORKSPACE otherwise, before any device work.  All calls
 * on one GPU share its array: calls that overlap on one GPU (other streams or
 * threads) race.  The first call on a device looks up the array's address on
 * the current device (not a stream operation); every call then only launches
 * the two stencils on `stream`.  Arguments, layouts and other errors as
 * ovl_q2_apply. */
OVL_API int ovl_q2_apply_noalloc(const ovl_lattice *lat, const ovl_gauge *U, double m0, double shift,
                                 const ovl_spinor *in, ovl_spinor *out, void *stream);

/* ---- sign function and overlap ------------------------------------------ */

/* Zolotarev coefficients (host only): shifts[n], weights[n] with
 * sign(x) ~ x sum_l weights[l]/(x^2+shifts[l]) for lambda_min <= |x| <= lambda_max,
 * and the relative error bound *delta on that range. */
OVL_API int ovl_zolotarev(double lambda_min, double lambda_max, int32_t npoles,
                  double *shifts, double *weights, double *delta);

/* Bounds of |Q| = sqrt(Q^2) from iters Lanczos steps on Q^2 in FP64 started
 * at the FP64 device spinor `start` (its random numbers are the caller's).
 * The extreme Ritz values lie inside the spectrum; the returned interval is
 * widened to [lo_margin*sqrt(theta_min), hi_margin*sqrt(theta_max)].
 * Synchronises the stream. */
OVL_API int ovl_spectral_bounds(const ovl_lattice *lat, const ovl_gauge *U, double m0, int32_t iters,
                        const ovl_spinor *start, double lo_margin, double hi_margin,
                        double *lambda_min, double *lambda_max,
                        void *ws, size_t ws_bytes, void *stream);

/* Low modes of Q (for ovl_deflation): the nev eigenpairs of
 * Q = Gamma_5 D_W(m0) smallest in |lambda|, in FP64.
 * A Lanczos run on Q^2 (`steps` steps, full reorthogonalisation by classical
 * Gram-Schmidt twice) from the FP64 device spinor `start` gives the top of the
 * spectrum theta_max and a block of nev + extra Ritz vectors.  Then
 * Chebyshev-filtered subspace iteration: the block is multiplied by
 * T_degree(a Q^2 + b), which is bounded by 1 on [theta_cut, theta_max] and
 * grows steeply below theta_cut, orthonormalised, and resolved into
 * eigenvectors of Q by Rayleigh-Ritz with Q on its span (Q^2 pairs
 * lambda^2 ~ (-lambda')^2, which only Q separates; H = Y^H Q Y diagonalised on
 * the host by Hermitian Jacobi).  The nev pairs with the smallest |Q x| are
 * tested against tol; theta_cut moves down to the block's largest Rayleigh-Ritz
 * value of Q^2 (an upper bound of that eigenvalue) times 1.05, at most
 * `stages` iterations; each iteration's degree is capped so that the filter's
 * gain at the lowest Rayleigh-Ritz value stays below 1e5, which keeps the
 * block's weaker directions above the rounding of its dominant ones.  The
 * filter runs on the whole block per stencil launch
 * (nrhs = nev + extra).  evecs: FP64, nrhs = nev fields, written; evals[nev]
 * (ascending |lambda|) and residuals[nev] = |Q xi_i - lambda_i xi_i|
 * (|xi_i| = 1) written on the host.  Returns OVL_OK when every residual is
 * <= tol, OVL_NOT_CONVERGED when the iterations ran out first (the best pairs
 * are still returned), or an error.  The start vector's random numbers are the
 * caller's.  Synchronises the stream. */
typedef struct {
    int32_t nev;             /* number of low modes, 1..OVL_MAX_NEV (16) */
    int32_t extra;           /* block size beyond nev (0: nev/2 + 4) */
    double tol;              /* residual target |Q xi - lambda xi| (1e-10) */
    int32_t degree;          /* Chebyshev degree of the filter, 1..200 (60) */
    int32_t steps;           /* steps of the seeding Lanczos run, >= nev + extra
                                (0: max(40, nev + extra + 8)) */
    int32_t stages;          /* cap on filtered subspace iterations, 1..200 (40) */
    int32_t check_every;     /* reserved (0) */
} ovl_eig_params;

typedef struct {
    int32_t steps;           /* steps of the seeding Lanczos run */
    int32_t stages;          /* filtered subspace iterations run */
    int64_t q2_applies;      /* applications of Q^2 (two stencils each) */
    int32_t converged;       /* 1 if every residual met tol */
    int32_t reserved;
    double max_residual;     /* max_i |Q xi_i - lambda_i xi_i| */
    double lambda_next;      /* the smallest |lambda| of the Rayleigh-Ritz pairs
                                not returned: an estimate of |lambda_{nev+1}|,
                                not a bound (|evals[nev-1]| is a safe lower
                                edge for the deflated Zolotarev interval) */
    double theta_cut;        /* the filter's final lower edge */
    double mean_degree;      /* mean filter degree over the iterations */
    double seconds;
} ovl_eig_stats;

OVL_API void ovl_default_eig_params(ovl_eig_params *prm);
OVL_API size_t ovl_low_modes_workspace_bytes(const ovl_lattice *lat, const ovl_eig_params *prm);
OVL_API int ovl_low_modes(const ovl_lattice *lat, const ovl_gauge *U, double m0, const ovl_spinor *start,
                          const ovl_eig_params *prm, ovl_spinor *evecs, double *evals, double *residuals,
                          ovl_eig_stats *stats, void *ws, size_t ws_bytes, void *stream);

/* Multishift CG on (Q^2 + shifts[l]) x_l = b, l = 0..nshift-1, every RHS of b
 * independently.  If weights is NULL, x holds nshift*b->nrhs fields
 * (field index l*nrhs + r, FP64; this count may exceed OVL_MAX_RHS);
 * otherwise x holds b->nrhs FP64 fields
 * y_r = sum_l weights[l] x_{l,r}.  b: FP64 spinor.  Synchronises the stream;
 * fills stats if non-NULL. */
OVL_API int ovl_multishift_cg(const ovl_lattice *lat, const ovl_gauge *U, double m0,
                      int32_t nshift, const double *shifts, const double *weights,
                      const ovl_spinor *b, ovl_spinor *x, const ovl_solver_params *prm,
                      ovl_solver_stats *stats, void *ws, size_t ws_bytes, void *stream);

/* out = sign(Q) b ~ Q sum_l w_l (Q^2 + s_l)^{-1} b, Q = Gamma_5 D_W(m0).
 * b, out: FP64 spinors with equal nrhs.  With prm->deflation the low modes
 * are projected out first and added back exactly (see ovl_deflation).
 * Synchronises the stream. */
OVL_API int ovl_sign_q_apply(const ovl_lattice *lat, const ovl_gauge *U, double m0, const ovl_zolo *z,
                     const ovl_spinor *b, ovl_spinor *out, const ovl_solver_params *prm,
                     ovl_solver_stats *stats, void *ws, size_t ws_bytes, void *stream);

/* out = D_ov b = rho (b + Gamma_5 sign(Q) b) = rho (b + D_W(-rho) y),
 * y = sum_l w_l (Q^2 + s_l)^{-1} b, Q = Gamma_5 D_W(-rho) (eq. (overlap_def),
 * massless normalisation).  b, out: FP64 spinors with equal nrhs; the final
 * combination and stencil are FP64 in every mode.  With prm->deflation,
 * sign(Q) b is formed as for ovl_sign_q_apply.  Synchronises the stream. */
OVL_API int ovl_overlap_apply(const ovl_lattice *lat, const ovl_gauge *U, double rho, const ovl_zolo *z,
                      const ovl_spinor *b, ovl_spinor *out, const ovl_solver_params *prm,
                      ovl_solver_stats *stats, void *ws, size_t ws_bytes, void *stream);

/* ---- outer solver ---------------------------------------------------------- */

#define OVL_MAX_RESTART 512   /* longest restart length of ovl_overlap_solve */

/* Parameters of ovl_overlap_solve (defaults from ovl_default_outer_params,
 * after Table (allparms1)). */
typedef struct {
    double tol;              /* eps_outer: required reduction |r|/|eta| (1e-8) */
    int32_t restart;         /* FGMRES restart length m_restart, 1..OVL_MAX_RESTART (100) */
    int32_t maxiter;         /* cap on Krylov steps (D_ov applications) (1000) */
    int32_t relax;           /* 1: at step k the multishift tolerance of the D_ov
                                application is min(sign_tol_max,
                                tol * relax_factor / (|r_k|/|eta|)); 0: the fixed
                                tol * relax_factor (1) */
    double relax_factor;     /* 1e-2 */
    double sign_tol_max;     /* cap of the relaxed tolerance (1e-2) */
    ovl_solver_params inner; /* the D_ov applications' multishift CG (its tol is
                                set per step; mixed mode scales sloppy_below with
                                it); defaults of ovl_default_params in mixed mode */
    int32_t precondition;    /* 1: right preconditioner D_W(prec_m0)^{-1} applied
                                by ovl_wilson_solve's method (0) */
    double prec_m0;          /* m0^prec (eq. (default_m)); no default: the caller's */
    double prec_tol;         /* eps_prec, the preconditioner's relative residual
                                on its normal equations (1e-1) */
    int32_t prec_maxiter;    /* cap on each preconditioner solve's CG iterations (200) */
    int32_t prec_block;      /* block length of that CG, 1..OVL_MAX_BLOCK (16) */
    int32_t prec_even_odd;   /* 1: the preconditioner solves are ovl_wilson_solve's
                                even-odd form, prec_tol then bounding the true
                                residual |v - D_W z| / |v| of each (the paper's
                                eps_prec) and prec_maxiter its CGLS iterations;
                                0: the normal-equations CG (1) */
} ovl_outer_params;

typedef struct {
    int32_t iterations;        /* Krylov steps (each one D_ov application) */
    int32_t restarts;          /* FGMRES cycles after the first */
    int32_t overlap_applies;   /* all D_ov applications (steps and residual checks) */
    int32_t mscg_iterations;   /* multishift CG iterations over all of them */
    int32_t prec_iterations;   /* CG iterations over all preconditioner solves */
    double residual;           /* |eta - D_ov psi| / |eta| of the returned psi, from a
                                  D_ov applied with multishift tolerance
                                  tol * relax_factor */
    double estimated_residual; /* the FGMRES estimate at the last step */
    double seconds;            /* wall time of the call (it synchronises) */
} ovl_outer_stats;

OVL_API void ovl_default_outer_params(ovl_outer_params *prm);

/* Workspace bytes of ovl_overlap_solve for npoles Zolotarev poles. */
OVL_API size_t ovl_overlap_solve_workspace_bytes(const ovl_lattice *lat, int32_t npoles,
                                                 const ovl_outer_params *prm);

/* psi = D_ov^{-1} eta, D_ov = rho (I + Gamma_5 sign(Q)) as in ovl_overlap_apply
 * (eq. (linsys) with the overlap operator of eq. (overlap_def)), by restarted
 * flexible GMRES in FP64 with relaxed D_ov applications and an optional
 * Wilson-Dirac right preconditioner D_W(m0^prec)^{-1} (Section 3).  eta, psi:
 * FP64 spinors with nrhs = 1.  The gauge field needs its FP64 and FP32 copies.
 * Returns OVL_OK when |eta - D_ov psi| <= tol |eta| (the check applies D_ov with
 * multishift tolerance tol * relax_factor), OVL_NOT_CONVERGED at maxiter with
 * psi the last iterate, or an error.  Synchronises the stream. */
OVL_API int ovl_overlap_solve(const ovl_lattice *lat, const ovl_gauge *U, double rho, const ovl_zolo *z,
                              const ovl_spinor *eta, ovl_spinor *psi, const ovl_outer_params *prm,
                              ovl_outer_stats *stats, void *ws, size_t ws_bytes, void *stream);

/* x = D_W(m0)^{-1} b (eq. (Wilson-Dirac)) for each RHS, the Wilson solve of
 * the outer iteration's preconditioner (Section 5.1).  prm->even_odd = 0:
 * through the normal equations D_W^H D_W x = D_W^H b with D_W^H = Gamma_5 D_W
 * Gamma_5 (eq. (gamma_5_symmetry)): an FP32 CG (block length prm->block, 0
 * meaning 16) with FP64 residual replacement, to prm->tol relative residual of
 * the normal equations or prm->maxiter iterations.  prm->even_odd = 1: the
 * even-site Schur complement system M x_e = b_e + H_eo b_o / (2(m0+4)),
 * M = (m0+4) - H_eo H_oe / (4(m0+4)), by an FP32 CGLS inside FP64 defect
 * correction, then x_o = (b_o + H_oe x_e / 2) / (m0+4); it stops when the true
 * residual |b - D_W x| <= prm->tol |b| or after prm->maxiter CGLS iterations
 * (m0 = -4 is rejected).  b, x: FP64 spinors, equal nrhs, distinct.  stats (optional): iterations[q] and true_residual[q][0] =
 * |b - D_W x| / |b| in FP64.  ws: ovl_workspace_bytes(lat, OVL_OP_WILSON_SOLVE,
 * OVL_F64, nrhs, 0, prm) bytes.  Returns OVL_OK, OVL_NOT_CONVERGED or an
 * error.  Synchronises the stream. */
OVL_API int ovl_wilson_solve(const ovl_lattice *lat, const ovl_gauge *U, double m0, const ovl_spinor *b,
                             ovl_spinor *x, const ovl_solver_params *prm, ovl_solver_stats *stats, void *ws,
                             size_t ws_bytes, void *stream);

/* ---- workspace and diagnostics ------------------------------------------ */

enum ovl_op {
    OVL_OP_Q2 = 0,
    OVL_OP_LANCZOS = 1,
    OVL_OP_MSCG = 2,      /* ovl_multishift_cg, sign_q_apply, overlap_apply */
    OVL_OP_TUNE = 3,      /* ovl_autotune_stencil (prec ignored) */
    OVL_OP_WILSON_SOLVE = 4 /* ovl_wilson_solve (prm: its block length) */
};

/* Workspace bytes for an operation; prm may be NULL for OVL_OP_Q2/LANCZOS. */
OVL_API size_t ovl_workspace_bytes(const ovl_lattice *lat, int32_t op, int32_t prec, int32_t nrhs,
                           int32_t nshift, const ovl_solver_params *prm);

/* Defaults: tol 1e-10, maxiter 2000, FP64 mode, reliable_delta 0.1,
 * check_every 10, refine 1, verify 0, profile 0, block 0, sloppy_below 3e-5,
 * block_f64 0, rhs_group 0, deflation NULL, sloppy_f16 0, even_odd 0, store48 1. */
OVL_API void ovl_default_params(ovl_solver_params *prm);

/* Stencil autotuner.  Times the Wilson stencil (D_W, eq. (Wilson-Dirac)) on
 * nrhs fields of a fixed pattern in every precision whose links U provides,
 * over the candidate site orders -- lat->tile_t in {1,2,4,8,16} for the
 * one-site form (timed on FP16 links when given, else FP32); then, for each
 * RHS tile lat->rhs_tile in {1,2,4,8} (only 1 for one RHS; tiles up to the
 * next power of two of nrhs), lat->stream_t in {0,2,4,8,16,32} on FP32 and
 * lat->stream_t64 likewise on FP64 (lengths that divide dims[0]; streaming
 * only when dims[1]*dims[2]*dims[3] % 256 == 0), keeping the tile whose FP32
 * and FP64 times add up least -- and writes the fastest into *lat (a
 * candidate replaces the current value only when more than 5% faster).
 * Outputs of every operator depend on these fields only through summation
 * order.  ws: device workspace of ovl_workspace_bytes(lat, OVL_OP_TUNE, 0,
 * nrhs, 0, NULL) bytes.  tried/times_us (host, optional, max_tried entries):
 * candidate k as 10000*what + 100*tile + value (what 0 tile_t, 1 stream_t,
 * 2 stream_t64; tile the RHS tile it ran with) and its average launch time in
 * microseconds; with FP32 links and nrhs >= 2 the matrix-core FP32 stencil
 * (lat->mfma) is timed against the chosen vector form as what = 3 (value 1).
 * Returns the number of candidates timed (>= 0) or a negative error.
 * Synchronises the stream. */
OVL_API int ovl_autotune_stencil(ovl_lattice *lat, const ovl_gauge *U, int32_t nrhs, void *ws, size_t ws_bytes,
                                 int32_t *tried, float *times_us, int32_t max_tried, void *stream);

/* ovl_autotune_stencil with a file of earlier choices: cache_path (host
 * string, may be NULL for none) holds one JSON object per line,
 *   {"key": "<arch> <L0>x<L1>x<L2>x<L3> bc<b0>,<b1>,<b2>,<b3> nrhs<n> links<f64><f32><f16>",
 *    "tile_t": t, "stream_t": s, "stream_t64": s64, "rhs_tile": k}
 * keyed by the current device's architecture name, the lattice, its boundary
 * phases, nrhs and which link copies U holds.  If a line matches (the last
 * one wins) and its values are valid for *lat, they are written into *lat
 * and 0 is returned without timing; otherwise the autotuner runs and its
 * choice is appended to the file (not locked: concurrent writers may
 * interleave lines).  Returns as ovl_autotune_stencil. */
OVL_API int ovl_autotune_stencil_cached(ovl_lattice *lat, const ovl_gauge *U, int32_t nrhs, void *ws,
                                        size_t ws_bytes, const char *cache_path, int32_t *tried, float *times_us,
                                        int32_t max_tried, void *stream);

OVL_API const char *ovl_status_string(int status);
OVL_API int ovl_last_hip_error(void);
OVL_API const char *ovl_version(void);

#ifdef __cplusplus
}
#endif
#endif /* OVL_H */
