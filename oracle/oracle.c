/*
 * FP64 CPU oracle for the overlap-operator apply.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load or call this file's library; the
 * GPU library shares no code with it and never calls it.
 *
 * Everything is complex128 in the canonical host layout
 *   gauge  U[site][mu][3][3],  spinor psi[site][4][3],
 *   site = ((x0*L1 + x1)*L2 + x2)*L3 + x3, x0 = time,
 * with plain loops (OpenMP over sites only).  Each function names the part of
 * Brannick et al., "Multigrid preconditioning for the overlap operator in
 * lattice QCD" (arXiv:1410.7170) it follows.  Steps the paper does not
 * specify (Zolotarev coefficients, multishift CG, Lanczos bounds) are written
 * from their textbook definitions, named where used.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------ */
/* gamma matrices: Hermitian chiral basis.  gamma_0 = [[0,I],[I,0]],
 * gamma_k = [[0,-i sigma_k],[i sigma_k,0]]; gamma_5 is formed as the product
 * gamma_0 gamma_1 gamma_2 gamma_3 (Section 2, eqs. (commutativity_rel) and
 * (gamma_commutativity)); the basis itself is left open by the paper. */
static cplx G[5][4][4];
static int g_init = 0;

static void init_gamma(void)
{
    if (g_init) return;
    memset(G, 0, sizeof G);
    const cplx sig[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    for (int a = 0; a < 2; a++) {
        G[0][a][2 + a] = 1;
        G[0][2 + a][a] = 1;
    }
    for (int k = 0; k < 3; k++)
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
                G[k + 1][a][2 + b] = -I * sig[k][a][b];
                G[k + 1][2 + a][b] = I * sig[k][a][b];
            }
    cplx t[4][4], u[4][4];
    memcpy(t, G[0], sizeof t);
    for (int m = 1; m < 4; m++) {
        for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++) {
                cplx s = 0;
                for (int k = 0; k < 4; k++) s += t[i][k] * G[m][k][j];
                u[i][j] = s;
            }
        memcpy(t, u, sizeof t);
    }
    memcpy(G[4], t, sizeof t);
    g_init = 1;
}

void orc_gamma(int mu, double *out /* 4x4 complex */)
{
    init_gamma();
    memcpy(out, G[mu], sizeof(G[mu]));
}

/* ------------------------------------------------------------------ */
static inline int64_t vol(const int *L) { return (int64_t)L[0] * L[1] * L[2] * L[3]; }

static inline void coords(const int *L, int64_t s, int *x)
{
    for (int m = 3; m >= 0; m--) { x[m] = (int)(s % L[m]); s /= L[m]; }
}

static inline int64_t lex(const int *L, const int *x)
{
    return (((int64_t)x[0] * L[1] + x[1]) * L[2] + x[2]) * L[3] + x[3];
}

/*
 * Wilson-Dirac operator, eq. (Wilson-Dirac) with a = 1:
 *   (D psi)(x) = (m0+4) psi(x)
 *              - 1/2 sum_mu [(I - gamma_mu) (x) U_mu(x)]      psi(x+mu)
 *              - 1/2 sum_mu [(I + gamma_mu) (x) U_mu(x-mu)^H] psi(x-mu).
 * Hops that cross the lattice boundary in direction mu carry the phase
 * bc[mu] (+1 periodic, -1 antiperiodic); the links themselves stay SU(3).
 */
void orc_dw(const int *L, const int *bc, const double *Ud, double m0, const double *ind, double *outd)
{
    init_gamma();
    const cplx *U = (const cplx *)Ud;
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    int64_t V = vol(L);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; s++) {
        int x[4];
        coords(L, s, x);
        cplx acc[4][3];
        for (int a = 0; a < 4; a++)
            for (int c = 0; c < 3; c++) acc[a][c] = (m0 + 4.0) * in[12 * s + 3 * a + c];
        for (int mu = 0; mu < 4; mu++) {
            for (int dir = -1; dir <= 1; dir += 2) {
                int y[4] = {x[0], x[1], x[2], x[3]};
                double ph = 1.0;
                y[mu] += dir;
                if (y[mu] == L[mu]) { y[mu] = 0; ph = bc[mu]; }
                if (y[mu] < 0) { y[mu] = L[mu] - 1; ph = bc[mu]; }
                int64_t n = lex(L, y);
                /* colour matrix: U_mu(x) forward, U_mu(x-mu)^H backward */
                cplx W[3][3];
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++)
                        W[i][j] = (dir > 0) ? U[9 * (4 * s + mu) + 3 * i + j]
                                            : conj(U[9 * (4 * n + mu) + 3 * j + i]);
                for (int a = 0; a < 4; a++)
                    for (int c = 0; c < 3; c++) {
                        cplx t = 0;
                        for (int b = 0; b < 4; b++) {
                            cplx sp = (a == b ? 1.0 : 0.0) - dir * G[mu][a][b];
                            if (sp == 0) continue;
                            for (int d = 0; d < 3; d++) t += sp * W[c][d] * in[12 * n + 3 * b + d];
                        }
                        acc[a][c] -= 0.5 * ph * t;
                    }
            }
        }
        for (int a = 0; a < 4; a++)
            for (int c = 0; c < 3; c++) out[12 * s + 3 * a + c] = acc[a][c];
    }
}

/* Gamma_5 = I_{n_L} (x) gamma_5 (x) I_3, applied in place-safe form */
void orc_gamma5(int64_t V, const double *ind, double *outd)
{
    init_gamma();
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; s++) {
        cplx t[4][3];
        for (int a = 0; a < 4; a++)
            for (int c = 0; c < 3; c++) {
                cplx v = 0;
                for (int b = 0; b < 4; b++) v += G[4][a][b] * in[12 * s + 3 * b + c];
                t[a][c] = v;
            }
        for (int a = 0; a < 4; a++)
            for (int c = 0; c < 3; c++) out[12 * s + 3 * a + c] = t[a][c];
    }
}

/* Q = Gamma_5 D_W(m0), Hermitian by eq. (gamma_5_symmetry) */
void orc_q(const int *L, const int *bc, const double *U, double m0, const double *in, double *out)
{
    orc_dw(L, bc, U, m0, in, out);
    orc_gamma5(vol(L), out, out);
}

/* (Q^2 + shift) in, with Q^2 = Q Q = D_W^H D_W */
void orc_q2(const int *L, const int *bc, const double *U, double m0, double shift,
            const double *in, double *out, double *tmp)
{
    int64_t n = 12 * vol(L);
    orc_q(L, bc, U, m0, in, tmp);
    orc_q(L, bc, U, m0, tmp, out);
    cplx *o = (cplx *)out;
    const cplx *i = (const cplx *)in;
    if (shift != 0.0)
        for (int64_t k = 0; k < n; k++) o[k] += shift * i[k];
}

/* ------------------------------------------------------------------ */
/* BLAS-1 */
static double nrm2(int64_t n, const cplx *a)
{
    double s = 0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (int64_t k = 0; k < n; k++) s += creal(a[k]) * creal(a[k]) + cimag(a[k]) * cimag(a[k]);
    return s;
}

static cplx dotc(int64_t n, const cplx *a, const cplx *b)
{
    double re = 0, im = 0;
#pragma omp parallel for reduction(+ : re, im) schedule(static)
    for (int64_t k = 0; k < n; k++) {
        cplx t = conj(a[k]) * b[k];
        re += creal(t);
        im += cimag(t);
    }
    return re + I * im;
}

double orc_norm2(int64_t n, const double *a) { return nrm2(n, (const cplx *)a); }

void orc_dot(int64_t n, const double *a, const double *b, double *out)
{
    cplx d = dotc(n, (const cplx *)a, (const cplx *)b);
    out[0] = creal(d);
    out[1] = cimag(d);
}

/* ------------------------------------------------------------------ */
/* Conjugate gradients for (Q^2 + shift) x = b, x starts at 0.  Stops when the
 * recursive residual satisfies ||r|| <= tol ||b||.  Returns iterations. */
int orc_cg(const int *L, const int *bc, const double *U, double m0, double shift,
           const double *bd, double *xd, double tol, int maxit)
{
    int64_t n = 12 * vol(L);
    const cplx *b = (const cplx *)bd;
    cplx *x = (cplx *)xd;
    cplx *r = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n);
    cplx *q = malloc(sizeof(cplx) * n), *t = malloc(sizeof(cplx) * n);
    for (int64_t k = 0; k < n; k++) { x[k] = 0; r[k] = b[k]; p[k] = b[k]; }
    double bb = nrm2(n, b), rr = bb;
    int it = 0;
    while (it < maxit && rr > tol * tol * bb) {
        orc_q2(L, bc, U, m0, shift, (double *)p, (double *)q, (double *)t);
        double alpha = rr / creal(dotc(n, p, q));
        for (int64_t k = 0; k < n; k++) { x[k] += alpha * p[k]; r[k] -= alpha * q[k]; }
        double rr_new = nrm2(n, r);
        double beta = rr_new / rr;
        for (int64_t k = 0; k < n; k++) p[k] = r[k] + beta * p[k];
        rr = rr_new;
        it++;
    }
    free(r); free(p); free(q); free(t);
    return it;
}

/*
 * Multishift CG (Jegerlehner's shifted recurrences) for
 *   (Q^2 + s_j) x_j = b,  j = 0..ns-1,
 * one Krylov space shared by all shifts.  The base system uses the smallest
 * shift s0; delta_j = s_j - s0.  With alpha, beta the base CG coefficients:
 *   zeta_j' = zeta_j zeta_j^old alpha_old /
 *             (alpha beta_old (zeta_j^old - zeta_j) + zeta_j^old alpha_old (1 + alpha delta_j))
 *   alpha_j = alpha zeta_j' / zeta_j,        x_j += alpha_j p_j
 *   beta_j  = beta (zeta_j' / zeta_j)^2,     p_j  = zeta_j' r + beta_j p_j
 * Shift j's residual is zeta_j r; once |zeta_j| ||r|| <= tol ||b|| it is frozen
 * (no further updates, which also keeps zeta_j from underflowing).  Stops when
 * every shift is frozen or after maxit iterations.  iters[j] receives the
 * iteration at which shift j froze (maxit if it never did).  Returns the
 * number of base iterations.
 */
int orc_mscg(const int *L, const int *bc, const double *U, double m0, int ns, const double *shifts,
             const double *bd, double *xd, double tol, int maxit, int *iters)
{
    int64_t n = 12 * vol(L);
    const cplx *b = (const cplx *)bd;
    cplx *x = (cplx *)xd;
    int j0 = 0;
    for (int j = 1; j < ns; j++)
        if (shifts[j] < shifts[j0]) j0 = j;
    double s0 = shifts[j0];
    cplx *r = malloc(sizeof(cplx) * n), *q = malloc(sizeof(cplx) * n), *t = malloc(sizeof(cplx) * n);
    cplx *p = malloc(sizeof(cplx) * n * ns);
    double *zeta = malloc(sizeof(double) * ns), *zeta_old = malloc(sizeof(double) * ns);
    double *zeta_new = malloc(sizeof(double) * ns), *aj = malloc(sizeof(double) * ns);
    int *active = malloc(sizeof(int) * ns);
    for (int j = 0; j < ns; j++) {
        zeta[j] = zeta_old[j] = 1.0;
        active[j] = 1;
        iters[j] = maxit;
        for (int64_t k = 0; k < n; k++) { x[n * j + k] = 0; p[n * j + k] = b[k]; }
    }
    for (int64_t k = 0; k < n; k++) r[k] = b[k];
    double bb = nrm2(n, b), rr = bb;
    double alpha_old = 1.0, beta = 0.0;
    int it = 0, nact = ns;
    while (it < maxit && nact > 0) {
        cplx *p0 = p + n * j0;
        orc_q2(L, bc, U, m0, s0, (double *)p0, (double *)q, (double *)t);
        double alpha = rr / creal(dotc(n, p0, q));
        for (int j = 0; j < ns; j++) {
            if (!active[j]) continue;
            double dj = shifts[j] - s0;
            zeta_new[j] = zeta[j] * zeta_old[j] * alpha_old /
                          (alpha * beta * (zeta_old[j] - zeta[j]) + zeta_old[j] * alpha_old * (1.0 + alpha * dj));
            aj[j] = alpha * zeta_new[j] / zeta[j];
            for (int64_t k = 0; k < n; k++) x[n * j + k] += aj[j] * p[n * j + k];
        }
        for (int64_t k = 0; k < n; k++) r[k] -= alpha * q[k];
        double rr_new = nrm2(n, r);
        beta = rr_new / rr;
        it++;
        for (int j = 0; j < ns; j++) {
            if (!active[j]) continue;
            double bj = beta * (zeta_new[j] / zeta[j]) * (zeta_new[j] / zeta[j]);
            for (int64_t k = 0; k < n; k++) p[n * j + k] = zeta_new[j] * r[k] + bj * p[n * j + k];
            zeta_old[j] = zeta[j];
            zeta[j] = zeta_new[j];
            if (fabs(zeta[j]) * sqrt(rr_new) <= tol * sqrt(bb)) {
                active[j] = 0;
                iters[j] = it;
                nact--;
            }
        }
        rr = rr_new;
        alpha_old = alpha;
    }
    free(r); free(q); free(t); free(p);
    free(zeta); free(zeta_old); free(zeta_new); free(aj); free(active);
    return it;
}

/* ||b - (Q^2 + shift) x|| / ||b|| computed from scratch */
double orc_true_residual(const int *L, const int *bc, const double *U, double m0, double shift,
                         const double *bd, const double *xd)
{
    int64_t n = 12 * vol(L);
    cplx *q = malloc(sizeof(cplx) * n), *t = malloc(sizeof(cplx) * n);
    orc_q2(L, bc, U, m0, shift, xd, (double *)q, (double *)t);
    const cplx *b = (const cplx *)bd;
    for (int64_t k = 0; k < n; k++) q[k] = b[k] - q[k];
    double r = sqrt(nrm2(n, q) / nrm2(n, b));
    free(q); free(t);
    return r;
}

/* ------------------------------------------------------------------ */
/*
 * Zolotarev's optimal rational approximation of sign(x) on [-1,-k] U [k,1]
 * (the paper computes sign(Gamma_5 D_W) by a Krylov method instead; the
 * rational form replaces it):
 *   sign(x) ~ D x prod_{i=1}^{n-1} (x^2 + c_{2i}) / prod_{j=1}^{n} (x^2 + c_{2j-1})
 *           = D x sum_j a_j / (x^2 + sigma_j),
 *   c_l = k^2 sn^2(l K'/(2n); k') / cn^2(l K'/(2n); k'),  k' = sqrt(1-k^2),
 *   K'  = K(k') = pi / (2 AGM(1, k)),  sigma_j = c_{2j-1},
 *   a_j = prod_i (c_{2i} - sigma_j) / prod_{i != j} (sigma_i - sigma_j).
 * sn, cn from the descending Landen (AGM) scheme of Abramowitz & Stegun 16.4,
 * started from the complementary modulus k itself (forming sqrt(1-k'^2) from
 * k' ~ 1 would cancel).
 * D and the error delta follow from the extremes of R(x) = x sum a_j/(x^2+sigma_j)
 * on [k,1]:  D = 2/(max+min), delta = (max-min)/(max+min).
 */
static void sncn(double u, double m /* modulus */, double mc /* sqrt(1-m^2) */, double *sn, double *cn)
{
    double a[64], c[64];
    double an = 1.0, bn = mc;
    int N = 0;
    a[0] = an;
    c[0] = m;
    while (fabs(c[N]) > 1e-17 && N < 60) {
        double an1 = 0.5 * (an + bn), bn1 = sqrt(an * bn);
        N++;
        c[N] = 0.5 * (an - bn);
        a[N] = an1;
        an = an1;
        bn = bn1;
    }
    double phi = ldexp(1.0, N) * a[N] * u;
    for (int i = N; i >= 1; i--) phi = 0.5 * (phi + asin(c[i] / a[i] * sin(phi)));
    *sn = sin(phi);
    *cn = cos(phi);
}

static double agm(double a, double b)
{
    for (int i = 0; i < 60 && fabs(a - b) > 1e-16 * a; i++) {
        double t = 0.5 * (a + b);
        b = sqrt(a * b);
        a = t;
    }
    return 0.5 * (a + b);
}

static double zolo_R(double x, int n, const double *sig, const double *a)
{
    double s = 0;
    for (int j = 0; j < n; j++) s += a[j] / (x * x + sig[j]);
    return x * s;
}

/* sigma[n], a[n] (unnormalised), *D, *delta for the interval [k,1] */
void orc_zolotarev(double k, int n, double *sigma, double *a, double *D, double *delta)
{
    double kp = sqrt(1.0 - k * k);
    double Kp = 1.5707963267948966192 / agm(1.0, k);
    double *c = malloc(sizeof(double) * 2 * n);
    for (int l = 1; l <= 2 * n - 1; l++) {
        double sn, cn;
        sncn(l * Kp / (2.0 * n), kp, k, &sn, &cn);
        c[l] = k * k * sn * sn / (cn * cn);
    }
    for (int j = 0; j < n; j++) sigma[j] = c[2 * j + 1];
    for (int j = 0; j < n; j++) {
        double num = 1.0, den = 1.0;
        for (int i = 1; i <= n - 1; i++) num *= c[2 * i] - sigma[j];
        for (int i = 0; i < n; i++)
            if (i != j) den *= sigma[i] - sigma[j];
        a[j] = num / den;
    }
    /* extremes of R on [k,1]: dense logarithmic grid, each interior local
     * maximum refined by golden-section search */
    const int G = 20000;
    double lo = log(k), hi = 0.0;
    double rmin = zolo_R(k, n, sigma, a), rmax = rmin;
    double prev2 = 0, prev1 = rmin;
    for (int g = 1; g <= G; g++) {
        double x = exp(lo + (hi - lo) * g / G);
        double v = zolo_R(x, n, sigma, a);
        if (v < rmin) rmin = v;
        if (v > rmax) rmax = v;
        if (g >= 2 && prev1 >= prev2 && prev1 >= v) {
            double ga = lo + (hi - lo) * (g - 2) / G, gb = lo + (hi - lo) * g / G;
            const double gr = 0.6180339887498949;
            for (int it = 0; it < 100; it++) {
                double m1 = gb - gr * (gb - ga), m2 = ga + gr * (gb - ga);
                if (zolo_R(exp(m1), n, sigma, a) > zolo_R(exp(m2), n, sigma, a)) gb = m2; else ga = m1;
            }
            double vm = zolo_R(exp(0.5 * (ga + gb)), n, sigma, a);
            if (vm > rmax) rmax = vm;
        }
        prev2 = prev1;
        prev1 = v;
    }
    *D = 2.0 / (rmax + rmin);
    *delta = (rmax - rmin) / (rmax + rmin);
    free(c);
}

/* ------------------------------------------------------------------ */
/*
 * Lanczos on Q^2 started from v0 (the random start vector is an input):
 * m steps of the three-term recurrence, no reorthogonalisation, then the
 * extreme eigenvalues of the tridiagonal matrix by Sturm-sequence bisection.
 * Returns the smallest and largest Ritz values.
 */
static int sturm_count(int m, const double *al, const double *be, double x)
{
    int cnt = 0;
    double d = al[0] - x;
    if (d < 0) cnt++;
    for (int i = 1; i < m; i++) {
        if (d == 0) d = 1e-300;
        d = al[i] - x - be[i - 1] * be[i - 1] / d;
        if (d < 0) cnt++;
    }
    return cnt;
}

static double tri_eig(int m, const double *al, const double *be, int idx, double lo, double hi)
{
    for (int it = 0; it < 200; it++) {
        double mid = 0.5 * (lo + hi);
        if (sturm_count(m, al, be, mid) > idx) hi = mid; else lo = mid;
    }
    return 0.5 * (lo + hi);
}

int orc_lanczos_q2(const int *L, const int *bc, const double *U, double m0, const double *v0d,
                   int m, double *theta_min, double *theta_max)
{
    int64_t n = 12 * vol(L);
    cplx *v = malloc(sizeof(cplx) * n), *vp = calloc(n, sizeof(cplx));
    cplx *w = malloc(sizeof(cplx) * n), *t = malloc(sizeof(cplx) * n);
    double *al = malloc(sizeof(double) * m), *be = malloc(sizeof(double) * m);
    double nv = sqrt(nrm2(n, (const cplx *)v0d));
    for (int64_t k = 0; k < n; k++) v[k] = ((const cplx *)v0d)[k] / nv;
    double bprev = 0;
    int steps = 0;
    for (int i = 0; i < m; i++) {
        orc_q2(L, bc, U, m0, 0.0, (double *)v, (double *)w, (double *)t);
        al[i] = creal(dotc(n, v, w));
        for (int64_t k = 0; k < n; k++) w[k] -= al[i] * v[k] + bprev * vp[k];
        be[i] = sqrt(nrm2(n, w));
        steps = i + 1;
        if (be[i] < 1e-14) break;
        for (int64_t k = 0; k < n; k++) { vp[k] = v[k]; v[k] = w[k] / be[i]; }
        bprev = be[i];
    }
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < steps; i++) {
        double r = fabs(i > 0 ? be[i - 1] : 0) + fabs(i < steps - 1 ? be[i] : 0);
        if (al[i] - r < lo) lo = al[i] - r;
        if (al[i] + r > hi) hi = al[i] + r;
    }
    *theta_min = tri_eig(steps, al, be, 0, lo, hi);
    *theta_max = tri_eig(steps, al, be, steps - 1, lo, hi);
    free(v); free(vp); free(w); free(t); free(al); free(be);
    return steps;
}

/* ------------------------------------------------------------------ */
/*
 * Overlap operator with the Wilson kernel at m0 = -rho (eq. (overlap_def),
 * in the normalisation D_ov = rho (I + Gamma_5 sign(Q)), Q = Gamma_5 D_W(-rho)):
 *   sign(Q) b ~ Q y,   y = sum_j w_j (Q^2 + s_j)^{-1} b   (multishift CG),
 *   D_ov b = rho (b + Gamma_5 Q y) = rho (b + D_W(-rho) y).
 * y_out (may be NULL) receives y.
 */
int orc_overlap(const int *L, const int *bc, const double *U, double rho, int ns, const double *shifts,
                const double *weights, const double *bd, double *outd, double *y_out, double tol,
                int maxit, int *iters)
{
    int64_t n = 12 * vol(L);
    double m0 = -rho;
    cplx *x = malloc(sizeof(cplx) * n * ns), *y = malloc(sizeof(cplx) * n);
    int it = orc_mscg(L, bc, U, m0, ns, shifts, bd, (double *)x, tol, maxit, iters);
    for (int64_t k = 0; k < n; k++) {
        cplx s = 0;
        for (int j = 0; j < ns; j++) s += weights[j] * x[n * j + k];
        y[k] = s;
    }
    orc_dw(L, bc, U, m0, (double *)y, outd);
    cplx *out = (cplx *)outd;
    const cplx *b = (const cplx *)bd;
    for (int64_t k = 0; k < n; k++) out[k] = rho * (b[k] + out[k]);
    if (y_out) memcpy(y_out, y, sizeof(cplx) * n);
    free(x); free(y);
    return it;
}

/* sign(Q) b ~ Q sum_j w_j (Q^2 + s_j)^{-1} b, Q = Gamma_5 D_W(m0) */
int orc_sign_q(const int *L, const int *bc, const double *U, double m0, int ns, const double *shifts,
               const double *weights, const double *bd, double *outd, double tol, int maxit, int *iters)
{
    int64_t n = 12 * vol(L);
    cplx *x = malloc(sizeof(cplx) * n * ns), *y = malloc(sizeof(cplx) * n);
    int it = orc_mscg(L, bc, U, m0, ns, shifts, bd, (double *)x, tol, maxit, iters);
    for (int64_t k = 0; k < n; k++) {
        cplx s = 0;
        for (int j = 0; j < ns; j++) s += weights[j] * x[n * j + k];
        y[k] = s;
    }
    orc_q(L, bc, U, m0, (double *)y, outd);
    free(x); free(y);
    return it;
}

/* ------------------------------------------------------------------ */
/* Sum over sites and mu < nu of Re tr P^{mu,nu}_x with the plaquette of eq.
 * (plaquette_def1): P = U_nu(x) U_mu(x+nu) U_nu(x+mu)^H U_mu(x)^H. */
double orc_plaquette_sum(const int *L, const double *Ud)
{
    const cplx *U = (const cplx *)Ud;
    int64_t V = vol(L);
    double total = 0;
#pragma omp parallel for reduction(+ : total) schedule(static)
    for (int64_t s = 0; s < V; s++) {
        int x[4];
        coords(L, s, x);
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++) {
                int y[4];
                memcpy(y, x, sizeof y);
                y[nu] = (y[nu] + 1) % L[nu];
                int64_t xpn = lex(L, y);
                memcpy(y, x, sizeof y);
                y[mu] = (y[mu] + 1) % L[mu];
                int64_t xpm = lex(L, y);
                const cplx *A = U + 9 * (4 * s + nu), *B = U + 9 * (4 * xpn + mu);
                const cplx *C = U + 9 * (4 * xpm + nu), *D = U + 9 * (4 * s + mu);
                /* tr(A B C^H D^H) = sum_{ijkl} A_ij B_jk conj(C_lk) conj(D_il) */
                cplx tr = 0;
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++)
                        for (int k = 0; k < 3; k++)
                            for (int l = 0; l < 3; l++)
                                tr += A[3 * i + j] * B[3 * j + k] * conj(C[3 * l + k]) * conj(D[3 * i + l]);
                total += creal(tr);
            }
    }
    return total;
}

/* ------------------------------------------------------------------ */
/* OpenMP thread count of the loops above (timing runs on one core or all). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }
