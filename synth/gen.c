/*
 * Seeded synthetic inputs: SU(3) gauge fields, stout smearing, Gaussian
 * spinor sources.  Shared, as bytes, by the FP64 oracle and the GPU library;
 * it contains none of the overlap operator's arithmetic.
 *
 * Canonical host layouts (complex128, C order):
 *   gauge  U[site][mu][row][col]   U_mu(x) is the link from x to x+mu
 *   spinor psi[site][spin][colour]
 *   site = ((x0*L1 + x1)*L2 + x2)*L3 + x3, x0 is time.
 *
 * Random numbers are counter based: uniform(seed, ctr) hashes the pair with
 * the SplitMix64 finaliser (Steele, Lea, Flood, OOPSLA 2014), so every value
 * depends only on (seed, ctr) and the OpenMP loops are reproducible.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <string.h>
#include <stdlib.h>

typedef double complex cplx;

static inline uint64_t sm64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* uniform in the open interval (0,1) */
static inline double uni(uint64_t seed, uint64_t ctr)
{
    uint64_t h = sm64(sm64(seed) ^ sm64(ctr * 0xD1B54A32D192ED03ULL + 1));
    return ((double)(h >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

/* standard normal by Box-Muller (cosine branch), from counters 2c, 2c+1 */
static inline double gauss(uint64_t seed, uint64_t c)
{
    double u1 = uni(seed, 2 * c), u2 = uni(seed, 2 * c + 1);
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
}

/* complex normal (N(0,1) + i N(0,1)) / sqrt(2), from counters 2c, 2c+1 */
static inline cplx cgauss(uint64_t seed, uint64_t c)
{
    return (gauss(seed, 2 * c) + I * gauss(seed, 2 * c + 1)) * 0.70710678118654752440;
}

/* ---- 3x3 complex helpers (row major) ---- */
static void m_mul(const cplx *a, const cplx *b, cplx *c)
{
    cplx t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cplx s = 0;
            for (int k = 0; k < 3; k++) s += a[3 * i + k] * b[3 * k + j];
            t[3 * i + j] = s;
        }
    memcpy(c, t, sizeof t);
}
static void m_dag(const cplx *a, cplx *c)
{
    cplx t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) t[3 * i + j] = conj(a[3 * j + i]);
    memcpy(c, t, sizeof t);
}

/* exp(X) by scaling and squaring of a degree-18 Taylor polynomial */
static void m_exp(const cplx *x, cplx *out)
{
    double nrm = 0;
    for (int i = 0; i < 9; i++) nrm += cabs(x[i]);
    int s = 0;
    while (nrm > 0.125) { nrm *= 0.5; s++; }
    double sc = ldexp(1.0, -s);
    cplx a[9], term[9], sum[9];
    for (int i = 0; i < 9; i++) a[i] = x[i] * sc;
    for (int i = 0; i < 9; i++) sum[i] = term[i] = (i % 4 == 0) ? 1.0 : 0.0;
    for (int n = 1; n <= 18; n++) {
        m_mul(term, a, term);
        for (int i = 0; i < 9; i++) { term[i] /= n; sum[i] += term[i]; }
    }
    for (int k = 0; k < s; k++) m_mul(sum, sum, sum);
    memcpy(out, sum, sizeof sum);
}

/* Project onto SU(3): Gram-Schmidt on rows 0,1, row 2 = conj(row0 x row1). */
static void m_su3_project(cplx *u)
{
    double n0 = 0;
    for (int j = 0; j < 3; j++) n0 += creal(u[j] * conj(u[j]));
    n0 = 1.0 / sqrt(n0);
    for (int j = 0; j < 3; j++) u[j] *= n0;
    cplx d = 0;
    for (int j = 0; j < 3; j++) d += conj(u[j]) * u[3 + j];
    for (int j = 0; j < 3; j++) u[3 + j] -= d * u[j];
    double n1 = 0;
    for (int j = 0; j < 3; j++) n1 += creal(u[3 + j] * conj(u[3 + j]));
    n1 = 1.0 / sqrt(n1);
    for (int j = 0; j < 3; j++) u[3 + j] *= n1;
    u[6] = conj(u[1] * u[5] - u[2] * u[4]);
    u[7] = conj(u[2] * u[3] - u[0] * u[5]);
    u[8] = conj(u[0] * u[4] - u[1] * u[3]);
}

static inline int64_t site_of(const int *L, int x0, int x1, int x2, int x3)
{
    return (((int64_t)x0 * L[1] + x1) * L[2] + x2) * L[3] + x3;
}

/* neighbour of site s one step in direction mu (dir=+1 or -1), periodic */
static inline int64_t hop(const int *L, int64_t s, int mu, int dir)
{
    int x[4];
    int64_t r = s;
    for (int m = 3; m >= 0; m--) { x[m] = (int)(r % L[m]); r /= L[m]; }
    x[mu] = (x[mu] + dir + L[mu]) % L[mu];
    return site_of(L, x[0], x[1], x[2], x[3]);
}

/*
 * U_mu(x) = exp(i eps0 H), H = traceless Hermitian part of a complex Gaussian
 * 3x3 matrix A, H = (A + A^H)/2 - tr((A + A^H)/2)/3.  Counter of entry e of
 * link (x,mu): ((x*4+mu)*9 + e).
 */
void synth_gauge(const int *L, double eps0, uint64_t seed, double *out)
{
    int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
    cplx *U = (cplx *)out;
#pragma omp parallel for schedule(static)
    for (int64_t l = 0; l < 4 * V; l++) {
        cplx a[9], h[9], x[9];
        for (int e = 0; e < 9; e++) a[e] = cgauss(seed, (uint64_t)l * 9 + e);
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) h[3 * i + j] = 0.5 * (a[3 * i + j] + conj(a[3 * j + i]));
        cplx tr = (h[0] + h[4] + h[8]) / 3.0;
        h[0] -= tr; h[4] -= tr; h[8] -= tr;
        for (int e = 0; e < 9; e++) x[e] = I * eps0 * h[e];
        m_exp(x, U + 9 * l);
        m_su3_project(U + 9 * l);
    }
}

/*
 * Stout smearing, one step of U_mu(x) -> exp(eps Z_mu(x)) U_mu(x) for all
 * links simultaneously from the old field (Morningstar & Peardon), with
 *   M_mu(x) = sum_{nu != mu} P^{mu,nu}_x + P^{mu,-nu}_x,
 *   P^{mu,nu}_x  = U_nu(x) U_mu(x+nu) U_nu(x+mu)^H U_mu(x)^H,
 *   P^{mu,-nu}_x = U_nu(x-nu)^H U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^H,
 *   Z = (M - M^H)/2 - tr(M - M^H)/6.
 * This orientation of Z is the one that lowers the Wilson action, as the
 * Lie-Euler/Wilson-flow reading of stout smearing requires.
 */
static void stout_step(const int *L, double eps, const cplx *U, cplx *Un)
{
    int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < V; x++) {
        for (int mu = 0; mu < 4; mu++) {
            cplx M[9] = {0}, t[9], w[9];
            const cplx *Umx = U + 9 * (4 * x + mu);
            cplx Umx_d[9];
            m_dag(Umx, Umx_d);
            int64_t xpm = hop(L, x, mu, +1);
            for (int nu = 0; nu < 4; nu++) {
                if (nu == mu) continue;
                int64_t xpn = hop(L, x, nu, +1), xmn = hop(L, x, nu, -1);
                int64_t xmnpm = hop(L, xmn, mu, +1);
                /* upper plaquette */
                m_mul(U + 9 * (4 * x + nu), U + 9 * (4 * xpn + mu), t);
                m_dag(U + 9 * (4 * xpm + nu), w);
                m_mul(t, w, t);
                m_mul(t, Umx_d, t);
                for (int e = 0; e < 9; e++) M[e] += t[e];
                /* lower plaquette */
                m_dag(U + 9 * (4 * xmn + nu), w);
                m_mul(w, U + 9 * (4 * xmn + mu), t);
                m_mul(t, U + 9 * (4 * xmnpm + nu), t);
                m_mul(t, Umx_d, t);
                for (int e = 0; e < 9; e++) M[e] += t[e];
            }
            cplx Z[9];
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) Z[3 * i + j] = 0.5 * (M[3 * i + j] - conj(M[3 * j + i]));
            cplx tr = (Z[0] + Z[4] + Z[8]) / 3.0;
            Z[0] -= tr; Z[4] -= tr; Z[8] -= tr;
            for (int e = 0; e < 9; e++) Z[e] *= eps;
            m_exp(Z, t);
            m_mul(t, Umx, Un + 9 * (4 * x + mu));
            m_su3_project(Un + 9 * (4 * x + mu));
        }
    }
}

/* nsteps stout steps in place; work must hold 4*V*9 complex numbers */
void synth_stout(const int *L, double eps, int nsteps, double *u, double *work)
{
    int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
    cplx *a = (cplx *)u, *b = (cplx *)work;
    for (int s = 0; s < nsteps; s++) {
        stout_step(L, eps, a, b);
        memcpy(a, b, sizeof(cplx) * 36 * V);
    }
}

/* nrhs Gaussian spinor fields, component (r, site, spin, colour) uses counter
 * ((r*V + site)*12 + spin*3 + colour). */
void synth_gaussian_spinor(int64_t V, int nrhs, uint64_t seed, double *out)
{
    cplx *p = (cplx *)out;
    int64_t n = (int64_t)nrhs * V * 12;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) p[i] = cgauss(seed, (uint64_t)i);
}

/* uniform integers in [0, n) for picking e.g. a point-source site */
int64_t synth_randint(uint64_t seed, uint64_t ctr, int64_t n)
{
    return (int64_t)(uni(seed, ctr) * (double)n) % n;
}
