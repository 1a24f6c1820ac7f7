/*
 * Plain FP64 CPU oracle for the data-parallel hot path of Nf=2 Wilson-fermion
 * Hybrid Monte Carlo (Winter, "Gauge Field Generation on Large-Scale
 * GPU-Enabled Systems", Lattice 2012; the HMC operations listed in Sec. 1:
 * pseudofermion refresh, momentum update, force terms, projection,
 * reunitarisation, random numbers, SU(3) exponentiation, matrix inversion,
 * and the global sums of Sec. 1's QDP-JIT feature list).
 *
 * TEST INFRASTRUCTURE.  This file is the checker, not the product: only the
 * test-suite, the smoke check and the benchmark's CPU-baseline leg load it.
 * It shares no code, header, table or helper with the HIP library.
 *
 * The paper names these operations but prints no formula for any of them, so
 * every definition below is the textbook one under an explicit convention
 * (DeGrand-Rossi gamma basis, M = 1 - kappa*D, T^a = lambda^a/2, U' = i P U,
 * antiperiodic fermion time boundary).  The code is deliberately literal:
 * full lattice, canonical array-of-structures layout, explicit 4x4 gamma
 * matrices, plain loops, C99 complex arithmetic, serial global sums.
 *
 * Canonical layouts (all complex double, row-major):
 *   site      i = x + Lx*(y + Ly*(z + Lz*t)),  parity = (x+y+z+t) mod 2
 *   gauge     U[i][mu][row][col]        (V*4*9)
 *   spinor    psi[i][spin][colour]       (V*12)
 *   momentum  P[i][mu][row][col]        (V*4*9, traceless Hermitian)
 * A field that lives on one parity is stored full-size with zeros elsewhere.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* Threads of the site loops (the CPU baseline is timed at several counts);
 * returns the previous count.  Results do not depend on it: every global
 * sum is serial. */
int or_set_threads(int n)
{
    int old = omp_get_max_threads();
    if (n > 0) omp_set_num_threads(n);
    return old;
}

/* ------------------------------------------------------------------ */
/* Geometry: lexicographic sites, parity, periodic neighbours.         */
/* ------------------------------------------------------------------ */

static long vol4(const int *L) { return (long)L[0] * L[1] * L[2] * L[3]; }

static void coords_of(const int *L, long i, int c[4])
{
    c[0] = (int)(i % L[0]); i /= L[0];
    c[1] = (int)(i % L[1]); i /= L[1];
    c[2] = (int)(i % L[2]); i /= L[2];
    c[3] = (int)i;
}

static long index_of(const int *L, const int c[4])
{
    return c[0] + (long)L[0] * (c[1] + (long)L[1] * (c[2] + (long)L[2] * c[3]));
}

static int parity_of(const int c[4]) { return (c[0] + c[1] + c[2] + c[3]) & 1; }

/* Neighbour of site c one step along +mu (dir=+1) or -mu (dir=-1), periodic.
 * *crosses_t is set when the step crosses the t = Lt-1 <-> 0 boundary. */
static long hop(const int *L, const int c[4], int mu, int dir, int *crosses_t)
{
    int n[4] = {c[0], c[1], c[2], c[3]};
    n[mu] += dir;
    int crossed = 0;
    if (n[mu] == L[mu]) { n[mu] = 0; crossed = 1; }
    if (n[mu] < 0) { n[mu] = L[mu] - 1; crossed = 1; }
    if (crosses_t) *crosses_t = (mu == 3) && crossed;
    return index_of(L, n);
}

long or_lex_index(const int *L, int x, int y, int z, int t)
{
    int c[4] = {x, y, z, t};
    return index_of(L, c);
}

int or_site_parity(const int *L, long i)
{
    int c[4];
    coords_of(L, i, c);
    return parity_of(c);
}

/* Neighbour table for tests: nb[i*8 + 2*mu + (dir<0)] = lex index. */
void or_neighbor_table(const int *L, long *nb)
{
    long V = vol4(L);
    for (long i = 0; i < V; ++i) {
        int c[4];
        coords_of(L, i, c);
        for (int mu = 0; mu < 4; ++mu) {
            nb[i * 8 + 2 * mu] = hop(L, c, mu, +1, NULL);
            nb[i * 8 + 2 * mu + 1] = hop(L, c, mu, -1, NULL);
        }
    }
}

/* ------------------------------------------------------------------ */
/* 3x3 complex matrices (row-major arrays of 9).                       */
/* ------------------------------------------------------------------ */

static void mat_mul(const cplx *a, const cplx *b, cplx *out)
{
    cplx r[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0;
            for (int k = 0; k < 3; ++k) s += a[3 * i + k] * b[3 * k + j];
            r[3 * i + j] = s;
        }
    memcpy(out, r, sizeof r);
}

static void mat_dag(const cplx *a, cplx *out)
{
    cplx r[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r[3 * i + j] = conj(a[3 * j + i]);
    memcpy(out, r, sizeof r);
}

static void mat_add_to(cplx *acc, const cplx *a)
{
    for (int k = 0; k < 9; ++k) acc[k] += a[k];
}

static cplx mat_trace(const cplx *a) { return a[0] + a[4] + a[8]; }

static void mat_identity(cplx *a)
{
    for (int k = 0; k < 9; ++k) a[k] = 0;
    a[0] = a[4] = a[8] = 1;
}

/* Traceless anti-Hermitian part used by both force terms:
 * Z = W - W^dagger,  out = Z - (1/3) Tr(Z) * 1. */
static void traceless_antiherm(const cplx *W, cplx *out)
{
    cplx Wd[9];
    mat_dag(W, Wd);
    for (int k = 0; k < 9; ++k) out[k] = W[k] - Wd[k];
    cplx tr = mat_trace(out) / 3.0;
    out[0] -= tr; out[4] -= tr; out[8] -= tr;
}

/* ------------------------------------------------------------------ */
/* Dirac matrices, DeGrand-Rossi basis; mu = 0..3 <-> gamma_1..gamma_4. */
/* ------------------------------------------------------------------ */

/* (re, im) of gamma_{mu+1}[row][col]. */
static const int gamma_tab[4][4][4][2] = {
    /* gamma_1 */
    {{{0, 0}, {0, 0}, {0, 0}, {0, 1}},
     {{0, 0}, {0, 0}, {0, 1}, {0, 0}},
     {{0, 0}, {0, -1}, {0, 0}, {0, 0}},
     {{0, -1}, {0, 0}, {0, 0}, {0, 0}}},
    /* gamma_2 */
    {{{0, 0}, {0, 0}, {0, 0}, {-1, 0}},
     {{0, 0}, {0, 0}, {1, 0}, {0, 0}},
     {{0, 0}, {1, 0}, {0, 0}, {0, 0}},
     {{-1, 0}, {0, 0}, {0, 0}, {0, 0}}},
    /* gamma_3 */
    {{{0, 0}, {0, 0}, {0, 1}, {0, 0}},
     {{0, 0}, {0, 0}, {0, 0}, {0, -1}},
     {{0, -1}, {0, 0}, {0, 0}, {0, 0}},
     {{0, 0}, {0, 1}, {0, 0}, {0, 0}}},
    /* gamma_4 */
    {{{0, 0}, {0, 0}, {1, 0}, {0, 0}},
     {{0, 0}, {0, 0}, {0, 0}, {1, 0}},
     {{1, 0}, {0, 0}, {0, 0}, {0, 0}},
     {{0, 0}, {1, 0}, {0, 0}, {0, 0}}},
};

static cplx gamma_el(int mu, int a, int b)
{
    return gamma_tab[mu][a][b][0] + I * gamma_tab[mu][a][b][1];
}

/* (1 + sgn*gamma_mu)[a][b] */
static cplx proj_el(int mu, int sgn, int a, int b)
{
    return (a == b ? 1.0 : 0.0) + sgn * gamma_el(mu, a, b);
}

/* Export the basis for tests. out[mu][a][b] complex. */
void or_gamma_matrices(cplx *out)
{
    for (int mu = 0; mu < 4; ++mu)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) out[(mu * 4 + a) * 4 + b] = gamma_el(mu, a, b);
}

/* ------------------------------------------------------------------ */
/* Wilson hopping term.                                                */
/*   (D psi)(x) = sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)            */
/*                       + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]   */
/* with a factor -1 on every hop across the time boundary.  dagger=1   */
/* gives D^dagger = gamma5 D gamma5, i.e. the projector signs swapped. */
/* out_parity = 0/1 writes only that parity (the rest set to zero);    */
/* -1 writes every site.                                               */
/* ------------------------------------------------------------------ */

/* The hopping term at one site i, written to out_site[12]. */
static void dslash_site(const int *L, const cplx *U, const cplx *in, long i, int dagger, cplx *out_site)
{
    int s_fwd = dagger ? +1 : -1; /* forward hop carries (1 + s_fwd*gamma) */
    int c[4];
    coords_of(L, i, c);
    cplx acc[4][3];
    memset(acc, 0, sizeof acc);
    for (int mu = 0; mu < 4; ++mu) {
        for (int dir = +1; dir >= -1; dir -= 2) {
            int wraps;
            long j = hop(L, c, mu, dir, &wraps);
            double bc = wraps ? -1.0 : 1.0;
            /* colour matrix: U_mu(x) forward, U_mu(x-mu)^dag backward */
            cplx Um[9];
            if (dir > 0)
                memcpy(Um, &U[(i * 4 + mu) * 9], sizeof Um);
            else
                mat_dag(&U[(j * 4 + mu) * 9], Um);
            cplx Upsi[4][3];
            for (int sp = 0; sp < 4; ++sp)
                for (int a = 0; a < 3; ++a) {
                    cplx s = 0;
                    for (int b = 0; b < 3; ++b) s += Um[3 * a + b] * in[(j * 4 + sp) * 3 + b];
                    Upsi[sp][a] = s;
                }
            int sgn = (dir > 0) ? s_fwd : -s_fwd;
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) {
                    cplx pr = proj_el(mu, sgn, a, b);
                    if (pr == 0) continue;
                    for (int col = 0; col < 3; ++col) acc[a][col] += bc * pr * Upsi[b][col];
                }
        }
    }
    for (int sp = 0; sp < 4; ++sp)
        for (int a = 0; a < 3; ++a) out_site[sp * 3 + a] = acc[sp][a];
}

void or_dslash(const int *L, const cplx *U, const cplx *in, cplx *out, int out_parity, int dagger)
{
    long V = vol4(L);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; ++i) {
        int c[4];
        coords_of(L, i, c);
        if (out_parity < 0 || parity_of(c) == out_parity)
            dslash_site(L, U, in, i, dagger, &out[i * 12]);
        else
            for (int k = 0; k < 12; ++k) out[i * 12 + k] = 0;
    }
}

/* The hopping term at the n listed sites only: out[k*12..] for sites[k].
 * U and in are full-size canonical arrays of which only the links and
 * spinors touching the listed sites are read. */
void or_dslash_sites(const int *L, const cplx *U, const cplx *in, const long *sites, long n, int dagger, cplx *out)
{
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k) dslash_site(L, U, in, sites[k], dagger, &out[k * 12]);
}

/* Full Wilson matrix M = 1 - kappa D (or M^dagger with dagger=1). */
void or_wilson_m(const int *L, const cplx *U, double kappa, const cplx *in, cplx *out, int dagger)
{
    long n = vol4(L) * 12;
    cplx *t = malloc(sizeof(cplx) * n);
    or_dslash(L, U, in, t, -1, dagger);
    for (long k = 0; k < n; ++k) out[k] = in[k] - kappa * t[k];
    free(t);
}

/* Even-even Schur operator Mhat = 1 - kappa^2 D_eo D_oe on even sites
 * (dagger=1: Mhat^dagger = 1 - kappa^2 (D^dag)_eo (D^dag)_oe).  The odd
 * half of the input is ignored and the odd half of the output is zero. */
void or_mhat(const int *L, const cplx *U, double kappa, const cplx *in, cplx *out, int dagger)
{
    long V = vol4(L);
    long n = V * 12;
    cplx *t = malloc(sizeof(cplx) * n);
    cplx *u = malloc(sizeof(cplx) * n);
    or_dslash(L, U, in, t, 1, dagger); /* odd <- even */
    or_dslash(L, U, t, u, 0, dagger);  /* even <- odd */
    for (long i = 0; i < V; ++i) {
        int c[4];
        coords_of(L, i, c);
        int even = parity_of(c) == 0;
        for (int k = 0; k < 12; ++k)
            out[i * 12 + k] = even ? in[i * 12 + k] - kappa * kappa * u[i * 12 + k] : 0;
    }
    free(t);
    free(u);
}

/* ------------------------------------------------------------------ */
/* Global sums (QDP++ sum / innerProduct / sumMulti), serial order.    */
/* ------------------------------------------------------------------ */

double or_norm2(long n, const cplx *a)
{
    double s = 0;
    for (long k = 0; k < n; ++k) s += creal(a[k]) * creal(a[k]) + cimag(a[k]) * cimag(a[k]);
    return s;
}

/* <a, b> = sum conj(a) b */
void or_inner(long n, const cplx *a, const cplx *b, double *re_im)
{
    cplx s = 0;
    for (long k = 0; k < n; ++k) s += conj(a[k]) * b[k];
    re_im[0] = creal(s);
    re_im[1] = cimag(s);
}

/* sumMulti: out[subset[i]] += sum over the `per_site` reals of site i of
 * f[i*per_site + k].  Subsets index 0..nsub-1. */
void or_sum_multi(long nsites, int per_site, const double *f, const int *subset, int nsub, double *out)
{
    for (int s = 0; s < nsub; ++s) out[s] = 0;
    for (long i = 0; i < nsites; ++i)
        for (int k = 0; k < per_site; ++k) out[subset[i]] += f[i * per_site + k];
}

/* ------------------------------------------------------------------ */
/* Gauge action and plaquette (Wilson plaquette action).               */
/*   U_munu(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag         */
/*   plaquette = (1/18V) sum_{x, mu<nu} Re Tr U_munu(x)                */
/*   S_g = beta sum_{x, mu<nu} (1 - Re Tr U_munu(x) / 3)               */
/* ------------------------------------------------------------------ */

static double site_plaquette_sum(const int *L, const cplx *U, long i)
{
    int c[4];
    coords_of(L, i, c);
    double s = 0;
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = mu + 1; nu < 4; ++nu) {
            long xmu = hop(L, c, mu, +1, NULL);
            long xnu = hop(L, c, nu, +1, NULL);
            cplx a[9], b[9], t[9];
            mat_mul(&U[(i * 4 + mu) * 9], &U[(xmu * 4 + nu) * 9], a);
            mat_dag(&U[(xnu * 4 + mu) * 9], t);
            mat_mul(a, t, a);
            mat_dag(&U[(i * 4 + nu) * 9], b);
            mat_mul(a, b, a);
            s += creal(mat_trace(a));
        }
    return s;
}

double or_plaquette(const int *L, const cplx *U)
{
    long V = vol4(L);
    double *ps = malloc(sizeof(double) * V);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; ++i) ps[i] = site_plaquette_sum(L, U, i);
    double s = 0;
    for (long i = 0; i < V; ++i) s += ps[i];
    free(ps);
    return s / (18.0 * V);
}

double or_gauge_action(const int *L, const cplx *U, double beta)
{
    long V = vol4(L);
    double *ps = malloc(sizeof(double) * V);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; ++i) ps[i] = site_plaquette_sum(L, U, i);
    double s = 0;
    for (long i = 0; i < V; ++i) s += 6.0 - ps[i] / 3.0;
    free(ps);
    return beta * s;
}

/* ------------------------------------------------------------------ */
/* Forces.  With U' = i P U and P' = -F, F = sum_a T^a d_a S where      */
/* d_a S = d/dt S(exp(i t T^a) U_mu(x)) at t = 0, so that dS/dt =       */
/* 2 sum Re Tr(P F) and H = sum Tr P^2 + S is conserved.               */
/* ------------------------------------------------------------------ */

/* Staple sum A_mu(x) = sum_{nu != mu} [ U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
 *                     + U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu) ]. */
static void staple_sum(const int *L, const cplx *U, long i, int mu, cplx *A)
{
    int c[4];
    coords_of(L, i, c);
    for (int k = 0; k < 9; ++k) A[k] = 0;
    long xmu = hop(L, c, mu, +1, NULL);
    int cmu[4];
    coords_of(L, xmu, cmu);
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        cplx a[9], b[9], t[9];
        /* upper staple */
        long xnu = hop(L, c, nu, +1, NULL);
        mat_dag(&U[(xnu * 4 + mu) * 9], t);
        mat_mul(&U[(xmu * 4 + nu) * 9], t, a);
        mat_dag(&U[(i * 4 + nu) * 9], b);
        mat_mul(a, b, a);
        mat_add_to(A, a);
        /* lower staple */
        long xmu_mnu = hop(L, cmu, nu, -1, NULL);
        long xmnu = hop(L, c, nu, -1, NULL);
        mat_dag(&U[(xmu_mnu * 4 + nu) * 9], a);
        mat_dag(&U[(xmnu * 4 + mu) * 9], t);
        mat_mul(a, t, a);
        mat_mul(a, &U[(xmnu * 4 + nu) * 9], a);
        mat_add_to(A, a);
    }
}

/* Gauge force F_g = -(i beta / 12) TA(U_mu(x) A_mu(x)),
 * TA(W) = (W - W^dag) - Tr(W - W^dag)/3. */
static void gauge_force_link(const int *L, const cplx *U, double beta, long i, int mu, cplx *F9)
{
    cplx A[9], W[9], Z[9];
    staple_sum(L, U, i, mu, A);
    mat_mul(&U[(i * 4 + mu) * 9], A, W);
    traceless_antiherm(W, Z);
    for (int k = 0; k < 9; ++k) F9[k] = -I * beta / 12.0 * Z[k];
}

void or_gauge_force(const int *L, const cplx *U, double beta, cplx *F)
{
    long V = vol4(L);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; ++i)
        for (int mu = 0; mu < 4; ++mu) gauge_force_link(L, U, beta, i, mu, &F[(i * 4 + mu) * 9]);
}

/* The same force at the listed lexicographic sites only: F[n][4][9]. */
void or_gauge_force_sites(const int *L, const cplx *U, double beta, const long *sites, long n, cplx *F)
{
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k)
        for (int mu = 0; mu < 4; ++mu) gauge_force_link(L, U, beta, sites[k], mu, &F[(k * 4 + mu) * 9]);
}

/* Wilson fermion force for S_f = phi^dag (Mhat^dag Mhat)^-1 phi.
 * X and Y are full-lattice spinors: X = (X_e, D_oe X_e), Y = (Mhat X_e,
 * (D^dag)_oe Mhat X_e).  With s the time-boundary sign of the hop x -> x+mu,
 *   M1 = s sum_{ab} (1 - gamma_mu)_{ab} X_b(x+mu) Y_a(x)^dag
 *   M2 = s sum_{ab} (1 + gamma_mu)_{ab} X_b(x) Y_a(x+mu)^dag
 *   W  = U_mu(x) M1 - M2 U_mu(x)^dag,   F_f = (i coef / 2) TA(W),
 * where coef = kappa^2 for the even/odd preconditioned action (and kappa
 * for the unpreconditioned one, with X = (M^dag M)^-1 phi, Y = M X). */
/* The force on the link (site i, direction mu), nine entries. */
static void fermion_force_link(const int *L, const cplx *U, double coef, const cplx *X, const cplx *Y, long i,
                               int mu, cplx *Fl)
{
    int c[4];
    coords_of(L, i, c);
    int wraps;
    long j = hop(L, c, mu, +1, &wraps);
    double s = wraps ? -1.0 : 1.0;
    cplx M1[9], M2[9];
    for (int k = 0; k < 9; ++k) M1[k] = M2[k] = 0;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            cplx pm = proj_el(mu, -1, a, b), pp = proj_el(mu, +1, a, b);
            for (int r = 0; r < 3; ++r)
                for (int q = 0; q < 3; ++q) {
                    M1[3 * r + q] += s * pm * X[(j * 4 + b) * 3 + r] * conj(Y[(i * 4 + a) * 3 + q]);
                    M2[3 * r + q] += s * pp * X[(i * 4 + b) * 3 + r] * conj(Y[(j * 4 + a) * 3 + q]);
                }
        }
    cplx W[9], t[9], Ud[9], Z[9];
    const cplx *Ul = &U[(i * 4 + mu) * 9];
    mat_mul(Ul, M1, W);
    mat_dag(Ul, Ud);
    mat_mul(M2, Ud, t);
    for (int k = 0; k < 9; ++k) W[k] -= t[k];
    traceless_antiherm(W, Z);
    for (int k = 0; k < 9; ++k) Fl[k] = I * coef / 2.0 * Z[k];
}

void or_fermion_force(const int *L, const cplx *U, double coef, const cplx *X, const cplx *Y, cplx *F)
{
    long V = vol4(L);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; ++i)
        for (int mu = 0; mu < 4; ++mu) fermion_force_link(L, U, coef, X, Y, i, mu, &F[(i * 4 + mu) * 9]);
}

/* The same at the listed sites only (X and Y needed at those sites and
 * their forward neighbours): F is (n, 4, 3, 3). */
void or_fermion_force_sites(const int *L, const cplx *U, double coef, const cplx *X, const cplx *Y, const long *sites,
                            long n, cplx *F)
{
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k)
        for (int mu = 0; mu < 4; ++mu) fermion_force_link(L, U, coef, X, Y, sites[k], mu, &F[(k * 4 + mu) * 9]);
}

/* ------------------------------------------------------------------ */
/* Exponential and reunitarisation.                                    */
/* ------------------------------------------------------------------ */

/* Matrix exponential by its Taylor series, summed until the next term is
 * below 1e-19 in every entry (the series of a 3x3 matrix of norm a few
 * units converges to full double precision well within 60 terms). */
void or_mat_exp(const cplx *A, cplx *E)
{
    cplx term[9];
    mat_identity(term);
    mat_identity(E);
    for (int n = 1; n <= 60; ++n) {
        mat_mul(term, A, term);
        double mx = 0;
        for (int k = 0; k < 9; ++k) {
            term[k] /= n;
            if (cabs(term[k]) > mx) mx = cabs(term[k]);
        }
        mat_add_to(E, term);
        if (mx < 1e-19) break;
    }
}

/* Row-wise Gram-Schmidt projection to SU(3): normalise row 0, orthogonalise
 * row 1 against it and normalise, row 2 = conj(row0 x row1). */
void or_reunit(cplx *u)
{
    double n0 = 0;
    for (int k = 0; k < 3; ++k) n0 += creal(u[k] * conj(u[k]));
    n0 = 1.0 / sqrt(n0);
    for (int k = 0; k < 3; ++k) u[k] *= n0;
    cplx ov = 0; /* row0^dag . row1 */
    for (int k = 0; k < 3; ++k) ov += conj(u[k]) * u[3 + k];
    for (int k = 0; k < 3; ++k) u[3 + k] -= ov * u[k];
    double n1 = 0;
    for (int k = 0; k < 3; ++k) n1 += creal(u[3 + k] * conj(u[3 + k]));
    n1 = 1.0 / sqrt(n1);
    for (int k = 0; k < 3; ++k) u[3 + k] *= n1;
    u[6] = conj(u[1] * u[5] - u[2] * u[4]);
    u[7] = conj(u[2] * u[3] - u[0] * u[5]);
    u[8] = conj(u[0] * u[4] - u[1] * u[3]);
}

/* Link update of the leapfrog: U_mu(x) <- reunit(exp(i eps P_mu(x)) U_mu(x)). */
void or_update_links(const int *L, cplx *U, const cplx *P, double eps)
{
    long n = vol4(L) * 4;
#pragma omp parallel for schedule(static)
    for (long l = 0; l < n; ++l) {
        cplx A[9], E[9];
        for (int k = 0; k < 9; ++k) A[k] = I * eps * P[l * 9 + k];
        or_mat_exp(A, E);
        mat_mul(E, &U[l * 9], &U[l * 9]);
        or_reunit(&U[l * 9]);
    }
}

/* Momentum update P <- P - eps F. */
void or_momentum_update(const int *L, cplx *P, const cplx *F, double eps)
{
    long n = vol4(L) * 36;
    for (long k = 0; k < n; ++k) P[k] -= eps * F[k];
}

/* Kinetic term sum_{x,mu} Tr P_mu(x)^2 (P Hermitian, so sum |P_ij|^2). */
double or_kinetic(const int *L, const cplx *P)
{
    long n = vol4(L) * 4;
    double s = 0;
    for (long l = 0; l < n; ++l) {
        cplx sq[9];
        mat_mul(&P[l * 9], &P[l * 9], sq);
        s += creal(mat_trace(sq));
    }
    return s;
}

/* ------------------------------------------------------------------ */
/* Counter-based random numbers: Philox4x64-10 (Salmon, Moraes, Dror,  */
/* Shaw, SC'11), u53 uniforms, Box-Muller Gaussians.                   */
/* ------------------------------------------------------------------ */

void or_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    const uint64_t mul0 = 0xD2E7470EE14C6C93ULL, mul1 = 0xCA5A826395121157ULL;
    const uint64_t inc0 = 0x9E3779B97F4A7C15ULL, inc1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += inc0; k1 += inc1; }
        unsigned __int128 p0 = (unsigned __int128)mul0 * x0;
        unsigned __int128 p1 = (unsigned __int128)mul1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        x0 = hi1 ^ x1 ^ k0;
        x1 = lo1;
        x2 = hi0 ^ x3 ^ k1;
        x3 = lo0;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Uniform in (0,1): top 53 bits plus one half, times 2^-53 (exact). */
double or_u53(uint64_t w) { return ((double)(w >> 11) + 0.5) * 0x1p-53; }

/* Random-stream assignment (counter word c2). */
enum { ST_WEAKFIELD = 0, ST_MOMENTA = 1, ST_ETA = 2, ST_ACCEPT = 3, ST_SOURCE = 4, ST_ETA2 = 5 };

/* `nblocks` Philox blocks for site i: counter (block, i, stream, epoch),
 * key (seed, 0); words written in block order. */
static void site_words(uint64_t seed, long i, uint64_t stream, uint64_t epoch, int nblocks, uint64_t *w)
{
    uint64_t key[2] = {seed, 0};
    for (int b = 0; b < nblocks; ++b) {
        uint64_t ctr[4] = {(uint64_t)b, (uint64_t)i, stream, epoch};
        or_philox4x64_10(ctr, key, &w[4 * b]);
    }
}

/* Box-Muller on consecutive uniform pairs. */
static void gaussians_from_words(const uint64_t *w, int n, double *g)
{
    const double two_pi = 6.283185307179586476925286766559;
    for (int k = 0; k < n; k += 2) {
        double u0 = or_u53(w[k]), u1 = or_u53(w[k + 1]);
        double r = sqrt(-2.0 * log(u0));
        double th = two_pi * u1;
        g[k] = r * cos(th);
        g[k + 1] = r * sin(th);
    }
}

/* Raw words for tests: out[b*4..] for blocks 0..nblocks-1. */
void or_site_words(uint64_t seed, long i, uint64_t stream, uint64_t epoch, int nblocks, uint64_t *w)
{
    site_words(seed, i, stream, epoch, nblocks, w);
}

/* The 32 Gaussians of a site for an su(3)-valued field: g[mu*8 + (a-1)]. */
void or_site_gaussians(uint64_t seed, long i, uint64_t stream, uint64_t epoch, int n, double *g)
{
    uint64_t w[32];
    site_words(seed, i, stream, epoch, (n + 3) / 4, w);
    gaussians_from_words(w, n, g);
}

/* Hermitian traceless matrix sum_a omega_a T^a with T^a = lambda^a / 2
 * (Gell-Mann matrices). */
void or_algebra_matrix(const double *om, cplx *H)
{
    const double r3 = 1.0 / sqrt(3.0);
    H[0] = 0.5 * (om[2] + r3 * om[7]);
    H[4] = 0.5 * (-om[2] + r3 * om[7]);
    H[8] = 0.5 * (-2.0 * r3 * om[7]);
    H[1] = 0.5 * (om[0] - I * om[1]);
    H[3] = conj(H[1]);
    H[2] = 0.5 * (om[3] - I * om[4]);
    H[6] = conj(H[2]);
    H[5] = 0.5 * (om[5] - I * om[6]);
    H[7] = conj(H[5]);
}

/* Momentum refresh: P_mu(x) = sum_a omega_a T^a, omega ~ N(0,1) from the
 * momentum stream at epoch = trajectory index. */
void or_refresh_momenta(const int *L, uint64_t seed, uint64_t traj, cplx *P)
{
    long V = vol4(L);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; ++i) {
        double g[32];
        or_site_gaussians(seed, i, ST_MOMENTA, traj, 32, g);
        for (int mu = 0; mu < 4; ++mu) or_algebra_matrix(&g[mu * 8], &P[(i * 4 + mu) * 9]);
    }
}

/* Weak-field start U_mu(x) = reunit(exp(i eps H_mu(x))), H from stream 0. */
void or_weak_field(const int *L, uint64_t seed, double eps, cplx *U)
{
    long V = vol4(L);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; ++i) {
        double g[32];
        or_site_gaussians(seed, i, ST_WEAKFIELD, 0, 32, g);
        for (int mu = 0; mu < 4; ++mu) {
            cplx H[9], A[9];
            or_algebra_matrix(&g[mu * 8], H);
            for (int k = 0; k < 9; ++k) A[k] = I * eps * H[k];
            or_mat_exp(A, &U[(i * 4 + mu) * 9]);
            or_reunit(&U[(i * 4 + mu) * 9]);
        }
    }
}

static void eta_stream(const int *L, uint64_t seed, uint64_t traj, int parity, int stream, cplx *eta);

/* Pseudofermion noise eta on the sites of `parity`: complex Gaussian with
 * E|eta_k|^2 = 1, components (spin, colour, re/im) in that order. */
void or_eta(const int *L, uint64_t seed, uint64_t traj, int parity, cplx *eta)
{
    eta_stream(L, seed, traj, parity, ST_ETA, eta);
}

/* The same noise from another Philox stream (the second pseudofermion of
 * the mass-preconditioned action uses stream 5). */
void or_eta2(const int *L, uint64_t seed, uint64_t traj, int parity, cplx *eta)
{
    eta_stream(L, seed, traj, parity, ST_ETA2, eta);
}

static void eta_stream(const int *L, uint64_t seed, uint64_t traj, int parity, int stream, cplx *eta)
{
    long V = vol4(L);
    const double s = sqrt(0.5); /* 1/sqrt2, correctly rounded */
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; ++i) {
        int c[4];
        coords_of(L, i, c);
        double g[24];
        or_site_gaussians(seed, i, stream, traj, 24, g);
        for (int k = 0; k < 12; ++k)
            eta[i * 12 + k] = (parity_of(c) == parity) ? s * (g[2 * k] + I * g[2 * k + 1]) : 0;
    }
}

/* Solver sources on the full lattice.  kind 0: Gaussian (unit variance per
 * real component); 1: Z2 noise (+-1 +-i)/sqrt2 with the sign of each real
 * component from bit 63 of successive Philox words; 2: point source at
 * site 0, spin 0, colour 0.  epoch = source index. */
void or_source(const int *L, int kind, uint64_t seed, uint64_t epoch, cplx *b)
{
    long V = vol4(L);
    const double s = sqrt(0.5); /* 1/sqrt2, correctly rounded */
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; ++i) {
        if (kind == 0) {
            double g[24];
            or_site_gaussians(seed, i, ST_SOURCE, epoch, 24, g);
            for (int k = 0; k < 12; ++k) b[i * 12 + k] = g[2 * k] + I * g[2 * k + 1];
        } else if (kind == 1) {
            uint64_t w[24];
            site_words(seed, i, ST_SOURCE, epoch, 6, w);
            for (int k = 0; k < 12; ++k) {
                double re = (w[2 * k] >> 63) ? -s : s;
                double im = (w[2 * k + 1] >> 63) ? -s : s;
                b[i * 12 + k] = re + I * im;
            }
        } else {
            for (int k = 0; k < 12; ++k) b[i * 12 + k] = (i == 0 && k == 0) ? 1.0 : 0.0;
        }
    }
}

/* Site-list variants of the weak-field start and the sources: fill only the
 * listed sites (and the 4 links of each) of full-size canonical arrays. */
void or_weak_field_sites(const int *L, uint64_t seed, double eps, const long *sites, long n, cplx *U)
{
    (void)L;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k) {
        long i = sites[k];
        double g[32];
        or_site_gaussians(seed, i, ST_WEAKFIELD, 0, 32, g);
        for (int mu = 0; mu < 4; ++mu) {
            cplx H[9], A[9];
            or_algebra_matrix(&g[mu * 8], H);
            for (int m = 0; m < 9; ++m) A[m] = I * eps * H[m];
            or_mat_exp(A, &U[(i * 4 + mu) * 9]);
            or_reunit(&U[(i * 4 + mu) * 9]);
        }
    }
}

void or_gauss_source_sites(uint64_t seed, uint64_t epoch, const long *sites, long n, cplx *b)
{
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k) {
        long i = sites[k];
        double g[24];
        or_site_gaussians(seed, i, ST_SOURCE, epoch, 24, g);
        for (int m = 0; m < 12; ++m) b[i * 12 + m] = g[2 * m] + I * g[2 * m + 1];
    }
}

/* Metropolis uniform of trajectory `traj`: word 0 of block 0, site 0. */
double or_accept_uniform(uint64_t seed, uint64_t traj)
{
    uint64_t w[4];
    site_words(seed, 0, ST_ACCEPT, traj, 1, w);
    return or_u53(w[0]);
}

/* ------------------------------------------------------------------ */
/* Krylov solvers.                                                     */
/* ------------------------------------------------------------------ */

typedef struct {
    int iters;
    double rel_res;      /* recursively updated residual norm / ||b|| */
    double true_rel_res; /* recomputed ||b - A x|| / ||b|| */
} or_cg_stats;

static void normal_op(const int *L, const cplx *U, double kappa, const cplx *in, cplx *out, cplx *tmp)
{
    or_mhat(L, U, kappa, in, tmp, 0);
    or_mhat(L, U, kappa, tmp, out, 1);
}

/* Conjugate gradient (Hestenes-Stiefel) on A = Mhat^dag Mhat, x0 = 0.
 * Stops at the first k with ||r_k|| <= tol ||b|| (recursive residual), or
 * after exactly `fixed_iters` iterations when that is positive.
 * Returns 0 on convergence, -4 when maxiter is reached first. */
static int cg_mhat_from(const int *L, const cplx *U, double kappa, const cplx *b, cplx *x, int start_zero,
                        double tol, int maxiter, int fixed_iters, or_cg_stats *st);

int or_cg_mhat(const int *L, const cplx *U, double kappa, const cplx *b, cplx *x, double tol, int maxiter,
               int fixed_iters, or_cg_stats *st)
{
    return cg_mhat_from(L, U, kappa, b, x, 1, tol, maxiter, fixed_iters, st);
}

/* The same iteration started from the x passed in (r0 = b - A x0). */
int or_cg_mhat_x0(const int *L, const cplx *U, double kappa, const cplx *b, cplx *x, double tol, int maxiter,
                  or_cg_stats *st)
{
    return cg_mhat_from(L, U, kappa, b, x, 0, tol, maxiter, 0, st);
}

static int cg_mhat_from(const int *L, const cplx *U, double kappa, const cplx *b, cplx *x, int start_zero,
                        double tol, int maxiter, int fixed_iters, or_cg_stats *st)
{
    long V = vol4(L), n = V * 12;
    cplx *r = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n);
    cplx *q = malloc(sizeof(cplx) * n), *tmp = malloc(sizeof(cplx) * n);
    if (start_zero) {
        for (long k = 0; k < n; ++k) { x[k] = 0; r[k] = b[k]; p[k] = b[k]; }
    } else {
        normal_op(L, U, kappa, x, q, tmp);
        for (long k = 0; k < n; ++k) { r[k] = b[k] - q[k]; p[k] = r[k]; }
    }
    double bb = or_norm2(n, b), rr = or_norm2(n, r);
    int k = 0, status = 0;
    int limit = fixed_iters > 0 ? fixed_iters : maxiter;
    while (1) {
        if (fixed_iters > 0) {
            if (k == fixed_iters) break;
        } else if (rr <= tol * tol * bb) {
            break;
        }
        if (k == limit) { status = -4; break; }
        normal_op(L, U, kappa, p, q, tmp);
        double ri[2];
        or_inner(n, p, q, ri);
        double alpha = rr / ri[0];
        for (long m = 0; m < n; ++m) { x[m] += alpha * p[m]; r[m] -= alpha * q[m]; }
        double rr_new = or_norm2(n, r);
        double beta = rr_new / rr;
        for (long m = 0; m < n; ++m) p[m] = r[m] + beta * p[m];
        rr = rr_new;
        ++k;
    }
    if (st) {
        st->iters = k;
        st->rel_res = bb > 0 ? sqrt(rr / bb) : 0;
        normal_op(L, U, kappa, x, q, tmp);
        for (long m = 0; m < n; ++m) q[m] = b[m] - q[m];
        st->true_rel_res = bb > 0 ? sqrt(or_norm2(n, q) / bb) : 0;
    }
    free(r); free(p); free(q); free(tmp);
    return status;
}

/* Wilson solve M x = b on the full lattice through the even/odd Schur
 * complement: bhat_e = b_e + kappa D_eo b_o; CGLS on Mhat x_e = bhat_e
 * (stop at ||bhat - Mhat x_e|| <= tol ||b||); x_o = b_o + kappa D_oe x_e.
 * true_rel_res is ||b - M x|| / ||b|| recomputed with the full operator. */
int or_wilson_solve(const int *L, const cplx *U, double kappa, const cplx *b, cplx *x, double tol, int maxiter,
                    or_cg_stats *st)
{
    long V = vol4(L), n = V * 12;
    cplx *bh = malloc(sizeof(cplx) * n), *t = malloc(sizeof(cplx) * n);
    cplx *r = malloc(sizeof(cplx) * n), *s = malloc(sizeof(cplx) * n);
    cplx *p = malloc(sizeof(cplx) * n), *q = malloc(sizeof(cplx) * n);
    double bnorm2 = or_norm2(n, b);

    or_dslash(L, U, b, t, 0, 0); /* (D b)_e: reads odd sites of b */
    for (long i = 0; i < V; ++i) {
        int even = or_site_parity(L, i) == 0;
        for (int k = 0; k < 12; ++k) bh[i * 12 + k] = even ? b[i * 12 + k] + kappa * t[i * 12 + k] : 0;
    }
    for (long m = 0; m < n; ++m) { x[m] = 0; r[m] = bh[m]; }
    or_mhat(L, U, kappa, r, s, 1);
    for (long m = 0; m < n; ++m) p[m] = s[m];
    double gam = or_norm2(n, s), rr = or_norm2(n, r);
    int k = 0, status = 0;
    while (rr > tol * tol * bnorm2) {
        if (k == maxiter) { status = -4; break; }
        or_mhat(L, U, kappa, p, q, 0);
        double alpha = gam / or_norm2(n, q);
        for (long m = 0; m < n; ++m) { x[m] += alpha * p[m]; r[m] -= alpha * q[m]; }
        or_mhat(L, U, kappa, r, s, 1);
        double gam_new = or_norm2(n, s);
        double beta = gam_new / gam;
        for (long m = 0; m < n; ++m) p[m] = s[m] + beta * p[m];
        gam = gam_new;
        rr = or_norm2(n, r);
        ++k;
    }
    /* odd half: x_o = b_o + kappa D_oe x_e */
    or_dslash(L, U, x, t, 1, 0);
    for (long i = 0; i < V; ++i)
        if (or_site_parity(L, i) == 1)
            for (int c = 0; c < 12; ++c) x[i * 12 + c] = b[i * 12 + c] + kappa * t[i * 12 + c];
    if (st) {
        st->iters = k;
        st->rel_res = bnorm2 > 0 ? sqrt(rr / bnorm2) : 0;
        or_wilson_m(L, U, kappa, x, t, 0);
        for (long m = 0; m < n; ++m) t[m] = b[m] - t[m];
        st->true_rel_res = bnorm2 > 0 ? sqrt(or_norm2(n, t) / bnorm2) : 0;
    }
    free(bh); free(t); free(r); free(s); free(p); free(q);
    return status;
}

/* ------------------------------------------------------------------ */
/* Hybrid Monte Carlo.                                                 */
/* ------------------------------------------------------------------ */

typedef struct {
    double beta, kappa;
    double tol;
    int maxiter;
} or_action;

typedef struct {
    int solves, iters_total, iters_max, nonconverged;
} or_md_stats;

/* X, Y of the fermion force from the CG solution X_e (full-lattice arrays). */
static void force_vectors(const int *L, const cplx *U, double kappa, const cplx *Xe, cplx *X, cplx *Y)
{
    long V = vol4(L), n = V * 12;
    cplx *t = malloc(sizeof(cplx) * n), *ye = malloc(sizeof(cplx) * n);
    or_dslash(L, U, Xe, t, 1, 0); /* D_oe X_e */
    or_mhat(L, U, kappa, Xe, ye, 0);
    for (long i = 0; i < V; ++i) {
        int even = or_site_parity(L, i) == 0;
        for (int k = 0; k < 12; ++k) {
            X[i * 12 + k] = even ? Xe[i * 12 + k] : t[i * 12 + k];
            Y[i * 12 + k] = even ? ye[i * 12 + k] : 0;
        }
    }
    or_dslash(L, U, Y, t, 1, 1); /* (D^dag)_oe Y_e */
    for (long i = 0; i < V; ++i)
        if (or_site_parity(L, i) == 1)
            for (int k = 0; k < 12; ++k) Y[i * 12 + k] = t[i * 12 + k];
    free(t);
    free(ye);
}

/* P <- P - coef (F_g + F_f); the solve result X_e is left in Xe. */
static int force_kick(const int *L, const cplx *U, cplx *P, const cplx *phi, const or_action *a, double coef,
                      cplx *Xe, or_md_stats *ms)
{
    long V = vol4(L), n = V * 12;
    cplx *F = malloc(sizeof(cplx) * V * 36);
    or_gauge_force(L, U, a->beta, F);
    or_momentum_update(L, P, F, coef);
    or_cg_stats st;
    int status = or_cg_mhat(L, U, a->kappa, phi, Xe, a->tol, a->maxiter, 0, &st);
    ms->solves++;
    ms->iters_total += st.iters;
    if (st.iters > ms->iters_max) ms->iters_max = st.iters;
    if (status) ms->nonconverged++;
    cplx *X = malloc(sizeof(cplx) * n), *Y = malloc(sizeof(cplx) * n);
    force_vectors(L, U, a->kappa, Xe, X, Y);
    or_fermion_force(L, U, a->kappa * a->kappa, X, Y, F);
    or_momentum_update(L, P, F, coef);
    free(X); free(Y); free(F);
    return status;
}

/* Leapfrog (PQP) over time tau in nsteps steps: a half kick, then nsteps
 * times [links by eps, kick by eps] with the last kick halved.  tau may be
 * negative (used by the reversibility check).  Xe receives the solve of
 * the final force evaluation. */
int or_leapfrog(const int *L, cplx *U, cplx *P, const cplx *phi, const or_action *a, double tau, int nsteps,
                cplx *Xe, or_md_stats *ms)
{
    double eps = tau / nsteps;
    int status = 0;
    memset(ms, 0, sizeof *ms);
    status |= force_kick(L, U, P, phi, a, 0.5 * eps, Xe, ms);
    for (int k = 1; k <= nsteps; ++k) {
        or_update_links(L, U, P, eps);
        status |= force_kick(L, U, P, phi, a, k < nsteps ? eps : 0.5 * eps, Xe, ms);
    }
    return status;
}

typedef struct {
    double H_old, H_new, dH;
    double S_g_old, S_g_new, S_f_old, S_f_new, KE_old, KE_new;
    double plaquette; /* after the accept/reject step */
    double u;         /* Metropolis uniform */
    int accepted;
    int cg_iters_total, cg_iters_max, nonconverged;
} or_traj_result;

/* Accept iff every solve converged and u < exp(-dH) (always for dH <= 0);
 * a non-finite dH rejects. */
static int metropolis_accept(int status, double dH, double u)
{
    if (dH != dH) return 0;
    return (status == 0) && (dH <= 0 || u < exp(-dH));
}

/* One HMC trajectory at index `traj` (momenta from stream 1, pseudofermion
 * noise from stream 2 on even sites, Metropolis uniform from stream 3, all
 * at epoch traj).  S_f(old) = eta^dag eta exactly, since phi = Mhat^dag eta. */
int or_hmc_trajectory(const int *L, cplx *U, const or_action *a, uint64_t seed, uint64_t traj, double tau,
                      int nsteps, or_traj_result *res)
{
    long V = vol4(L), n = V * 12;
    cplx *U_old = malloc(sizeof(cplx) * V * 36), *P = malloc(sizeof(cplx) * V * 36);
    cplx *eta = malloc(sizeof(cplx) * n), *phi = malloc(sizeof(cplx) * n), *Xe = malloc(sizeof(cplx) * n);
    memcpy(U_old, U, sizeof(cplx) * V * 36);
    or_refresh_momenta(L, seed, traj, P);
    or_eta(L, seed, traj, 0, eta);
    or_mhat(L, U, a->kappa, eta, phi, 1);

    res->KE_old = or_kinetic(L, P);
    res->S_g_old = or_gauge_action(L, U, a->beta);
    res->S_f_old = or_norm2(n, eta);
    res->H_old = res->KE_old + res->S_g_old + res->S_f_old;

    or_md_stats ms;
    int status = or_leapfrog(L, U, P, phi, a, tau, nsteps, Xe, &ms);

    double ri[2];
    or_inner(n, phi, Xe, ri);
    res->KE_new = or_kinetic(L, P);
    res->S_g_new = or_gauge_action(L, U, a->beta);
    res->S_f_new = ri[0];
    res->H_new = res->KE_new + res->S_g_new + res->S_f_new;
    res->dH = res->H_new - res->H_old;
    res->u = or_accept_uniform(seed, traj);
    res->accepted = metropolis_accept(status, res->dH, res->u);
    if (!res->accepted) memcpy(U, U_old, sizeof(cplx) * V * 36);
    res->plaquette = or_plaquette(L, U);
    res->cg_iters_total = ms.iters_total;
    res->cg_iters_max = ms.iters_max;
    res->nonconverged = ms.nonconverged;
    free(U_old); free(P); free(eta); free(phi); free(Xe);
    return status;
}

/* ------------------------------------------------------------------ */
/* Mass-preconditioned (Hasenbusch) action on several time scales.     */
/* ------------------------------------------------------------------ */
/* The paper's production run (Sec. 7) splits the two-flavour determinant
 * with a heavier hopping parameter kappa_h < kappa,
 *   det(A) = det(A_h) * det(A) / det(A_h),   A = Mhat^dag Mhat,
 * with one pseudofermion per factor:
 *   S_1 = phi_1^dag A_h^-1 phi_1,            phi_1 = Mhat_h^dag eta_1,
 *   S_2 = chi^dag A^-1 chi, chi = Mhat_h^dag phi_2,
 *                                            phi_2 = Mhat_h A_h^-1 Mhat^dag eta_2,
 * so that S_1 = |eta_1|^2 and S_2 = |eta_2|^2 at the start (eta_1 from
 * stream 2, eta_2 from stream 5).  The ratio force follows from
 *   dS_2 = 2 Re(phi_2^dag dMhat_h X_2) - 2 Re((Mhat X_2)^dag dMhat X_2),
 * X_2 = A^-1 chi: the fermion-force bilinear with (X_2, Mhat X_2, kappa)
 * minus the same bilinear with (X_2, phi_2, kappa_h).  The monomials run on
 * nested leapfrog time scales (Sexton-Weingarten): ratio (outer), heavy,
 * gauge (inner), n_r, n_h, n_g steps per enclosing step. */

typedef struct {
    double beta, kappa, kappa_h;
    double tol;
    int maxiter;
    int n_ratio, n_heavy, n_gauge;
} or_mts_action;

typedef struct {
    double S1_old, S2_old, S1_new, S2_new;
    int solves_ratio, solves_heavy, gauge_forces, link_updates;
} or_mts_stats;

/* Full-lattice X = (X_e, D_oe X_e) and Y = (Y_e, (D^dag)_oe Y_e). */
static void bilinear_vectors(const int *L, const cplx *U, const cplx *Xe, const cplx *Ye, cplx *X, cplx *Y)
{
    long V = vol4(L), n = V * 12;
    cplx *t = malloc(sizeof(cplx) * n);
    or_dslash(L, U, Xe, t, 1, 0);
    for (long i = 0; i < V; ++i) {
        int even = or_site_parity(L, i) == 0;
        for (int k = 0; k < 12; ++k) {
            X[i * 12 + k] = even ? Xe[i * 12 + k] : t[i * 12 + k];
            Y[i * 12 + k] = even ? Ye[i * 12 + k] : 0;
        }
    }
    or_dslash(L, U, Y, t, 1, 1);
    for (long i = 0; i < V; ++i)
        if (or_site_parity(L, i) == 1)
            for (int k = 0; k < 12; ++k) Y[i * 12 + k] = t[i * 12 + k];
    free(t);
}

/* Force of the heavy monomial S_1 at U; X_1 = A_h^-1 phi_1 left in X1. */
static int heavy_force(const int *L, const cplx *U, const or_mts_action *a, const cplx *phi1, cplx *X1, cplx *F,
                       or_mts_stats *ms)
{
    long n = vol4(L) * 12;
    or_cg_stats st;
    int status = or_cg_mhat(L, U, a->kappa_h, phi1, X1, a->tol, a->maxiter, 0, &st);
    ms->solves_heavy++;
    cplx *ye = malloc(sizeof(cplx) * n), *X = malloc(sizeof(cplx) * n), *Y = malloc(sizeof(cplx) * n);
    or_mhat(L, U, a->kappa_h, X1, ye, 0);
    bilinear_vectors(L, U, X1, ye, X, Y);
    or_fermion_force(L, U, a->kappa_h * a->kappa_h, X, Y, F);
    free(ye); free(X); free(Y);
    return status;
}

/* Force of the ratio monomial S_2 at U; X_2 = A^-1 chi left in X2 and chi
 * = Mhat_h^dag phi_2 in chi. */
static int ratio_force(const int *L, const cplx *U, const or_mts_action *a, const cplx *phi2, cplx *X2, cplx *chi,
                       cplx *F, or_mts_stats *ms)
{
    long V = vol4(L), n = V * 12;
    or_mhat(L, U, a->kappa_h, phi2, chi, 1);
    or_cg_stats st;
    int status = or_cg_mhat(L, U, a->kappa, chi, X2, a->tol, a->maxiter, 0, &st);
    ms->solves_ratio++;
    cplx *ye = malloc(sizeof(cplx) * n), *X = malloc(sizeof(cplx) * n), *Y = malloc(sizeof(cplx) * n);
    cplx *F2 = malloc(sizeof(cplx) * V * 36);
    or_mhat(L, U, a->kappa, X2, ye, 0);
    bilinear_vectors(L, U, X2, ye, X, Y);
    or_fermion_force(L, U, a->kappa * a->kappa, X, Y, F);
    bilinear_vectors(L, U, X2, phi2, X, Y);
    or_fermion_force(L, U, a->kappa_h * a->kappa_h, X, Y, F2);
    for (long k = 0; k < V * 36; ++k) F[k] -= F2[k];
    free(ye); free(X); free(Y); free(F2);
    return status;
}

/* Monomial force (level 0 ratio, 1 heavy, 2 gauge), exposed for the force
 * checks; returns the solver status. */
int or_mts_force(const int *L, const cplx *U, const or_mts_action *a, int level, const cplx *phi, cplx *X,
                 cplx *F)
{
    or_mts_stats ms;
    memset(&ms, 0, sizeof ms);
    long n = vol4(L) * 12;
    if (level == 2) {
        or_gauge_force(L, U, a->beta, F);
        return 0;
    }
    if (level == 1) return heavy_force(L, U, a, phi, X, F, &ms);
    cplx *chi = malloc(sizeof(cplx) * n);
    int s = ratio_force(L, U, a, phi, X, chi, F, &ms);
    free(chi);
    return s;
}

/* The nested leapfrog as a flat list of operations: kicks (level, coef)
 * and link updates (eps).  integrate(l, t): with e = t / n_l, a kick of
 * e/2, then n_l times [the next level over e (links by e at the innermost
 * level), a kick of e (e/2 after the last)].  Kicks between two link
 * updates act on the same links and are summed per level. */
typedef struct {
    int kind;  /* 0..2 kick of that level, 3 link update */
    double c;
} mts_op;

static void mts_emit(mts_op *ops, int *nops, int kind, double c)
{
    ops[*nops].kind = kind;
    ops[*nops].c = c;
    ++*nops;
}

static void mts_gen(const int *steps, int level, double t, mts_op *ops, int *nops)
{
    int n = steps[level];
    double e = t / n;
    mts_emit(ops, nops, level, 0.5 * e);
    for (int k = 1; k <= n; ++k) {
        if (level == 2)
            mts_emit(ops, nops, 3, e);
        else
            mts_gen(steps, level + 1, e, ops, nops);
        mts_emit(ops, nops, level, k < n ? e : 0.5 * e);
    }
}

/* Coalesced schedule: for each stretch between link updates one summed
 * coefficient per level (0 = not evaluated), then the update.  Returns the
 * number of stretches; coef[s*3 + l], eps[s] (eps of the update that ends
 * stretch s; 0 for the last). */
int or_mts_schedule(int n_ratio, int n_heavy, int n_gauge, double tau, double *coef, double *eps, int max_stretch)
{
    int steps[3] = {n_ratio, n_heavy, n_gauge};
    long cap = 4L * (2L * n_ratio + 2) * (2L * n_heavy + 2) * (2L * n_gauge + 2);
    mts_op *ops = malloc(sizeof(mts_op) * cap);
    int nops = 0;
    mts_gen(steps, 0, tau, ops, &nops);
    int s = 0;
    double pend[3] = {0, 0, 0};
    for (int k = 0; k < nops; ++k) {
        if (ops[k].kind < 3) {
            pend[ops[k].kind] += ops[k].c;
            continue;
        }
        if (s >= max_stretch) { free(ops); return -1; }
        for (int l = 0; l < 3; ++l) coef[s * 3 + l] = pend[l], pend[l] = 0;
        eps[s] = ops[k].c;
        ++s;
    }
    if (s >= max_stretch) { free(ops); return -1; }
    for (int l = 0; l < 3; ++l) coef[s * 3 + l] = pend[l];
    eps[s] = 0;
    free(ops);
    return s + 1;
}

/* Integrate over tau with the coalesced schedule; at each stretch the
 * forces are applied in the order ratio, heavy, gauge.  X1/X2/chi receive
 * the last solves. */
int or_mts_integrate(const int *L, cplx *U, cplx *P, const cplx *phi1, const cplx *phi2, const or_mts_action *a,
                     double tau, cplx *X1, cplx *X2, cplx *chi, or_mts_stats *ms)
{
    long V = vol4(L);
    int maxs = a->n_ratio * a->n_heavy * a->n_gauge + 1;
    double *coef = malloc(sizeof(double) * 3 * maxs), *eps = malloc(sizeof(double) * maxs);
    int ns = or_mts_schedule(a->n_ratio, a->n_heavy, a->n_gauge, tau, coef, eps, maxs);
    cplx *F = malloc(sizeof(cplx) * V * 36);
    int status = ns < 0 ? -1 : 0;
    for (int s = 0; s < ns; ++s) {
        if (coef[s * 3 + 0] != 0) {
            status |= ratio_force(L, U, a, phi2, X2, chi, F, ms);
            or_momentum_update(L, P, F, coef[s * 3 + 0]);
        }
        if (coef[s * 3 + 1] != 0) {
            status |= heavy_force(L, U, a, phi1, X1, F, ms);
            or_momentum_update(L, P, F, coef[s * 3 + 1]);
        }
        if (coef[s * 3 + 2] != 0) {
            or_gauge_force(L, U, a->beta, F);
            ms->gauge_forces++;
            or_momentum_update(L, P, F, coef[s * 3 + 2]);
        }
        if (eps[s] != 0) {
            or_update_links(L, U, P, eps[s]);
            ms->link_updates++;
        }
    }
    free(coef); free(eps); free(F);
    return status;
}

/* One mass-preconditioned HMC trajectory (momenta stream 1, eta_1 stream
 * 2, eta_2 stream 5, Metropolis stream 3, all at epoch traj). */
int or_hmc_trajectory_mts(const int *L, cplx *U, const or_mts_action *a, uint64_t seed, uint64_t traj, double tau,
                          or_traj_result *res, or_mts_stats *ms)
{
    long V = vol4(L), n = V * 12;
    cplx *U_old = malloc(sizeof(cplx) * V * 36), *P = malloc(sizeof(cplx) * V * 36);
    cplx *eta1 = malloc(sizeof(cplx) * n), *eta2 = malloc(sizeof(cplx) * n);
    cplx *phi1 = malloc(sizeof(cplx) * n), *phi2 = malloc(sizeof(cplx) * n), *t = malloc(sizeof(cplx) * n);
    cplx *X1 = malloc(sizeof(cplx) * n), *X2 = malloc(sizeof(cplx) * n), *chi = malloc(sizeof(cplx) * n);
    memset(ms, 0, sizeof *ms);
    memcpy(U_old, U, sizeof(cplx) * V * 36);
    or_refresh_momenta(L, seed, traj, P);
    or_eta(L, seed, traj, 0, eta1);
    or_eta2(L, seed, traj, 0, eta2);
    or_mhat(L, U, a->kappa_h, eta1, phi1, 1);
    /* phi_2 = Mhat_h A_h^-1 Mhat^dag eta_2 */
    or_mhat(L, U, a->kappa, eta2, t, 1);
    or_cg_stats st;
    int status = or_cg_mhat(L, U, a->kappa_h, t, X1, a->tol, a->maxiter, 0, &st);
    ms->solves_heavy++;
    or_mhat(L, U, a->kappa_h, X1, phi2, 0);

    res->KE_old = or_kinetic(L, P);
    res->S_g_old = or_gauge_action(L, U, a->beta);
    ms->S1_old = or_norm2(n, eta1);
    ms->S2_old = or_norm2(n, eta2);
    res->S_f_old = ms->S1_old + ms->S2_old;
    res->H_old = res->KE_old + res->S_g_old + res->S_f_old;

    status |= or_mts_integrate(L, U, P, phi1, phi2, a, tau, X1, X2, chi, ms);

    double ri[2];
    or_inner(n, phi1, X1, ri);
    ms->S1_new = ri[0];
    or_inner(n, chi, X2, ri);
    ms->S2_new = ri[0];
    res->KE_new = or_kinetic(L, P);
    res->S_g_new = or_gauge_action(L, U, a->beta);
    res->S_f_new = ms->S1_new + ms->S2_new;
    res->H_new = res->KE_new + res->S_g_new + res->S_f_new;
    res->dH = res->H_new - res->H_old;
    res->u = or_accept_uniform(seed, traj);
    res->accepted = metropolis_accept(status, res->dH, res->u);
    if (!res->accepted) memcpy(U, U_old, sizeof(cplx) * V * 36);
    res->plaquette = or_plaquette(L, U);
    res->cg_iters_total = 0;
    res->cg_iters_max = 0;
    res->nonconverged = status != 0;
    free(U_old); free(P); free(eta1); free(eta2); free(phi1); free(phi2); free(t);
    free(X1); free(X2); free(chi);
    return status;
}

/* S_2 at U for a given phi_2 (converged solve), for the force checks. */
double or_ratio_action(const int *L, const cplx *U, const or_mts_action *a, const cplx *phi2)
{
    long n = vol4(L) * 12;
    cplx *chi = malloc(sizeof(cplx) * n), *X = malloc(sizeof(cplx) * n);
    or_mhat(L, U, a->kappa_h, phi2, chi, 1);
    or_cg_stats st;
    or_cg_mhat(L, U, a->kappa, chi, X, a->tol, a->maxiter, 0, &st);
    double ri[2];
    or_inner(n, chi, X, ri);
    free(chi); free(X);
    return ri[0];
}

/* ------------------------------------------------------------------ */
/* Chronological initial guess (minimal-residual extrapolation).       */
/* ------------------------------------------------------------------ */
/* Brower, Ivanenko, Levi, Orginos, Nucl. Phys. B 484 (1997) 353: the
 * initial guess for A x = b is the Galerkin projection onto the span of the
 * last m solutions y_1..y_m, x0 = sum_k c_k y_k with
 *   sum_k <y_j, A y_k> c_k = <y_j, b>   (j = 1..m),
 * i.e. the x0 in the span with the smallest A-norm error.  G is Hermitian
 * positive definite for independent y; solved here by Gaussian elimination
 * with partial pivoting.  Returns 0, or -1 when G is singular (then x0 = 0). */
int or_chrono_guess(const int *L, const cplx *U, double kappa, const cplx *b, const cplx *Y, int m, cplx *x0)
{
    long n = vol4(L) * 12;
    cplx *AY = malloc(sizeof(cplx) * n * m), *tmp = malloc(sizeof(cplx) * n);
    cplx G[64], f[8];
    for (int k = 0; k < m; ++k) normal_op(L, U, kappa, &Y[k * n], &AY[k * n], tmp);
    for (int j = 0; j < m; ++j) {
        double ri[2];
        for (int k = 0; k < m; ++k) {
            or_inner(n, &Y[j * n], &AY[k * n], ri);
            G[j * m + k] = ri[0] + I * ri[1];
        }
        or_inner(n, &Y[j * n], b, ri);
        f[j] = ri[0] + I * ri[1];
    }
    int status = 0;
    /* forward elimination with partial pivoting */
    for (int c = 0; c < m && !status; ++c) {
        int piv = c;
        for (int r = c + 1; r < m; ++r)
            if (cabs(G[r * m + c]) > cabs(G[piv * m + c])) piv = r;
        if (cabs(G[piv * m + c]) == 0) { status = -1; break; }
        if (piv != c) {
            for (int k = 0; k < m; ++k) { cplx t = G[c * m + k]; G[c * m + k] = G[piv * m + k]; G[piv * m + k] = t; }
            cplx t = f[c]; f[c] = f[piv]; f[piv] = t;
        }
        for (int r = c + 1; r < m; ++r) {
            cplx l = G[r * m + c] / G[c * m + c];
            for (int k = c; k < m; ++k) G[r * m + k] -= l * G[c * m + k];
            f[r] -= l * f[c];
        }
    }
    cplx coef[8];
    for (int c = m - 1; c >= 0 && !status; --c) {
        cplx s = f[c];
        for (int k = c + 1; k < m; ++k) s -= G[c * m + k] * coef[k];
        coef[c] = s / G[c * m + c];
    }
    for (long i = 0; i < n; ++i) {
        cplx s = 0;
        if (!status)
            for (int k = 0; k < m; ++k) s += coef[k] * Y[k * n + i];
        x0[i] = s;
    }
    free(AY); free(tmp);
    return status;
}

/* Plain HMC trajectory whose force solves start from the chronological
 * guess over the last n_chrono solutions of the same trajectory (the
 * history is cleared at the start; n_chrono <= 8). */
static int force_kick_chrono(const int *L, const cplx *U, cplx *P, const cplx *phi, const or_action *a, double coef,
                             cplx *Xe, cplx *hist, int *nh, int n_chrono, or_md_stats *ms)
{
    long V = vol4(L), n = V * 12;
    cplx *F = malloc(sizeof(cplx) * V * 36);
    or_gauge_force(L, U, a->beta, F);
    or_momentum_update(L, P, F, coef);
    or_cg_stats st;
    int status;
    if (*nh > 0) {
        or_chrono_guess(L, U, a->kappa, phi, hist, *nh, Xe);
        status = or_cg_mhat_x0(L, U, a->kappa, phi, Xe, a->tol, a->maxiter, &st);
    } else {
        status = or_cg_mhat(L, U, a->kappa, phi, Xe, a->tol, a->maxiter, 0, &st);
    }
    ms->solves++;
    ms->iters_total += st.iters;
    if (st.iters > ms->iters_max) ms->iters_max = st.iters;
    if (status) ms->nonconverged++;
    /* push the solution, oldest dropped */
    if (*nh == n_chrono) {
        memmove(hist, hist + n, sizeof(cplx) * n * (n_chrono - 1));
        --*nh;
    }
    memcpy(hist + *nh * n, Xe, sizeof(cplx) * n);
    ++*nh;
    cplx *X = malloc(sizeof(cplx) * n), *Y = malloc(sizeof(cplx) * n);
    force_vectors(L, U, a->kappa, Xe, X, Y);
    or_fermion_force(L, U, a->kappa * a->kappa, X, Y, F);
    or_momentum_update(L, P, F, coef);
    free(X); free(Y); free(F);
    return status;
}

int or_hmc_trajectory_chrono(const int *L, cplx *U, const or_action *a, uint64_t seed, uint64_t traj, double tau,
                             int nsteps, int n_chrono, or_traj_result *res)
{
    long V = vol4(L), n = V * 12;
    if (n_chrono < 1 || n_chrono > 8) return -1;
    cplx *U_old = malloc(sizeof(cplx) * V * 36), *P = malloc(sizeof(cplx) * V * 36);
    cplx *eta = malloc(sizeof(cplx) * n), *phi = malloc(sizeof(cplx) * n), *Xe = malloc(sizeof(cplx) * n);
    cplx *hist = malloc(sizeof(cplx) * n * n_chrono);
    int nh = 0;
    memcpy(U_old, U, sizeof(cplx) * V * 36);
    or_refresh_momenta(L, seed, traj, P);
    or_eta(L, seed, traj, 0, eta);
    or_mhat(L, U, a->kappa, eta, phi, 1);
    res->KE_old = or_kinetic(L, P);
    res->S_g_old = or_gauge_action(L, U, a->beta);
    res->S_f_old = or_norm2(n, eta);
    res->H_old = res->KE_old + res->S_g_old + res->S_f_old;

    or_md_stats ms;
    memset(&ms, 0, sizeof ms);
    double eps = tau / nsteps;
    int status = force_kick_chrono(L, U, P, phi, a, 0.5 * eps, Xe, hist, &nh, n_chrono, &ms);
    for (int k = 1; k <= nsteps; ++k) {
        or_update_links(L, U, P, eps);
        status |= force_kick_chrono(L, U, P, phi, a, k < nsteps ? eps : 0.5 * eps, Xe, hist, &nh, n_chrono, &ms);
    }

    double ri[2];
    or_inner(n, phi, Xe, ri);
    res->KE_new = or_kinetic(L, P);
    res->S_g_new = or_gauge_action(L, U, a->beta);
    res->S_f_new = ri[0];
    res->H_new = res->KE_new + res->S_g_new + res->S_f_new;
    res->dH = res->H_new - res->H_old;
    res->u = or_accept_uniform(seed, traj);
    res->accepted = metropolis_accept(status, res->dH, res->u);
    if (!res->accepted) memcpy(U, U_old, sizeof(cplx) * V * 36);
    res->plaquette = or_plaquette(L, U);
    res->cg_iters_total = ms.iters_total;
    res->cg_iters_max = ms.iters_max;
    res->nonconverged = ms.nonconverged;
    free(U_old); free(P); free(eta); free(phi); free(Xe); free(hist);
    return status;
}
