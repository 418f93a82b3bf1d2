/*
 * clgc_oracle.c -- plain, slow FP64 CPU oracle for complex Langevin (CL)
 * dynamics of SU(3) lattice gauge theory with a theta term, plus adaptive
 * SL(3,C) gauge cooling (Bongiovanni, Aarts, Seiler, Sexty, Stamatescu,
 * "Adaptive gauge cooling for complex Langevin dynamics", LATTICE 2013).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker for the HIP library:
 * only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code with the GPU path (no common headers,
 * helpers or tables); the two agree only on the documented conventions:
 *
 *   host link layout  links[((s*4 + mu)*9 + 3*i + j)*2 + {0: re, 1: im}],
 *                     s = x0 + L0*(x1 + L1*(x2 + L2*x3))  (x0 fastest);
 *   inverse           U^{-1} := adj(U) (exact for det U = 1);
 *   generators        standard Gell-Mann lambda_a, Tr(lambda_a lambda_b) = 2 delta_ab;
 *   noise             Philox4x32-10 (Salmon et al., SC'11), counter
 *                     (4*s+mu, step, draw, tag), key (seed lo, seed hi).
 *
 * Everything is written for clarity, not speed: matrices are 3x3 arrays of
 * C99 double complex, every matrix exponential is a Taylor series with
 * scaling and squaring, loops run over lexicographic sites, and every
 * global sum is taken serially in site order after a parallel map.
 *
 * Parity pins (what fixes each function other than itself) live in
 * tests/test_oracle_*.py; each function below names its passage.
 * Parity unpinned: none of these functions.  What no pin fixes is the
 * absolute physics value of <P> and <Q> at given (beta, theta), which the
 * paper's figures do not give in recoverable form.
 */
#include "clgc_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef double complex cplx;
typedef struct { cplx a[3][3]; } M3;

/* ------------------------------------------------------------------ */
/* 3x3 complex matrix algebra                                          */
/* ------------------------------------------------------------------ */

static M3 m_zero(void) { M3 r; memset(&r, 0, sizeof r); return r; }

static M3 m_id(void)
{
    M3 r = m_zero();
    r.a[0][0] = r.a[1][1] = r.a[2][2] = 1.0;
    return r;
}

static M3 m_mul(M3 x, M3 y)
{
    M3 r = m_zero();
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
                r.a[i][j] += x.a[i][k] * y.a[k][j];
    return r;
}

static M3 m_add(M3 x, M3 y)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) x.a[i][j] += y.a[i][j];
    return x;
}

static M3 m_sub(M3 x, M3 y)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) x.a[i][j] -= y.a[i][j];
    return x;
}

static M3 m_scale(M3 x, cplx c)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) x.a[i][j] *= c;
    return x;
}

/* Hermitian conjugate U^dagger. */
static M3 m_dag(M3 x)
{
    M3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r.a[i][j] = conj(x.a[j][i]);
    return r;
}

static cplx m_tr(M3 x) { return x.a[0][0] + x.a[1][1] + x.a[2][2]; }

static cplx m_det(M3 x)
{
    return x.a[0][0] * (x.a[1][1] * x.a[2][2] - x.a[1][2] * x.a[2][1])
         - x.a[0][1] * (x.a[1][0] * x.a[2][2] - x.a[1][2] * x.a[2][0])
         + x.a[0][2] * (x.a[1][0] * x.a[2][1] - x.a[1][1] * x.a[2][0]);
}

/* Adjugate (transposed cofactor matrix): x * adj(x) = det(x) * 1.  For
 * links in SL(3,C) this is the group inverse. */
static M3 m_inv(M3 x)
{
    M3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            /* cofactor C_ji goes to r[i][j] */
            int r0 = (j + 1) % 3, r1 = (j + 2) % 3;
            int c0 = (i + 1) % 3, c1 = (i + 2) % 3;
            r.a[i][j] = x.a[r0][c0] * x.a[r1][c1] - x.a[r0][c1] * x.a[r1][c0];
        }
    return r;
}

/* Traceless part TL(M) = M - (1/3) Tr M. */
static M3 m_tl(M3 x)
{
    cplx t = m_tr(x) / 3.0;
    for (int i = 0; i < 3; ++i) x.a[i][i] -= t;
    return x;
}

static double m_norm1(M3 x)
{
    double best = 0.0;
    for (int j = 0; j < 3; ++j) {
        double c = 0.0;
        for (int i = 0; i < 3; ++i) c += cabs(x.a[i][j]);
        if (c > best) best = c;
    }
    return best;
}

static double m_maxabs(M3 x)
{
    double m = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            if (cabs(x.a[i][j]) > m) m = cabs(x.a[i][j]);
    return m;
}

/* Matrix exponential by its Taylor series, after scaling A by 2^-k so that
 * ||A||_1 <= 1/2, followed by k squarings.  The series is summed until a
 * term no longer changes the sum. */
static M3 m_exp(M3 A)
{
    int k = 0;
    double nrm = m_norm1(A);
    /* bounded: a finite double needs at most ~1025 halvings, and an infinite
     * norm (a runaway) must not loop forever; its result is non-finite anyway */
    while (nrm > 0.5 && k < 1100) { nrm *= 0.5; ++k; }
    A = m_scale(A, ldexp(1.0, -k));
    M3 sum = m_id(), term = m_id();
    for (int n = 1; n < 60; ++n) {
        term = m_scale(m_mul(term, A), 1.0 / n);
        sum = m_add(sum, term);
        if (m_maxabs(term) <= 1e-19 * m_maxabs(sum)) break;
    }
    for (int i = 0; i < k; ++i) sum = m_mul(sum, sum);
    return sum;
}

/* ------------------------------------------------------------------ */
/* Gell-Mann matrices lambda_1..lambda_8 (index a = 0..7 here)         */
/* ------------------------------------------------------------------ */

static M3 gell_mann(int a)
{
    M3 r = m_zero();
    switch (a) {
    case 0: r.a[0][1] = 1; r.a[1][0] = 1; break;
    case 1: r.a[0][1] = -I; r.a[1][0] = I; break;
    case 2: r.a[0][0] = 1; r.a[1][1] = -1; break;
    case 3: r.a[0][2] = 1; r.a[2][0] = 1; break;
    case 4: r.a[0][2] = -I; r.a[2][0] = I; break;
    case 5: r.a[1][2] = 1; r.a[2][1] = 1; break;
    case 6: r.a[1][2] = -I; r.a[2][1] = I; break;
    case 7:
        r.a[0][0] = 1.0 / sqrt(3.0); r.a[1][1] = 1.0 / sqrt(3.0);
        r.a[2][2] = -2.0 / sqrt(3.0);
        break;
    }
    return r;
}

/* sum_a c_a lambda_a for complex coefficients c_a */
static M3 lie_combination(const cplx c[8])
{
    M3 r = m_zero();
    for (int a = 0; a < 8; ++a) r = m_add(r, m_scale(gell_mann(a), c[a]));
    return r;
}

/* ------------------------------------------------------------------ */
/* Lattice geometry                                                    */
/* ------------------------------------------------------------------ */

typedef struct { int L[4]; long V; } Geom;

static Geom geom(const int *dims)
{
    Geom g;
    g.V = 1;
    for (int m = 0; m < 4; ++m) { g.L[m] = dims[m]; g.V *= dims[m]; }
    return g;
}

static void coords(const Geom *g, long s, int x[4])
{
    for (int m = 0; m < 4; ++m) { x[m] = (int)(s % g->L[m]); s /= g->L[m]; }
}

static long site_of(const Geom *g, const int x[4])
{
    long s = 0;
    for (int m = 3; m >= 0; --m) s = s * g->L[m] + ((x[m] % g->L[m]) + g->L[m]) % g->L[m];
    return s;
}

/* the site one lattice spacing away from s in direction mu (d = +1 or -1) */
static long shift(const Geom *g, long s, int mu, int d)
{
    int x[4];
    coords(g, s, x);
    x[mu] += d;
    return site_of(g, x);
}

static int parity_of(const Geom *g, long s)
{
    int x[4];
    coords(g, s, x);
    return (x[0] + x[1] + x[2] + x[3]) & 1;
}

static M3 get_link(const double *links, long s, int mu)
{
    M3 r;
    const double *p = links + (s * 4 + mu) * 18;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r.a[i][j] = p[2 * (3 * i + j)] + I * p[2 * (3 * i + j) + 1];
    return r;
}

static void set_link(double *links, long s, int mu, M3 u)
{
    double *p = links + (s * 4 + mu) * 18;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            p[2 * (3 * i + j)] = creal(u.a[i][j]);
            p[2 * (3 * i + j) + 1] = cimag(u.a[i][j]);
        }
}

static M3 get_mat(const double *p)
{
    M3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r.a[i][j] = p[2 * (3 * i + j)] + I * p[2 * (3 * i + j) + 1];
    return r;
}

static void put_mat(double *p, M3 u)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            p[2 * (3 * i + j)] = creal(u.a[i][j]);
            p[2 * (3 * i + j) + 1] = cimag(u.a[i][j]);
        }
}

/* One hop of a lattice path: starting at *s, move in signed direction
 * dir (+(mu+1) forward, -(mu+1) backward).  Forward hops multiply by
 * U_mu(s); backward hops move to s - mu and multiply by U_mu(s - mu)^{-1}
 * (holomorphic continuation: inverse, never dagger). */
static M3 hop(const Geom *g, const double *links, long *s, int dir)
{
    int mu = abs(dir) - 1;
    if (dir > 0) {
        M3 u = get_link(links, *s, mu);
        *s = shift(g, *s, mu, +1);
        return u;
    }
    *s = shift(g, *s, mu, -1);
    return m_inv(get_link(links, *s, mu));
}

/* Ordered product of links along a closed or open path of n signed hops. */
static M3 path(const Geom *g, const double *links, long s, const int *dirs, int n)
{
    M3 r = m_id();
    for (int k = 0; k < n; ++k) r = m_mul(r, hop(g, links, &s, dirs[k]));
    return r;
}

/* Plaquette U_{mu nu}(x) for signed directions mu, nu (1-based signs as in
 * the theta-term density): x -> x+mu -> x+mu+nu -> x+nu -> x. */
static M3 plaquette_signed(const Geom *g, const double *links, long s, int smu, int snu)
{
    int dirs[4] = {smu, snu, -smu, -snu};
    return path(g, links, s, dirs, 4);
}

/* ------------------------------------------------------------------ */
/* Philox4x32-10 and Gaussian draws                                    */
/* ------------------------------------------------------------------ */

/* Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw ("Parallel
 * random numbers: as easy as 1, 2, 3", SC'11): ten rounds of the 4x32
 * S-box with multipliers 0xD2511F53 and 0xCD9E8D57, the key bumped by the
 * Weyl constants 0x9E3779B9 and 0xBB67AE85 between rounds. */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0;
        uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
    memcpy(out, c, sizeof c);
}

/* Two standard normals from one Philox call: two 53-bit uniforms in (0,1)
 * from word pairs (w0,w1) and (w2,w3), then the Box-Muller transform. */
void orc_normal_pair(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                     double out[2])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    double uA = ((double)(w[0] >> 5) * 67108864.0 + (double)(w[1] >> 6) + 0.5) / 9007199254740992.0;
    double uB = ((double)(w[2] >> 5) * 67108864.0 + (double)(w[3] >> 6) + 0.5) / 9007199254740992.0;
    double r = sqrt(-2.0 * log(uA));
    out[0] = r * cos(2.0 * M_PI * uB);
    out[1] = r * sin(2.0 * M_PI * uB);
}

/* Langevin noise eta_1..eta_8 for link (s, mu) at CL step n, with
 * <eta_a eta_b> = 2 delta_ab: draws j = 0..3 of stream tag 0. */
void orc_cl_noise(uint64_t seed, long s, int mu, uint32_t step, double eta[8])
{
    for (int j = 0; j < 4; ++j) {
        double n[2];
        orc_normal_pair(seed, (uint32_t)(4 * s + mu), step, (uint32_t)j, 0u, n);
        eta[2 * j] = sqrt(2.0) * n[0];
        eta[2 * j + 1] = sqrt(2.0) * n[1];
    }
}

/* ------------------------------------------------------------------ */
/* Initial configurations                                              */
/* ------------------------------------------------------------------ */

void orc_cold_links(const int *dims, double *links)
{
    Geom g = geom(dims);
    for (long s = 0; s < g.V; ++s)
        for (int mu = 0; mu < 4; ++mu) set_link(links, s, mu, m_id());
}

/* Perturbed SL(3,C) start U = exp(i lambda_a (x_a + i y_a)), with
 * x_a ~ N(0, sigma_x^2), y_a ~ N(0, sigma_y^2) from Philox stream tag 1:
 * draws j = 0..3 give x_1..x_8, draws j = 4..7 give y_1..y_8. */
void orc_init_links(const int *dims, uint64_t seed, double sigma_x, double sigma_y, double *links)
{
    Geom g = geom(dims);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < g.V; ++s)
        for (int mu = 0; mu < 4; ++mu) {
            double xr[8], yr[8];
            for (int j = 0; j < 8; ++j) {
                double n[2];
                orc_normal_pair(seed, (uint32_t)(4 * s + mu), 0u, (uint32_t)j, 1u, n);
                double *dst = j < 4 ? xr : yr;
                int a = 2 * (j & 3);
                double sig = j < 4 ? sigma_x : sigma_y;
                dst[a] = sig * n[0];
                dst[a + 1] = sig * n[1];
            }
            cplx c[8];
            for (int a = 0; a < 8; ++a) c[a] = xr[a] + I * yr[a];
            set_link(links, s, mu, m_exp(m_scale(lie_combination(c), I)));
        }
}

/* ------------------------------------------------------------------ */
/* Observables                                                         */
/* ------------------------------------------------------------------ */

/* Sum over sites and planes mu<nu of Tr U_{mu nu}(x) (complex). */
static cplx plaquette_trace_sum(const Geom *g, const double *links)
{
    cplx *per = malloc(sizeof(cplx) * g->V);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < g->V; ++s) {
        cplx t = 0;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu)
                t += m_tr(plaquette_signed(g, links, s, mu + 1, nu + 1));
        per[s] = t;
    }
    cplx sum = 0;
    for (long s = 0; s < g->V; ++s) sum += per[s];
    free(per);
    return sum;
}

/* Average plaquette P = (1/(18 V)) sum_x sum_{mu<nu} Tr U_{mu nu}(x); P = 1
 * on a cold start. */
void orc_plaquette(const int *dims, const double *links, double out[2])
{
    Geom g = geom(dims);
    cplx p = plaquette_trace_sum(&g, links) / (18.0 * g.V);
    out[0] = creal(p);
    out[1] = cimag(p);
}

/* Wilson action S_W = beta sum_x sum_{mu<nu} [1 - (1/6) Tr(U_{mu nu} + U_{mu nu}^{-1})]
 * (holomorphic in the links). */
void orc_wilson_action(const int *dims, const double *links, double beta, double out[2])
{
    Geom g = geom(dims);
    cplx *per = malloc(sizeof(cplx) * g.V);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < g.V; ++s) {
        cplx t = 0;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                M3 p = plaquette_signed(&g, links, s, mu + 1, nu + 1);
                t += 1.0 - (m_tr(p) + m_tr(m_inv(p))) / 6.0;
            }
        per[s] = t;
    }
    cplx sum = 0;
    for (long s = 0; s < g.V; ++s) sum += per[s];
    free(per);
    out[0] = beta * creal(sum);
    out[1] = beta * cimag(sum);
}

static int plane_index(int mu, int nu)
{
    /* planes (0,1) (0,2) (0,3) (1,2) (1,3) (2,3) -> 0..5 */
    static const int tab[4][4] = {{-1, 0, 1, 2}, {0, -1, 3, 4}, {1, 3, -1, 5}, {2, 4, 5, -1}};
    return tab[mu][nu];
}

/* Clover field F_{mu nu}(x) = sum over the four counter-clockwise leaves L
 * at x in the (mu, nu) plane of (L - L^{-1}), mu < nu.  Grouping the
 * signed-index sum of the theta-term density by plane gives
 *   q_L(x) = -(1/(2^8 pi^2)) [Tr F01 F23 - Tr F02 F13 + Tr F03 F12]. */
static M3 clover(const Geom *g, const double *links, long s, int mu, int nu)
{
    int m = mu + 1, n = nu + 1;
    M3 leaves[4] = {
        plaquette_signed(g, links, s, m, n),
        plaquette_signed(g, links, s, n, -m),
        plaquette_signed(g, links, s, -m, -n),
        plaquette_signed(g, links, s, -n, m),
    };
    M3 f = m_zero();
    for (int k = 0; k < 4; ++k) f = m_add(f, m_sub(leaves[k], m_inv(leaves[k])));
    return f;
}

/* All six clover matrices of every site, indexed [s*6 + plane]. */
static M3 *clover_field(const Geom *g, const double *links)
{
    M3 *F = malloc(sizeof(M3) * 6 * g->V);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < g->V; ++s)
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu)
                F[s * 6 + plane_index(mu, nu)] = clover(g, links, s, mu, nu);
    return F;
}

/* Topological charge Q_L = sum_x q_L(x) (complex for SL(3,C) links). */
void orc_topological_charge(const int *dims, const double *links, double out[2])
{
    Geom g = geom(dims);
    M3 *F = clover_field(&g, links);
    cplx sum = 0;
    const double c = -1.0 / (256.0 * M_PI * M_PI);
    for (long s = 0; s < g.V; ++s) {
        const M3 *f = F + s * 6;
        cplx t = m_tr(m_mul(f[0], f[5])) - m_tr(m_mul(f[1], f[4])) + m_tr(m_mul(f[2], f[3]));
        sum += c * t;
    }
    free(F);
    out[0] = creal(sum);
    out[1] = cimag(sum);
}

/* Sum over all links of Tr U U^dagger (the unitarity norm, UN). */
double orc_unitarity_norm(const int *dims, const double *links)
{
    Geom g = geom(dims);
    double *per = malloc(sizeof(double) * g.V);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < g.V; ++s) {
        double t = 0;
        for (int mu = 0; mu < 4; ++mu)
            t += creal(m_tr(m_mul(get_link(links, s, mu), m_dag(get_link(links, s, mu)))));
        per[s] = t;
    }
    double sum = 0;
    for (long s = 0; s < g.V; ++s) sum += per[s];
    free(per);
    return sum;
}

/* ------------------------------------------------------------------ */
/* Drift                                                               */
/* ------------------------------------------------------------------ */

/* Dual clover matrix Ft_{mu nu} = (1/2) eps_{mu nu rho sigma} F_{rho sigma}
 * for mu < nu: Ft01 = F23, Ft02 = -F13, Ft03 = F12, Ft12 = F03,
 * Ft13 = -F02, Ft23 = F01, so that sum_P Tr(F_P Ft_P) is twice the bracket
 * of the clover form of q_L. */
static M3 dual_clover(const Geom *g, const double *links, const M3 *F, long s, int mu, int nu)
{
    int a = mu < nu ? mu : nu, b = mu < nu ? nu : mu;
    int p = plane_index(a, b);
    static const int partner[6] = {5, 4, 3, 2, 1, 0};
    static const int pa[6] = {0, 0, 0, 1, 1, 2}, pb[6] = {1, 2, 3, 2, 3, 3};
    static const double sgn[6] = {+1, -1, +1, +1, -1, +1};
    int q = partner[p];
    /* from the precomputed field, or evaluated at this site when F is NULL */
    M3 f = F ? F[s * 6 + q] : clover(g, links, s, pa[q], pb[q]);
    return m_scale(f, sgn[p]);
}

/* Drift Khat = sum_a K_a lambda_a of link (s, mu), K_a = -D_a S,
 * D_a f(U) = d/dt f(exp(i t lambda_a) U) at t = 0, for S = S_W - i theta Q_L.
 *
 * Each of the six plaquettes through the link is the loop
 *   Gamma = e0 e1 e2 e3,  corners d0 = x, d1 = x+mu, d2 = x+mu+s nu, d3 = x+s nu,
 * hops (+mu, +s nu, -mu, -s nu).  Wilson part:
 *   Khat_W = (i beta / 3) TL( sum_loops (Gamma - Gamma^{-1}) ).
 * Theta part: with X_k the dual clover of the loop's plane at corner d_k and
 * sigma = s * sign(nu - mu) (+1 when the loop is counter-clockwise in its
 * plane),
 *   Khat_theta = theta/(2^7 pi^2) TL( sum_loops sigma sum_k (Lam_k + Lam'_k) ),
 *   Lam_0 = e0 e1 e2 e3 X0,  Lam_1 = e0 X1 e1 e2 e3,
 *   Lam_2 = e0 e1 X2 e2 e3,  Lam_3 = e0 e1 e2 X3 e3,
 *   Lam'_0 = X0 e3' e2' e1' e0',  Lam'_1 = e3' e2' e1' X1 e0',
 *   Lam'_2 = e3' e2' X2 e1' e0',  Lam'_3 = e3' X3 e2' e1' e0'   (e' = e^{-1}).
 * The derivation (D_a inserts i lambda_a left of e0, and -i lambda_a right
 * of e0^{-1}, in every clover leaf that contains the link) is checked
 * against central finite differences of S_W and Q_L in the tests. */
static M3 link_drift(const Geom *g, const double *links, const M3 *F, long s, int mu,
                     double beta, cplx theta, int with_theta)
{
    M3 wil = m_zero(), top = m_zero();
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        for (int sg = -1; sg <= 1; sg += 2) {
            int dirs[4] = {mu + 1, sg * (nu + 1), -(mu + 1), -sg * (nu + 1)};
            long d[4];
            M3 e[4];
            long cur = s;
            for (int k = 0; k < 4; ++k) { d[k] = cur; e[k] = hop(g, links, &cur, dirs[k]); }
            M3 gam = m_mul(m_mul(e[0], e[1]), m_mul(e[2], e[3]));
            wil = m_add(wil, m_sub(gam, m_inv(gam)));
            if (with_theta) {
                double sigma = sg * (nu > mu ? 1.0 : -1.0);
                M3 ei[4];
                for (int k = 0; k < 4; ++k) ei[k] = m_inv(e[k]);
                M3 X[4];
                for (int k = 0; k < 4; ++k) X[k] = dual_clover(g, links, F, d[k], mu, nu);
                M3 acc = m_zero();
                /* Lam_k: X_k inserted at corner d_k of e0 e1 e2 e3 */
                acc = m_add(acc, m_mul(gam, X[0]));
                acc = m_add(acc, m_mul(m_mul(e[0], X[1]), m_mul(m_mul(e[1], e[2]), e[3])));
                acc = m_add(acc, m_mul(m_mul(m_mul(e[0], e[1]), X[2]), m_mul(e[2], e[3])));
                acc = m_add(acc, m_mul(m_mul(m_mul(e[0], e[1]), m_mul(e[2], X[3])), e[3]));
                /* Lam'_k: X_k inserted at corner d_k of e3' e2' e1' e0' */
                acc = m_add(acc, m_mul(m_mul(X[0], ei[3]), m_mul(m_mul(ei[2], ei[1]), ei[0])));
                acc = m_add(acc, m_mul(m_mul(m_mul(ei[3], ei[2]), m_mul(ei[1], X[1])), ei[0]));
                acc = m_add(acc, m_mul(m_mul(m_mul(ei[3], ei[2]), X[2]), m_mul(ei[1], ei[0])));
                acc = m_add(acc, m_mul(m_mul(ei[3], X[3]), m_mul(m_mul(ei[2], ei[1]), ei[0])));
                top = m_add(top, m_scale(acc, sigma));
            }
        }
    }
    M3 K = m_scale(m_tl(wil), I * beta / 3.0);
    if (with_theta) K = m_add(K, m_scale(m_tl(top), theta / (128.0 * M_PI * M_PI)));
    return K;
}

/* Drift of every link, written in the host link layout (4V matrices). */
void orc_drift(const int *dims, const double *links, double beta, double theta_re,
               double theta_im, double *K)
{
    Geom g = geom(dims);
    cplx theta = theta_re + I * theta_im;
    M3 *F = (theta_re != 0.0 || theta_im != 0.0) ? clover_field(&g, links) : NULL;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < g.V; ++s)
        for (int mu = 0; mu < 4; ++mu)
            set_link(K, s, mu, link_drift(&g, links, F, s, mu, beta, theta, F != NULL));
    free(F);
}

/* Drift of selected links only (for sampled checks on large lattices); the
 * clover matrices are evaluated where the selected links need them. */
void orc_drift_links(const int *dims, const double *links, double beta, double theta_re,
                     double theta_im, const long *sel, long nsel, double *K)
{
    Geom g = geom(dims);
    cplx theta = theta_re + I * theta_im;
    int with_theta = theta_re != 0.0 || theta_im != 0.0;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < nsel; ++i)
        put_mat(K + 18 * i, link_drift(&g, links, NULL, sel[i] / 4, (int)(sel[i] % 4), beta, theta,
                                       with_theta));
}

/* ||Khat||^2 = (1/2) Tr(Khat Khat^dagger) = sum_a |K_a|^2. */
static double drift_norm2(M3 K)
{
    return 0.5 * creal(m_tr(m_mul(K, m_dag(K))));
}

/* ------------------------------------------------------------------ */
/* Langevin update                                                     */
/* ------------------------------------------------------------------ */

/* U <- exp(i (eps Khat + sqrt(eps) eta_hat)) U, eta_hat = sum_a eta_a lambda_a,
 * then U <- U det(U)^{-1/3} (principal branch) to stay on SL(3,C).  All
 * links are updated from the same drift (Jacobi order). */
void orc_langevin_update(const int *dims, double *links, const double *K, double eps,
                         uint64_t seed, uint32_t step)
{
    Geom g = geom(dims);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < g.V; ++s)
        for (int mu = 0; mu < 4; ++mu) {
            double eta[8];
            orc_cl_noise(seed, s, mu, step, eta);
            cplx c[8];
            for (int a = 0; a < 8; ++a) c[a] = sqrt(eps) * eta[a];
            M3 X = m_add(m_scale(get_link(K, s, mu), eps), lie_combination(c));
            M3 U = m_mul(m_exp(m_scale(X, I)), get_link(links, s, mu));
            cplx w = cpow(m_det(U), -1.0 / 3.0);
            set_link(links, s, mu, m_scale(U, w));
        }
}

/* One CL step: drift, step size, update.  Adaptive step size (absent from
 * the paper; a common CL control): eps_n = min(eps0, B / Kmax_n) with
 * Kmax_n = max over links of ||Khat||; B = eps0 * Kmax_0 is fixed on the
 * first adaptive step unless a positive drift_bound is given.  *bound
 * holds B between calls (<= 0: not yet set).  out = {eps_n, Kmax_n}. */
int orc_langevin_step(const int *dims, double *links, double beta, double theta_re,
                      double theta_im, uint64_t seed, uint32_t step, double eps0,
                      int adaptive, double drift_bound, double *bound, double out[2])
{
    Geom g = geom(dims);
    double *K = malloc(sizeof(double) * 72 * g.V);
    if (!K) return -2;
    orc_drift(dims, links, beta, theta_re, theta_im, K);
    double kmax2 = 0.0;
    for (long l = 0; l < 4 * g.V; ++l) {
        double n2 = drift_norm2(get_mat(K + 18 * l));
        if (n2 > kmax2) kmax2 = n2;
    }
    double kmax = sqrt(kmax2);
    double eps = eps0;
    if (adaptive) {
        if (*bound <= 0.0) *bound = drift_bound > 0.0 ? drift_bound : eps0 * kmax;
        if (kmax > 0.0 && *bound / kmax < eps0) eps = *bound / kmax;
    }
    orc_langevin_update(dims, links, K, eps, seed, step);
    free(K);
    out[0] = eps;
    out[1] = kmax;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Gauge cooling                                                       */
/* ------------------------------------------------------------------ */

/* Cooling gradient at site x: f_ax = 2 Tr[lambda_a sum_mu (U_{x,mu} U_{x,mu}^dagger
 * - U_{x-mu,mu}^dagger U_{x-mu,mu})]; returns the eight real f_a. */
static void cool_gradient(const Geom *g, const double *links, long s, double f[8])
{
    M3 G = m_zero();
    for (int mu = 0; mu < 4; ++mu) {
        M3 uf = get_link(links, s, mu);
        M3 ub = get_link(links, shift(g, s, mu, -1), mu);
        G = m_add(G, m_sub(m_mul(uf, m_dag(uf)), m_mul(m_dag(ub), ub)));
    }
    for (int a = 0; a < 8; ++a) f[a] = creal(2.0 * m_tr(m_mul(gell_mann(a), G)));
}

void orc_cool_gradient(const int *dims, const double *links, long s, double f[8])
{
    Geom g = geom(dims);
    cool_gradient(&g, links, s, f);
}

/* Gauge transformation at site x: U_{x,mu} -> Omega U_{x,mu},
 * U_{x-mu,mu} -> U_{x-mu,mu} Omega^{-1}. */
static void transform_site(const Geom *g, double *links, long s, M3 om, M3 om_inv)
{
    for (int mu = 0; mu < 4; ++mu) {
        set_link(links, s, mu, m_mul(om, get_link(links, s, mu)));
        long b = shift(g, s, mu, -1);
        set_link(links, b, mu, m_mul(get_link(links, b, mu), om_inv));
    }
}

/* One cooling half-sweep over the sites of one parity: at each such site,
 * Omega_x = exp(-eps alpha f_ax lambda_a), applied as above.  Sites of one
 * parity touch disjoint sets of links (even extents), so their order does
 * not matter; every link is written exactly once. */
void orc_cool_halfsweep(const int *dims, double *links, int parity, double eps_alpha)
{
    Geom g = geom(dims);
    for (long s = 0; s < g.V; ++s) {
        if (parity_of(&g, s) != parity) continue;
        double f[8];
        cool_gradient(&g, links, s, f);
        cplx c[8];
        for (int a = 0; a < 8; ++a) c[a] = -eps_alpha * f[a];
        M3 A = lie_combination(c);
        transform_site(&g, links, s, m_exp(A), m_exp(m_scale(A, -1.0)));
    }
}

/* n_steps cooling steps (even half-sweep, then odd), each with
 * alpha_ad = alpha / D:  D_0 = 1 (mode 0),  D_1 = Tr UU^dagger averaged over
 * links, UN/(4V), on the configuration entering the step (mode 1),
 * D_2 = mean over (a, x) of |f_ax| on that configuration (mode 2).
 * unorm[i] receives UN entering step i, unorm[n_steps] UN after the last;
 * alpha_used[i] (if not NULL) the alpha_ad of step i. */
int orc_gauge_cool(const int *dims, double *links, int n_steps, double eps_c, double alpha,
                   int mode, double *unorm, double *alpha_used)
{
    Geom g = geom(dims);
    for (int m = 0; m < 4; ++m)
        if (g.L[m] < 2 || (g.L[m] & 1)) return -1;
    for (int it = 0; it < n_steps; ++it) {
        double un = orc_unitarity_norm(dims, links);
        if (unorm) unorm[it] = un;
        double D = 1.0;
        if (mode == 1) {
            D = un / (4.0 * g.V);
        } else if (mode == 2) {
            double *per = malloc(sizeof(double) * g.V);
#pragma omp parallel for schedule(static)
            for (long s = 0; s < g.V; ++s) {
                double f[8], t = 0;
                cool_gradient(&g, links, s, f);
                for (int a = 0; a < 8; ++a) t += fabs(f[a]);
                per[s] = t;
            }
            double sum = 0;
            for (long s = 0; s < g.V; ++s) sum += per[s];
            free(per);
            D = sum / (8.0 * g.V);
        }
        double a_ad = alpha / D;
        if (alpha_used) alpha_used[it] = a_ad;
        if (!(D > 0.0) || !isfinite(a_ad)) return -4;
        orc_cool_halfsweep(dims, links, 0, eps_c * a_ad);
        orc_cool_halfsweep(dims, links, 1, eps_c * a_ad);
    }
    if (unorm) unorm[n_steps] = orc_unitarity_norm(dims, links);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Utilities for tests                                                 */
/* ------------------------------------------------------------------ */

/* Apply an arbitrary gauge transformation Omega_x (V matrices, row-major
 * interleaved complex, assumed invertible) to every site at once:
 * U_mu(x) -> Omega_x U_mu(x) Omega_{x+mu}^{-1}. */
void orc_gauge_transform(const int *dims, double *links, const double *omega)
{
    Geom g = geom(dims);
    double *out = malloc(sizeof(double) * 72 * g.V);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < g.V; ++s)
        for (int mu = 0; mu < 4; ++mu) {
            M3 om = get_mat(omega + 18 * s);
            M3 omn = m_inv(get_mat(omega + 18 * shift(&g, s, mu, +1)));
            set_link(out, s, mu, m_mul(m_mul(om, get_link(links, s, mu)), omn));
        }
    memcpy(links, out, sizeof(double) * 72 * g.V);
    free(out);
}

/* exp of one 3x3 complex matrix (18 doubles in, 18 out). */
void orc_expm(const double *A, double *out)
{
    put_mat(out, m_exp(get_mat(A)));
}

/* Product of the links along a path of signed hops from site s. */
void orc_path(const int *dims, const double *links, long s, const int *dirs, int n, double *out)
{
    Geom g = geom(dims);
    put_mat(out, path(&g, links, s, dirs, n));
}

/* Per-link checks: max |det U - 1| and min (1/3) Tr U U^dagger. */
void orc_link_stats(const int *dims, const double *links, double out[2])
{
    Geom g = geom(dims);
    double dmax = 0, tmin = 1e300;
    for (long l = 0; l < 4 * g.V; ++l) {
        M3 u = get_mat(links + 18 * l);
        double dd = cabs(m_det(u) - 1.0);
        double t = creal(m_tr(m_mul(u, m_dag(u)))) / 3.0;
        if (dd > dmax) dmax = dd;
        if (t < tmin) tmin = t;
    }
    out[0] = dmax;
    out[1] = tmin;
}

/* ------------------------------------------------------------------ */
/* Whole runs                                                          */
/* ------------------------------------------------------------------ */

/* A run: n_steps CL steps, each followed by n_cool cooling steps, then the
 * observables (measured after cooling).  Per step i, obs[i*8 + ...] =
 * {d before cooling, d after cooling, Re P, Im P, Re Q, Im Q, eps_n, Kmax_n}.
 * links holds the starting configuration on entry and the final one on exit;
 * step0 is the Philox step index of the first step, *bound the adaptive
 * step-size bound (<= 0: fix it on the first step). */
int orc_run(const int *dims, double *links, double beta, double theta_re, double theta_im,
            uint64_t seed, uint32_t step0, int n_steps, double eps0, int adaptive,
            double drift_bound, double *bound, int n_cool, double eps_c, double alpha,
            int mode, double *obs)
{
    Geom g = geom(dims);
    double *un = malloc(sizeof(double) * (n_cool + 1));
    for (int i = 0; i < n_steps; ++i) {
        double eo[2];
        int rc = orc_langevin_step(dims, links, beta, theta_re, theta_im, seed, step0 + i, eps0,
                                   adaptive, drift_bound, bound, eo);
        if (rc) { free(un); return rc; }
        double d_pre = orc_unitarity_norm(dims, links) / (12.0 * g.V) - 1.0;
        rc = orc_gauge_cool(dims, links, n_cool, eps_c, alpha, mode, un, NULL);
        if (rc) { free(un); return rc; }
        double d_post = un[n_cool] / (12.0 * g.V) - 1.0;
        double p[2], q[2];
        orc_plaquette(dims, links, p);
        orc_topological_charge(dims, links, q);
        double *o = obs + 8 * i;
        o[0] = d_pre; o[1] = d_post; o[2] = p[0]; o[3] = p[1]; o[4] = q[0]; o[5] = q[1];
        o[6] = eo[0]; o[7] = eo[1];
    }
    free(un);
    return 0;
}

/* Langevin noise of every link at step n, as (V, 4, 8) doubles. */
void orc_cl_noise_field(const int *dims, uint64_t seed, uint32_t step, double *eta)
{
    Geom g = geom(dims);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < g.V; ++s)
        for (int mu = 0; mu < 4; ++mu) orc_cl_noise(seed, s, mu, step, eta + (s * 4 + mu) * 8);
}

/* Thread count of the OpenMP loops (timing of the oracle only; results do not
 * depend on it: every reduction runs serially in a fixed order). */
int orc_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}
