/*
 * chain_oracle.c -- plain FP64 CPU oracle for the SU(2) Polyakov chain with
 * complex Langevin (CL) dynamics and adaptive gauge cooling (section
 * "Adaptive gauge cooling in the SU(2) Polyakov chain model": the action of
 * eq. (eq:s); cooling of section "Gauge cooling", eq. (eq:24); the distance
 * d of eq. (d)).
 *
 * TEST INFRASTRUCTURE ONLY, like clgc_oracle.c: only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark load it, and it shares no
 * code with the GPU path.  Conventions shared with the GPU by definition
 * only:
 *
 *   chain       links U_0 .. U_{n-1}, link k from site k to site k+1 (mod n);
 *               action S = -(beta/2) Tr(U_0 U_1 ... U_{n-1}), beta complex;
 *   host layout links[((c*n + k)*4 + 2*i + j)*2 + {0: re, 1: im}] for chain c;
 *   generators  Pauli sigma_a, Tr(sigma_a sigma_b) = 2 delta_ab (the Gell-Mann
 *               normalisation of the SU(3) path; the paper's one-link
 *               formulas use sigma_a/2, which rescales cooling rates by 4);
 *   noise       Philox4x32-10, key (seed lo, seed hi), counter
 *               (link k, step, chain, tag << 16 | draw); tag 2 = CL noise,
 *               tag 3 = start; draws 0, 1 give eta_1, eta_2 and eta_3 (x sqrt 2).
 *   cooling     Jacobi order: every Omega_k from the same links, then
 *               U_k <- Omega_k U_k Omega_{k+1}^{-1} (a periodic chain of odd
 *               length, the one-link chain included, has no checkerboard).
 *
 * Parity unpinned: none of these functions; the pins are in
 * tests/test_oracle_chain.py.
 */
#include "clgc_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double complex a[2][2];
} M2;

static M2 m2_id(void)
{
    M2 r = {{{1, 0}, {0, 1}}};
    return r;
}

static M2 m2_zero(void)
{
    M2 r;
    memset(&r, 0, sizeof r);
    return r;
}

static M2 m2_mul(M2 x, M2 y)
{
    M2 r;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) r.a[i][j] = x.a[i][0] * y.a[0][j] + x.a[i][1] * y.a[1][j];
    return r;
}

static M2 m2_add(M2 x, M2 y)
{
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) x.a[i][j] += y.a[i][j];
    return x;
}

static M2 m2_scale(M2 x, double complex s)
{
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) x.a[i][j] *= s;
    return x;
}

static M2 m2_dag(M2 x)
{
    M2 r;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) r.a[i][j] = conj(x.a[j][i]);
    return r;
}

static double complex m2_tr(M2 x) { return x.a[0][0] + x.a[1][1]; }

static double complex m2_det(M2 x) { return x.a[0][0] * x.a[1][1] - x.a[0][1] * x.a[1][0]; }

static double m2_maxabs(M2 x)
{
    double m = 0.0;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            if (cabs(x.a[i][j]) > m) m = cabs(x.a[i][j]);
    return m;
}

/* Traceless part M - Tr(M)/2 */
static M2 m2_tl(M2 x)
{
    double complex t = 0.5 * m2_tr(x);
    x.a[0][0] -= t;
    x.a[1][1] -= t;
    return x;
}

/* Pauli matrices sigma_1..sigma_3 (index a = 0..2) */
static M2 pauli(int a)
{
    M2 r = m2_zero();
    if (a == 0) {
        r.a[0][1] = 1;
        r.a[1][0] = 1;
    } else if (a == 1) {
        r.a[0][1] = -I;
        r.a[1][0] = I;
    } else {
        r.a[0][0] = 1;
        r.a[1][1] = -1;
    }
    return r;
}

/* exp(A): Taylor series after scaling A by 2^-k (||A||_1 <= 1/2), then k
 * squarings; the halving is bounded so that a non-finite A ends. */
static M2 m2_exp(M2 A)
{
    double nrm = 0.0;
    for (int j = 0; j < 2; ++j) {
        double c = cabs(A.a[0][j]) + cabs(A.a[1][j]);
        if (c > nrm) nrm = c;
    }
    int k = 0;
    while (nrm > 0.5 && k < 1100) {
        nrm *= 0.5;
        ++k;
    }
    A = m2_scale(A, ldexp(1.0, -k));
    M2 sum = m2_id(), term = m2_id();
    for (int n = 1; n < 60; ++n) {
        term = m2_scale(m2_mul(term, A), 1.0 / n);
        sum = m2_add(sum, term);
        if (m2_maxabs(term) <= 1e-19 * m2_maxabs(sum)) break;
    }
    for (int i = 0; i < k; ++i) sum = m2_mul(sum, sum);
    return sum;
}

static M2 m2_load(const double *p)
{
    M2 r;
    for (int e = 0; e < 4; ++e) r.a[e / 2][e % 2] = p[2 * e] + I * p[2 * e + 1];
    return r;
}

static void m2_store(M2 x, double *p)
{
    for (int e = 0; e < 4; ++e) {
        p[2 * e] = creal(x.a[e / 2][e % 2]);
        p[2 * e + 1] = cimag(x.a[e / 2][e % 2]);
    }
}

/* sum_a c_a sigma_a */
static M2 pauli_comb(const double complex c[3])
{
    M2 r = m2_zero();
    for (int a = 0; a < 3; ++a) r = m2_add(r, m2_scale(pauli(a), c[a]));
    return r;
}

/* ------------------------------------------------------------------ */
/* noise and start                                                     */
/* ------------------------------------------------------------------ */

/* eta_1..eta_3 of link k of chain c at CL step n, <eta_a eta_b> = 2 delta_ab */
void orc_chain_noise(uint64_t seed, long chain, int k, uint32_t step, double eta[3])
{
    double n0[2], n1[2];
    orc_normal_pair(seed, (uint32_t)k, step, (uint32_t)chain, (2u << 16) | 0u, n0);
    orc_normal_pair(seed, (uint32_t)k, step, (uint32_t)chain, (2u << 16) | 1u, n1);
    eta[0] = sqrt(2.0) * n0[0];
    eta[1] = sqrt(2.0) * n0[1];
    eta[2] = sqrt(2.0) * n1[0];
}

/* U_k = exp(i sigma_a (x_a + i y_a)), x_a ~ N(0, sx), y_a ~ N(0, sy) (the
 * start of the SU(3) path, with Pauli generators) */
void orc_chain_init(int n, long chain, uint64_t seed, double sx, double sy, double *links)
{
    for (int k = 0; k < n; ++k) {
        double p[4][2];
        for (int j = 0; j < 4; ++j) orc_normal_pair(seed, (uint32_t)k, 0u, (uint32_t)chain, (3u << 16) | (uint32_t)j, p[j]);
        const double x[3] = {sx * p[0][0], sx * p[0][1], sx * p[1][0]};
        const double y[3] = {sy * p[2][0], sy * p[2][1], sy * p[3][0]};
        double complex c[3];
        for (int a = 0; a < 3; ++a) c[a] = I * (x[a] + I * y[a]);
        m2_store(m2_exp(pauli_comb(c)), links + (size_t)k * 8);
    }
}

/* ------------------------------------------------------------------ */
/* action, drift, observables                                          */
/* ------------------------------------------------------------------ */

/* P_k = U_k U_{k+1} ... U_{n-1} U_0 ... U_{k-1}: the chain's loop opened at link k */
void orc_chain_loop(int n, const double *links, int k, double out[8])
{
    M2 P = m2_id();
    for (int j = 0; j < n; ++j) P = m2_mul(P, m2_load(links + (size_t)((k + j) % n) * 8));
    m2_store(P, out);
}

/* Drift of link k (eq. (eq:s) with K_a = -D_a S, D_a f = d/dt f(e^{i t sigma_a} U_k)):
 * K_a = (i beta / 2) Tr(sigma_a P_k), so Khat = sum_a K_a sigma_a = i beta TL(P_k). */
void orc_chain_drift(int n, const double *links, double beta_re, double beta_im, double *K)
{
    const double complex beta = beta_re + I * beta_im;
    for (int k = 0; k < n; ++k) {
        double p[8];
        orc_chain_loop(n, links, k, p);
        m2_store(m2_scale(m2_tl(m2_load(p)), I * beta), K + (size_t)k * 8);
    }
}

/* sum_k Tr U_k U_k^dagger */
double orc_chain_unorm(int n, const double *links)
{
    double s = 0.0;
    for (int k = 0; k < n; ++k) {
        M2 U = m2_load(links + (size_t)k * 8);
        s += creal(m2_tr(m2_mul(U, m2_dag(U))));
    }
    return s;
}

/* out = (Re L, Im L, d, Re S, Im S) with the Polyakov loop L = Tr(U_0...U_{n-1})/2,
 * S = -beta L (eq. (eq:s)) and d = (1/2n) sum_k Tr(U U^dag - 1) (eq. (d) per link) */
void orc_chain_measure(int n, const double *links, double beta_re, double beta_im, double out[5])
{
    double p[8];
    orc_chain_loop(n, links, 0, p);
    const double complex L = 0.5 * m2_tr(m2_load(p));
    const double complex S = -(beta_re + I * beta_im) * L;
    out[0] = creal(L);
    out[1] = cimag(L);
    out[2] = orc_chain_unorm(n, links) / (2.0 * n) - 1.0;
    out[3] = creal(S);
    out[4] = cimag(S);
}

/* ------------------------------------------------------------------ */
/* CL update                                                           */
/* ------------------------------------------------------------------ */

/* U_k <- exp(i (eps Khat_k + sqrt(eps) eta_a sigma_a)) U_k, then U_k <- U_k / sqrt(det U_k)
 * (principal branch; the SU(3) path's det renormalisation for N = 2) */
void orc_chain_update(int n, double *links, const double *K, double eps, uint64_t seed, long chain,
                      uint32_t step)
{
    for (int k = 0; k < n; ++k) {
        double eta[3];
        orc_chain_noise(seed, chain, k, step, eta);
        double complex c[3];
        for (int a = 0; a < 3; ++a) c[a] = sqrt(eps) * eta[a];
        const M2 X = m2_scale(m2_add(m2_scale(m2_load(K + (size_t)k * 8), eps), pauli_comb(c)), I);
        M2 U = m2_mul(m2_exp(X), m2_load(links + (size_t)k * 8));
        U = m2_scale(U, 1.0 / csqrt(m2_det(U)));
        m2_store(U, links + (size_t)k * 8);
    }
}

/* One CL step of one chain: drift, adaptive step eps = min(eps0, B/K_max)
 * (B fixed from the first step: eps0 K_max,0 unless given), update.
 * Returns 0, or 1 if the drift is not finite (links untouched). */
int orc_chain_step(int n, double *links, double beta_re, double beta_im, uint64_t seed, long chain,
                   uint32_t step, double eps0, int adaptive, double drift_bound, double *bound,
                   double *eps_used, double *kmax_out)
{
    double *K = malloc(sizeof(double) * 8 * (size_t)n);
    orc_chain_drift(n, links, beta_re, beta_im, K);
    double km2 = 0.0;
    for (int k = 0; k < n; ++k) {
        const M2 Kk = m2_load(K + (size_t)k * 8);
        double v = 0.5 * creal(m2_tr(m2_mul(Kk, m2_dag(Kk))));
        if (!isfinite(v)) v = INFINITY;
        if (v > km2) km2 = v;
    }
    const double kmax = sqrt(km2);
    if (kmax_out) *kmax_out = kmax;
    if (!isfinite(kmax)) {
        free(K);
        return 1;
    }
    double eps = eps0;
    if (adaptive) {
        if (*bound <= 0.0) *bound = drift_bound > 0.0 ? drift_bound : eps0 * kmax;
        if (kmax > 0.0 && *bound / kmax < eps0) eps = *bound / kmax;
    }
    if (eps_used) *eps_used = eps;
    orc_chain_update(n, links, K, eps, seed, chain, step);
    free(K);
    return 0;
}

/* ------------------------------------------------------------------ */
/* gauge cooling                                                       */
/* ------------------------------------------------------------------ */

/* G_k = U_k U_k^dag - U_{k-1}^dag U_{k-1} at site k (eq. (eq:24) for one direction);
 * f_ak = 2 Tr(sigma_a G_k) is written to f[3*k + a] if f is not NULL */
static M2 chain_gradient(int n, const double *links, int k, double *f)
{
    const M2 U = m2_load(links + (size_t)k * 8);
    const M2 W = m2_load(links + (size_t)((k + n - 1) % n) * 8);
    const M2 G = m2_add(m2_mul(U, m2_dag(U)), m2_scale(m2_mul(m2_dag(W), W), -1.0));
    if (f)
        for (int a = 0; a < 3; ++a) f[3 * k + a] = creal(2.0 * m2_tr(m2_mul(pauli(a), G)));
    return G;
}

void orc_chain_gradient(int n, const double *links, double *f)
{
    for (int k = 0; k < n; ++k) chain_gradient(n, links, k, f);
}

/* One cooling step: Omega_k = exp(-eps alpha_ad f_ak sigma_a) at every site from
 * the same links, then U_k <- Omega_k U_k Omega_{k+1}^{-1} (Omega^{-1} = exp of the
 * negated exponent). */
void orc_chain_cool_step(int n, double *links, double eps_alpha)
{
    M2 *Om = malloc(sizeof(M2) * (size_t)n), *Oi = malloc(sizeof(M2) * (size_t)n);
    double *f = malloc(sizeof(double) * 3 * (size_t)n);
    orc_chain_gradient(n, links, f);
    for (int k = 0; k < n; ++k) {
        double complex c[3];
        for (int a = 0; a < 3; ++a) c[a] = -eps_alpha * f[3 * k + a];
        const M2 A = pauli_comb(c);
        Om[k] = m2_exp(A);
        Oi[k] = m2_exp(m2_scale(A, -1.0));
    }
    for (int k = 0; k < n; ++k) {
        const M2 U = m2_load(links + (size_t)k * 8);
        m2_store(m2_mul(m2_mul(Om[k], U), Oi[(k + 1) % n]), links + (size_t)k * 8);
    }
    free(Om);
    free(Oi);
    free(f);
}

/* n_cool cooling steps with alpha_ad = alpha / D (section on adaptive cooling):
 * mode 0: D_0 = 1; mode 1: D_1 = Tr UU^dag per link, UN / n; mode 2: D_2 = mean
 * over (a, k) of |f_ak|; each on the chain entering the step.  un[0..n_cool]
 * receives UN before every step and after the last, alpha_used[i] alpha_ad.
 * Returns 0, or 1 if the unitarity norm became non-finite. */
int orc_chain_cool(int n, double *links, int n_cool, double eps_c, double alpha, int mode, double *un,
                   double *alpha_used)
{
    double *f = malloc(sizeof(double) * 3 * (size_t)n);
    int rc = 0;
    for (int i = 0; i < n_cool; ++i) {
        const double u = orc_chain_unorm(n, links);
        if (un) un[i] = u;
        if (!isfinite(u)) {
            rc = 1;
            break;
        }
        double D = 1.0;
        if (mode == 1) D = u / n;
        if (mode == 2) {
            orc_chain_gradient(n, links, f);
            double s = 0.0;
            for (int j = 0; j < 3 * n; ++j) s += fabs(f[j]);
            D = s / (3.0 * n);
        }
        const double al = alpha / D;
        if (alpha_used) alpha_used[i] = al;
        orc_chain_cool_step(n, links, eps_c * al);
    }
    if (!rc && un) un[n_cool] = orc_chain_unorm(n, links);
    if (!rc && !isfinite(orc_chain_unorm(n, links))) rc = 1;
    free(f);
    return rc;
}

/* n_steps CL steps of one chain, each followed by n_cool cooling steps and a
 * measurement: obs[i*6 + {0..5}] = (Re L, Im L, d, eps, kmax, d before cooling).
 * Returns 0, or the 1-based step whose drift or cooling was not finite. */
int orc_chain_run(int n, double *links, double beta_re, double beta_im, uint64_t seed, long chain,
                  uint32_t step0, int n_steps, double eps0, int adaptive, double drift_bound, double *bound,
                  int n_cool, double eps_c, double alpha, int mode, double *obs)
{
    for (int i = 0; i < n_steps; ++i) {
        double eps = 0.0, kmax = 0.0, m[5];
        if (orc_chain_step(n, links, beta_re, beta_im, seed, chain, step0 + (uint32_t)i, eps0, adaptive,
                           drift_bound, bound, &eps, &kmax))
            return i + 1;
        const double d_pre = orc_chain_unorm(n, links) / (2.0 * n) - 1.0;
        if (orc_chain_cool(n, links, n_cool, eps_c, alpha, mode, NULL, NULL)) return i + 1;
        orc_chain_measure(n, links, beta_re, beta_im, m);
        if (obs) {
            double *o = obs + (size_t)i * 6;
            o[0] = m[0];
            o[1] = m[1];
            o[2] = m[2];
            o[3] = eps;
            o[4] = kmax;
            o[5] = d_pre;
        }
    }
    return 0;
}

/* exp of a 2x2 complex matrix (for the pins) */
void orc_chain_expm(const double *A, double *out) { m2_store(m2_exp(m2_load(A)), out); }
