/*
 * clgc_oracle.h -- FP64 CPU oracle for complex Langevin + adaptive gauge
 * cooling of SU(3) with a theta term.  TEST INFRASTRUCTURE ONLY: loaded by
 * the tests, the smoke check and the benchmark's CPU-baseline leg, never by
 * the library.  Conventions are documented at the top of clgc_oracle.c.
 */
#ifndef CLGC_ORACLE_H
#define CLGC_ORACLE_H
#include <stdint.h>

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_normal_pair(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, double out[2]);
void orc_cl_noise(uint64_t seed, long s, int mu, uint32_t step, double eta[8]);
void orc_cold_links(const int *dims, double *links);
void orc_init_links(const int *dims, uint64_t seed, double sigma_x, double sigma_y, double *links);
void orc_plaquette(const int *dims, const double *links, double out[2]);
void orc_wilson_action(const int *dims, const double *links, double beta, double out[2]);
void orc_topological_charge(const int *dims, const double *links, double out[2]);
double orc_unitarity_norm(const int *dims, const double *links);
void orc_drift(const int *dims, const double *links, double beta, double theta_re, double theta_im, double *K);
void orc_drift_links(const int *dims, const double *links, double beta, double theta_re, double theta_im,
                     const long *sel, long nsel, double *K);
void orc_langevin_update(const int *dims, double *links, const double *K, double eps, uint64_t seed, uint32_t step);
int orc_langevin_step(const int *dims, double *links, double beta, double theta_re, double theta_im,
                      uint64_t seed, uint32_t step, double eps0, int adaptive, double drift_bound,
                      double *bound, double out[2]);
void orc_cool_gradient(const int *dims, const double *links, long s, double f[8]);
void orc_cool_halfsweep(const int *dims, double *links, int parity, double eps_alpha);
int orc_gauge_cool(const int *dims, double *links, int n_steps, double eps_c, double alpha, int mode,
                   double *unorm, double *alpha_used);
void orc_gauge_transform(const int *dims, double *links, const double *omega);
void orc_expm(const double *A, double *out);
void orc_path(const int *dims, const double *links, long s, const int *dirs, int n, double *out);
void orc_link_stats(const int *dims, const double *links, double out[2]);
void orc_cl_noise_field(const int *dims, uint64_t seed, uint32_t step, double *eta);
int orc_run(const int *dims, double *links, double beta, double theta_re, double theta_im, uint64_t seed,
            uint32_t step0, int n_steps, double eps0, int adaptive, double drift_bound, double *bound,
            int n_cool, double eps_c, double alpha, int mode, double *obs);

/* Set (n > 0) and return the OpenMP thread count; timing only. */
int orc_set_threads(int n);

/* SU(2) Polyakov chain (chain_oracle.c); links: n x 8 doubles (2x2, row-major, re/im) */
void orc_chain_noise(uint64_t seed, long chain, int k, uint32_t step, double eta[3]);
void orc_chain_init(int n, long chain, uint64_t seed, double sx, double sy, double *links);
void orc_chain_loop(int n, const double *links, int k, double out[8]);
void orc_chain_drift(int n, const double *links, double beta_re, double beta_im, double *K);
double orc_chain_unorm(int n, const double *links);
void orc_chain_measure(int n, const double *links, double beta_re, double beta_im, double out[5]);
void orc_chain_update(int n, double *links, const double *K, double eps, uint64_t seed, long chain,
                      uint32_t step);
int orc_chain_step(int n, double *links, double beta_re, double beta_im, uint64_t seed, long chain,
                   uint32_t step, double eps0, int adaptive, double drift_bound, double *bound,
                   double *eps_used, double *kmax_out);
void orc_chain_gradient(int n, const double *links, double *f);
void orc_chain_cool_step(int n, double *links, double eps_alpha);
int orc_chain_cool(int n, double *links, int n_cool, double eps_c, double alpha, int mode, double *un,
                   double *alpha_used);
int orc_chain_run(int n, double *links, double beta_re, double beta_im, uint64_t seed, long chain,
                  uint32_t step0, int n_steps, double eps0, int adaptive, double drift_bound, double *bound,
                  int n_cool, double eps_c, double alpha, int mode, double *obs);
void orc_chain_expm(const double *A, double *out);

#endif
