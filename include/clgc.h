/*
 * clgc.h -- C ABI of the MI355X (gfx950) library for complex Langevin (CL)
 * dynamics of SU(3) lattice gauge theory with a theta term and adaptive
 * SL(3,C) gauge cooling (Bongiovanni, Aarts, Seiler, Sexty, Stamatescu,
 * "Adaptive gauge cooling for complex Langevin dynamics", LATTICE 2013).
 *
 * The library holds no torch types: callers pass plain device pointers (a
 * buffer they own, e.g. a torch tensor's data_ptr) and a hipStream_t as
 * void*.  Every entry point returns a cl_status; on failure the thread-local
 * message from cl_last_error() says why.  Calls on one lattice are
 * stream-ordered and must come from one thread at a time; distinct lattices
 * are independent.
 *
 * Conventions (shared with the host link layout used by set/get_links):
 *   sites   s = x0 + L0*(x1 + L1*(x2 + L2*x3)), x0 fastest; periodic;
 *   links   host array of V*4*18 doubles: [s][mu][row][col][re,im];
 *   inverse U^{-1} = adj(U) (links stay in SL(3,C): det U = 1);
 *   basis   Gell-Mann lambda_a, Tr(lambda_a lambda_b) = 2 delta_ab;
 *   noise   Philox4x32-10, counter (4*s+mu, CL step n, draw j, stream tag),
 *           key = seed; eta_a with <eta_a eta_b> = 2 delta_ab;
 *   extents even and >= 2 (the cooling sweep is checkerboarded).
 */
#ifndef CLGC_H
#define CLGC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cl_lattice cl_lattice;

typedef enum {
    CL_OK = 0,
    CL_EINVAL = -1,      /* bad argument: odd/too small extent, NULL pointer, size mismatch */
    CL_ENOMEM = -2,      /* caller's device buffer too small */
    CL_EHIP = -3,        /* a HIP runtime call failed */
    CL_ENONFINITE = -4,  /* drift or unitarity norm became non-finite: the run is not advanced */
    CL_EBUDGET = -5      /* a served run can never fit the server's HBM budget */
} cl_status;

typedef enum { CL_FP64 = 0, CL_MIXED = 1 } cl_precision;

/* Adaptive cooling strength alpha_ad = alpha / D (section on adaptive gauge
 * cooling): D_0 = 1, D_1 = Tr U U^dagger averaged over links (UN / 4V),
 * D_2 = mean over (a, x) of |f_ax|, each on the configuration entering the
 * cooling step. */
typedef enum { CL_ALPHA_FIXED = 0, CL_ALPHA_UNORM = 1, CL_ALPHA_GRAD = 2 } cl_alpha_mode;

typedef struct {
    int32_t dims[4];     /* L0..L3, each even and >= 2 */
    double beta;         /* Wilson coupling, > 0 */
    double theta_re;     /* theta_L (complex: real theta -> complex action, */
    double theta_im;     /*   imaginary theta -> real action) */
    int32_t precision;   /* cl_precision */
    uint64_t seed;       /* Philox key */
} cl_lattice_desc;

typedef struct {
    double eps0;         /* nominal Langevin step */
    int32_t adaptive;    /* 0: eps = eps0; 1: eps_n = min(eps0, B / Kmax_n) */
    double drift_bound;  /* B; <= 0: B = eps0 * Kmax of the first adaptive step */
} cl_step_desc;

typedef struct {
    int32_t n_steps;     /* cooling steps (each an even then an odd half-sweep), 0..64 */
    double eps_c;        /* epsilon of Omega_x = exp(-eps alpha_ad f_ax lambda_a) */
    double alpha;        /* alpha_gf */
    int32_t mode;        /* cl_alpha_mode */
} cl_cool_desc;

typedef struct {
    double plaq[2];      /* (1/18V) sum_x sum_{mu<nu} Tr U_{mu nu}(x), complex */
    double q[2];         /* Q_L = sum_x q_L(x), clover form, complex */
    double action[2];    /* S = S_W - i theta Q_L, complex */
    double unorm_d;      /* d = (1/12V) sum Tr(U U^dagger - 1) of the current links */
    double d_pre;        /* d right after the last CL update, before cooling */
    double eps;          /* step size of the last CL update */
    double kmax;         /* max over links of ||Khat|| of the last CL update */
    double alpha;        /* alpha_ad of the last cooling step */
    double bound;        /* adaptive step-size bound B (<= 0: not set yet) */
    int64_t step;        /* CL steps taken (the next update uses Philox step = this) */
} cl_obs;

/* Bytes of device memory a lattice needs (links, clover field, drift,
 * reduction scratch, control block).  desc as for cl_lattice_create. */
cl_status cl_lattice_bytes(const cl_lattice_desc* desc, size_t* device_bytes);

/* Create a lattice inside dev_buf (device memory of at least
 * cl_lattice_bytes, 256-byte aligned, owned by the caller and kept alive
 * until cl_lattice_destroy).  hip_stream: the hipStream_t every call on this
 * lattice is ordered on (NULL = the default stream).  The links start cold
 * (U = 1). */
cl_status cl_lattice_create(const cl_lattice_desc* desc, void* dev_buf, size_t buf_bytes,
                            void* hip_stream, cl_lattice** out);
cl_status cl_lattice_destroy(cl_lattice* lat);

/* Start configuration.  The paper does not give one; the perturbed start has
 * the form of the SL(3,C) elements of the section on gauge cooling (the
 * exponential of i omega_a lambda_a with complex omega_a).
 * perturbed = 0: cold start U = 1.  perturbed = 1: U = exp(i lambda_a (x_a + i y_a))
 * with x_a ~ N(0, sigma_x^2), y_a ~ N(0, sigma_y^2) from Philox stream tag 1
 * (draws 0..3 give x_1..x_8, draws 4..7 give y_1..y_8).  Resets the step counter
 * and the adaptive bound and clears the per-step record.  Asynchronous. */
cl_status cl_lattice_init(cl_lattice* lat, int perturbed, double sigma_x, double sigma_y);

/* Copy all links from / to a host array of V*4*18 doubles (layout above).
 * Synchronous on the lattice's stream. */
cl_status cl_lattice_set_links(cl_lattice* lat, const double* host, size_t n_doubles);
cl_status cl_lattice_get_links(cl_lattice* lat, double* host, size_t n_doubles);

/* Step counter n and adaptive bound B (for checkpoint / resume).  set_state
 * clears the per-step record.  Synchronous. */
cl_status cl_lattice_get_state(cl_lattice* lat, int64_t* step, double* bound);
cl_status cl_lattice_set_state(cl_lattice* lat, int64_t step, double bound);

/* One CL update of every link (section on SU(3) with a theta term; the
 * update itself is the standard CL step the paper alternates with cooling):
 *   Khat = -sum_a lambda_a D_a S,  S = S_W - i theta Q_L,
 *   U <- exp(i (eps_n Khat + sqrt(eps_n) eta_a lambda_a)) U,  U <- U det(U)^{-1/3}.
 * All links move from the same configuration.  eps_used: if non-NULL the
 * call waits for the stream and returns eps_n; if NULL it is asynchronous.
 * Returns CL_ENONFINITE (and leaves the links unchanged) if the drift is not
 * finite -- detected at the next synchronising call when asynchronous. */
cl_status cl_langevin_step(cl_lattice* lat, const cl_step_desc* step, double* eps_used);

/* n_steps adaptive gauge-cooling steps (section on gauge cooling, eq. for
 * Omega_x and f_ax): at every site x of one parity, then the other,
 *   f_ax = 2 Tr[lambda_a sum_mu (U_{x,mu} U_{x,mu}^dagger - U_{x-mu,mu}^dagger U_{x-mu,mu})],
 *   Omega_x = exp(-eps_c alpha_ad f_ax lambda_a),
 *   U_{x,mu} <- Omega_x U_{x,mu},  U_{x-mu,mu} <- U_{x-mu,mu} Omega_x^{-1}.
 * unorm_after: if non-NULL, waits and returns d of the cooled links. */
cl_status cl_gauge_cool(cl_lattice* lat, const cl_cool_desc* cool, double* unorm_after);

/* d = (1/12V) sum_{x,mu} Tr(U U^dagger - 1) of the current links: the
 * one-link distance from the unitary manifold, eq. (d) of the section on the
 * one-link model, averaged over links; (1/N) Tr U U^dagger >= 1 (section on
 * gauge cooling) makes it >= 0, with 0 exactly on SU(3).  Synchronous.
 * CL_ENONFINITE if the lattice's state went non-finite. */
cl_status cl_unitarity_norm(cl_lattice* lat, double* d);

/* Observables of the current links (section on SU(3) with a theta term):
 * the plaquette, the topological charge Q_L = sum_x q_L(x) with the density of
 * eq. (eq:st) in its equivalent clover form, the action S = S_W - i theta Q_L
 * of the same section (S_W the Wilson action), the distance d of eq. (d), and
 * the control state (step size, Kmax, alpha_ad, bound, step counter).
 * Accumulated in FP64 in both precisions; a mixed-precision lattice forms the
 * clover matrices in FP64 from its FP32 links.  Synchronous.  CL_ENONFINITE if
 * the state went non-finite (out is still filled). */
cl_status cl_measure(cl_lattice* lat, cl_obs* out);

/* Drift Khat of every link for the current configuration, copied to a host
 * array in the link layout (V*4*18 doubles).  Synchronous; for inspection
 * and tests, not needed by a simulation. */
cl_status cl_compute_drift(cl_lattice* lat, double* host_K, size_t n_doubles);

/* Per-cooling-step history of the last cl_gauge_cool / cl_run_steps call:
 * unorm[i] = sum Tr U U^dagger entering cooling step i (i = 0..n), alpha[i] =
 * alpha_ad used by step i.  cap: room in each array.  Synchronous. */
cl_status cl_cool_history(cl_lattice* lat, double* unorm, double* alpha, int cap, int* n);

/* n_steps x (one CL update + cooling), all enqueued without host
 * synchronisation (what a production loop runs): the alternation of Langevin
 * updates and cooling steps of the section on the SU(2) Polyakov chain model,
 * applied to the SU(3) lattice.  Replayed from captured graphs (blocks of
 * eight steps, then single steps), captured on first use for these
 * parameters.  With the record on (cl_record_enable) every step's
 * observables are written to the device record as well.  Asynchronous. */
cl_status cl_run_steps(cl_lattice* lat, const cl_step_desc* step, const cl_cool_desc* cool,
                       int n_steps);

/* Capture and instantiate the graphs cl_run_steps replays for these
 * parameters (and the current record setting) without running them, so that
 * no later call pays for a capture.  Sets the step and cooling parameters as
 * cl_run_steps would.  Synchronous on the host (no device work). */
cl_status cl_run_prepare(cl_lattice* lat, const cl_step_desc* step, const cl_cool_desc* cool);

/* Per-step record of cl_run_steps (the paper's results are Langevin-time
 * series: the running <Q_L> and the distance along the Langevin time).  While
 * enabled, each CL step's observables, measured on the links it leaves after
 * its cooling, go to a ring of the last 4096 steps in the lattice's device
 * buffer, with no host synchronisation: the measurement runs at the start of
 * the next step (with a theta term in FP64 it reuses the clover field that
 * step builds for its drift) and after each call's last step.  Disabled by
 * default.  Each entry is 12 doubles:
 *   step, d_pre, d, Re P, Im P, Re Q, Im Q, Re S, Im S, eps, Kmax, alpha_ad
 * (as in cl_obs; d_pre before and d after the step's cooling). */
cl_status cl_record_enable(cl_lattice* lat, int enable);
/* Copy the entries of CL steps first_step .. first_step + n - 1 (1-based,
 * counted by the step counter) to host[n * 12].  CL_EINVAL if a step is not
 * in the record (not taken yet, or more than 4096 steps ago).  Synchronous. */
cl_status cl_record_read(cl_lattice* lat, int64_t first_step, int n, double* host);

/* Allocation-free variant of cl_measure, for callers that cannot allocate
 * device memory or wait for a stream: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Measures a link field the
 * caller already holds on the device, in the host link layout (V*4*18
 * doubles, lexicographic sites, x0 fastest), with the formulas of cl_measure
 * (every sum in FP64, the clover matrices formed per site):
 *   dev_out[0..1] plaquette (re, im), [2..3] Q_L, [4..5] S = S_W - i theta Q_L,
 *   [6] d = (1/12V) sum Tr(U U^dagger - 1)
 * (7 doubles of device memory the caller owns).  dims: four even extents >= 2
 * with at most 2^20 sites (32^4); larger fields get CL_EINVAL.  The kernels
 * run on hip_stream (NULL: the default stream) of the current device and the
 * call returns without waiting; nothing is allocated at any call.  Their
 * per-block partials live in a 224 KiB device array of the library's own,
 * one per GPU, held until the process ends: calls that overlap on one GPU
 * (e.g. on two streams) race on it and must be ordered by the caller. */
cl_status cl_measure_links(const double* dev_links, const int32_t* dims, double beta, double theta_re,
                           double theta_im, double* dev_out, void* hip_stream);

/* Kernel kinds reported by cl_timing_read. */
typedef enum {
    CL_K_INIT = 0, CL_K_UNORM = 1, CL_K_PACK = 2, CL_K_CLOVER = 3, CL_K_DRIFT = 4, CL_K_UPDATE = 5,
    CL_K_COOL_OMEGA = 6,  /* even-site Omega of a cooling step */
    CL_K_COOL_APPLY = 7,  /* both half-sweeps applied, odd-site Omega, every link written once */
    CL_K_GRADNORM = 8, CL_K_MEASURE = 9, CL_K_FINALIZE = 10, CL_K_COUNT = 11
} cl_kernel_kind;

/* Benchmark instrumentation: while enabled, every kernel the lattice
 * launches is bracketed by a pair of HIP events on its stream.  Disabled by
 * default.  Enabling clears the previous record. */
cl_status cl_timing_enable(cl_lattice* lat, int enable);

/* Waits for the stream, then gives per kernel kind (cap >= CL_K_COUNT
 * entries) the summed event-measured milliseconds and launch count recorded
 * since cl_timing_enable(lat, 1). */
cl_status cl_timing_read(cl_lattice* lat, double* total_ms, int64_t* launches, int cap);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of independent CL runs on one GPU.
 *
 * A server owns a caller-provided device arena.  Submitted runs wait in a
 * FIFO queue until their device footprint (cl_lattice_bytes) fits in the
 * arena; admitted runs are initialised and then advance together: every
 * cl_server_step performs one CL update plus that run's own number of
 * cooling steps for every active run, with one launch per kernel kind over
 * the concatenated logical blocks of all runs of a precision (replayed from a
 * captured graph).  Finished runs are measured, retired and their memory
 * reused by the next admissions.  A run's arithmetic does not depend on what
 * it is batched with.
 * ------------------------------------------------------------------------- */
typedef struct cl_server cl_server;

typedef struct {
    cl_lattice_desc lattice;   /* extents, beta, theta, precision, seed */
    cl_step_desc step;         /* eps0, adaptive, drift bound */
    cl_cool_desc cool;         /* cooling steps per update (0..64), eps_c, alpha, mode */
    int32_t n_steps;           /* CL steps to run (>= 1) */
    double sigma_x, sigma_y;   /* perturbed start as in cl_lattice_init */
    uint64_t tag;              /* caller's label, returned with the result */
    int32_t keep_links;        /* != 0: keep the final links for cl_server_take_links */
    int32_t pad;
} cl_run_desc;

typedef struct {
    uint64_t run_id, tag;
    int32_t status;            /* CL_OK, or CL_ENONFINITE for a run retired on a runaway */
    int32_t steps_done;
    cl_obs obs;                /* measured after the last step */
    double t_submit, t_admit, t_finish;  /* seconds on the server's clock */
    double step_ms_p50, step_ms_p99;     /* wall time of the batch steps the run advanced in */
    int64_t link_updates;      /* 4 V x steps_done */
} cl_run_result;

typedef struct {
    int32_t pending, active, finished;
    size_t bytes_in_use, bytes_budget;
    int64_t batch_steps, link_updates;
    double busy_s;                       /* summed wall time of batch steps */
    double step_ms_p50, step_ms_p99;     /* over all (run, step) samples */
    double wait_s_p50, wait_s_p99;       /* queue wait (admit - submit) of finished runs */
} cl_server_stats;

/* arena: device memory owned by the caller (256-byte aligned) holding the
 * server's tables and every admitted run; its size is the HBM budget. */
cl_status cl_server_create(void* arena, size_t arena_bytes, void* hip_stream, cl_server** out);
/* Queue a run (non-blocking).  CL_EBUDGET if it can never fit the arena. */
cl_status cl_server_submit(cl_server* srv, const cl_run_desc* run, uint64_t* run_id);
/* Admit what fits, advance every active run by one step, retire finished
 * runs.  Waits for the GPU at the end of the step.  n_active / n_pending may
 * be NULL.  The same as cl_server_steps(srv, 1, ...). */
cl_status cl_server_step(cl_server* srv, int* n_active, int* n_pending);
/* Admit what fits, then advance every active run by n batch steps with one
 * wait for the GPU at the end, n = min(max_steps, the fewest steps any
 * active run has left), so that no run goes past its last step; retire
 * finished runs.  Runs submitted meanwhile are admitted by the next call.
 * A run's step_ms samples are the call's wall time over n.  A run that runs
 * away during the call stops advancing at that point (its steps_done is its
 * own step counter) and is retired at the end of the call.  CL_EINVAL if
 * max_steps < 1. */
cl_status cl_server_steps(cl_server* srv, int max_steps, int* n_active, int* n_pending);
/* Move up to cap finished results into out (oldest first). */
cl_status cl_server_poll(cl_server* srv, cl_run_result* out, int cap, int* n_done);
cl_status cl_server_stats_get(cl_server* srv, cl_server_stats* out);
/* The final links of a finished run submitted with keep_links (host link
 * layout, V*4*18 doubles), copied once and then released.  CL_EINVAL if the
 * run is not finished, kept no links or was already taken, or n_doubles does
 * not match. */
cl_status cl_server_take_links(cl_server* srv, uint64_t run_id, double* host, size_t n_doubles);
cl_status cl_server_destroy(cl_server* srv);

/* ------------------------------------------------------------------------
 * SU(2) Polyakov chain (section "Adaptive gauge cooling in the SU(2) Polyakov
 * chain model"): n_chains independent chains of n_links SL(2,C) links with
 * S = -(beta/2) Tr(U_0 U_1 ... U_{n-1}), eq. (eq:s), beta complex, evolved by
 * complex Langevin (Pauli generators, <eta_a eta_b> = 2 delta_ab, the update
 * and det renormalisation of the SU(3) path) alternated with gauge cooling of
 * eq. (eq:24) on the chain's sites (Omega_k = exp(-4 eps_c alpha_ad TL(G_k)),
 * G_k = U_k U_k^dag - U_{k-1}^dag U_{k-1}, all sites from the same links) with
 * the adaptive alpha_ad = alpha / D of the same section (D_0 = 1, D_1 = Tr UU^dag
 * per link, D_2 = mean |f_ak|).  The model reduces to one link, so the exact
 * equilibrium is <Tr P / 2> = I_2(beta) / I_1(beta).  FP64 only.
 *
 * Host (and device) link layout: links[((c * n_links + k) * 4 + 2 i + j) * 2 +
 * {0: re, 1: im}], 8 doubles per link.  Noise: Philox4x32-10 with key = seed
 * and counter (link k, CL step, chain c, tag 2 << 16 | draw), draws 0 and 1
 * giving eta_1..eta_3; the start of cl_chain_init uses tag 3 (draws 0..3).
 * ------------------------------------------------------------------------ */
typedef struct cl_chain cl_chain;

typedef struct {
    int32_t n_links;     /* 1 .. 1024 */
    int32_t n_chains;    /* 1 .. 2^24 */
    double beta_re, beta_im;
    uint64_t seed;
    int32_t obs_cap;     /* steps of per-step record kept on the device (may be 0) */
} cl_chain_desc;

/* one chain after the last call (see cl_chain_run for the sums) */
typedef struct {
    int64_t step;        /* CL steps done */
    int32_t status;      /* 0, or 1 once a drift or norm was not finite (chain frozen) */
    int32_t pad;
    double L[2];         /* Polyakov loop Tr(U_0 ... U_{n-1}) / 2 */
    double d;            /* (1/2n) sum_k Tr(U U^dag - 1), after cooling */
    double d_pre;        /* the same before the cooling of the last step */
    double eps, kmax;    /* of the last CL step */
    double sum_L[2];     /* Langevin-time integrals sum_n eps_n L_n and sum_n eps_n d_n over */
    double sum_d;        /* the steps of the last cl_chain_run (an adaptive step visits */
                         /* configurations of small eps more often: the time average     */
                         /* sum / t_sum is the equilibrium estimate, the plain step      */
                         /* average is not) */
    double n_sum;        /* steps in those sums */
    double t_sum;        /* their Langevin time sum_n eps_n */
} cl_chain_obs;

/* Device bytes for the chains, their control blocks and obs_cap steps of record.
 * CL_EINVAL: n_links outside 1..1024, n_chains outside 1..2^24, obs_cap < 0, beta not
 * finite. */
cl_status cl_chain_bytes(const cl_chain_desc* desc, size_t* device_bytes);
/* dev_buf: caller-owned, at least cl_chain_bytes, 256-byte aligned; the stream is
 * the caller's.  The chains start at the identity (a cold start). */
cl_status cl_chain_create(const cl_chain_desc* desc, void* dev_buf, size_t buf_bytes, void* hip_stream,
                          cl_chain** out);
cl_status cl_chain_destroy(cl_chain* ch);
/* U_k = exp(i sigma_a (x_a + i y_a)), x_a ~ N(0, sigma_x), y_a ~ N(0, sigma_y);
 * resets every control block (step 0, adaptive bound unset, status 0). */
cl_status cl_chain_init(cl_chain* ch, double sigma_x, double sigma_y);
/* host copies of all links (n_doubles = n_chains * n_links * 8); set_links
 * resets the control blocks like cl_chain_init.  Synchronous. */
cl_status cl_chain_set_links(cl_chain* ch, const double* host, size_t n_doubles);
cl_status cl_chain_get_links(cl_chain* ch, double* host, size_t n_doubles);
/* n_steps CL steps of every chain, each followed by cool->n_steps cooling
 * steps (cool may be NULL: none) and a measurement, in one launch (a chain
 * is owned by T threads of a workgroup, T the smallest power of two with
 * PT T >= n_links, PT = 2 up to 512 links and 4 above, and its links stay in
 * registers between steps).  Adaptive step
 * eps = min(eps0, B/K_max) per chain, B fixed on its first step (drift_bound if
 * > 0).  record != 0 keeps (Re L, Im L, d, eps, kmax, d_pre) of every step in
 * the device record (n_steps <= obs_cap), read with cl_chain_record.  A chain
 * whose drift, norm or loop turns non-finite gets status 1, keeps the links it
 * had when the call started and is not advanced again; the other chains are
 * not affected.  Asynchronous on the stream.
 * CL_EINVAL: n_steps < 0, record with n_steps > obs_cap, bad eps0/cooling. */
cl_status cl_chain_run(cl_chain* ch, const cl_step_desc* step, const cl_cool_desc* cool, int n_steps, int record);
/* cooling only: cool->n_steps steps of every chain (eq. (eq:24)), then L and d. */
cl_status cl_chain_cool(cl_chain* ch, const cl_cool_desc* cool);
/* the drift Khat_k = i beta TL(U_k ... U_{k-1}) of every link (host, same layout
 * as the links) and, if kmax != NULL, K_max of every chain.  Synchronous;
 * overwrites the device record. */
cl_status cl_chain_drift(cl_chain* ch, double* host_K, size_t n_doubles, double* kmax);
/* every chain's observables (cap >= n_chains); recomputes L and d from the
 * current links.  Synchronous. */
cl_status cl_chain_measure(cl_chain* ch, cl_chain_obs* out, int cap);
/* the per-step record of the last recording cl_chain_run: n_steps x n_chains x 6. */
cl_status cl_chain_record(cl_chain* ch, double* host, size_t n_doubles);

/* Message for the last failing call on this thread ("" if none). */
const char* cl_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CLGC_H */
