// chain.hpp -- the SU(2) Polyakov chain workload (section "Adaptive gauge
// cooling in the SU(2) Polyakov chain model"): many independent chains of n
// SL(2,C) links, S = -(beta/2) Tr(U_0 U_1 ... U_{n-1}) with complex beta,
// evolved by complex Langevin with adaptive gauge cooling.
//
// Device layout (equal to the host layout, so that set/get are copies):
//   links  [chain][k][8] doubles: link k of a chain as a row-major 2x2
//          complex matrix, (re, im) interleaved (64 B);
//   ctrl   [chain] ChainCtrl;
//   obs    [step][chain][kChainObs] doubles, the per-step record of the
//          last cl_chain_run call (capacity obs_cap steps);
//   K      [chain][k][8], the drift written by cl_chain_drift (aliases obs).
#pragma once
#include <stdint.h>

namespace clgc {

constexpr int kChainBlock = 256;      // most threads per chain (and per workgroup)
// links per thread: two up to kChainShortMax links (two waves per SIMD), four
// for longer chains (one wave, fewer threads to scan over)
constexpr int kChainShortPT = 2, kChainLongPT = 4;
constexpr int kChainShortMax = kChainBlock * kChainShortPT;
constexpr int kChainMaxLinks = kChainBlock * kChainLongPT;
constexpr int kChainObs = 6;          // Re L, Im L, d, eps, kmax, d before cooling

// Philox stream tags of the chain (counter word 3 = tag << 16 | draw)
constexpr uint32_t kChainTagNoise = 2u;
constexpr uint32_t kChainTagInit = 3u;

struct ChainCtrl {
    int64_t step;       // CL steps done
    double bound;       // adaptive-step bound B (0: fixed at the next step)
    int status;         // 0 ok, 1 non-finite (the chain is no longer advanced)
    int pad;
    double eps, kmax;   // of the last CL step
    double d_pre, d;    // distance after the last update, after its cooling
    double L_re, L_im;  // Polyakov loop Tr(U_0 ... U_{n-1}) / 2 after the last step
    // eps-weighted sums (Langevin-time integrals) of L and d, the step count and
    // the Langevin time, over the steps of the last run call
    double sum_L_re, sum_L_im, sum_d, sum_n, sum_t;
};

// everything one launch needs, passed by value in the kernel arguments
struct ChainArgs {
    int n;              // links per chain, 1 .. kChainMaxLinks
    int n_chains;
    double beta_re, beta_im;
    uint64_t seed;
    double* links;
    ChainCtrl* ctrl;
    double* obs;        // per-step record (nullptr: none)
    int obs_cap;
    int record;         // write obs in this launch
    double* K;          // drift output (cl_chain_drift)
    double eps0, drift_bound;
    int adaptive;
    int n_cool;
    double eps_c, alpha;
    int mode;           // cl_alpha_mode: 0 D_0, 1 D_1, 2 D_2
};

}  // namespace clgc
