// kernels.hip -- gfx950 kernels of the complex Langevin + adaptive gauge
// cooling hot path.  No MFMA: the work is 3x3 complex products, which do not
// map onto dense matrix-core tiles; everything is FP64 (or FP32) VALU code
// with coalesced complex-element SoA loads (see lattice.hpp).
//
// Every kernel walks logical blocks of a batch of runs (a single lattice is a
// batch of one).  Per-run scalars (max drift, unitarity norm, observables) are
// reduced deterministically: each logical block stores its partial and a
// one-block-per-run finalize kernel sums them in a fixed order and updates the
// run's control block on the device, so no host round trip sits between the
// kernels of a step and no grid-wide fence is needed inside a sweep.
#include "engine.hpp"
#include "host.hpp"
#include "reduce.hpp"

#include <hip/hip_ext.h>
#include <math.h>

#include <cstring>
#include <mutex>

namespace clgc {

// ---------------------------------------------------------------------------
// reductions

// Sum / max over the wavefront, the same bits in every lane (reduce.hpp).
__device__ __forceinline__ double wave_sum(double v) { return group_reduce<false>(v, 64); }

__device__ __forceinline__ double wave_max(double v) { return group_reduce<true>(v, 64); }

// Sum (or max) of NV values over the block; the result is valid in thread 0.
// The order of operations is fixed, so the result depends on the inputs only.
template <int NV, bool MAX = false>
__device__ __forceinline__ void block_reduce(double (&v)[NV], double* lds /* NV*4 */)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const double w = MAX ? wave_max(v[j]) : wave_sum(v[j]);
        if (lane == 0) lds[j * 4 + wave] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            v[j] = MAX ? fmax(fmax(lds[j * 4], lds[j * 4 + 1]), fmax(lds[j * 4 + 2], lds[j * 4 + 3]))
                       : (lds[j * 4] + lds[j * 4 + 1]) + (lds[j * 4 + 2] + lds[j * 4 + 3]);
        }
    }
    __syncthreads();
}

// Store this logical block's partials (thread 0 holds v[] from block_reduce).
template <int NV>
__device__ __forceinline__ void store_partials(const RunArgs& ra, int kind, int lb, const double (&v)[NV])
{
    if (threadIdx.x == 0) {
        const int nblk = ra.nblk[kind];
#pragma unroll
        for (int j = 0; j < NV; ++j) ra.part[j * nblk + lb] = v[j];
    }
}

// Partials of a recorded step, FP64 with a theta term (the measurement
// rides on the step's own clover kernel): value j of logical block b at
// part[j * nblk[KIND_PLANE] + b].  The clover kernel leaves j = 1..4 (Tr P
// re / im, Tr P^-1 re / im) and 5 (link norms), k_record_charge j = 6, 7 (the
// clover bracket re / im, one block per 256 sites, fewer than the clover's
// blocks); j = 0 stays the drift's own K_max partial, written in between.
__device__ __forceinline__ double* record_partial(const RunArgs& ra, int j)
{
    return ra.part + (size_t)j * ra.nblk[KIND_PLANE];
}

// Fixed-order sum (or max) of n partials at p_in; valid in thread 0.  Each
// thread issues eight independent loads before combining them, so the gather
// costs a few memory round trips rather than one per loop trip.
template <bool MAX = false>
__device__ __forceinline__ double gather_values(const double* p_in, int n, double* lds)
{
    typedef __attribute__((address_space(1))) const double* gcd;
    const gcd p = (gcd)p_in;
    double acc = 0.0;
    for (int base = 0; base < n; base += 8 * kBlock) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = base + u * kBlock + (int)threadIdx.x;
            v[u] = i < n ? p[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = MAX ? (isnan(v[u]) || isnan(acc) ? NAN : fmax(acc, v[u])) : acc + v[u];
    }
    double r[1] = {acc};
    block_reduce<1, MAX>(r, lds);
    return r[0];
}

// partial j of every logical block of one kind
template <bool MAX = false>
__device__ __forceinline__ double gather_partials(const RunArgs& ra, int kind, int j, double* lds)
{
    const int nblk = ra.nblk[kind];
    return gather_values<MAX>(ra.part + (size_t)j * nblk, nblk, lds);
}

// n <= kMaxCoolBlocks partials (the cooling step's unitarity norm, the D_2
// gradient norm) summed by one wavefront on its own: each lane adds its values in index order, then a
// butterfly; every wavefront of every block gets the same value, with no
// barrier, so the sum can wait until a wavefront's link loads are in flight
__device__ __forceinline__ double wave_sum_of(const double* p_in, int n)
{
    typedef __attribute__((address_space(1))) const double* gcd;
    const gcd p = (gcd)p_in;
    const int lane = (int)threadIdx.x & 63;
    double acc = 0.0;
    for (int base = 0; base < n; base += 8 * 64) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = base + u * 64 + lane;
            v[u] = i < n ? p[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    return wave_sum(acc);
}

__device__ __forceinline__ double wave_cool_sum(const RunArgs& ra) { return wave_sum_of(ra.cpart, ra.nblk[KIND_COOL]); }

// ---------------------------------------------------------------------------
// logical-block iteration

// Logical blocks are dealt to launch slots by logical_block (lattice.hpp), so
// that each XCD works through a contiguous range of the lattice.  Grids are
// launched as a multiple of eight (or grid-stride with a multiple-of-eight
// stride), so the XCD of a logical slot never changes.
// The body between CLGC_FOR_BLOCKS and CLGC_END_BLOCKS runs once per logical
// block (ra, lb, tid); it is written once, as a lambda, and each kernel
// instance inlines it into one of two loops: FAST, a single run whose RunArgs
// sit in the kernel arguments, or a batch, where the run of each block is
// looked up in the device tables.
#define CLGC_FOR_BLOCKS(KIND)                                                  \
    constexpr int kind_ = (KIND);                                              \
    auto body_ = [&](const RunArgs& ra, const int lb) __attribute__((always_inline)) { \
        const int tid = lb * kBlock + (int)threadIdx.x;                        \
        (void)tid;

#define CLGC_END_BLOCKS                                                        \
    };                                                                         \
    if constexpr (FAST) {                                                      \
        const int total_ = ka.one.nblk[kind_];                                 \
        const int q_ = (total_ + kXcds - 1) / kXcds;                           \
        for (int gb0_ = blockIdx.x; gb0_ < kXcds * q_; gb0_ += gridDim.x) {    \
            const int gb_ = logical_block(gb0_, total_);                       \
            if (gb_ < total_) body_(ka.one, gb_);                              \
        }                                                                      \
    } else {                                                                   \
        /* the batch tables do not change during a launch: read through the   \
           constant address space, like the kernel arguments (scalar loads,   \
           and no re-reads of RunArgs fields after every store of the body) */ \
        const __attribute__((address_space(4))) BatchHdr* hdr_ =               \
            (const __attribute__((address_space(4))) BatchHdr*)ka.hdr;          \
        const __attribute__((address_space(4))) RunArgs* runs4_ =              \
            (const __attribute__((address_space(4))) RunArgs*)ka.runs;          \
        const int total_ = hdr_->total[kind_];                                 \
        const int q_ = (total_ + kXcds - 1) / kXcds;                           \
        for (int gb0_ = blockIdx.x; gb0_ < kXcds * q_; gb0_ += gridDim.x) {    \
            const int gb_ = logical_block(gb0_, total_);                       \
            if (gb_ >= total_) continue;                                       \
            const int run_ = find_run(hdr_, kind_, gb_);                       \
            body_(*(const RunArgs*)&runs4_[run_], gb_ - hdr_->begin[kind_][run_]); \
        }                                                                      \
    }


template <typename T>
__device__ __forceinline__ mat3<T> ldU(const RunArgs& ra, int mu, const Site& s)
{
    return load_mat((const cx<T>*)ra.U, link_off(ra, mu, s), 4 * ra.V);
}

// ---------------------------------------------------------------------------
// initial configuration

template <typename T, bool FAST>
__global__ void __launch_bounds__(kBlock) k_init(const KArgs ka,
                                                 int perturbed, double sx, double sy)
{
    __shared__ double lds[8];
    CLGC_FOR_BLOCKS(KIND_LINK)
    double un = 0.0;
    if (tid < 4 * ra.V) {
        int mu, p, h;
        link_decompose(ra, tid, mu, p, h);
        mat3<double> U = m_id<double>();
        if (perturbed) {
            const Site s = site_coords(ra, p, h);
            const uint32_t c0 = (uint32_t)(4 * site_lex(ra, s) + mu);
            double xr[8], yr[8];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                double n0, n1;
                normal_pair<double>(ra.seed, c0, 0u, (uint32_t)j, kStreamInit, n0, n1);
                xr[2 * j] = sx * n0;
                xr[2 * j + 1] = sx * n1;
                normal_pair<double>(ra.seed, c0, 0u, (uint32_t)(j + 4), kStreamInit, n0, n1);
                yr[2 * j] = sy * n0;
                yr[2 * j + 1] = sy * n1;
            }
            // A = i sum_a (x_a + i y_a) lambda_a = sum_a (-y_a + i x_a) lambda_a
            cx<double> c[8];
#pragma unroll
            for (int a = 0; a < 8; ++a) c[a] = {-yr[a], xr[a]};
            const double r3 = 0.57735026918962576451;  // 1/sqrt(3)
            mat3<double> A;
            A.e[0][0] = c[2] + r3 * c[7];
            A.e[1][1] = r3 * c[7] - c[2];
            A.e[2][2] = (-2.0 * r3) * c[7];
            // lambda_1, lambda_2: (0,1) = c1 - i c2, (1,0) = c1 + i c2
            A.e[0][1] = c[0] + cx<double>{c[1].im, -c[1].re};
            A.e[1][0] = c[0] + cx<double>{-c[1].im, c[1].re};
            A.e[0][2] = c[3] + cx<double>{c[4].im, -c[4].re};
            A.e[2][0] = c[3] + cx<double>{-c[4].im, c[4].re};
            A.e[1][2] = c[5] + cx<double>{c[6].im, -c[6].re};
            A.e[2][1] = c[5] + cx<double>{-c[6].im, c[6].re};
            U = m_exp_traceless(A);
        }
        const mat3<T> Ut = m_cast_from<T>(U);
        store_mat((cx<T>*)ra.U, tid, 4 * ra.V, Ut);
        un = (double)m_norm2(Ut);
    }
    double v[1] = {un};
    block_reduce<1>(v, lds);
    store_partials(ra, KIND_LINK, lb, v);
    CLGC_END_BLOCKS
}

// unitarity norm of the current links (after links are written from the host)
template <typename T, bool FAST>
__global__ void __launch_bounds__(kBlock) k_unorm(const KArgs ka)
{
    __shared__ double lds[8];
    CLGC_FOR_BLOCKS(KIND_LINK)
    double un = 0.0;
    if (tid < 4 * ra.V) un = (double)m_norm2(load_mat((const cx<T>*)ra.U, tid, 4 * ra.V));
    double v[1] = {un};
    block_reduce<1>(v, lds);
    store_partials(ra, KIND_LINK, lb, v);
    CLGC_END_BLOCKS
}

// host AoS (double, lexicographic) <-> device SoA (T, checkerboard)
template <typename T, bool FAST>
__global__ void __launch_bounds__(kBlock) k_unpack(const KArgs ka,
                                                   const double* __restrict__ aos)
{
    CLGC_FOR_BLOCKS(KIND_LINK)
    if (tid < 4 * ra.V) {
        int mu, p, h;
        link_decompose(ra, tid, mu, p, h);
        const Site s = site_coords(ra, p, h);
        const double* src = aos + ((size_t)site_lex(ra, s) * 4 + mu) * 18;
        mat3<T> m;
#pragma unroll
        for (int e = 0; e < 9; ++e) m.e[e / 3][e % 3] = {T(src[2 * e]), T(src[2 * e + 1])};
        store_mat((cx<T>*)ra.U, tid, 4 * ra.V, m);
    }
    CLGC_END_BLOCKS
}

template <typename T, bool FAST>
__global__ void __launch_bounds__(kBlock) k_pack(const KArgs ka,
                                                 const void* __restrict__ field, double* __restrict__ aos)
{
    CLGC_FOR_BLOCKS(KIND_LINK)
    if (tid < 4 * ra.V) {
        int mu, p, h;
        link_decompose(ra, tid, mu, p, h);
        const Site s = site_coords(ra, p, h);
        double* dst = aos + ((size_t)site_lex(ra, s) * 4 + mu) * 18;
        const mat3<T> m = load_mat((const cx<T>*)field, tid, 4 * ra.V);
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            dst[2 * e] = (double)m.e[e / 3][e % 3].re;
            dst[2 * e + 1] = (double)m.e[e / 3][e % 3].im;
        }
    }
    CLGC_END_BLOCKS
}

// ---------------------------------------------------------------------------
// clover field: F_{mu nu}(x) = sum over the four counter-clockwise leaves L at
// x in the (mu, nu) plane of (L - L^{-1})

template <typename T, bool FAST>
__global__ void __launch_bounds__(kBlock, 2) k_clover(const KArgs ka,
                                                   int only_theta, int record)
{
    __shared__ double lds[5 * 4];
    CLGC_FOR_BLOCKS(KIND_PLANE)
    // record (FP64): the first leaf is the plaquette of the plane at x; with
    // the norm of one of the site's links in four of the six planes (mu's
    // link in 01, 12, 23, the 3-link in 03) the blocks cover every plaquette
    // and every link once
    constexpr bool kRec = sizeof(T) == 8;
    double rv[5] = {0, 0, 0, 0, 0};
    // logical block -> (region of 256 half-indices, plane, parity), regions major
    const int P = (lb % 12) >> 1, p = lb & 1;
    const int h = xcd_region_order(ra, lb / 12, ra.nblk[KIND_PLANE] / 12) * kBlock + (int)threadIdx.x;
    // in a batched step only the runs with a theta term need the field
    if (h < ra.Vh && !(only_theta && !ra.has_theta)) {
        const int tid_f = P * ra.V + p * ra.Vh + h;
        const int mu = P < 3 ? 0 : (P < 5 ? 1 : 2);
        const int nu = P < 3 ? P + 1 : (P < 5 ? P - 1 : 3);
        const Site x = site_coords(ra, p, h);
        const Site xpm = site_move(ra, x, mu, +1), xpn = site_move(ra, x, nu, +1);
        const Site xmm = site_move(ra, x, mu, -1), xmn = site_move(ra, x, nu, -1);
        const Site xmmpn = site_move(ra, xmm, nu, +1), xmmmn = site_move(ra, xmm, nu, -1);
        const Site xmnpm = site_move(ra, xmn, mu, +1);
        mat3<T> F, L;
        if constexpr (sizeof(T) == 8) {
            // FP64: the scheduling barriers keep the next leaf's loads from being
            // hoisted, which holds two waves per SIMD without spilling; a link
            // shared with the next leaf stays in registers (U_nu(x), U_mu(x-mu),
            // U_nu(x-nu)), the one shared by the first and the last leaf,
            // U_mu(x), is loaded again (a cache hit)
            // U_mu(x) U_nu(x+mu) [U_nu(x) U_mu(x+nu)]^{-1}
            mat3<T> S = ldU<T>(ra, nu, x);
            const mat3<T> Umx = ldU<T>(ra, mu, x);
            L = (Umx * ldU<T>(ra, nu, xpm)) * m_adj(S * ldU<T>(ra, mu, xpn));
            if (kRec && record) {
                const cx<T> tp = m_tr(L);
                const cx<T> ti = (L.e[1][1] * L.e[2][2] - L.e[1][2] * L.e[2][1]) +
                                 (L.e[0][0] * L.e[2][2] - L.e[0][2] * L.e[2][0]) +
                                 (L.e[0][0] * L.e[1][1] - L.e[0][1] * L.e[1][0]);
                rv[0] = tp.re;
                rv[1] = tp.im;
                rv[2] = ti.re;
                rv[3] = ti.im;
                if (P == 0 || P == 3 || P == 5) rv[4] = m_norm2(Umx);
                else if (P == 2) rv[4] = m_norm2(S);
            }
            F = L - m_adj(L);
            __builtin_amdgcn_sched_barrier(0);
            // U_nu(x) [U_nu(x-mu) U_mu(x-mu+nu)]^{-1} U_mu(x-mu)
            {
                const mat3<T> Umm = ldU<T>(ra, mu, xmm);
                L = S * (m_adj(ldU<T>(ra, nu, xmm) * ldU<T>(ra, mu, xmmpn)) * Umm);
                S = Umm;
            }
            F = F + (L - m_adj(L));
            __builtin_amdgcn_sched_barrier(0);
            // [U_nu(x-mu-nu) U_mu(x-mu)]^{-1} U_mu(x-mu-nu) U_nu(x-nu)
            {
                const mat3<T> Unn = ldU<T>(ra, nu, xmn);
                L = m_adj(ldU<T>(ra, nu, xmmmn) * S) * (ldU<T>(ra, mu, xmmmn) * Unn);
                S = Unn;
            }
            F = F + (L - m_adj(L));
            __builtin_amdgcn_sched_barrier(0);
            // U_nu(x-nu)^{-1} U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^{-1}
            L = m_adj(S) * ((ldU<T>(ra, mu, xmn) * ldU<T>(ra, nu, xmnpm)) * m_adj(ldU<T>(ra, mu, x)));
            F = F + (L - m_adj(L));
        } else {
            const mat3<T> Umx = ldU<T>(ra, mu, x), Unx = ldU<T>(ra, nu, x);
            const mat3<T> Umxmm = ldU<T>(ra, mu, xmm), Unxmn = ldU<T>(ra, nu, xmn);
            // U_mu(x) U_nu(x+mu) [U_nu(x) U_mu(x+nu)]^{-1}
            L = (Umx * ldU<T>(ra, nu, xpm)) * m_adj(Unx * ldU<T>(ra, mu, xpn));
            F = L - m_adj(L);
            // U_nu(x) [U_nu(x-mu) U_mu(x-mu+nu)]^{-1} U_mu(x-mu)
            L = Unx * (m_adj(ldU<T>(ra, nu, xmm) * ldU<T>(ra, mu, xmmpn)) * Umxmm);
            F = F + (L - m_adj(L));
            // [U_nu(x-mu-nu) U_mu(x-mu)]^{-1} U_mu(x-mu-nu) U_nu(x-nu)
            L = m_adj(ldU<T>(ra, nu, xmmmn) * Umxmm) * (ldU<T>(ra, mu, xmmmn) * Unxmn);
            F = F + (L - m_adj(L));
            // U_nu(x-nu)^{-1} U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^{-1}
            L = m_adj(Unxmn) * ((ldU<T>(ra, mu, xmn) * ldU<T>(ra, nu, xmnpm)) * m_adj(Umx));
            F = F + (L - m_adj(L));
        }
        store_mat((cx<T>*)ra.F, tid_f, 6 * ra.V, F);
    }
    if (kRec && record) {
        block_reduce<5>(rv, lds);
        if (threadIdx.x == 0)
            for (int j = 0; j < 5; ++j) record_partial(ra, 1 + j)[lb] = rv[j];
    }
    CLGC_END_BLOCKS
}

// ---------------------------------------------------------------------------
// drift
//
// For link (x, mu) each of the six loops through it is e0 e1 e2 e3 with
// corners d0 = x, d1 = x+mu, d2 = x+mu+s nu, d3 = x+s nu (e0 = U_mu(x)) and
// staple P = e1 e2 e3 (d1 -> d0).  With X_k the dual clover matrix of the
// loop's plane at d_k, the theta term inserts X_k at each corner of the loop
// and of its inverse in turn:
//   I = X1 e1e2e3 + e1 X2 e2e3 + e1e2 X3 e3 + e1e2e3 X0,
//   J = X0 e3'e2'e1' + e3' X3 e2'e1' + e3'e2' X2 e1' + e3'e2'e1' X1
// (' the inverse), and
//   Khat = TL( e0 sum (cb P + cts I) - sum (cb P' - cts J) e0' ),
// cb = i beta/3, cts = sigma theta/(128 pi^2), sigma = s sign(nu - mu) times
// the sign of the dual plane.  With the paths R_1 = 1, R_2 = e1, R_3 = e1 e2
// from d1 to the corners and the transported clover Q = sum_k R_k X_k R_k^-1,
//   I = Q P + P X0,    J = X0 P' + P' Q,
// so one walk along the staple gives both chains.  Inverses are adjugates
// (the inverse on SL(3,C)); adj(AB) = adj(B) adj(A) makes P' = adj(P) exact.
// Q is summed nested, X1 + e1 (X2 + e2 X3 e2^-1) e1^-1, with e1^-1 and e2^-1
// from the raw links' adjugates and determinants, which keeps both identities
// exact for any links.  One lane per link loads each of a loop's seven
// matrices once.

// 1 / det M from the first row of M and the first column of adj(M)
template <typename T>
__device__ __forceinline__ cx<T> inv_det(const mat3<T>& M, const mat3<T>& Ma)
{
    const cx<T> d = cfma(M.e[0][2], Ma.e[2][0], cfma(M.e[0][1], Ma.e[1][0], M.e[0][0] * Ma.e[0][0]));
    const T r = T(1) / fma(d.re, d.re, d.im * d.im);
    return {d.re * r, -d.im * r};
}

// A lane's accumulator matrix kept in LDS: 18 values in a column of its own
// (acc[j * kBlock + thread]), so no lane reads another's and no barrier is
// needed.
template <typename T>
__device__ __forceinline__ void lds_acc_add(T* acc, const mat3<T>& m)
{
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        T* c = acc + (2 * e) * kBlock + threadIdx.x;
        c[0] += m.e[e / 3][e % 3].re;
        c[kBlock] += m.e[e / 3][e % 3].im;
    }
}
template <typename T>
__device__ __forceinline__ mat3<T> lds_acc_get(const T* acc)
{
    mat3<T> m;
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        const T* c = acc + (2 * e) * kBlock + threadIdx.x;
        m.e[e / 3][e % 3] = {c[0], c[kBlock]};
    }
    return m;
}

// One loop (nu, s = S) of the theta drift with the lane's A and B in LDS:
// the loop's terms cb P + Q P + P X0 and -cb P' + P' Q + X0 P' are formed in
// registers and added to the accumulators there.  The products are those of
// the walk in k_drift, in the same order.
template <typename T, int S>
__device__ __forceinline__ void theta_loop_lds(const RunArgs& ra, const cx<T>* __restrict__ Ub,
                                               const cx<T>* __restrict__ Fb, int fo, const Site& x,
                                               const Site& d1, int mu, int nu, int p, int h, cx<T> cb, cx<T> mcb,
                                               cx<T> cts, T* accA, T* accB)
{
    const int us = 4 * ra.V, fs = 6 * ra.V;
    const Site d3 = site_move(ra, x, nu, S);
    const Site d2 = site_move(ra, d1, nu, S);
    const mat3<T> ub = load_mat(Ub, link_off(ra, mu, d3), us);
    const mat3<T> X3 = load_mat(Fb, fo + link_off(ra, 0, d3), fs);
    const mat3<T> e2 = m_adj(ub);
    mat3<T> Y = (e2 * X3) * ub;
    Y = m_scale(Y, inv_det(ub, e2)) + load_mat(Fb, fo + link_off(ra, 0, d2), fs);
    __builtin_amdgcn_sched_barrier(0);
    const mat3<T> ua = load_mat(Ub, link_off(ra, nu, S > 0 ? d1 : d2), us);
    const mat3<T> ua_adj = m_adj(ua);
    const cx<T> ida = inv_det(ua, ua_adj);
    const mat3<T>& e1 = S > 0 ? ua : ua_adj;
    const mat3<T>& e1i = S > 0 ? ua_adj : ua;
    const mat3<T> R = e1 * e2;
    mat3<T> Q = m_scale((e1 * Y) * e1i, ida) + load_mat(Fb, fo + link_off(ra, 0, d1), fs);
    __builtin_amdgcn_sched_barrier(0);
    mat3<T> e3 = load_mat(Ub, link_off(ra, nu, S > 0 ? x : d3), us);
    if (S > 0) e3 = m_adj(e3);
    const mat3<T> Pm = R * e3;
    Q = m_scale(Q, cts);
    const mat3<T> X0s = m_scale(load_mat(Fb, fo + p * ra.Vh + h, fs), cts);
    mat3<T> a = m_scale_i(Pm, cb.im);
    m_mac(a, Q, Pm);
    m_mac(a, Pm, X0s);
    lds_acc_add(accA, a);
    const mat3<T> Pa = m_adj(Pm);
    mat3<T> b = m_scale_i(Pa, mcb.im);
    m_mac(b, Pa, Q);
    m_mac(b, X0s, Pa);
    lds_acc_add(accB, b);
}

// FP64 with the theta term keeps each lane's A and B in LDS (36 doubles a
// lane, 72 KB a block): the walk then fits in 256 registers and two waves
// run per SIMD, where A and B in registers (about 440 with the walk) allow
// one.  FP32 (two waves with them in registers, three in LDS, at the same
// speed: it is bound by its arithmetic) and the Wilson-only drift keep them
// in registers.
template <typename T, bool THETA, bool FAST>
__global__ void __launch_bounds__(kBlock, 2) k_drift(const KArgs ka)
{
    __shared__ double lds[8];
    constexpr bool kAccLds = sizeof(T) == 8 && THETA;
    // FP64 forms e^-1 = adj(e) / det e, exact for any links.  FP32 links are
    // in SL(3,C) to their rounding (|det - 1| ~ 1e-7, renormalised in FP64
    // at every update), so the FP32 walk takes adj(e) itself: that changes
    // its drift by as much, far inside the mixed path's tolerance, and saves
    // the two reciprocals and scalings of every loop (the FP32 drift is
    // bound by instruction issue)
    constexpr bool kExactInverse = sizeof(T) == 8;
    __shared__ T accl[kAccLds ? 36 * kBlock : 1];
    CLGC_FOR_BLOCKS(KIND_DRIFT)
    // logical block -> (region of 256 half-indices, direction, parity): the eight
    // (mu, parity) blocks of a region are adjacent, so one XCD covers all the
    // links of a contiguous slab of sites (its regions in xcd_region_order)
    const int mu = (lb & 7) >> 1, p = lb & 1;
    const int h = xcd_region_order(ra, lb >> 3, ra.nblk[KIND_DRIFT] >> 3) * kBlock + (int)threadIdx.x;
    const int l = (mu * 2 + p) * ra.Vh + h;
    double kn2 = 0.0;
    if (h < ra.Vh) {
        const Site x = site_coords(ra, p, h);
        const Site d1 = site_move(ra, x, mu, +1);
        const cx<T> cb = {T(0), T(ra.beta / 3.0)};
        const cx<T> mcb = {T(0), T(-ra.beta / 3.0)};
        const double tn = 1.0 / (128.0 * M_PI * M_PI);
        const cx<T> ct = {T(ra.th_re * tn), T(ra.th_im * tn)};
        const cx<T>* __restrict__ Ub = (const cx<T>*)ra.U;
        const cx<T>* __restrict__ Fb = (const cx<T>*)ra.F;
        const int us = 4 * ra.V, fs = 6 * ra.V;
        // block-uniform: a batch can mix runs with and without a theta term
        const bool th = THETA && ra.has_theta;
        // A = sum (cb P + cts I),  B = sum (cts J - cb P'):  Khat = TL(e0 A + B e0')
        mat3<T> A = m_zero<T>(), B = m_zero<T>();
        if (kAccLds && th) {
            T* accA = accl;
            T* accB = accl + 18 * kBlock;
#pragma unroll
            for (int j = 0; j < 18; ++j) accA[j * kBlock + threadIdx.x] = accB[j * kBlock + threadIdx.x] = T(0);
#pragma unroll 1
            for (int nn = 0; nn < 3; ++nn) {
                const int nu = nn + (nn >= mu);
                const int Pl = mu < nu ? plane_of(mu, nu) : plane_of(nu, mu);
                const int fo = dual_plane(Pl) * ra.V;
                const T sig = T((nu > mu ? 1 : -1) * dual_sign(Pl));
                theta_loop_lds<T, 1>(ra, Ub, Fb, fo, x, d1, mu, nu, p, h, cb, mcb, cx<T>{sig * ct.re, sig * ct.im},
                                     accA, accB);
                __builtin_amdgcn_sched_barrier(0);
                theta_loop_lds<T, -1>(ra, Ub, Fb, fo, x, d1, mu, nu, p, h, cb, mcb,
                                      cx<T>{-sig * ct.re, -sig * ct.im}, accA, accB);
                __builtin_amdgcn_sched_barrier(0);
            }
            A = lds_acc_get(accA);
            B = lds_acc_get(accB);
        } else
#pragma unroll 1
        for (int nn = 0; nn < 3; ++nn) {
            const int nu = nn + (nn >= mu);
            const int Pl = mu < nu ? plane_of(mu, nu) : plane_of(nu, mu);
            const int fo = dual_plane(Pl) * ra.V;
            // unrolled over the sign: a compile-time s selects the raw link or its
            // adjugate
#pragma unroll
            for (int si = 0; si < 2; ++si) {
                const int s = si ? -1 : 1;
                const Site d3 = site_move(ra, x, nu, s);
                const Site d2 = site_move(ra, d1, nu, s);
                // e1 = U_nu(d1) (s>0) or U_nu(d2)^-1, e2 = U_mu(d3)^-1, e3 = U_nu(x)^-1 (s>0) or U_nu(d3)
                const int oa = link_off(ra, nu, s > 0 ? d1 : d2);
                if (!th) {
                    const mat3<T> ua = load_mat(Ub, oa, us);
                    const mat3<T> e1 = s > 0 ? ua : m_adj(ua);
                    mat3<T> Pm = e1 * m_adj(load_mat(Ub, link_off(ra, mu, d3), us));
                    mat3<T> e3 = load_mat(Ub, link_off(ra, nu, s > 0 ? x : d3), us);
                    if (s > 0) e3 = m_adj(e3);
                    Pm = Pm * e3;
                    m_axpy_i(A, cb.im, Pm);
                    m_axpy_i(B, mcb.im, m_adj(Pm));
                } else {
                    const T sig = T(s * (nu > mu ? 1 : -1) * dual_sign(Pl));
                    const cx<T> cts = {sig * ct.re, sig * ct.im};
                    // Q = X1 + e1 X2 e1^-1 + (e1 e2) X3 (e1 e2)^-1 = X1 + e1 Y e1^-1 with
                    // Y = X2 + e2 X3 e2^-1.  Inverses from the raw links: e2 =
                    // adj(ub) has e2^-1 = ub / det ub, and e1^-1 is adj(ua) / det ua
                    // (s > 0) or ua / det ua (s < 0, e1 = adj(ua)); exact for any
                    // links, not only det U = 1 (the determinants only in FP64,
                    // kExactInverse).
                    const mat3<T> ub = load_mat(Ub, link_off(ra, mu, d3), us);
                    const mat3<T> X3 = load_mat(Fb, fo + link_off(ra, 0, d3), fs);
                    const mat3<T> e2 = m_adj(ub);
                    mat3<T> Y = (e2 * X3) * ub;
                    if constexpr (kExactInverse) Y = m_scale(Y, inv_det(ub, e2));
                    Y = Y + load_mat(Fb, fo + link_off(ra, 0, d2), fs);
                    const mat3<T> ua = load_mat(Ub, oa, us);
                    const mat3<T> ua_adj = m_adj(ua);
                    mat3<T> e1, e1i;
                    if (s > 0) {
                        e1 = ua;
                        e1i = ua_adj;
                    } else {
                        e1 = ua_adj;
                        e1i = ua;
                    }
                    const mat3<T> R = e1 * e2;
                    mat3<T> Q = (e1 * Y) * e1i;
                    if constexpr (kExactInverse) Q = m_scale(Q, inv_det(ua, ua_adj));
                    Q = Q + load_mat(Fb, fo + link_off(ra, 0, d1), fs);
                    mat3<T> e3 = load_mat(Ub, link_off(ra, nu, s > 0 ? x : d3), us);
                    if (s > 0) e3 = m_adj(e3);
                    const mat3<T> Pm = R * e3;
                    const mat3<T> Pa = m_adj(Pm);
                    m_axpy_i(A, cb.im, Pm);
                    m_axpy_i(B, mcb.im, Pa);
                    Q = m_scale_z(Q, cts);
                    m_mac(A, Q, Pm);
                    m_mac(B, Pa, Q);
                    const mat3<T> X0s = m_scale_z(load_mat(Fb, fo + p * ra.Vh + h, fs), cts);
                    m_mac(A, Pm, X0s);
                    m_mac(B, X0s, Pa);
                }
            }
        }
        if constexpr (sizeof(T) == 8) __builtin_amdgcn_sched_barrier(0);
        const mat3<T> e0 = load_mat(Ub, l, us);
        mat3<T> M = e0 * A;
        m_mac(M, B, m_adj(e0));
        const mat3<T> K = m_traceless(M);
        store_mat((cx<T>*)ra.K, l, us, K);
        kn2 = 0.5 * (double)m_norm2(K);
        if (!isfinite(kn2)) kn2 = INFINITY;
    }
    double v[1] = {kn2};
    block_reduce<1, true>(v, lds);
    store_partials(ra, KIND_DRIFT, lb, v);
    // the step's K_max for the update kernel, with no finalize launch between
    if (threadIdx.x == 0) {
        const int par = (int)(ra.ctrl->step & 1);
        atomicMax(&ra.ctrl->kslot[par][blockIdx.x & (kXcds - 1)][0],
                  (unsigned long long)__double_as_longlong(v[0]));
    }
    CLGC_END_BLOCKS
}

// d^(-1/3) on the principal branch.  The updated link's determinant differs
// from 1 only by rounding (the exponential of a traceless matrix has
// determinant 1), so d = 1 + delta with |delta| ~ 1e-16 in FP64 and ~1e-7
// from FP32 links: for |delta| < 2^-12 the binomial series of
// (1 + delta)^(-1/3) to delta^5 is exact to 2e-23 and replaces the
// logarithm, arctangent, exponential and sine/cosine; otherwise those are
// evaluated.
__device__ __forceinline__ cx<double> det_renorm_factor(cx<double> d)
{
    const cx<double> dl = {d.re - 1.0, d.im};
    if (fabs(dl.re) < 0x1p-13 && fabs(dl.im) < 0x1p-13) {
        // binomial coefficients of (1 + x)^(-1/3): -1/3, 2/9, -14/81, 35/243, -91/729
        cx<double> w = {-91.0 / 729.0, 0.0};
        w = cfma(w, dl, cx<double>{35.0 / 243.0, 0.0});
        w = cfma(w, dl, cx<double>{-14.0 / 81.0, 0.0});
        w = cfma(w, dl, cx<double>{2.0 / 9.0, 0.0});
        w = cfma(w, dl, cx<double>{-1.0 / 3.0, 0.0});
        return cfma(w, dl, cx<double>{1.0, 0.0});
    }
    const double lr = -log(sqrt(fma(d.re, d.re, d.im * d.im))) / 3.0;
    const double ph = -atan2(d.im, d.re) / 3.0;
    double sn, cs;
    sincos(ph, &sn, &cs);
    const double mg = exp(lr);
    return {mg * cs, mg * sn};
}

// ---------------------------------------------------------------------------
// Langevin update: U <- exp(i (eps K + sqrt(eps) eta_a lambda_a)) U, then
// U <- U det(U)^{-1/3} in FP64.

// Every wavefront forms the step size itself from the drift's K_max (the
// per-XCD maxima its blocks left in the control block), so no finalize runs
// between the two kernels; block 0 records eps, K_max and the bound and
// clears the slots the next step's drift will use.  The update runs on the
// applying cooling kernel's logical blocks (KIND_COOL: at most
// kMaxCoolBlocks, each looping over chunks of 256 links) and leaves its
// unitarity-norm partials where the next omega kernel's wavefronts sum them.
template <typename T, bool FAST>
__global__ void __launch_bounds__(kBlock) k_update(const KArgs ka)
{
    __shared__ double lds[8];
    CLGC_FOR_BLOCKS(KIND_COOL)
    Ctrl* cr = ra.ctrl;
    const int64_t step = cr->step;
    const int par = (int)(step & 1);
    unsigned long long km = 0;
#pragma unroll
    for (int x = 0; x < kXcds; ++x) {
        const unsigned long long b = __hip_atomic_load(&cr->kslot[par][x][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        km = b > km ? b : km;
    }
    const double kmax = sqrt(__longlong_as_double((long long)km));
    // eps_n = min(eps0, B / K_max), B fixed on the first adaptive step; the
    // bound block 0 may be writing below is the value computed here either way
    const double bound = cr->bound;
    double B = bound, eps = ra.eps0;
    if (ra.adaptive) {
        if (B <= 0.0) B = ra.drift_bound > 0.0 ? ra.drift_bound : ra.eps0 * kmax;
        if (kmax > 0.0 && B / kmax < ra.eps0) eps = B / kmax;
    }
    const int ok = cr->status == ST_OK && isfinite(kmax);
    if (lb == 0 && threadIdx.x == 0) {
        cr->kmax = kmax;
        cr->eps = eps;
        if (ra.adaptive && bound <= 0.0) cr->bound = B;
        if (!isfinite(kmax)) cr->status = ST_NONFINITE;
        if (ok) cr->upd_pending = 1;
#pragma unroll
        for (int x = 0; x < kXcds; ++x)
            __hip_atomic_store(&cr->kslot[par ^ 1][x][0], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const int nch = (4 * ra.V + kBlock - 1) / kBlock;
    int cb0, cb1;
    chunk_range(nch, ra.nblk[KIND_COOL], lb, cb0, cb1);
    double un = 0.0;
    for (int c = cb0; c < cb1; ++c) {
        const int t = c * kBlock + (int)threadIdx.x;
        if (t < 4 * ra.V && ok) {
            int mu, p, h;
            link_decompose(ra, t, mu, p, h);
            const Site s = site_coords(ra, p, h);
            const uint32_t c0 = (uint32_t)(4 * site_lex(ra, s) + mu);
            const T se = T(sqrt(eps) * 1.41421356237309504880);  // sqrt(eps) * sqrt(2)
            T eta[8];
#pragma unroll
            for (int j = 0; j < 4; ++j) normal_pair<T>(ra.seed, c0, (uint32_t)step, (uint32_t)j, kStreamNoise,
                                                       eta[2 * j], eta[2 * j + 1]);
#pragma unroll
            for (int a = 0; a < 8; ++a) eta[a] *= se;
            // A = i (eps K + H),  H = sum_a eta_a lambda_a (Hermitian)
            const mat3<T> K = load_mat((const cx<T>*)ra.K, t, 4 * ra.V);
            const T r3 = T(0.57735026918962576451);
            mat3<T> H;
            H.e[0][0] = {eta[2] + r3 * eta[7], T(0)};
            H.e[1][1] = {r3 * eta[7] - eta[2], T(0)};
            H.e[2][2] = {T(-2) * r3 * eta[7], T(0)};
            H.e[0][1] = {eta[0], -eta[1]};
            H.e[1][0] = {eta[0], eta[1]};
            H.e[0][2] = {eta[3], -eta[4]};
            H.e[2][0] = {eta[3], eta[4]};
            H.e[1][2] = {eta[5], -eta[6]};
            H.e[2][1] = {eta[5], eta[6]};
            const T te = T(eps);
            mat3<T> A;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const cx<T> x = {fma(te, K.e[i][j].re, H.e[i][j].re), fma(te, K.e[i][j].im, H.e[i][j].im)};
                    A.e[i][j] = {-x.im, x.re};
                }
            const mat3<T> R = m_exp_traceless(A);
            const mat3<T> U = load_mat((const cx<T>*)ra.U, t, 4 * ra.V);
            // det renormalisation in FP64 on the principal branch
            const mat3<double> W = m_to_double(R * U);
            const cx<double> w = det_renorm_factor(m_det(W));
            const mat3<T> Un = m_cast_from<T>(m_scale(W, w));
            store_mat((cx<T>*)ra.U, t, 4 * ra.V, Un);
            un += (double)m_norm2(Un);
        }
    }
    double v[1] = {un};
    block_reduce<1>(v, lds);
    if (threadIdx.x == 0) ra.cpart[lb] = v[0];
    CLGC_END_BLOCKS
}

// ---------------------------------------------------------------------------
// gauge cooling half-sweep
//
// Four lanes per site x of the active parity (one per wavefront of a chunk of
// 64 sites), lane mu owning U_mu(x) and U_mu(x - mu): every link has exactly
// one end of each parity, so the half-sweep reads and writes every link
// exactly once.  The four lanes' shares of G_x = sum_mu (U_mu(x)
// U_mu(x)^dagger - U_mu(x-mu)^dagger U_mu(x-mu)) are added through LDS
// (site_sum); sum_a f_ax lambda_a = 4 G_x (G_x is traceless
// Hermitian), so Omega_x = exp(-4 eps alpha G_x), a Hermitian matrix whose
// exponential has real Cayley-Hamilton coefficients; Omega_x^{-1} =
// exp(+4 eps alpha G_x) uses the same series with det -> -det.



// real Horner series for exp of a Hermitian traceless matrix (the Hermitian
// counterpart of ch_exp_coeffs: s, t and the coefficients are real), N terms
// (f0m1 = f0 - 1 without the cancellation: the last step's t z)
template <typename T, int N>
__device__ __forceinline__ void ch_exp_coeffs_real(T s, T t, T& f0, T& f1, T& f2, T& f0m1)
{
    T x = T(1), y = T(0), z = T(0), last = T(0);
#pragma unroll
    for (int n = N; n >= 1; --n) {
        const T inv = T(1) / T(n);
        const T nx = t * z;
        const T ny = fma(s, z, x);
        const T nz = y;
        x = fma(inv, nx, T(1));
        y = inv * ny;
        z = inv * nz;
        last = nx;
    }
    f0 = x;
    f1 = y;
    f2 = z;
    f0m1 = last;
}

// square of a Hermitian matrix (Hermitian again)
template <typename T>
__device__ __forceinline__ herm3<T> h_square(const herm3<T>& A)
{
    const T n01 = norm2(A.u01), n02 = norm2(A.u02), n12 = norm2(A.u12);
    herm3<T> R;
    R.d0 = A.d0 * A.d0 + n01 + n02;
    R.d1 = n01 + A.d1 * A.d1 + n12;
    R.d2 = n02 + n12 + A.d2 * A.d2;
    R.u01 = cfma(A.u02, conj(A.u12), (A.d0 + A.d1) * A.u01);
    R.u02 = cfma(A.u01, A.u12, (A.d0 + A.d2) * A.u02);
    R.u12 = cfma(conj(A.u01), A.u02, (A.d1 + A.d2) * A.u12);
    return R;
}

// c0 + c1 A + c2 A2 for Hermitian A, A2 and real coefficients
template <typename T>
__device__ __forceinline__ herm3<T> h_poly(T c0, T c1, T c2, const herm3<T>& A, const herm3<T>& A2)
{
    herm3<T> R;
    R.d0 = fma(c2, A2.d0, fma(c1, A.d0, c0));
    R.d1 = fma(c2, A2.d1, fma(c1, A.d1, c0));
    R.d2 = fma(c2, A2.d2, fma(c1, A.d2, c0));
    R.u01 = {fma(c2, A2.u01.re, c1 * A.u01.re), fma(c2, A2.u01.im, c1 * A.u01.im)};
    R.u02 = {fma(c2, A2.u02.re, c1 * A.u02.re), fma(c2, A2.u02.im, c1 * A.u02.im)};
    R.u12 = {fma(c2, A2.u12.re, c1 * A.u12.re), fma(c2, A2.u12.im, c1 * A.u12.im)};
    return R;
}

// 2 D + D^2: (1 + D)^2 - 1
template <typename T>
__device__ __forceinline__ herm3<T> h_double_plus_square(const herm3<T>& D)
{
    const herm3<T> Q = h_square(D);
    herm3<T> R;
    R.d0 = fma(T(2), D.d0, Q.d0);
    R.d1 = fma(T(2), D.d1, Q.d1);
    R.d2 = fma(T(2), D.d2, Q.d2);
    R.u01 = {fma(T(2), D.u01.re, Q.u01.re), fma(T(2), D.u01.im, Q.u01.im)};
    R.u02 = {fma(T(2), D.u02.re, Q.u02.re), fma(T(2), D.u02.im, Q.u02.im)};
    R.u12 = {fma(T(2), D.u12.re, Q.u12.re), fma(T(2), D.u12.im, Q.u12.im)};
    return R;
}

// E = exp(A), Ei = exp(-A) for Hermitian traceless A, both kept Hermitian.
// DELTA: E - 1 and Ei - 1 instead, formed without cancellation (the series'
// constant term minus one, then (1 + D)^2 = 1 + 2 D + D^2 for each squaring),
// which FP32 can store with all its digits when A is small
template <typename T, bool DELTA = false>
__device__ __forceinline__ void herm_exp_pair(herm3<T> A, herm3<T>& E, herm3<T>& Ei)
{
    const T fro2 = A.d0 * A.d0 + A.d1 * A.d1 + A.d2 * A.d2 +
                   T(2) * (norm2(A.u01) + norm2(A.u02) + norm2(A.u12));
    int k = 0;
    if (fro2 > T(1)) {
        // a non-finite norm (a runaway) takes no squarings; its infinite log
        // converted to int would give a loop of 2^31 squarings
        const T lk = T(0.5) * log2(fro2);
        k = lk < T(1100) ? (int)ceil(lk) : 0;
        const T sc = ldexp(T(1), -k);
        A.d0 *= sc;
        A.d1 *= sc;
        A.d2 *= sc;
        A.u01 = sc * A.u01;
        A.u02 = sc * A.u02;
        A.u12 = sc * A.u12;
    }
    const herm3<T> A2 = h_square(A);
    const T s = T(0.5) * (A2.d0 + A2.d1 + A2.d2);
    // det of a Hermitian matrix (real)
    const cx<T> w = A.u01 * A.u12 * conj(A.u02);
    const T t = A.d0 * A.d1 * A.d2 + T(2) * w.re - A.d0 * norm2(A.u12) - A.d1 * norm2(A.u02) -
                A.d2 * norm2(A.u01);
    T f0, f1, f2, g0, g1, g2, f0m1, g0m1;
    // The series needs exp_terms terms for |A|_F <= 1; a cooling step's A is
    // usually far smaller, and for |A|_F <= 1/8 the terms after the first 10
    // (FP64; 6 in FP32) add at most 3e-18 (1e-10) relative.  The choice is
    // taken per wavefront, so the loop stays uniform.
    constexpr int kShort = sizeof(T) == 8 ? 10 : 6;
    if (__all(fro2 * ldexp(T(1), -2 * k) <= T(1.0 / 64.0))) {
        ch_exp_coeffs_real<T, kShort>(s, t, f0, f1, f2, f0m1);
        ch_exp_coeffs_real<T, kShort>(s, -t, g0, g1, g2, g0m1);
    } else {
        ch_exp_coeffs_real<T, exp_terms<T>::n>(s, t, f0, f1, f2, f0m1);
        ch_exp_coeffs_real<T, exp_terms<T>::n>(s, -t, g0, g1, g2, g0m1);
    }
    if constexpr (DELTA) {
        E = h_poly(f0m1, f1, f2, A, A2);
        Ei = h_poly(g0m1, -g1, g2, A, A2);
        for (int i = 0; i < k; ++i) {
            E = h_double_plus_square(E);
            Ei = h_double_plus_square(Ei);
        }
    } else {
        E = h_poly(f0, f1, f2, A, A2);
        Ei = h_poly(g0, -g1, g2, A, A2);
        for (int i = 0; i < k; ++i) {
            E = h_square(E);
            Ei = h_square(Ei);
        }
    }
}
// exp(A) alone (DELTA: exp(A) - 1), with the same operations herm_exp_pair
// applies to A: for -A it reproduces that function's exp(-A) bit for bit (A^2
// and the scaling do not see the sign, det flips it, and c1 (-a) equals
// (-c1) a)
template <typename T, bool DELTA = false>
__device__ __forceinline__ void herm_exp_one(herm3<T> A, herm3<T>& E)
{
    const T fro2 = A.d0 * A.d0 + A.d1 * A.d1 + A.d2 * A.d2 +
                   T(2) * (norm2(A.u01) + norm2(A.u02) + norm2(A.u12));
    int k = 0;
    if (fro2 > T(1)) {
        // a non-finite norm (a runaway) takes no squarings; its infinite log
        // converted to int would give a loop of 2^31 squarings
        const T lk = T(0.5) * log2(fro2);
        k = lk < T(1100) ? (int)ceil(lk) : 0;
        const T sc = ldexp(T(1), -k);
        A.d0 *= sc;
        A.d1 *= sc;
        A.d2 *= sc;
        A.u01 = sc * A.u01;
        A.u02 = sc * A.u02;
        A.u12 = sc * A.u12;
    }
    const herm3<T> A2 = h_square(A);
    const T s = T(0.5) * (A2.d0 + A2.d1 + A2.d2);
    // det of a Hermitian matrix (real)
    const cx<T> w = A.u01 * A.u12 * conj(A.u02);
    const T t = A.d0 * A.d1 * A.d2 + T(2) * w.re - A.d0 * norm2(A.u12) - A.d1 * norm2(A.u02) -
                A.d2 * norm2(A.u01);
    T f0, f1, f2, f0m1;
    // The series needs exp_terms terms for |A|_F <= 1; a cooling step's A is
    // usually far smaller, and for |A|_F <= 1/8 the terms after the first 10
    // (FP64; 6 in FP32) add at most 3e-18 (1e-10) relative.  The choice is
    // taken per wavefront, so the loop stays uniform.
    constexpr int kShort = sizeof(T) == 8 ? 10 : 6;
    if (__all(fro2 * ldexp(T(1), -2 * k) <= T(1.0 / 64.0)))
        ch_exp_coeffs_real<T, kShort>(s, t, f0, f1, f2, f0m1);
    else
        ch_exp_coeffs_real<T, exp_terms<T>::n>(s, t, f0, f1, f2, f0m1);
    if constexpr (DELTA) {
        E = h_poly(f0m1, f1, f2, A, A2);
        for (int i = 0; i < k; ++i) E = h_double_plus_square(E);
    } else {
        E = h_poly(f0, f1, f2, A, A2);
        for (int i = 0; i < k; ++i) E = h_square(E);
    }
}

// H U for Hermitian H
template <typename T>
__device__ __forceinline__ mat3<T> h_mul(const herm3<T>& H, const mat3<T>& U)
{
    mat3<T> r;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        r.e[0][j] = cfma(H.u02, U.e[2][j], cfma(H.u01, U.e[1][j], H.d0 * U.e[0][j]));
        r.e[1][j] = cfma(H.u12, U.e[2][j], cfma(conj(H.u01), U.e[0][j], H.d1 * U.e[1][j]));
        r.e[2][j] = cfma(conj(H.u12), U.e[1][j], cfma(conj(H.u02), U.e[0][j], H.d2 * U.e[2][j]));
    }
    return r;
}

// U H for Hermitian H
template <typename T>
__device__ __forceinline__ mat3<T> mul_h(const mat3<T>& U, const herm3<T>& H)
{
    mat3<T> r;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        r.e[i][0] = cfma(U.e[i][2], conj(H.u02), cfma(U.e[i][1], conj(H.u01), H.d0 * U.e[i][0]));
        r.e[i][1] = cfma(U.e[i][2], conj(H.u12), cfma(U.e[i][0], H.u01, H.d1 * U.e[i][1]));
        r.e[i][2] = cfma(U.e[i][1], H.u12, cfma(U.e[i][0], H.u02, H.d2 * U.e[i][2]));
    }
    return r;
}

// One cooling step (an even, then an odd half-sweep) in two kernels.
//
// k_cool_omega: at every even site x, Omega_x = exp(-4 eps alpha G_x) and its
// inverse from the links entering the step; the 18 reals are stored per even
// site in the drift buffer, which is idle during cooling.  Nothing else is
// written.
//
// k_cool_apply: at every odd site y, lane mu takes U_mu(y) and U_mu(y - mu),
// applies the even-site transforms those links received (U_mu(y) ends at the
// even site y + mu: U -> U Omega_{y+mu}^{-1}; U_mu(y - mu) starts at the even
// site y - mu: U -> Omega_{y-mu} U), forms G_y from the transformed links,
// Omega_y, and writes the two links with the odd transform applied.  Every
// link is read and written once per cooling step, and each product is the one
// the separate half-sweeps would evaluate, in the same order.

// How the cooling transforms are staged and applied.  FP64 stages Omega and
// Omega^-1 themselves.  FP32 (mixed precision) stages Omega - 1 and
// Omega^-1 - 1, whose entries are of the order of eps alpha G, so FP32 keeps
// all their digits, and applies U + (Omega - 1) U: the product is rounded at
// its own small scale and the sum once at the link's, where a product with
// Omega itself (diagonal entries near 1) rounds at the link's scale in every
// term.
template <typename T>
constexpr bool kCoolDelta = sizeof(T) == 4;

// FP64 stages Omega alone (9 reals per even site) and the applying kernel
// inverts it (h_inverse: Omega is Hermitian positive definite and near 1,
// so the adjugate over the determinant is accurate to rounding); the
// cooling pair is bound by its bytes there, and this drops a ninth of them.
// FP32 stages both Omega - 1 and Omega^-1 - 1, each formed without
// cancellation by the series.
template <typename T>
constexpr bool kStageInverse = kCoolDelta<T>;

// H^-1 for Hermitian H with det H > 0: adj(H) / det H, Hermitian again
template <typename T>
__device__ __forceinline__ herm3<T> h_inverse(const herm3<T>& H)
{
    herm3<T> a;
    a.d0 = H.d1 * H.d2 - norm2(H.u12);
    a.d1 = H.d0 * H.d2 - norm2(H.u02);
    a.d2 = H.d0 * H.d1 - norm2(H.u01);
    a.u01 = H.u02 * conj(H.u12) - H.d2 * H.u01;
    a.u02 = H.u01 * H.u12 - H.d1 * H.u02;
    a.u12 = H.u02 * conj(H.u01) - H.d0 * H.u12;
    const T det = H.d0 * a.d0 + (H.u01.re * a.u01.re + H.u01.im * a.u01.im) +
                  (H.u02.re * a.u02.re + H.u02.im * a.u02.im);
    const T r = T(1) / det;
    a.d0 *= r;
    a.d1 *= r;
    a.d2 *= r;
    a.u01 = r * a.u01;
    a.u02 = r * a.u02;
    a.u12 = r * a.u12;
    return a;
}

// Omega^-1 of the even site from what the omega kernel staged at value
// offset 9 (the inverse itself) or 0 (Omega, inverted here)
template <typename T>
__device__ __forceinline__ herm3<T> staged_inverse(const herm3<T>& S)
{
    if constexpr (kStageInverse<T>) return S;
    else return h_inverse(S);
}

// The even half-sweep on an odd site's lane, Uf Omega^-1 (the even site at
// the link's end) and Omega Ub (the even site at its start).  FP64 transforms
// Uf and Ub in place.  FP32 keeps the entering links and returns the small
// corrections Tf = Uf (Omega^-1 - 1), Tb = (Omega - 1) Ub: the transformed
// links are Uf + Tf and Ub + Tb (half_swept), and odd_transforms rounds the
// cooling step's result once at the scale of the link.
template <typename T>
__device__ __forceinline__ void even_transforms(mat3<T>& Uf, mat3<T>& Ub, const herm3<T>& Rf, const herm3<T>& Lb,
                                                mat3<T>& Tf, mat3<T>& Tb)
{
    if constexpr (kCoolDelta<T>) {
        Tf = mul_h(Uf, Rf);
        Tb = h_mul(Lb, Ub);
    } else {
        Uf = mul_h(Uf, Rf);
        Ub = h_mul(Lb, Ub);
    }
}

template <typename T>
__device__ __forceinline__ mat3<T> half_swept(const mat3<T>& U, const mat3<T>& Tc)
{
    if constexpr (kCoolDelta<T>) return U + Tc;
    else return U;
}

// The odd half-sweep: Nf = Omega_y (Uf Omega^-1), Nb = (Omega Ub) Omega_y^-1
// with the staged (E, Ei) of the odd site.  FP32: Nf = Uf + (Tf + (Omega_y -
// 1) (Uf + Tf)), every term but the last sum at its own small scale (and
// likewise Nb).
template <typename T>
__device__ __forceinline__ void odd_transforms(const mat3<T>& Uf, const mat3<T>& Ub, const mat3<T>& Tf,
                                               const mat3<T>& Tb, const herm3<T>& E, const herm3<T>& Ei, mat3<T>& Nf,
                                               mat3<T>& Nb)
{
    if constexpr (kCoolDelta<T>) {
        Nf = Uf + (Tf + h_mul(E, Uf + Tf));
        Nb = Ub + (Tb + mul_h(Ub + Tb, Ei));
    } else {
        Nf = h_mul(E, Uf);
        Nb = mul_h(Ub, Ei);
    }
}

// the staged transform of even site h, value j at OM[j * Vh + h] in the link
// type: 18 reals (Omega, Omega^-1) where kStageInverse, else the 9 of Omega
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t omega_rsrc(const RunArgs& ra)
{
    const uint32_t bytes = (kStageInverse<T> ? 18u : 9u) * (uint32_t)ra.Vh * (uint32_t)sizeof(T);
    return __builtin_amdgcn_make_buffer_rsrc(ra.K, (short)0, (int)bytes, kBufferWord3);
}

template <typename T>
__device__ __forceinline__ T buf_load_scalar(__amdgpu_buffer_rsrc_t rs, uint32_t lane_bytes, int elem_bytes)
{
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)lane_bytes, elem_bytes, 0));
    else
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)lane_bytes, elem_bytes, 0));
}

template <typename T>
__device__ __forceinline__ void buf_store_scalar(__amdgpu_buffer_rsrc_t rs, uint32_t lane_bytes, int elem_bytes, T v)
{
    if constexpr (sizeof(T) == 8)
    {
        typedef unsigned int u2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), rs, (int)lane_bytes, elem_bytes, 0);
    }
    else
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), rs, (int)lane_bytes, elem_bytes, 0);
}

template <typename T>
__device__ __forceinline__ herm3<T> load_herm(__amdgpu_buffer_rsrc_t rs, int h, int Vh, int j0)
{
    const uint32_t lane = (uint32_t)h * (uint32_t)sizeof(T);
    const int es = Vh * (int)sizeof(T);
    herm3<T> H;
    H.d0 = buf_load_scalar<T>(rs, lane, (j0 + 0) * es);
    H.d1 = buf_load_scalar<T>(rs, lane, (j0 + 1) * es);
    H.d2 = buf_load_scalar<T>(rs, lane, (j0 + 2) * es);
    H.u01 = {buf_load_scalar<T>(rs, lane, (j0 + 3) * es), buf_load_scalar<T>(rs, lane, (j0 + 4) * es)};
    H.u02 = {buf_load_scalar<T>(rs, lane, (j0 + 5) * es), buf_load_scalar<T>(rs, lane, (j0 + 6) * es)};
    H.u12 = {buf_load_scalar<T>(rs, lane, (j0 + 7) * es), buf_load_scalar<T>(rs, lane, (j0 + 8) * es)};
    return H;
}

template <typename T>
__device__ __forceinline__ void store_herm(__amdgpu_buffer_rsrc_t rs, int h, int Vh, int j0, const herm3<T>& H)
{
    // (j0 may differ between lanes: it goes into the lane offset, since the
    // scalar offset must be uniform -- a divergent one costs a loop over its
    // distinct values)
    const uint32_t lane = ((uint32_t)j0 * (uint32_t)Vh + (uint32_t)h) * (uint32_t)sizeof(T);
    const int es = Vh * (int)sizeof(T);
    buf_store_scalar<T>(rs, lane, 0 * es, H.d0);
    buf_store_scalar<T>(rs, lane, 1 * es, H.d1);
    buf_store_scalar<T>(rs, lane, 2 * es, H.d2);
    buf_store_scalar<T>(rs, lane, 3 * es, H.u01.re);
    buf_store_scalar<T>(rs, lane, 4 * es, H.u01.im);
    buf_store_scalar<T>(rs, lane, 5 * es, H.u02.re);
    buf_store_scalar<T>(rs, lane, 6 * es, H.u02.im);
    buf_store_scalar<T>(rs, lane, 7 * es, H.u12.re);
    buf_store_scalar<T>(rs, lane, 8 * es, H.u12.im);
}

// The four wavefronts of a cooling chunk hold the direction shares s_mu of
// G at the chunk's 64 sites (wave mu, lane = site).  They exchange them
// through LDS and every wavefront forms G = (s_0 + s_1) + (s_2 + s_3), the
// same bits in all four.  Two buffers, used in turn: a buffer is written
// again only two exchanges later, after every lane has passed the barrier of
// the exchange in between, so one barrier per exchange suffices.
template <typename T>
struct CoolShare {
    T g[2][4][9][kCoolSites];
};

template <typename T>
__device__ __forceinline__ herm3<T> site_sum(const herm3<T>& S, CoolShare<T>& sh, int& buf)
{
    const int lane = (int)threadIdx.x & (kCoolSites - 1), mu = (int)threadIdx.x / kCoolSites;
    T (*g)[9][kCoolSites] = sh.g[buf];
    buf ^= 1;
    const T v[9] = {S.d0, S.d1, S.d2, S.u01.re, S.u01.im, S.u02.re, S.u02.im, S.u12.re, S.u12.im};
#pragma unroll
    for (int j = 0; j < 9; ++j) g[mu][j][lane] = v[j];
    __syncthreads();
    T r[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) r[j] = (g[0][j][lane] + g[1][j][lane]) + (g[2][j][lane] + g[3][j][lane]);
    herm3<T> G;
    G.d0 = r[0];
    G.d1 = r[1];
    G.d2 = r[2];
    G.u01 = {r[3], r[4]};
    G.u02 = {r[5], r[6]};
    G.u12 = {r[7], r[8]};
    return G;
}

// coef TL(G) for the site sum G
template <typename T>
__device__ __forceinline__ herm3<T> scaled_traceless(const herm3<T>& G, T coef)
{
    const T tr = (G.d0 + G.d1 + G.d2) * T(1.0 / 3.0);
    herm3<T> A;
    A.d0 = coef * (G.d0 - tr);
    A.d1 = coef * (G.d1 - tr);
    A.d2 = coef * (G.d2 - tr);
    A.u01 = coef * G.u01;
    A.u02 = coef * G.u02;
    A.u12 = coef * G.u12;
    return A;
}

// Omega = exp(coef TL(G)) and its inverse, as the cooling kernels stage them
// (kCoolDelta)
template <typename T>
__device__ __forceinline__ void site_omega(const herm3<T>& G, T coef, herm3<T>& E, herm3<T>& Ei)
{
    herm_exp_pair<T, kCoolDelta<T>>(scaled_traceless(G, coef), E, Ei);
}
// the same for one of the pair: coef < 0 gives Omega, coef > 0 Omega^-1
template <typename T>
__device__ __forceinline__ void site_omega_one(const herm3<T>& G, T coef, herm3<T>& E)
{
    herm_exp_one<T, kCoolDelta<T>>(scaled_traceless(G, coef), E);
}

// In both kernels the link loads are issued first: the run's state (status,
// the unitarity norm entering the step, alpha) only sets the coefficient,
// which is needed once G is formed, so its dependent reads overlap the loads.
template <typename T, bool FAST>
__global__ void __launch_bounds__(kBlock) k_cool_omega(const KArgs ka, int iter)
{
    __shared__ CoolShare<T> sh;
    int buf = 0;
    CLGC_FOR_BLOCKS(KIND_OMEGA)
    Ctrl* cr = ra.ctrl;
    if (iter < ra.n_cool) {
        const int nch = cool_chunks_total(ra.V);
        int cb0, cb1;
        chunk_range(nch, ra.nblk[KIND_OMEGA], lb, cb0, cb1);
        for (int c = cb0; c < cb1; ++c) {
            int h, mu;
            cool_lane(c, (int)threadIdx.x, h, mu);
            const bool lane_ok = h < ra.Vh;
            herm3<T> G = h_zero<T>();
            if (lane_ok) {
                int of, ob;
                cool_lane_links(ra, 0, h, mu, of, ob);
                const cx<T>* __restrict__ Uc = (const cx<T>*)ra.U;
                h_add_uudag(G, load_mat(Uc, of, 4 * ra.V));
                h_sub_udagu(G, load_mat(Uc, ob, 4 * ra.V));
            }
            // wavefront 0 forms Omega, wavefront 1 Omega^-1 where it is staged;
            // the others only contribute their shares of G and need no run state
            const bool expw = mu < (kStageInverse<T> ? 2 : 1);
            bool ok = false;
            double alpha_ad = 0.0;
            if (expw) {
                // Each of these wavefronts reads the status for itself (there is
                // no barrier here).  Within this launch the word changes only
                // below, in block 0, when the norm that every one of them
                // computes identically is not finite: then every Omega is
                // non-finite and nothing reads them.
                ok = cr->status == ST_OK;
                // unitarity norm entering the step: the partials of the CL update
                // just applied or of the previous cooling step; else (a cooling
                // call on its own) the finalized norm
                const bool pend = iter == 0 && cr->upd_pending;
                const double un = iter == 0 && !pend ? cr->unorm : wave_cool_sum(ra);
                // D_2 = mean |f_ax| from the gradient-norm pass just before (its
                // partials, one per logical block of the applying kernel)
                const double d2 = ra.mode == 2 ? wave_sum_of(ra.part, ra.nblk[KIND_COOL]) / (8.0 * ra.V) : 1.0;
                alpha_ad = ra.mode == 1 ? ra.alpha / (un / (4.0 * ra.V)) : (ra.mode == 2 ? ra.alpha / d2 : ra.alpha);
                if (ok && lb == 0 && c == 0 && threadIdx.x == 0) {
                    cr->alpha_cur = alpha_ad;
                    cr->unorm = un;
                    if (pend) {
                        // the update's finalization: its norm, and the step is taken
                        cr->d_pre = un / (12.0 * ra.V) - 1.0;
                        cr->step = cr->step + 1;
                    }
                    if (!isfinite(un) || !(d2 > 0.0) || !isfinite(alpha_ad)) cr->status = ST_NONFINITE;
                    if (iter < kMaxCoolHist) {
                        cr->hist_alpha[iter] = alpha_ad;
                        cr->hist_un[iter] = un;
                        cr->hist_n = iter + 1;
                    }
                }
            }
            const herm3<T> Gx = site_sum(G, sh, buf);
            if (expw) {
                const T coef = T(-4.0 * ra.eps_c * alpha_ad);
                herm3<T> E;
                site_omega_one(Gx, mu == 1 ? -coef : coef, E);
                if (ok && lane_ok) store_herm(omega_rsrc<T>(ra), h, ra.Vh, mu == 0 ? 0 : 9, E);
            }
        }
    }
    CLGC_END_BLOCKS
}

template <typename T, bool FAST>
__global__ void __launch_bounds__(kBlock) k_cool_apply(const KArgs ka, int iter)
{
    __shared__ double lds[8];
    __shared__ CoolShare<T> sh;
    int buf = 0;
    CLGC_FOR_BLOCKS(KIND_COOL)
    Ctrl* cr = ra.ctrl;
    if (iter < ra.n_cool) {
        const int nch = cool_chunks_total(ra.V);
        int cb0, cb1;
        chunk_range(nch, ra.nblk[KIND_COOL], lb, cb0, cb1);
        // (no kernel writes the status during this launch: every wavefront
        // reads the same value, so the block reduction below is reached by all)
        bool ok = true;
        double un = 0.0;
        for (int c = cb0; c < cb1; ++c) {
            int h, mu;
            cool_lane(c, (int)threadIdx.x, h, mu);
            const bool lane_ok = h < ra.Vh;
            herm3<T> G = h_zero<T>();
            mat3<T> Uf, Ub, Tf, Tb;
            int of = 0, ob = 0;
            if (lane_ok) {
                const Site y = site_coords(ra, 1, h);
                const Site yb = site_move(ra, y, mu, -1), yf = site_move(ra, y, mu, +1);
                cool_lane_links(ra, 1, h, mu, of, ob);
                const cx<T>* __restrict__ Uc = (const cx<T>*)ra.U;
                const __amdgpu_buffer_rsrc_t om = omega_rsrc<T>(ra);
                Uf = load_mat(Uc, of, 4 * ra.V);
                Ub = load_mat(Uc, ob, 4 * ra.V);
                even_transforms(Uf, Ub,
                                staged_inverse(load_herm<T>(om, site_half(ra, yf), ra.Vh, kStageInverse<T> ? 9 : 0)),
                                load_herm<T>(om, site_half(ra, yb), ra.Vh, 0), Tf, Tb);
                h_add_uudag(G, half_swept(Uf, Tf));
                h_sub_udagu(G, half_swept(Ub, Tb));
            }
            ok = cr->status == ST_OK;
            herm3<T> E, Ei;
            site_omega(site_sum(G, sh, buf), T(-4.0 * ra.eps_c * cr->alpha_cur), E, Ei);
            if (ok && lane_ok) {
                mat3<T> Nf, Nb;
                odd_transforms(Uf, Ub, Tf, Tb, E, Ei, Nf, Nb);
                cx<T>* __restrict__ Uw = (cx<T>*)ra.U;
                store_mat(Uw, of, 4 * ra.V, Nf);
                store_mat(Uw, ob, 4 * ra.V, Nb);
                un += (double)m_norm2(Nf) + (double)m_norm2(Nb);
            }
        }
        // every link is written exactly once: the sum is the unitarity norm of
        // the cooled configuration
        double v[1] = {un};
        block_reduce<1>(v, lds);
        if (ok && threadIdx.x == 0) ra.cpart[lb] = v[0];
        // the omega kernel before this one consumed the update's partials
        if (iter == 0 && lb == 0 && threadIdx.x == 0) cr->upd_pending = 0;
    }
    CLGC_END_BLOCKS
}

// The same cooling step for a single lattice whose blocks loop over several
// chunks (more chunks than the kernel's logical blocks: the applying kernel
// above 16^4 sites, and in mixed precision the omega kernel): each wavefront
// issues the next chunk's loads before it works on the current one, so HBM
// keeps streaming while the chunk's arithmetic runs.  The run state is read
// once per wavefront.  Same products in the same order as k_cool_omega /
// k_cool_apply: the results are bitwise equal.

// lane (h, mu) of chunk c: U_mu(x) and U_mu(x - mu) of even site h
template <typename T>
__device__ __forceinline__ void omega_loads(const RunArgs& ra, int c, int& h, bool& lok, mat3<T>& Af, mat3<T>& Ab)
{
    int mu;
    cool_lane(c, (int)threadIdx.x, h, mu);
    lok = h < ra.Vh;
    if (lok) {
        int of, ob;
        cool_lane_links(ra, 0, h, mu, of, ob);
        const cx<T>* __restrict__ Uc = (const cx<T>*)ra.U;
        Af = load_mat(Uc, of, 4 * ra.V);
        Ab = load_mat(Uc, ob, 4 * ra.V);
    }
}

template <typename T, bool FAST>
__global__ void __launch_bounds__(kBlock) k_cool_omega_pf(const KArgs ka, int iter)
{
    __shared__ CoolShare<T> sh;
    int buf = 0;
    CLGC_FOR_BLOCKS(KIND_OMEGA)
    Ctrl* cr = ra.ctrl;
    if (iter < ra.n_cool) {
        const int nch = cool_chunks_total(ra.V);
        int c0, c1;
        chunk_range(nch, ra.nblk[KIND_OMEGA], lb, c0, c1);
        const int mu = (int)threadIdx.x / kCoolSites;
        int h = 0;
        bool lok = false;
        mat3<T> Af, Ab;
        if (c0 < c1) omega_loads(ra, c0, h, lok, Af, Ab);
        // the run state, as in k_cool_omega: read by the wavefronts that form
        // an exponential only
        const bool expw = mu < (kStageInverse<T> ? 2 : 1);
        bool ok = false;
        double alpha_ad = 0.0;
        if (expw) {
            ok = cr->status == ST_OK;
            const bool pend = iter == 0 && cr->upd_pending;
            const double un = iter == 0 && !pend ? cr->unorm : wave_cool_sum(ra);
            const double d2 = ra.mode == 2 ? wave_sum_of(ra.part, ra.nblk[KIND_COOL]) / (8.0 * ra.V) : 1.0;
            alpha_ad = ra.mode == 1 ? ra.alpha / (un / (4.0 * ra.V)) : (ra.mode == 2 ? ra.alpha / d2 : ra.alpha);
            if (ok && lb == 0 && c0 < c1 && threadIdx.x == 0) {
                cr->alpha_cur = alpha_ad;
                cr->unorm = un;
                if (pend) {
                    cr->d_pre = un / (12.0 * ra.V) - 1.0;
                    cr->step = cr->step + 1;
                }
                if (!isfinite(un) || !(d2 > 0.0) || !isfinite(alpha_ad)) cr->status = ST_NONFINITE;
                if (iter < kMaxCoolHist) {
                    cr->hist_alpha[iter] = alpha_ad;
                    cr->hist_un[iter] = un;
                    cr->hist_n = iter + 1;
                }
            }
        }
        const T coef = T(-4.0 * ra.eps_c * alpha_ad);
        for (int c = c0; c < c1; ++c) {
            int hn = 0;
            bool lokn = false;
            mat3<T> Nf, Nb;
            if (c + 1 < c1) omega_loads(ra, c + 1, hn, lokn, Nf, Nb);
            herm3<T> G = h_zero<T>();
            if (lok) {
                h_add_uudag(G, Af);
                h_sub_udagu(G, Ab);
            }
            const herm3<T> Gx = site_sum(G, sh, buf);
            if (expw) {
                herm3<T> E;
                site_omega_one(Gx, mu == 1 ? -coef : coef, E);
                if (ok && lok) store_herm(omega_rsrc<T>(ra), h, ra.Vh, mu == 0 ? 0 : 9, E);
            }
            h = hn;
            lok = lokn;
            Af = Nf;
            Ab = Nb;
        }
    }
    CLGC_END_BLOCKS
}

// lane (h, mu) of chunk c: U_mu(y), U_mu(y - mu) of odd site h and the even
// transforms they take (what is staged for Omega^-1 of y + mu -- the inverse
// itself or Omega, see staged_inverse -- and Omega of y - mu)
template <typename T>
struct ApplyIn {
    mat3<T> Uf, Ub;
    herm3<T> Eif, Eb;
    int of, ob;
    bool lok;
};

template <typename T>
__device__ __forceinline__ void apply_loads(const RunArgs& ra, int c, ApplyIn<T>& in)
{
    int h, mu;
    cool_lane(c, (int)threadIdx.x, h, mu);
    in.lok = h < ra.Vh;
    if (in.lok) {
        const Site y = site_coords(ra, 1, h);
        const Site yb = site_move(ra, y, mu, -1), yf = site_move(ra, y, mu, +1);
        cool_lane_links(ra, 1, h, mu, in.of, in.ob);
        const cx<T>* __restrict__ Uc = (const cx<T>*)ra.U;
        const __amdgpu_buffer_rsrc_t om = omega_rsrc<T>(ra);
        in.Uf = load_mat(Uc, in.of, 4 * ra.V);
        in.Eif = load_herm<T>(om, site_half(ra, yf), ra.Vh, kStageInverse<T> ? 9 : 0);
        in.Eb = load_herm<T>(om, site_half(ra, yb), ra.Vh, 0);
        in.Ub = load_mat(Uc, in.ob, 4 * ra.V);
    }
}

template <typename T, bool FAST>
__global__ void __launch_bounds__(kBlock) k_cool_apply_pf(const KArgs ka, int iter)
{
    __shared__ double lds[8];
    __shared__ CoolShare<T> sh;
    int buf = 0;
    CLGC_FOR_BLOCKS(KIND_COOL)
    Ctrl* cr = ra.ctrl;
    if (iter < ra.n_cool) {
        const int nch = cool_chunks_total(ra.V);
        int c0, c1;
        chunk_range(nch, ra.nblk[KIND_COOL], lb, c0, c1);
        ApplyIn<T> cur;
        cur.lok = false;
        if (c0 < c1) apply_loads(ra, c0, cur);
        // (no kernel writes the status during this launch)
        const bool ok = cr->status == ST_OK;
        const T coef = T(-4.0 * ra.eps_c * cr->alpha_cur);
        double un = 0.0;
        for (int c = c0; c < c1; ++c) {
            ApplyIn<T> nxt;
            nxt.lok = false;
            if (c + 1 < c1) apply_loads(ra, c + 1, nxt);
            herm3<T> G = h_zero<T>();
            mat3<T> Uf = cur.Uf, Ub = cur.Ub, Tf, Tb;
            if (cur.lok) {
                even_transforms(Uf, Ub, staged_inverse(cur.Eif), cur.Eb, Tf, Tb);
                h_add_uudag(G, half_swept(Uf, Tf));
                h_sub_udagu(G, half_swept(Ub, Tb));
            }
            herm3<T> E, Ei;
            site_omega(site_sum(G, sh, buf), coef, E, Ei);
            if (ok && cur.lok) {
                mat3<T> Nf, Nb;
                odd_transforms(Uf, Ub, Tf, Tb, E, Ei, Nf, Nb);
                cx<T>* __restrict__ Uw = (cx<T>*)ra.U;
                store_mat(Uw, cur.of, 4 * ra.V, Nf);
                store_mat(Uw, cur.ob, 4 * ra.V, Nb);
                un += (double)m_norm2(Nf) + (double)m_norm2(Nb);
            }
            cur = nxt;
        }
        double v[1] = {un};
        block_reduce<1>(v, lds);
        if (ok && threadIdx.x == 0) ra.cpart[lb] = v[0];
        if (iter == 0 && lb == 0 && threadIdx.x == 0) cr->upd_pending = 0;
    }
    CLGC_END_BLOCKS
}

// D_2 = mean over (a, x) of |f_ax| on the configuration entering a cooling
// step, f_ax = 2 Tr(lambda_a G_x).  Two lanes per site (directions 0, 1 and
// 2, 3, joined by one shuffle), on the applying kernel's logical blocks: the
// chunks of kBlock lanes are then exactly as many as the cooling chunks, so
// every block (and every XCD) has work, and the next omega kernel's
// wavefronts sum the <= kMaxCoolBlocks partials themselves.
template <typename T, bool FAST>
__global__ void __launch_bounds__(kBlock) k_gradnorm(const KArgs ka, int iter)
{
    __shared__ double lds[8];
    CLGC_FOR_BLOCKS(KIND_COOL)
    Ctrl* cr = ra.ctrl;
    if (ra.mode == 2 && iter < ra.n_cool && cr->status == ST_OK) {
        const int nch = (2 * ra.V + kBlock - 1) / kBlock;
        int cb0, cb1;
        chunk_range(nch, ra.nblk[KIND_COOL], lb, cb0, cb1);
        double fs = 0.0;
        for (int c = cb0; c < cb1; ++c) {
            const int t = c * kBlock + (int)threadIdx.x;
            const int sx = t >> 1, half = t & 1;
            herm3<T> G = h_zero<T>();
            if (sx < ra.V) {
                const int p = sx >= ra.Vh;
                const Site x = site_coords(ra, p, sx - p * ra.Vh);
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    const int mu = 2 * half + m;
                    h_add_uudag(G, ldU<T>(ra, mu, x));
                    h_sub_udagu(G, ldU<T>(ra, mu, site_move(ra, x, mu, -1)));
                }
            }
            G.d0 += dpp_move<0xB1>(G.d0);
            G.d1 += dpp_move<0xB1>(G.d1);
            G.d2 += dpp_move<0xB1>(G.d2);
            G.u01 = {G.u01.re + dpp_move<0xB1>(G.u01.re), G.u01.im + dpp_move<0xB1>(G.u01.im)};
            G.u02 = {G.u02.re + dpp_move<0xB1>(G.u02.re), G.u02.im + dpp_move<0xB1>(G.u02.im)};
            G.u12 = {G.u12.re + dpp_move<0xB1>(G.u12.re), G.u12.im + dpp_move<0xB1>(G.u12.im)};
            if (sx < ra.V && half == 0) {
                const double r3 = 0.57735026918962576451;
                fs += 4.0 * (fabs((double)G.u01.re) + fabs((double)G.u01.im) + fabs((double)G.u02.re) +
                             fabs((double)G.u02.im) + fabs((double)G.u12.re) + fabs((double)G.u12.im)) +
                      2.0 * fabs((double)G.d0 - (double)G.d1) +
                      2.0 * r3 * fabs((double)G.d0 + (double)G.d1 - 2.0 * (double)G.d2);
            }
        }
        double v[1] = {fs};
        block_reduce<1>(v, lds);
        if (threadIdx.x == 0) ra.part[lb] = v[0];
    }
    CLGC_END_BLOCKS
}

// ---------------------------------------------------------------------------
// measurement: plaquette traces (and of their inverses, for the Wilson
// action), topological charge density from the clover field, unitarity norm

template <typename T>
__device__ __forceinline__ mat3<double> ldU64(const RunArgs& ra, int mu, const Site& s)
{
    return m_to_double(ldU<T>(ra, mu, s));
}

// F_{mu nu}(x) = sum over the four counter-clockwise leaves L of (L - L^-1),
// formed in FP64 from the links ld(mu, site) returns, with the leaf products
// associated as in k_clover; tp / ti get the traces of the first leaf (the
// plaquette U_{mu nu}(x)) and of its inverse
template <typename LD>
__device__ __forceinline__ mat3<double> clover_f64(const RunArgs& ra, const LD& ld, const Site& x, int mu, int nu,
                                                   cx<double>& tp, cx<double>& ti)
{
    const Site xpm = site_move(ra, x, mu, +1), xpn = site_move(ra, x, nu, +1);
    const Site xmm = site_move(ra, x, mu, -1), xmn = site_move(ra, x, nu, -1);
    const Site xmmpn = site_move(ra, xmm, nu, +1), xmmmn = site_move(ra, xmm, nu, -1);
    const Site xmnpm = site_move(ra, xmn, mu, +1);
    mat3<double> S = ld(nu, x);
    // U_mu(x) U_nu(x+mu) [U_nu(x) U_mu(x+nu)]^{-1}
    mat3<double> L = (ld(mu, x) * ld(nu, xpm)) * m_adj(S * ld(mu, xpn));
    tp = m_tr(L);
    ti = (L.e[1][1] * L.e[2][2] - L.e[1][2] * L.e[2][1]) + (L.e[0][0] * L.e[2][2] - L.e[0][2] * L.e[2][0]) +
         (L.e[0][0] * L.e[1][1] - L.e[0][1] * L.e[1][0]);
    mat3<double> F = L - m_adj(L);
    __builtin_amdgcn_sched_barrier(0);
    // U_nu(x) [U_nu(x-mu) U_mu(x-mu+nu)]^{-1} U_mu(x-mu)
    {
        const mat3<double> Umm = ld(mu, xmm);
        L = S * (m_adj(ld(nu, xmm) * ld(mu, xmmpn)) * Umm);
        S = Umm;
    }
    F = F + (L - m_adj(L));
    __builtin_amdgcn_sched_barrier(0);
    // [U_nu(x-mu-nu) U_mu(x-mu)]^{-1} U_mu(x-mu-nu) U_nu(x-nu)
    {
        const mat3<double> Unn = ld(nu, xmn);
        L = m_adj(ld(nu, xmmmn) * S) * (ld(mu, xmmmn) * Unn);
        S = Unn;
    }
    F = F + (L - m_adj(L));
    __builtin_amdgcn_sched_barrier(0);
    // U_nu(x-nu)^{-1} U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^{-1}
    L = m_adj(S) * ((ld(mu, xmn) * ld(nu, xmnpm)) * m_adj(ld(mu, x)));
    return F + (L - m_adj(L));
}

// One site's measurement sums, all in FP64 from the links ld returns: v[0..3]
// the plaquette traces Tr P and Tr P^-1 (re, im) of its six planes, v[4..5]
// the clover bracket Tr F01 F23 - Tr F02 F13 + Tr F03 F12 (re, im), v[6] the
// norms Tr U U^dagger of its four links
template <typename LD>
__device__ __forceinline__ void site_obs_f64(const RunArgs& ra, const LD& ld, const Site& x, double (&v)[7])
{
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) v[6] += m_norm2(ld(mu, x));
    // planes in the pairs (01, 23), (02, 13), (03, 12) of the charge
    cx<double> q = {0.0, 0.0};
#pragma unroll 1
    for (int P = 0; P < 3; ++P) {
        const int mu2 = P == 0 ? 2 : 1, nu2 = P == 2 ? 2 : 3;
        cx<double> tp, ti;
        const mat3<double> Fa = clover_f64(ra, ld, x, 0, P + 1, tp, ti);
        v[0] += tp.re;
        v[1] += tp.im;
        v[2] += ti.re;
        v[3] += ti.im;
        __builtin_amdgcn_sched_barrier(0);
        const mat3<double> Fd = clover_f64(ra, ld, x, mu2, nu2, tp, ti);
        v[0] += tp.re;
        v[1] += tp.im;
        v[2] += ti.re;
        v[3] += ti.im;
        const cx<double> t = m_trmul(Fa, Fd);
        const double sg = P == 1 ? -1.0 : 1.0;
        q.re += sg * t.re;
        q.im += sg * t.im;
        __builtin_amdgcn_sched_barrier(0);
    }
    v[4] = q.re;
    v[5] = q.im;
}

// One lane per site.  FROM_F: the clover field of the current links is in F
// (FP64, built by k_clover); otherwise every site forms its six clover
// matrices itself, in FP64 whatever the link precision, so a mixed-precision
// lattice is measured without FP32 rounding of the near-identity leaves
// (L - L^-1 cancels most of their digits).
template <typename T, bool FAST, bool FROM_F>
__global__ void __launch_bounds__(kBlock) k_measure(const KArgs ka)
{
    __shared__ double lds[7 * 4];
    CLGC_FOR_BLOCKS(KIND_SITE)
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    if (tid < ra.V) {
        const int p = tid >= ra.Vh;
        const int h = tid - p * ra.Vh;
        const Site x = site_coords(ra, p, h);
        if constexpr (FROM_F) {
#pragma unroll 1
            for (int mu = 0; mu < 4; ++mu) {
                const mat3<T> Um = ldU<T>(ra, mu, x);
                v[6] += (double)m_norm2(Um);
#pragma unroll 1
                for (int nu = mu + 1; nu < 4; ++nu) {
                    const mat3<T> Un = ldU<T>(ra, nu, x);
                    const mat3<T> Pm = (Um * ldU<T>(ra, nu, site_move(ra, x, mu, +1))) *
                                       m_adj(Un * ldU<T>(ra, mu, site_move(ra, x, nu, +1)));
                    const cx<T> tp = m_tr(Pm);
                    const cx<T> ti = (Pm.e[1][1] * Pm.e[2][2] - Pm.e[1][2] * Pm.e[2][1]) +
                                     (Pm.e[0][0] * Pm.e[2][2] - Pm.e[0][2] * Pm.e[2][0]) +
                                     (Pm.e[0][0] * Pm.e[1][1] - Pm.e[0][1] * Pm.e[1][0]);
                    v[0] += (double)tp.re;
                    v[1] += (double)tp.im;
                    v[2] += (double)ti.re;
                    v[3] += (double)ti.im;
                }
            }
            const cx<T>* __restrict__ Fb = (const cx<T>*)ra.F;
            const int so = p * ra.Vh + h;
            cx<double> q = {0.0, 0.0};
#pragma unroll 1
            for (int P = 0; P < 3; ++P) {
                const cx<T> t = m_trmul(load_mat(Fb, P * ra.V + so, 6 * ra.V), load_mat(Fb, (5 - P) * ra.V + so, 6 * ra.V));
                const double sg = P == 1 ? -1.0 : 1.0;
                q.re += sg * (double)t.re;
                q.im += sg * (double)t.im;
            }
            v[4] = q.re;
            v[5] = q.im;
        } else {
            site_obs_f64(ra, [&](int m, const Site& y) { return ldU64<T>(ra, m, y); }, x, v);
        }
    }
    block_reduce<7>(v, lds);
    store_partials(ra, KIND_SITE, lb, v);
    CLGC_END_BLOCKS
}

// The charge density of a recorded FP64 step with a theta term, from the
// clover field the step's clover kernel built for the links it measures: one
// lane per site, Tr F01 F23 - Tr F02 F13 + Tr F03 F12 (re, im) into the record
// partials 6 and 7 (record_partial).  Summed on the drift's own lanes it
// pushed the drift past 256 registers (scratch), so it has its own launch.
template <bool FAST>
__global__ void __launch_bounds__(kBlock) k_record_charge(const KArgs ka)
{
    __shared__ double lds[2 * 4];
    CLGC_FOR_BLOCKS(KIND_SITE)
    double q[2] = {0.0, 0.0};
    if (tid < ra.V) {
        const cx<double>* __restrict__ Fb = (const cx<double>*)ra.F;
#pragma unroll 1
        for (int P = 0; P < 3; ++P) {
            const cx<double> t = m_trmul(load_mat(Fb, P * ra.V + tid, 6 * ra.V),
                                         load_mat(Fb, (5 - P) * ra.V + tid, 6 * ra.V));
            const double sg = P == 1 ? -1.0 : 1.0;
            q[0] += sg * t.re;
            q[1] += sg * t.im;
        }
    }
    block_reduce<2>(q, lds);
    if (threadIdx.x == 0) {
        record_partial(ra, 6)[lb] = q[0];
        record_partial(ra, 7)[lb] = q[1];
    }
    CLGC_END_BLOCKS
}

// ---------------------------------------------------------------------------
// finalize: one block per run sums (or maxes) the partials of the kernel that
// just ran, in a fixed order, and updates the run's control block.

template <bool FAST>
__global__ void __launch_bounds__(kBlock) k_finalize(const KArgs ka, int what, int iter)
{
    __shared__ double lds[8];
    auto fin_ = [&](const RunArgs& ra) __attribute__((always_inline)) {
        Ctrl* c = ra.ctrl;
        const bool ok = c->status == ST_OK;
        switch (what) {
        case FIN_INIT: {
            const double tot = gather_partials(ra, KIND_LINK, 0, lds);
            if (threadIdx.x == 0) {
                c->unorm = tot;
                c->step = 0;
                c->bound = 0.0;
                c->eps = 0.0;
                c->kmax = 0.0;
                c->d_pre = tot / (12.0 * ra.V) - 1.0;
                c->status = isfinite(tot) ? ST_OK : ST_NONFINITE;
                c->hist_n = 0;
                c->alpha_cur = 0.0;
                c->upd_pending = 0;
                for (int x = 0; x < kXcds; ++x) c->kslot[0][x][0] = c->kslot[1][x][0] = 0ull;
            }
            break;
        }
        case FIN_UNORM: {
            const double tot = gather_partials(ra, KIND_LINK, 0, lds);
            if (threadIdx.x == 0) {
                c->unorm = tot;
                c->upd_pending = 0;
                if (!isfinite(tot)) c->status = ST_NONFINITE;
            }
            break;
        }
        case FIN_DRIFT: {
            const double km2 = gather_partials<true>(ra, KIND_DRIFT, 0, lds);
            if (threadIdx.x == 0) {
                const double kmax = sqrt(km2);
                double eps = ra.eps0;
                if (ra.adaptive) {
                    if (c->bound <= 0.0) c->bound = ra.drift_bound > 0.0 ? ra.drift_bound : ra.eps0 * kmax;
                    if (kmax > 0.0 && c->bound / kmax < ra.eps0) eps = c->bound / kmax;
                }
                c->kmax = kmax;
                c->eps = eps;
                if (!isfinite(kmax)) c->status = ST_NONFINITE;
            }
            break;
        }
        case FIN_UPDATE: {
            // nothing to do if the update left the links untouched (not ok) or a
            // cooling step already finished it
            if (!ok || !c->upd_pending) break;
            // (summed as the cooling kernels sum these partials, so that every
            // path gives the same bits)
            const double tot = wave_cool_sum(ra);
            if (threadIdx.x == 0) {
                c->unorm = tot;
                c->d_pre = tot / (12.0 * ra.V) - 1.0;
                c->step = c->step + 1;
                c->upd_pending = 0;
                if (!isfinite(tot)) c->status = ST_NONFINITE;
            }
            break;
        }
        case FIN_COOL: {
            // iter < 0: the run's own last cooling step (runs in a batch differ)
            const int it = iter < 0 ? ra.n_cool - 1 : iter;
            if (!ok || it < 0 || it >= ra.n_cool) break;
            const double tot = wave_cool_sum(ra);
            if (threadIdx.x == 0) {
                c->unorm = tot;
                if (it + 1 <= kMaxCoolHist) c->hist_un[it + 1] = tot;
                if (!isfinite(tot)) c->status = ST_NONFINITE;
            }
            break;
        }
        case FIN_MEASURE:
        case FIN_RECORD:
        case FIN_RECORD_STEP: {
            // the seven measurement sums (Tr P re / im, Tr P^-1 re / im, the
            // clover bracket re / im, the link norms): from the measurement
            // kernel, or from the recorded step's clover and drift kernels
            double o[7];
            for (int j = 0; j < 7; ++j) {
                if (what == FIN_RECORD_STEP) {
                    const int rj = j < 4 ? 1 + j : (j < 6 ? 2 + j : 5);
                    const int n = j == 4 || j == 5 ? ra.nblk[KIND_SITE] : ra.nblk[KIND_PLANE];
                    o[j] = gather_values(record_partial(ra, rj), n, lds);
                } else {
                    o[j] = gather_partials(ra, KIND_SITE, j, lds);
                }
                if (threadIdx.x == 0) c->obs[j] = o[j];
            }
            // the record entry of CL step n (1-based), measured on the links that
            // step left after its cooling (the measurement runs before step n + 1
            // or after a call's last step: either way the step counter is n)
            if (what != FIN_MEASURE && threadIdx.x == 0 && ok && ra.rec && c->step >= 1) {
                const double V = ra.V;
                const double qs = -1.0 / (256.0 * M_PI * M_PI);
                const double qr = qs * o[4], qi = qs * o[5];
                // S = S_W - i theta Q,  S_W = beta sum_x sum_{mu<nu} [1 - (Tr P + Tr P^-1) / 6]
                const double swr = ra.beta * (6.0 * V - (o[0] + o[2]) / 6.0);
                const double swi = -ra.beta * (o[1] + o[3]) / 6.0;
                double* e = ra.rec + (size_t)((c->step - 1) % kRecCap) * kRecFields;
                e[0] = (double)c->step;
                e[1] = c->d_pre;
                e[2] = o[6] / (12.0 * V) - 1.0;
                e[3] = o[0] / (18.0 * V);
                e[4] = o[1] / (18.0 * V);
                e[5] = qr;
                e[6] = qi;
                e[7] = swr + (ra.th_im * qr + ra.th_re * qi);
                e[8] = swi - (ra.th_re * qr - ra.th_im * qi);
                e[9] = c->eps;
                e[10] = c->kmax;
                e[11] = c->alpha_cur;
            }
            break;
        }
        default:
            break;
        }
    };
    if constexpr (FAST) {
        if (blockIdx.x == 0) fin_(ka.one);
    } else {
        for (int r = blockIdx.x; r < ka.hdr->nrun; r += gridDim.x) fin_(ka.runs[r]);
    }
}

// compact per-run status for the host after a batched step
__global__ void k_gather(const KArgs ka, GatherRec* out)
{
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < ka.hdr->nrun; r += gridDim.x * blockDim.x) {
        const Ctrl* c = ka.runs[r].ctrl;
        GatherRec g;
        g.step = c->step;
        g.status = c->status;
        g.pad = 0;
        g.eps = c->eps;
        g.kmax = c->kmax;
        g.unorm = c->unorm;
        g.d_pre = c->d_pre;
        out[r] = g;
    }
}

// ---------------------------------------------------------------------------
// small control kernels (stream-ordered writes of host-side parameters)

__global__ void k_write_args(RunArgs* dst, RunArgs src)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = src;
}

// zero n doubles (a kernel rather than a memset: safe under graph capture)
__global__ void k_zero(double* p, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0.0;
}

__global__ void k_write_state(Ctrl* c, int64_t step, double bound)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->step = step;
        c->bound = bound;
        // the drift of step n leaves its maximum in the slots of parity n & 1
        for (int x = 0; x < kXcds; ++x) c->kslot[0][x][0] = c->kslot[1][x][0] = 0ull;
    }
}

// ---------------------------------------------------------------------------
// Measurement of a device-resident link field without any allocation
// (cl_measure_links): the per-block partials live in a file-scope device
// array, the result goes to the caller's device memory, and nothing waits for
// the stream, so the call also works where hipMalloc cannot be called.

constexpr int kScratchMaxSites = 1 << 20;                   // 32^4
constexpr int kScratchBlocks = kScratchMaxSites / kBlock;   // 4096 logical blocks
constexpr int kScratchParts = 7;                            // partials per block
// 7 x 4096 doubles = 224 KiB on every GPU the library runs on, held until the
// process ends; every call on a GPU shares it
static __device__ __align__(256) double scratch[kScratchParts * kScratchBlocks];

// link (mu, s) of a field in the host layout [site][mu][row][col][re, im]
__device__ __forceinline__ mat3<double> load_aos(const double* __restrict__ f, const RunArgs& ra, int mu, const Site& s)
{
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2* q = (const d2*)(f + ((size_t)site_lex(ra, s) * 4 + mu) * 18);
    mat3<double> m;
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        const d2 c = q[e];
        m.e[e / 3][e % 3] = {c.x, c.y};
    }
    return m;
}

// one lane per site (lexicographic); block b writes part[j * gridDim.x + b]
__global__ void __launch_bounds__(kBlock) k_measure_links(const RunArgs ra, const double* __restrict__ links,
                                                          double* __restrict__ part)
{
    __shared__ double lds[7 * 4];
    const int s = (int)(blockIdx.x * kBlock + threadIdx.x);
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    if (s < ra.V) {
        Site x;
        int r = s / ra.L[0];
        x.x0 = s - r * ra.L[0];
        int q = r / ra.L[1];
        x.x1 = r - q * ra.L[1];
        r = q;
        q = r / ra.L[2];
        x.x2 = r - q * ra.L[2];
        x.x3 = q;
        site_obs_f64(ra, [&](int m, const Site& y) { return load_aos(links, ra, m, y); }, x, v);
    }
    block_reduce<7>(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < 7; ++j) part[j * gridDim.x + blockIdx.x] = v[j];
    }
}

// fixed-order sums of the nblk partials; out = P (re, im), Q (re, im), S (re, im), d
__global__ void __launch_bounds__(kBlock) k_measure_links_final(const RunArgs ra, const double* __restrict__ part,
                                                                int nblk, double* __restrict__ out)
{
    __shared__ double lds[8];
    double o[7];
    for (int j = 0; j < 7; ++j) o[j] = gather_values(part + (size_t)j * nblk, nblk, lds);
    if (threadIdx.x == 0) {
        const double V = ra.V;
        const double qs = -1.0 / (256.0 * M_PI * M_PI);
        const double qr = qs * o[4], qi = qs * o[5];
        const double swr = ra.beta * (6.0 * V - (o[0] + o[2]) / 6.0);
        const double swi = -ra.beta * (o[1] + o[3]) / 6.0;
        out[0] = o[0] / (18.0 * V);
        out[1] = o[1] / (18.0 * V);
        out[2] = qr;
        out[3] = qi;
        out[4] = swr + (ra.th_im * qr + ra.th_re * qi);
        out[5] = swi - (ra.th_re * qr - ra.th_im * qi);
        out[6] = o[6] / (12.0 * V) - 1.0;
    }
}

namespace {

// device address of `scratch` on each GPU, taken once per device with that
// device current (the array's name is only a host-side stand-in)
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

hipError_t scratch_of_current_device(double** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = (double*)p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace

// ---------------------------------------------------------------------------
// host launchers

namespace {

// a multiple of the XCD count, so that a logical slot keeps its XCD (see CLGC_FOR_BLOCKS)
inline int grid_of(const Launch& L, int kind)
{
    const int b = L.blocks[kind] > 0 ? L.blocks[kind] : 1;
    return (b + kXcds - 1) / kXcds * kXcds;
}

}  // namespace

// With L.ev_start / L.ev_stop set, the dispatch itself records the two events
// at its start and end (hipExtLaunchKernelGGL), so the elapsed time is the
// kernel's own execution time with no marker packets around it.
#define CLGC_LAUNCH_1(KERNEL, KIND, ...)                                                                  \
    do {                                                                                                  \
        const KArgs ka_ = make_kargs(L);                                                                  \
        if (L.ev_start)                                                                                   \
            hipExtLaunchKernelGGL(KERNEL, dim3(grid_of(L, KIND)), dim3(kBlock), 0, L.stream, L.ev_start,  \
                                  L.ev_stop, 0, ka_, ##__VA_ARGS__);                                      \
        else                                                                                              \
            hipLaunchKernelGGL(KERNEL, dim3(grid_of(L, KIND)), dim3(kBlock), 0, L.stream, ka_,            \
                               ##__VA_ARGS__);                                                            \
    } while (0)

// KERNEL names its instance with FAST_, bound here to the launch's path
#define CLGC_LAUNCH(KERNEL, KIND, ...)                                                                    \
    do {                                                                                                  \
        if (L.fast) {                                                                                     \
            constexpr bool FAST_ = true;                                                                  \
            CLGC_LAUNCH_1(KERNEL, KIND, ##__VA_ARGS__);                                                   \
        } else {                                                                                          \
            constexpr bool FAST_ = false;                                                                 \
            CLGC_LAUNCH_1(KERNEL, KIND, ##__VA_ARGS__);                                                   \
        }                                                                                                 \
    } while (0)

KArgs make_kargs(const Launch& L)
{
    KArgs k;
    k.hdr = L.hdr;
    k.runs = L.runs;
    k.one = L.one;
    return k;
}

hipError_t launch_init(const Launch& L, int prec, int perturbed, double sx, double sy)
{
    if (prec) CLGC_LAUNCH((k_init<float, FAST_>), KIND_LINK, perturbed, sx, sy);
    else CLGC_LAUNCH((k_init<double, FAST_>), KIND_LINK, perturbed, sx, sy);
    return hipGetLastError();
}

hipError_t launch_unorm(const Launch& L, int prec)
{
    if (prec) CLGC_LAUNCH((k_unorm<float, FAST_>), KIND_LINK);
    else CLGC_LAUNCH((k_unorm<double, FAST_>), KIND_LINK);
    return hipGetLastError();
}

hipError_t launch_unpack(const Launch& L, int prec, const double* aos)
{
    if (prec) CLGC_LAUNCH((k_unpack<float, FAST_>), KIND_LINK, aos);
    else CLGC_LAUNCH((k_unpack<double, FAST_>), KIND_LINK, aos);
    return hipGetLastError();
}

hipError_t launch_pack(const Launch& L, int prec, const void* field, double* aos)
{
    if (prec) CLGC_LAUNCH((k_pack<float, FAST_>), KIND_LINK, field, aos);
    else CLGC_LAUNCH((k_pack<double, FAST_>), KIND_LINK, field, aos);
    return hipGetLastError();
}

hipError_t launch_clover(const Launch& L, int prec, int only_theta, bool record)
{
    const int rec = record ? 1 : 0;
    if (prec) CLGC_LAUNCH((k_clover<float, FAST_>), KIND_PLANE, only_theta, rec);
    else CLGC_LAUNCH((k_clover<double, FAST_>), KIND_PLANE, only_theta, rec);
    return hipGetLastError();
}

hipError_t launch_drift(const Launch& L, int prec, bool theta)
{
    if (prec) {
        if (theta) CLGC_LAUNCH((k_drift<float, true, FAST_>), KIND_DRIFT);
        else CLGC_LAUNCH((k_drift<float, false, FAST_>), KIND_DRIFT);
    } else {
        if (theta) CLGC_LAUNCH((k_drift<double, true, FAST_>), KIND_DRIFT);
        else CLGC_LAUNCH((k_drift<double, false, FAST_>), KIND_DRIFT);
    }
    return hipGetLastError();
}

hipError_t launch_record_charge(const Launch& L)
{
    CLGC_LAUNCH((k_record_charge<FAST_>), KIND_SITE);
    return hipGetLastError();
}

hipError_t launch_update(const Launch& L, int prec)
{
    if (prec) CLGC_LAUNCH((k_update<float, FAST_>), KIND_COOL);
    else CLGC_LAUNCH((k_update<double, FAST_>), KIND_COOL);
    return hipGetLastError();
}

hipError_t launch_cool(const Launch& L, int prec, int phase, int iter)
{
    // a single lattice whose blocks loop over several chunks takes the
    // prefetching kernel (a batch keeps the plain ones: its runs are mostly
    // small, and the prefetching ones hold more registers)
    const int kind = phase ? KIND_COOL : KIND_OMEGA;
    if (L.fast && cool_chunks_total(L.one.V) > L.one.nblk[kind]) {
        if (prec) {
            if (phase) CLGC_LAUNCH((k_cool_apply_pf<float, FAST_>), KIND_COOL, iter);
            else CLGC_LAUNCH((k_cool_omega_pf<float, FAST_>), KIND_OMEGA, iter);
        } else {
            if (phase) CLGC_LAUNCH((k_cool_apply_pf<double, FAST_>), KIND_COOL, iter);
            else CLGC_LAUNCH((k_cool_omega_pf<double, FAST_>), KIND_OMEGA, iter);
        }
        return hipGetLastError();
    }
    if (prec) {
        if (phase) CLGC_LAUNCH((k_cool_apply<float, FAST_>), KIND_COOL, iter);
        else CLGC_LAUNCH((k_cool_omega<float, FAST_>), KIND_OMEGA, iter);
    } else {
        if (phase) CLGC_LAUNCH((k_cool_apply<double, FAST_>), KIND_COOL, iter);
        else CLGC_LAUNCH((k_cool_omega<double, FAST_>), KIND_OMEGA, iter);
    }
    return hipGetLastError();
}

hipError_t launch_gradnorm(const Launch& L, int prec, int iter)
{
    if (prec) CLGC_LAUNCH((k_gradnorm<float, FAST_>), KIND_COOL, iter);
    else CLGC_LAUNCH((k_gradnorm<double, FAST_>), KIND_COOL, iter);
    return hipGetLastError();
}

hipError_t launch_measure(const Launch& L, int prec, bool from_f)
{
    if (prec) CLGC_LAUNCH((k_measure<float, FAST_, false>), KIND_SITE);
    else if (from_f) CLGC_LAUNCH((k_measure<double, FAST_, true>), KIND_SITE);
    else CLGC_LAUNCH((k_measure<double, FAST_, false>), KIND_SITE);
    return hipGetLastError();
}

hipError_t launch_finalize(const Launch& L, int what, int iter)
{
    const int g = L.fast ? 1 : (L.nrun > 0 ? L.nrun : 1);
    const KArgs ka = make_kargs(L);
    auto* const kern = L.fast ? k_finalize<true> : k_finalize<false>;
    if (L.ev_start)
        hipExtLaunchKernelGGL(kern, dim3(g), dim3(kBlock), 0, L.stream, L.ev_start, L.ev_stop, 0, ka, what, iter);
    else
        hipLaunchKernelGGL(kern, dim3(g), dim3(kBlock), 0, L.stream, ka, what, iter);
    return hipGetLastError();
}

hipError_t launch_gather(const Launch& L, GatherRec* out)
{
    hipLaunchKernelGGL(k_gather, dim3(1), dim3(kBlock), 0, L.stream, make_kargs(L), out);
    return hipGetLastError();
}

hipError_t launch_write_args(RunArgs* dst, const RunArgs& src, hipStream_t st)
{
    hipLaunchKernelGGL(k_write_args, dim3(1), dim3(64), 0, st, dst, src);
    return hipGetLastError();
}

hipError_t launch_zero(double* p, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero, dim3((n + 255) / 256 < 64 ? (n + 255) / 256 : 64), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_write_state(Ctrl* c, int64_t step, double bound, hipStream_t st)
{
    hipLaunchKernelGGL(k_write_state, dim3(1), dim3(64), 0, st, c, step, bound);
    return hipGetLastError();
}

}  // namespace clgc

extern "C" cl_status cl_measure_links(const double* dev_links, const int32_t* dims, double beta, double theta_re,
                                      double theta_im, double* dev_out, void* hip_stream)
{
    using namespace clgc;
    if (!dev_links || !dims || !dev_out) return fail(CL_EINVAL, "NULL argument");
    long long V = 1;
    for (int m = 0; m < 4; ++m) {
        if (dims[m] < 2 || (dims[m] & 1)) return fail(CL_EINVAL, "extent L%d = %d must be even and >= 2", m, dims[m]);
        V *= dims[m];
    }
    if (V > kScratchMaxSites)
        return fail(CL_EINVAL, "cl_measure_links: %lld sites, at most %d (its scratch is sized for 32^4)", V,
                    kScratchMaxSites);
    if (!(beta > 0) || !std::isfinite(beta) || !std::isfinite(theta_re) || !std::isfinite(theta_im))
        return fail(CL_EINVAL, "beta must be > 0 and finite, theta finite");
    double* part = nullptr;
    HIP_TRY(scratch_of_current_device(&part));
    RunArgs ra;
    std::memset(&ra, 0, sizeof ra);
    for (int m = 0; m < 4; ++m) ra.L[m] = dims[m];
    ra.Lh0 = dims[0] / 2;
    ra.V = (int)V;
    ra.Vh = (int)(V / 2);
    ra.beta = beta;
    ra.th_re = theta_re;
    ra.th_im = theta_im;
    const int nblk = (int)((V + kBlock - 1) / kBlock);
    const hipStream_t st = (hipStream_t)hip_stream;
    // every partial slot [0, nblk) is written before it is read: nothing of an
    // earlier call's scratch contents is used
    hipLaunchKernelGGL(k_measure_links, dim3(nblk), dim3(kBlock), 0, st, ra, dev_links, part);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_measure_links_final, dim3(1), dim3(kBlock), 0, st, ra, (const double*)part, nblk, dev_out);
    HIP_TRY(hipGetLastError());
    return CL_OK;
}

