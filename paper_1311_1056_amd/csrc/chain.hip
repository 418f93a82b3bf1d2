// chain.hip -- complex Langevin with adaptive gauge cooling for the SU(2)
// Polyakov chain (section "Adaptive gauge cooling in the SU(2) Polyakov chain
// model", action eq. (eq:s); cooling eq. (eq:24); distance eq. (d)).
//
// One workgroup owns one chain of n <= 1024 links for a whole call: four
// links per thread live in registers, so a call of many CL steps reads and
// writes HBM once.  Per CL step:
//   drift   K_k = -D_a S sigma_a = i beta TL(P_k), P_k = U_k ... U_{n-1} U_0 ... U_{k-1}
//           (the loop opened at link k), from an inclusive prefix and an
//           inclusive suffix scan of the chain's 2x2 products in LDS
//           (Hillis-Steele over the 256 per-thread products, 8 rounds);
//   step    eps = min(eps0, B / K_max), K_max = max_k ||K_k|| (block max);
//   update  U_k <- exp(i (eps K_k + sqrt(eps) eta_a sigma_a)) U_k, then
//           U_k <- U_k / sqrt(det U_k);
//   cooling n_c Jacobi steps: G_k = U_k U_k^dag - U_{k-1}^dag U_{k-1},
//           Omega_k = exp(-4 eps_c alpha_ad TL(G_k)) (sum_a f_ak sigma_a = 4 TL(G_k)
//           for f_ak = 2 Tr(sigma_a G_k)), U_k <- Omega_k U_k Omega_{k+1}^{-1};
//           alpha_ad = alpha / D with D_0 = 1, D_1 = UN / n, D_2 = mean |f_ak|;
//   measure L = Tr(U_0 ... U_{n-1}) / 2 (ordered tree product), d = UN/(2n) - 1.
// All block reductions are fixed-order, so a chain's result does not depend
// on the launch.  Exponentials of traceless 2x2 matrices use X^2 = w 1:
// exp(X) = C(w) 1 + S(w) X with the even and odd series C, S in w.
#include "chain.hpp"
#include "philox.hpp"
#include "su3.hpp"

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>

namespace clgc {
namespace {

using cxd = cx<double>;

// row-major 2x2 complex [[a, b], [c, d]]
struct m2 {
    cxd a, b, c, d;
};

__device__ __forceinline__ m2 m2_id() { return m2{{1.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {1.0, 0.0}}; }

__device__ __forceinline__ m2 mul(const m2& x, const m2& y)
{
    m2 r;
    r.a = cfma(x.b, y.c, x.a * y.a);
    r.b = cfma(x.b, y.d, x.a * y.b);
    r.c = cfma(x.d, y.c, x.c * y.a);
    r.d = cfma(x.d, y.d, x.c * y.b);
    return r;
}

__device__ __forceinline__ m2 dag(const m2& x) { return m2{conj(x.a), conj(x.c), conj(x.b), conj(x.d)}; }

__device__ __forceinline__ m2 scale(const m2& x, cxd s) { return m2{s * x.a, s * x.b, s * x.c, s * x.d}; }

__device__ __forceinline__ m2 sub(const m2& x, const m2& y) { return m2{x.a - y.a, x.b - y.b, x.c - y.c, x.d - y.d}; }

__device__ __forceinline__ double nrm2(const m2& x) { return norm2(x.a) + norm2(x.b) + norm2(x.c) + norm2(x.d); }

// traceless part
__device__ __forceinline__ m2 tl(m2 x)
{
    const cxd t = {0.5 * (x.a.re + x.d.re), 0.5 * (x.a.im + x.d.im)};
    x.a = x.a - t;
    x.d = x.d - t;
    return x;
}

// exp(X) for traceless X: scaled by 2^-k so that ||X||_F <= 1, then
// exp = C(w) 1 + S(w) X (w = X^2 / 1 = x_00^2 + x_01 x_10, |w| <= 1, 13 terms
// each, truncation below 1e-26), squared k times; k is bounded so that a
// non-finite X (a runaway, flagged by the drift maximum) ends at once.
__device__ __forceinline__ m2 exp_tl(m2 X)
{
    const double fro2 = nrm2(X);
    int k = 0;
    if (fro2 > 1.0) {
        const double lk = 0.5 * log2(fro2);
        k = lk < 1100.0 ? (int)ceil(lk) : 0;
        X = scale(X, cxd{ldexp(1.0, -k), 0.0});
    }
    const cxd w = cfma(X.b, X.c, X.a * X.a);
    cxd C = {1.0, 0.0}, S = {1.0, 0.0};
#pragma unroll
    for (int m = 12; m >= 1; --m) {
        // C_m-1 = 1 + w C_m / ((2m-1) 2m),  S_m-1 = 1 + w S_m / (2m (2m+1))
        const double rc = 1.0 / ((2.0 * m - 1.0) * (2.0 * m));
        const double rs = 1.0 / ((2.0 * m) * (2.0 * m + 1.0));
        const cxd wc = w * C, ws = w * S;
        C = cxd{fma(rc, wc.re, 1.0), rc * wc.im};
        S = cxd{fma(rs, ws.re, 1.0), rs * ws.im};
    }
    m2 E = scale(X, S);
    E.a = E.a + C;
    E.d = E.d + C;
    for (int i = 0; i < k; ++i) E = mul(E, E);
    return E;
}

// principal square root
__device__ __forceinline__ cxd csqrt_p(cxd z)
{
    const double r = sqrt(norm2(z));
    const double re = sqrt(0.5 * (r + z.re));
    const double im = copysign(sqrt(fmax(0.0, 0.5 * (r - z.re))), z.im);
    return {re, im};
}

// U / sqrt(det U)
__device__ __forceinline__ m2 renorm(const m2& U)
{
    const cxd s = csqrt_p(U.a * U.d - U.b * U.c);
    const double q = 1.0 / norm2(s);
    return scale(U, cxd{s.re * q, -s.im * q});
}

__device__ __forceinline__ m2 load_link(const double* p)
{
    return m2{{p[0], p[1]}, {p[2], p[3]}, {p[4], p[5]}, {p[6], p[7]}};
}

__device__ __forceinline__ void store_link(double* p, const m2& x)
{
    p[0] = x.a.re;
    p[1] = x.a.im;
    p[2] = x.b.re;
    p[3] = x.b.im;
    p[4] = x.c.re;
    p[5] = x.c.im;
    p[6] = x.d.re;
    p[7] = x.d.im;
}

// p ? x : y by components (a ?: on the structs would select their addresses)
__device__ __forceinline__ m2 pick(bool p, const m2& x, const m2& y)
{
    return m2{{p ? x.a.re : y.a.re, p ? x.a.im : y.a.im}, {p ? x.b.re : y.b.re, p ? x.b.im : y.b.im},
              {p ? x.c.re : y.c.re, p ? x.c.im : y.c.im}, {p ? x.d.re : y.d.re, p ? x.d.im : y.d.im}};
}

// LDS transfers element by element into component-major arrays (a
// whole-struct copy between address spaces would become a memcpy that keeps
// the registers' copy in scratch memory)
__device__ __forceinline__ void put(double (*arr)[kChainBlock], int i, const m2& x)
{
    arr[0][i] = x.a.re;
    arr[1][i] = x.a.im;
    arr[2][i] = x.b.re;
    arr[3][i] = x.b.im;
    arr[4][i] = x.c.re;
    arr[5][i] = x.c.im;
    arr[6][i] = x.d.re;
    arr[7][i] = x.d.im;
}

__device__ __forceinline__ m2 get(const double (*arr)[kChainBlock], int i)
{
    return m2{{arr[0][i], arr[1][i]}, {arr[2][i], arr[3][i]}, {arr[4][i], arr[5][i]}, {arr[6][i], arr[7][i]}};
}

// ---------------------------------------------------------------------------
// block reductions (fixed order: waves in order, lanes by butterfly)

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max_d(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

template <bool MAX>
__device__ __forceinline__ double block_all(double v, double* red)
{
    v = MAX ? wave_max_d(v) : wave_sum_d(v);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[wv] = v;
    __syncthreads();
    double r = red[0];
#pragma unroll
    for (int i = 1; i < kChainBlock / 64; ++i) r = MAX ? fmax(r, red[i]) : r + red[i];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// the per-chain workgroup state

// Matrices in LDS are stored component-major (component e of thread t at
// [e][t]), so that a wavefront's accesses fall on consecutive banks.
struct ChainLds {
    double pre[8][kChainBlock], suf[8][kChainBlock];  // scans / products
    double edge[8][kChainBlock];  // last link, then the first Omega^-1, of every thread
    double last[8];               // link n-1
    double red[kChainBlock / 64];
};

struct Chain {
    m2 U[kChainPerThread];
    int n, k0;  // chain length, first link of this thread
    __device__ bool valid(int j) const { return k0 + j < n; }
};

// The loops P_k of this thread's links (drift) and the chain's product.
__device__ __forceinline__ void chain_loops(const Chain& ch, ChainLds& s, m2 (&P)[kChainPerThread])
{
    const int t = threadIdx.x;
    m2 M = m2_id();
#pragma unroll
    for (int j = 0; j < kChainPerThread; ++j)
        if (ch.valid(j)) M = mul(M, ch.U[j]);
    // inclusive prefix I_t = M_0 ... M_t and suffix S_t = M_t ... M_last
    m2 I = M, S = M;
    for (int off = 1; off < kChainBlock; off <<= 1) {
        put(s.pre, t, I);
        put(s.suf, t, S);
        __syncthreads();
        if (t >= off) I = mul(get(s.pre, t - off), I);
        if (t + off < kChainBlock) S = mul(S, get(s.suf, t + off));
        __syncthreads();
    }
    put(s.pre, t, I);
    put(s.suf, t, S);
    __syncthreads();
    // (no ?: on matrix values below: it selects addresses and keeps the
    // operands in scratch memory)
    m2 E = m2_id(), F = m2_id();
    if (t > 0) E = get(s.pre, t - 1);                 // M_0 ... M_t-1
    if (t + 1 < kChainBlock) F = get(s.suf, t + 1);   // M_t+1 ... M_last
    __syncthreads();
    // A_j = E U_0 ... U_j-1 (links before), B_j = U_j ... U_3 F (links from j on)
    m2 A[kChainPerThread], B[kChainPerThread];
    // (invalid links are the identity, so they need no test)
    A[0] = E;
#pragma unroll
    for (int j = 1; j < kChainPerThread; ++j) A[j] = mul(A[j - 1], ch.U[j - 1]);
    B[kChainPerThread - 1] = mul(ch.U[kChainPerThread - 1], F);
#pragma unroll
    for (int j = kChainPerThread - 2; j >= 0; --j) B[j] = mul(ch.U[j], B[j + 1]);
#pragma unroll
    for (int j = 0; j < kChainPerThread; ++j) P[j] = mul(B[j], A[j]);
}

// ordered product U_0 ... U_{n-1} (valid in every thread)
__device__ __forceinline__ m2 chain_product(const Chain& ch, ChainLds& s)
{
    const int t = threadIdx.x;
    m2 M = m2_id();
#pragma unroll
    for (int j = 0; j < kChainPerThread; ++j)
        if (ch.valid(j)) M = mul(M, ch.U[j]);
    put(s.pre, t, M);
    __syncthreads();
    for (int off = 1; off < kChainBlock; off <<= 1) {
        if ((t & (2 * off - 1)) == 0) put(s.pre, t, mul(get(s.pre, t), get(s.pre, t + off)));
        __syncthreads();
    }
    const m2 r = get(s.pre, 0);
    __syncthreads();
    return r;
}

__device__ __forceinline__ double chain_unorm(const Chain& ch, ChainLds& s)
{
    double u = 0.0;
#pragma unroll
    for (int j = 0; j < kChainPerThread; ++j)
        if (ch.valid(j)) u += nrm2(ch.U[j]);
    return block_all<false>(u, s.red);
}

// the drift of this thread's links and K_max of the chain
__device__ __forceinline__ double chain_drift(const ChainArgs& a, const Chain& ch, ChainLds& s,
                                              m2 (&K)[kChainPerThread])
{
    chain_loops(ch, s, K);
    const cxd ib = {-a.beta_im, a.beta_re};  // i beta
    double kn2 = 0.0;
#pragma unroll
    for (int j = 0; j < kChainPerThread; ++j) {
        K[j] = scale(tl(K[j]), ib);
        if (ch.valid(j)) {
            double v = 0.5 * nrm2(K[j]);
            if (!isfinite(v)) v = INFINITY;
            kn2 = fmax(kn2, v);
        }
    }
    return sqrt(block_all<true>(kn2, s.red));
}

// Hermitian 2x2 [[p, q], [q*, r]] (p, r real)
struct h2 {
    double p, r;
    cxd q;
};

// H U and U H for Hermitian H
__device__ __forceinline__ m2 hmul(const h2& H, const m2& U)
{
    const cxd qc = conj(H.q);
    return m2{cfma(H.q, U.c, H.p * U.a), cfma(H.q, U.d, H.p * U.b), cfma(qc, U.a, H.r * U.c), cfma(qc, U.b, H.r * U.d)};
}

__device__ __forceinline__ m2 mulh(const m2& U, const h2& H)
{
    const cxd qc = conj(H.q);
    return m2{cfma(U.b, qc, H.p * U.a), cfma(U.b, cxd{H.r, 0.0}, U.a * H.q), cfma(U.d, qc, H.p * U.c),
              cfma(U.d, cxd{H.r, 0.0}, U.c * H.q)};
}

// Omega = exp(A) and Omega^-1 = exp(-A) for A = [[g, q], [q*, -g]] Hermitian
// traceless: A^2 = w 1 with w = g^2 + |q|^2 >= 0, so exp(+-A) = C 1 +- S A with
// C = cosh(sqrt w), S = sinh(sqrt w) / sqrt w (exact inverses: C^2 - S^2 w = 1).
__device__ __forceinline__ void herm_exp2(double g, cxd q, h2& Om, h2& Oi)
{
    const double w = fma(g, g, norm2(q));
    double C, S;
    if (w < 0.25) {
        // even and odd series in w: the first omitted terms, w^10 / 20! and
        // w^10 / 21!, are below 1e-24
        C = 1.0;
        S = 1.0;
#pragma unroll
        for (int m = 9; m >= 1; --m) {
            C = fma(w * (1.0 / ((2.0 * m - 1.0) * (2.0 * m))), C, 1.0);
            S = fma(w * (1.0 / ((2.0 * m) * (2.0 * m + 1.0))), S, 1.0);
        }
    } else {
        const double l = sqrt(w), e = exp(l), ei = 1.0 / e;
        C = 0.5 * (e + ei);
        S = 0.5 * (e - ei) / l;
    }
    const double Sg = S * g;
    const cxd Sq = {S * q.re, S * q.im};
    Om = h2{C + Sg, C - Sg, Sq};
    Oi = h2{C - Sg, C + Sg, cxd{-Sq.re, -Sq.im}};
}

// one Jacobi cooling step at eps_c alpha_ad chosen by the mode
__device__ __forceinline__ void chain_cool_step(const ChainArgs& a, Chain& ch, ChainLds& s)
{
    const int t = threadIdx.x;
    // neighbours: link k-1 of this thread's first link
    put(s.edge, t, ch.U[kChainPerThread - 1]);
    if (ch.valid(0) && (ch.n - 1) / kChainPerThread == t) {
        // link n-1 by compile-time selects (a runtime index would put U in scratch)
        const int jl = (ch.n - 1) % kChainPerThread;
        m2 u = ch.U[0];
#pragma unroll
        for (int j = 1; j < kChainPerThread; ++j) u = pick(j == jl, ch.U[j], u);
        s.last[0] = u.a.re;
        s.last[1] = u.a.im;
        s.last[2] = u.b.re;
        s.last[3] = u.b.im;
        s.last[4] = u.c.re;
        s.last[5] = u.c.im;
        s.last[6] = u.d.re;
        s.last[7] = u.d.im;
    }
    __syncthreads();
    m2 prev0 = m2{{s.last[0], s.last[1]}, {s.last[2], s.last[3]}, {s.last[4], s.last[5]}, {s.last[6], s.last[7]}};
    if (t > 0) prev0 = get(s.edge, t - 1);
    __syncthreads();
    // G_k = TL(U U^dag - W^dag W) = [[g, q], [q*, -g]]: sum_a f_ak sigma_a = 4 TL(G_k)
    // (the trace, the difference of the two links' norms, is no direction of the
    // gauge orbit), f_1 = 4 Re q, f_2 = -4 Im q, f_3 = 4 g
    double g[kChainPerThread];
    cxd q[kChainPerThread];
    double un = 0.0, fsum = 0.0;
#pragma unroll
    for (int j = 0; j < kChainPerThread; ++j) {
        m2 W = prev0;
        if (j > 0) W = ch.U[j - 1];
        const m2& U = ch.U[j];
        const double h00 = norm2(U.a) + norm2(U.b) - norm2(W.a) - norm2(W.c);
        const double h11 = norm2(U.c) + norm2(U.d) - norm2(W.b) - norm2(W.d);
        // (U U^dag)_01 = a c* + b d*,  (W^dag W)_01 = wa* wb + wc* wd
        const cxd uu = cfma(U.b, conj(U.d), U.a * conj(U.c));
        const cxd ww = cfma(conj(W.c), W.d, conj(W.a) * W.b);
        g[j] = 0.5 * (h00 - h11);
        q[j] = uu - ww;
        if (ch.valid(j)) {
            un += nrm2(U);
            fsum += 4.0 * (fabs(q[j].re) + fabs(q[j].im) + fabs(g[j]));
        }
    }
    double D = 1.0;
    if (a.mode == 1) D = block_all<false>(un, s.red) / ch.n;
    if (a.mode == 2) D = block_all<false>(fsum, s.red) / (3.0 * ch.n);
    const double c = -4.0 * a.eps_c * (a.alpha / D);
    h2 Om[kChainPerThread], Oi[kChainPerThread];
#pragma unroll
    for (int j = 0; j < kChainPerThread; ++j) herm_exp2(c * g[j], cxd{c * q[j].re, c * q[j].im}, Om[j], Oi[j]);
    s.edge[0][t] = Oi[0].p;
    s.edge[1][t] = Oi[0].r;
    s.edge[2][t] = Oi[0].q.re;
    s.edge[3][t] = Oi[0].q.im;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kChainPerThread; ++j) {
        if (!ch.valid(j)) continue;
        const int k = ch.k0 + j;
        // Omega^-1 of site k+1: this thread's next one, the next thread's first,
        // or (k = n-1) the first of the chain
        h2 On;
        if (k + 1 == ch.n || j + 1 == kChainPerThread) {
            const int o = k + 1 == ch.n ? 0 : (t + 1) % kChainBlock;
            On = h2{s.edge[0][o], s.edge[1][o], cxd{s.edge[2][o], s.edge[3][o]}};
        } else {
            On = Oi[(j + 1) % kChainPerThread];
        }
        ch.U[j] = mulh(hmul(Om[j], ch.U[j]), On);
    }
    __syncthreads();
}

__device__ __forceinline__ void chain_load(const ChainArgs& a, int chain, Chain& ch)
{
    ch.n = a.n;
    ch.k0 = (int)threadIdx.x * kChainPerThread;
    const double* base = a.links + (size_t)chain * a.n * 8;
#pragma unroll
    for (int j = 0; j < kChainPerThread; ++j) {
        ch.U[j] = m2_id();
        if (ch.valid(j)) ch.U[j] = load_link(base + (size_t)(ch.k0 + j) * 8);
    }
}

__device__ __forceinline__ void chain_store(const ChainArgs& a, int chain, const Chain& ch)
{
    double* base = a.links + (size_t)chain * a.n * 8;
#pragma unroll
    for (int j = 0; j < kChainPerThread; ++j)
        if (ch.valid(j)) store_link(base + (size_t)(ch.k0 + j) * 8, ch.U[j]);
}

// ---------------------------------------------------------------------------
// kernels

// U_k = exp(i sigma_a (x_a + i y_a)), x ~ N(0, sx), y ~ N(0, sy); fresh control block
__global__ void __launch_bounds__(kChainBlock) k_chain_init(ChainArgs a, double sx, double sy)
{
    const int chain = blockIdx.y;
    const int k = blockIdx.x * kChainBlock + (int)threadIdx.x;
    if (k < a.n) {
        double p[8];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            normal_pair<double>(a.seed, (uint32_t)k, 0u, (uint32_t)chain, (kChainTagInit << 16) | (uint32_t)j, p[2 * j],
                                p[2 * j + 1]);
        // c_a = i (x_a + i y_a) = -y_a + i x_a for x = (p0, p1, p2), y = (p4, p5, p6)
        const cxd c1 = {-sy * p[4], sx * p[0]}, c2 = {-sy * p[5], sx * p[1]}, c3 = {-sy * p[6], sx * p[2]};
        // sum_a c_a sigma_a = [[c3, c1 - i c2], [c1 + i c2, -c3]]
        const m2 X = {c3, c1 - cxd{-c2.im, c2.re}, c1 + cxd{-c2.im, c2.re}, cxd{-c3.re, -c3.im}};
        store_link(a.links + ((size_t)chain * a.n + k) * 8, exp_tl(X));
    }
    if (k == 0) {
        ChainCtrl c = {};
        a.ctrl[chain] = c;
    }
}

// n_steps CL steps of every chain, each followed by n_cool cooling steps and a
// measurement; the record of step i of chain c goes to obs[i][c] if asked.
__global__ void __launch_bounds__(kChainBlock) k_chain_run(ChainArgs a, int n_steps)
{
    __shared__ ChainLds s;
    const int chain = blockIdx.x;
    ChainCtrl* cc = a.ctrl + chain;
    __shared__ int s_status;
    __shared__ int64_t s_step;
    __shared__ double s_bound;
    if (threadIdx.x == 0) {
        s_status = cc->status;
        s_step = cc->step;
        s_bound = cc->bound;
    }
    __syncthreads();
    if (s_status != 0) return;  // block-uniform
    int64_t step = s_step;
    double bound = s_bound;
    Chain ch;
    chain_load(a, chain, ch);
    double sL_re = 0.0, sL_im = 0.0, sd = 0.0, eps = 0.0, kmax = 0.0, d_pre = 0.0, d = 0.0;
    cxd L = {0.0, 0.0};
    int status = 0, done = 0;
    for (int i = 0; i < n_steps; ++i) {
        m2 K[kChainPerThread];
        kmax = chain_drift(a, ch, s, K);
        if (!isfinite(kmax)) {  // block-uniform (a block maximum)
            status = 1;
            break;
        }
        eps = a.eps0;
        if (a.adaptive) {
            if (bound <= 0.0) bound = a.drift_bound > 0.0 ? a.drift_bound : a.eps0 * kmax;
            if (kmax > 0.0 && bound / kmax < a.eps0) eps = bound / kmax;
        }
        const double se = sqrt(eps) * 1.41421356237309504880;  // sqrt(eps) * sqrt(2)
#pragma unroll
        for (int j = 0; j < kChainPerThread; ++j) {
            if (!ch.valid(j)) continue;
            double n0, n1, n2, n3;
            const uint32_t k = (uint32_t)(ch.k0 + j);
            normal_pair<double>(a.seed, k, (uint32_t)step, (uint32_t)chain, (kChainTagNoise << 16) | 0u, n0, n1);
            normal_pair<double>(a.seed, k, (uint32_t)step, (uint32_t)chain, (kChainTagNoise << 16) | 1u, n2, n3);
            const double e1 = se * n0, e2 = se * n1, e3 = se * n2;
            // eps K + sum_a eta_a sigma_a, times i
            m2 Y = scale(K[j], cxd{eps, 0.0});
            Y.a = Y.a + cxd{e3, 0.0};
            Y.b = Y.b + cxd{e1, -e2};
            Y.c = Y.c + cxd{e1, e2};
            Y.d = Y.d + cxd{-e3, 0.0};
            ch.U[j] = renorm(mul(exp_tl(scale(Y, cxd{0.0, 1.0})), ch.U[j]));
        }
        ++step;
        d_pre = chain_unorm(ch, s) / (2.0 * ch.n) - 1.0;
        for (int ic = 0; ic < a.n_cool; ++ic) chain_cool_step(a, ch, s);
        const double un = chain_unorm(ch, s);
        d = un / (2.0 * ch.n) - 1.0;
        const m2 Pt = chain_product(ch, s);
        L = {0.5 * (Pt.a.re + Pt.d.re), 0.5 * (Pt.a.im + Pt.d.im)};
        if (!isfinite(un) || !isfinite(L.re) || !isfinite(L.im)) {
            status = 1;
            break;
        }
        sL_re += L.re;
        sL_im += L.im;
        sd += d;
        ++done;
        if (a.record && i < a.obs_cap && threadIdx.x == 0) {
            double* o = a.obs + ((size_t)i * a.n_chains + chain) * kChainObs;
            o[0] = L.re;
            o[1] = L.im;
            o[2] = d;
            o[3] = eps;
            o[4] = kmax;
            o[5] = d_pre;
        }
    }
    if (status == 0) chain_store(a, chain, ch);  // a runaway step leaves the links as they were
    if (threadIdx.x == 0) {
        cc->step = step;
        cc->bound = bound;
        cc->status = status;
        cc->eps = eps;
        cc->kmax = kmax;
        cc->d_pre = d_pre;
        cc->d = d;
        cc->L_re = L.re;
        cc->L_im = L.im;
        cc->sum_L_re = sL_re;
        cc->sum_L_im = sL_im;
        cc->sum_d = sd;
        cc->sum_n = done;
    }
}

// the drift of every link (K[chain][k][8]) and K_max (ctrl.kmax)
__global__ void __launch_bounds__(kChainBlock) k_chain_drift(ChainArgs a)
{
    __shared__ ChainLds s;
    const int chain = blockIdx.x;
    Chain ch;
    chain_load(a, chain, ch);
    m2 K[kChainPerThread];
    const double kmax = chain_drift(a, ch, s, K);
    double* base = a.K + (size_t)chain * a.n * 8;
#pragma unroll
    for (int j = 0; j < kChainPerThread; ++j)
        if (ch.valid(j)) store_link(base + (size_t)(ch.k0 + j) * 8, K[j]);
    if (threadIdx.x == 0) a.ctrl[chain].kmax = kmax;
}

// n_cool cooling steps of every chain, then L and d into the control block
__global__ void __launch_bounds__(kChainBlock) k_chain_cool(ChainArgs a)
{
    __shared__ ChainLds s;
    const int chain = blockIdx.x;
    Chain ch;
    chain_load(a, chain, ch);
    for (int ic = 0; ic < a.n_cool; ++ic) chain_cool_step(a, ch, s);
    const double un = chain_unorm(ch, s);
    const m2 Pt = chain_product(ch, s);
    chain_store(a, chain, ch);
    if (threadIdx.x == 0) {
        ChainCtrl* cc = a.ctrl + chain;
        cc->d = un / (2.0 * ch.n) - 1.0;
        cc->L_re = 0.5 * (Pt.a.re + Pt.d.re);
        cc->L_im = 0.5 * (Pt.a.im + Pt.d.im);
        if (!isfinite(un)) cc->status = 1;
    }
}

// L and d of every chain into the control block
__global__ void __launch_bounds__(kChainBlock) k_chain_measure(ChainArgs a)
{
    __shared__ ChainLds s;
    const int chain = blockIdx.x;
    Chain ch;
    chain_load(a, chain, ch);
    const double un = chain_unorm(ch, s);
    const m2 Pt = chain_product(ch, s);
    if (threadIdx.x == 0) {
        ChainCtrl* cc = a.ctrl + chain;
        cc->d = un / (2.0 * ch.n) - 1.0;
        cc->L_re = 0.5 * (Pt.a.re + Pt.d.re);
        cc->L_im = 0.5 * (Pt.a.im + Pt.d.im);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers (one workgroup per chain)

hipError_t chain_launch_init(const ChainArgs& a, double sx, double sy, hipStream_t st)
{
    hipLaunchKernelGGL(k_chain_init, dim3((a.n + kChainBlock - 1) / kChainBlock, a.n_chains), dim3(kChainBlock), 0, st,
                       a, sx, sy);
    return hipGetLastError();
}

hipError_t chain_launch_run(const ChainArgs& a, int n_steps, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1)
{
    if (ev0)
        hipExtLaunchKernelGGL(k_chain_run, dim3(a.n_chains), dim3(kChainBlock), 0, st, ev0, ev1, 0, a, n_steps);
    else
        hipLaunchKernelGGL(k_chain_run, dim3(a.n_chains), dim3(kChainBlock), 0, st, a, n_steps);
    return hipGetLastError();
}

hipError_t chain_launch_drift(const ChainArgs& a, hipStream_t st)
{
    hipLaunchKernelGGL(k_chain_drift, dim3(a.n_chains), dim3(kChainBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t chain_launch_cool(const ChainArgs& a, hipStream_t st)
{
    hipLaunchKernelGGL(k_chain_cool, dim3(a.n_chains), dim3(kChainBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t chain_launch_measure(const ChainArgs& a, hipStream_t st)
{
    hipLaunchKernelGGL(k_chain_measure, dim3(a.n_chains), dim3(kChainBlock), 0, st, a);
    return hipGetLastError();
}

}  // namespace clgc
