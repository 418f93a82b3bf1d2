// chain.hip -- complex Langevin with adaptive gauge cooling for the SU(2)
// Polyakov chain (section "Adaptive gauge cooling in the SU(2) Polyakov chain
// model", action eq. (eq:s); cooling eq. (eq:24); distance eq. (d)).
//
// A chain of n <= 1024 links is owned by T threads of one workgroup for a
// whole call (PT links per thread, two up to 512 links and four above; T the
// smallest power of two with PT T >= n; short chains share a workgroup): the
// links live in registers, so a call of many CL
// steps reads and writes HBM once.  Per CL step:
//   drift   K_k = -D_a S sigma_a = i beta TL(P_k), P_k = U_k ... U_{n-1} U_0 ... U_{k-1}
//           (the loop opened at link k), from an inclusive prefix and an
//           inclusive suffix scan of the chain's 2x2 products in LDS
//           (Hillis-Steele over the T per-thread products, log2 T rounds);
//   step    eps = min(eps0, B / K_max), K_max = max_k ||K_k|| (chain max);
//   update  U_k <- exp(i (eps K_k + sqrt(eps) eta_a sigma_a)) U_k, then
//           U_k <- U_k / sqrt(det U_k);
//   cooling n_c Jacobi steps: G_k = U_k U_k^dag - U_{k-1}^dag U_{k-1},
//           Omega_k = exp(-4 eps_c alpha_ad TL(G_k)) (sum_a f_ak sigma_a = 4 TL(G_k)
//           for f_ak = 2 Tr(sigma_a G_k)), U_k <- Omega_k U_k Omega_{k+1}^{-1};
//           alpha_ad = alpha / D with D_0 = 1, D_1 = UN / n, D_2 = mean |f_ak|;
//   measure L = Tr(U_0 ... U_{n-1}) / 2 (ordered tree product), d = UN/(2n) - 1.
// All reductions over a chain are fixed-order, so a chain's result does not
// depend on the launch or the other chains.  Exponentials of traceless 2x2 matrices use X^2 = w 1:
// exp(X) = C(w) 1 + S(w) X with the even and odd series C, S in w.
#include "chain.hpp"
#include "philox.hpp"
#include "reduce.hpp"
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

// LDS transfers element by element into component-major arrays (component e
// of slot i at [e][i], so that a wavefront's accesses fall on consecutive
// banks; a whole-struct copy between address spaces would become a memcpy
// that keeps the registers' copy in scratch memory)
template <int B>
__device__ __forceinline__ void put(double (*arr)[B], int i, const m2& x)
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

template <int B>
__device__ __forceinline__ m2 get(const double (*arr)[B], int i)
{
    return m2{{arr[0][i], arr[1][i]}, {arr[2][i], arr[3][i]}, {arr[4][i], arr[5][i]}, {arr[6][i], arr[7][i]}};
}

// ---------------------------------------------------------------------------
// workgroup layout: a chain of n links is owned by T threads (the smallest
// power of two with PT T >= n), PT consecutive links each; a workgroup of B
// threads (64 for T <= 64, else 256) holds B / T chains.  Two links per thread
// keep a thread's state within 256 registers, two waves per SIMD, which the
// dependent FP64 work of one thread needs to keep the SIMD busy; chains longer
// than 512 links take four per thread (one wave per SIMD), which measured
// faster there than 512 threads per chain with their longer scans.

template <int B>
struct ChainLds {
    double pre[8][B], suf[8][B];  // scans / products; suf[.][first] also holds link n-1
    double edge[8][B];            // last link, then the first Omega, of every thread
    double red[B / 64];
    int dead[B / 64];
};

struct Seg {
    int t;      // thread in the workgroup
    int lt;     // thread in the chain
    int T;      // threads per chain
    int first;  // the chain's first thread in the workgroup
};

__device__ __forceinline__ Seg make_seg(int T)
{
    Seg g;
    g.t = (int)threadIdx.x;
    g.T = T;
    g.lt = g.t & (T - 1);
    g.first = g.t - g.lt;
    return g;
}

template <int PT>
struct Chain {
    m2 U[PT];
    int n, k0;  // chain length, first link of this thread
    __device__ bool valid(int j) const { return k0 + j < n; }
};

// ---------------------------------------------------------------------------
// reductions over one chain's threads, in a fixed order (a butterfly within
// the wavefront, then the chain's wavefronts in order), so that a chain's
// result depends on n only; every thread of the chain gets the same value.

template <bool MAX, int B>
__device__ __forceinline__ double chain_all(double v, const Seg& g, ChainLds<B>& s)
{
    // the butterfly of reduce.hpp over the chain's lanes: every lane adds the
    // same pairs in the same order and ends with the same bits
    v = group_reduce<MAX>(v, g.T);
    if (B > 64 && g.T > 64) {
        if ((g.t & 63) == 0) s.red[g.t >> 6] = v;
        __syncthreads();
        const int w0 = g.first >> 6;
        double r = s.red[w0];
#pragma unroll
        for (int i = 1; i < (g.T >> 6); ++i) r = MAX ? fmax(r, s.red[w0 + i]) : r + s.red[w0 + i];
        __syncthreads();
        v = r;
    }
    return v;
}

// true in every thread when p holds in every thread of the workgroup
template <int B>
__device__ __forceinline__ bool block_all_true(bool p, ChainLds<B>& s)
{
    const bool w = __all(p);
    if (B == 64) return w;
    if ((threadIdx.x & 63) == 0) s.dead[threadIdx.x >> 6] = w;
    __syncthreads();
    bool r = true;
#pragma unroll
    for (int i = 0; i < B / 64; ++i) r = r && s.dead[i];
    __syncthreads();
    return r;
}

// E = M_0 ... M_t-1 and F = M_t+1 ... M_T-1, the chain's products before and
// after this thread's links (M_t = U_k0 ... U_k0+PT-1), from an inclusive prefix
// and an inclusive suffix scan over the chain's threads (Hillis-Steele)
template <int B, int PT>
__device__ __forceinline__ void chain_ends(const Chain<PT>& ch, const Seg& g, ChainLds<B>& s, m2& E, m2& F)
{
    m2 M = m2_id();
#pragma unroll
    for (int j = 0; j < PT; ++j)
        if (ch.valid(j)) M = mul(M, ch.U[j]);
    m2 I = M, S = M;
#pragma unroll
    for (int off = 1; off < g.T; off <<= 1) {
        put(s.pre, g.t, I);
        put(s.suf, g.t, S);
        __syncthreads();
        if (g.lt >= off) I = mul(get(s.pre, g.t - off), I);
        if (g.lt + off < g.T) S = mul(S, get(s.suf, g.t + off));
        __syncthreads();
    }
    put(s.pre, g.t, I);
    put(s.suf, g.t, S);
    __syncthreads();
    // (no ?: on matrix values: it selects addresses and keeps the operands in
    // scratch memory)
    E = m2_id();
    F = m2_id();
    if (g.lt > 0) E = get(s.pre, g.t - 1);
    if (g.lt + 1 < g.T) F = get(s.suf, g.t + 1);
    __syncthreads();
}

// The loop opened at each of this thread's links, P_j = U_j ... U_PT-1 F E U_0
// ... U_j-1 (invalid links are the identity and need no test): with A_j = E U_0
// ... U_j-1 and B_j = U_j ... U_PT-1 F, P_j = B_j A_j.
template <int PT>
__device__ __forceinline__ void chain_loops(const Chain<PT>& ch, const m2& E, const m2& F, m2 (&P)[PT])
{
    m2 A[PT], Bm[PT];
    A[0] = E;
#pragma unroll
    for (int j = 1; j < PT; ++j) A[j] = mul(A[j - 1], ch.U[j - 1]);
    Bm[PT - 1] = mul(ch.U[PT - 1], F);
#pragma unroll
    for (int j = PT - 2; j >= 0; --j) Bm[j] = mul(ch.U[j], Bm[j + 1]);
#pragma unroll
    for (int j = 0; j < PT; ++j) P[j] = mul(Bm[j], A[j]);
}

// ordered product U_0 ... U_{n-1} (valid in every thread of the chain)
template <int B, int PT>
__device__ __forceinline__ m2 chain_product(const Chain<PT>& ch, const Seg& g, ChainLds<B>& s)
{
    m2 M = m2_id();
#pragma unroll
    for (int j = 0; j < PT; ++j)
        if (ch.valid(j)) M = mul(M, ch.U[j]);
    put(s.pre, g.t, M);
    __syncthreads();
#pragma unroll
    for (int off = 1; off < g.T; off <<= 1) {
        if ((g.lt & (2 * off - 1)) == 0) put(s.pre, g.t, mul(get(s.pre, g.t), get(s.pre, g.t + off)));
        __syncthreads();
    }
    const m2 r = get(s.pre, g.first);
    __syncthreads();
    return r;
}

template <int B, int PT>
__device__ __forceinline__ double chain_unorm(const Chain<PT>& ch, const Seg& g, ChainLds<B>& s)
{
    double u = 0.0;
#pragma unroll
    for (int j = 0; j < PT; ++j)
        if (ch.valid(j)) u += nrm2(ch.U[j]);
    return chain_all<false>(u, g, s);
}

// the drift K_j = i beta TL(P_j) of this thread's links and K_max of the chain
template <int B, int PT>
__device__ __forceinline__ double chain_drift(const ChainArgs& a, const Chain<PT>& ch, const Seg& g, ChainLds<B>& s,
                                              m2 (&K)[PT])
{
    m2 E, F;
    chain_ends(ch, g, s, E, F);
    chain_loops(ch, E, F, K);
    const cxd ib = {-a.beta_im, a.beta_re};  // i beta
    double kn2 = 0.0;
#pragma unroll
    for (int j = 0; j < PT; ++j) {
        K[j] = scale(tl(K[j]), ib);
        if (ch.valid(j)) {
            double v = 0.5 * nrm2(K[j]);
            if (!isfinite(v)) v = INFINITY;
            kn2 = fmax(kn2, v);
        }
    }
    return sqrt(chain_all<true>(kn2, g, s));
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

// Omega = exp(A) = C 1 + S A and Omega^-1 = exp(-A) = C 1 - S A for
// A = [[g, q], [q*, -g]] Hermitian traceless: A^2 = w 1 with w = g^2 + |q|^2 >= 0,
// C = cosh(sqrt w), S = sinh(sqrt w) / sqrt w (exact inverses: C^2 - S^2 w = 1).
// Both are kept as (C, S g, S q).
struct hexp {
    double C, Sg;
    cxd Sq;
    __device__ h2 fwd() const { return h2{C + Sg, C - Sg, Sq}; }
    __device__ h2 inv() const { return h2{C - Sg, C + Sg, cxd{-Sq.re, -Sq.im}}; }
};

__device__ __forceinline__ hexp herm_exp2(double g, cxd q)
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
    return hexp{C, S * g, cxd{S * q.re, S * q.im}};
}

// one Jacobi cooling step at eps_c alpha_ad chosen by the mode
template <int B, int PT>
__device__ __forceinline__ void chain_cool_step(const ChainArgs& a, Chain<PT>& ch, const Seg& g, ChainLds<B>& s)
{
    // neighbours: link k-1 of this thread's first link (link n-1 for k = 0)
    put(s.edge, g.t, ch.U[PT - 1]);
    if (ch.valid(0) && (ch.n - 1) / PT == g.lt) {
        // link n-1 by compile-time selects (a runtime index would put U in scratch)
        const int jl = (ch.n - 1) % PT;
        m2 u = ch.U[0];
#pragma unroll
        for (int j = 1; j < PT; ++j) u = pick(j == jl, ch.U[j], u);
        put(s.suf, g.first, u);
    }
    __syncthreads();
    m2 prev0 = get(s.suf, g.first);
    if (g.lt > 0) prev0 = get(s.edge, g.t - 1);
    __syncthreads();
    // G_k = TL(U U^dag - W^dag W) = [[g, q], [q*, -g]]: sum_a f_ak sigma_a = 4 TL(G_k)
    // (the trace, the difference of the two links' norms, is no direction of the
    // gauge orbit), f_1 = 4 Re q, f_2 = -4 Im q, f_3 = 4 g
    double gd[PT];
    cxd q[PT];
    double un = 0.0, fsum = 0.0;
#pragma unroll
    for (int j = 0; j < PT; ++j) {
        m2 W = prev0;
        if (j > 0) W = ch.U[j - 1];
        const m2& U = ch.U[j];
        const double h00 = norm2(U.a) + norm2(U.b) - norm2(W.a) - norm2(W.c);
        const double h11 = norm2(U.c) + norm2(U.d) - norm2(W.b) - norm2(W.d);
        // (U U^dag)_01 = a c* + b d*,  (W^dag W)_01 = wa* wb + wc* wd
        const cxd uu = cfma(U.b, conj(U.d), U.a * conj(U.c));
        const cxd ww = cfma(conj(W.c), W.d, conj(W.a) * W.b);
        gd[j] = 0.5 * (h00 - h11);
        q[j] = uu - ww;
        if (ch.valid(j)) {
            un += nrm2(U);
            fsum += 4.0 * (fabs(q[j].re) + fabs(q[j].im) + fabs(gd[j]));
        }
    }
    double D = 1.0;
    if (a.mode == 1) D = chain_all<false>(un, g, s) / ch.n;
    if (a.mode == 2) D = chain_all<false>(fsum, g, s) / (3.0 * ch.n);
    const double c = -4.0 * a.eps_c * (a.alpha / D);
    hexp Om[PT];
#pragma unroll
    for (int j = 0; j < PT; ++j) Om[j] = herm_exp2(c * gd[j], cxd{c * q[j].re, c * q[j].im});
    s.edge[0][g.t] = Om[0].C;
    s.edge[1][g.t] = Om[0].Sg;
    s.edge[2][g.t] = Om[0].Sq.re;
    s.edge[3][g.t] = Om[0].Sq.im;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PT; ++j) {
        if (!ch.valid(j)) continue;
        const int k = ch.k0 + j;
        // Omega^-1 of site k+1: this thread's next one, the next thread's first
        // (always of the same chain: the chain's last thread holds link n-1),
        // or, for k = n-1, the chain's first
        hexp On;
        if (k + 1 == ch.n || j + 1 == PT) {
            const int o = k + 1 == ch.n ? g.first : g.t + 1;
            On = hexp{s.edge[0][o], s.edge[1][o], cxd{s.edge[2][o], s.edge[3][o]}};
        } else {
            On = Om[(j + 1) % PT];
        }
        ch.U[j] = mulh(hmul(Om[j].fwd(), ch.U[j]), On.inv());
    }
    __syncthreads();
}

// this thread's links of a chain; a chain index past the last (the padding
// of the last workgroup) gets identity links and is never stored
template <int PT>
__device__ __forceinline__ void chain_load(const ChainArgs& a, int chain, const Seg& g, Chain<PT>& ch)
{
    ch.n = a.n;
    ch.k0 = g.lt * PT;
    const double* base = a.links + (size_t)chain * a.n * 8;
#pragma unroll
    for (int j = 0; j < PT; ++j) {
        ch.U[j] = m2_id();
        if (chain < a.n_chains && ch.valid(j)) ch.U[j] = load_link(base + (size_t)(ch.k0 + j) * 8);
    }
}

template <int PT>
__device__ __forceinline__ void chain_store(const ChainArgs& a, int chain, const Chain<PT>& ch)
{
    double* base = a.links + (size_t)chain * a.n * 8;
#pragma unroll
    for (int j = 0; j < PT; ++j)
        if (ch.valid(j)) store_link(base + (size_t)(ch.k0 + j) * 8, ch.U[j]);
}

__device__ __forceinline__ int chain_of(const Seg& g, int B) { return (int)blockIdx.x * (B / g.T) + g.t / g.T; }

// ---------------------------------------------------------------------------
// kernels

// U_k = exp(i sigma_a (x_a + i y_a)), x ~ N(0, sx), y ~ N(0, sy); fresh control block
__global__ void __launch_bounds__(256) k_chain_init(ChainArgs a, double sx, double sy)
{
    // one lane per link of every chain (a one-dimensional grid: the chain count
    // may exceed the limit of a grid's second dimension)
    const size_t l = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (l >= (size_t)a.n * a.n_chains) return;
    const int chain = (int)(l / a.n);
    const int k = (int)(l - (size_t)chain * a.n);
    {
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
// A chain that runs away (a non-finite drift maximum, norm or loop) keeps its
// links of the call's start and is advanced no further; its workgroup goes on
// (every thread takes every barrier) until all of its chains are done.
template <int B, int T, int PT>
__global__ void __launch_bounds__(B) k_chain_run(ChainArgs a, int n_steps)
{
    __shared__ ChainLds<B> s;
    const Seg g = make_seg(T);
    const int chain = chain_of(g, B);
    const bool exists = chain < a.n_chains;
    ChainCtrl* cc = a.ctrl + chain;
    // (every thread of a chain reads the same words)
    int status = exists ? cc->status : 1;
    if (block_all_true(status != 0, s)) return;  // workgroup-uniform
    int64_t step = exists ? cc->step : 0;
    double bound = exists ? cc->bound : 0.0;
    Chain<PT> ch;
    chain_load(a, chain, g, ch);
    double sL_re = 0.0, sL_im = 0.0, sd = 0.0, st = 0.0, eps = 0.0, kmax = 0.0, d_pre = 0.0, d = 0.0;
    cxd L = {0.0, 0.0};
    int done = 0;
    for (int i = 0; i < n_steps; ++i) {
        m2 K[PT];
        const double km = chain_drift(a, ch, g, s, K);  // chain-uniform
        if (status == 0) {
            kmax = km;
            if (!isfinite(km)) status = 1;
        }
        const bool live = status == 0;  // this step advances the chain
        double e = a.eps0;
        if (a.adaptive) {
            if (live && bound <= 0.0) bound = a.drift_bound > 0.0 ? a.drift_bound : a.eps0 * km;
            if (km > 0.0 && bound / km < a.eps0) e = bound / km;
        }
        const double se = sqrt(e) * 1.41421356237309504880;  // sqrt(eps) * sqrt(2)
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            if (!ch.valid(j)) continue;
            double n0, n1, n2, n3;
            const uint32_t k = (uint32_t)(ch.k0 + j);
            normal_pair<double>(a.seed, k, (uint32_t)step, (uint32_t)chain, (kChainTagNoise << 16) | 0u, n0, n1);
            normal_pair<double>(a.seed, k, (uint32_t)step, (uint32_t)chain, (kChainTagNoise << 16) | 1u, n2, n3);
            const double e1 = se * n0, e2 = se * n1, e3 = se * n2;
            // eps K + sum_a eta_a sigma_a, times i
            m2 Y = scale(K[j], cxd{e, 0.0});
            Y.a = Y.a + cxd{e3, 0.0};
            Y.b = Y.b + cxd{e1, -e2};
            Y.c = Y.c + cxd{e1, e2};
            Y.d = Y.d + cxd{-e3, 0.0};
            ch.U[j] = renorm(mul(exp_tl(scale(Y, cxd{0.0, 1.0})), ch.U[j]));
        }
        const double dp = chain_unorm(ch, g, s) / (2.0 * ch.n) - 1.0;
        for (int ic = 0; ic < a.n_cool; ++ic) chain_cool_step(a, ch, g, s);
        const double un = chain_unorm(ch, g, s);
        const m2 Pt = chain_product(ch, g, s);
        if (live) {
            eps = e;
            ++step;
            d_pre = dp;
            d = un / (2.0 * ch.n) - 1.0;
            L = {0.5 * (Pt.a.re + Pt.d.re), 0.5 * (Pt.a.im + Pt.d.im)};
            if (!isfinite(un) || !isfinite(L.re) || !isfinite(L.im)) {
                status = 1;
            } else {
                // Langevin-time integrals: with an adaptive step the chain
                // spends more steps where eps is small, so each step weighs eps
                sL_re = fma(eps, L.re, sL_re);
                sL_im = fma(eps, L.im, sL_im);
                sd = fma(eps, d, sd);
                st += eps;
                ++done;
                if (a.record && i < a.obs_cap && g.lt == 0) {
                    double* o = a.obs + ((size_t)i * a.n_chains + chain) * kChainObs;
                    o[0] = L.re;
                    o[1] = L.im;
                    o[2] = d;
                    o[3] = eps;
                    o[4] = kmax;
                    o[5] = d_pre;
                }
            }
        }
        if (block_all_true(status != 0, s)) break;  // workgroup-uniform
    }
    if (!exists) return;
    if (status == 0) chain_store(a, chain, ch);  // a runaway leaves the links as they were
    if (g.lt == 0) {
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
        cc->sum_t = st;
    }
}

// the drift of every link (K[chain][k][8]) and K_max (ctrl.kmax)
template <int B, int T, int PT>
__global__ void __launch_bounds__(B) k_chain_drift(ChainArgs a)
{
    __shared__ ChainLds<B> s;
    const Seg g = make_seg(T);
    const int chain = chain_of(g, B);
    Chain<PT> ch;
    chain_load(a, chain, g, ch);
    m2 K[PT];
    const double kmax = chain_drift(a, ch, g, s, K);
    if (chain >= a.n_chains) return;
    double* base = a.K + (size_t)chain * a.n * 8;
#pragma unroll
    for (int j = 0; j < PT; ++j)
        if (ch.valid(j)) store_link(base + (size_t)(ch.k0 + j) * 8, K[j]);
    if (g.lt == 0) a.ctrl[chain].kmax = kmax;
}

// n_cool cooling steps of every chain, then L and d into the control block
template <int B, int T, int PT>
__global__ void __launch_bounds__(B) k_chain_cool(ChainArgs a)
{
    __shared__ ChainLds<B> s;
    const Seg g = make_seg(T);
    const int chain = chain_of(g, B);
    Chain<PT> ch;
    chain_load(a, chain, g, ch);
    for (int ic = 0; ic < a.n_cool; ++ic) chain_cool_step(a, ch, g, s);
    const double un = chain_unorm(ch, g, s);
    const m2 Pt = chain_product(ch, g, s);
    if (chain >= a.n_chains) return;
    chain_store(a, chain, ch);
    if (g.lt == 0) {
        ChainCtrl* cc = a.ctrl + chain;
        cc->d = un / (2.0 * ch.n) - 1.0;
        cc->L_re = 0.5 * (Pt.a.re + Pt.d.re);
        cc->L_im = 0.5 * (Pt.a.im + Pt.d.im);
        if (!isfinite(un)) cc->status = 1;
    }
}

// L and d of every chain into the control block
template <int B, int T, int PT>
__global__ void __launch_bounds__(B) k_chain_measure(ChainArgs a)
{
    __shared__ ChainLds<B> s;
    const Seg g = make_seg(T);
    const int chain = chain_of(g, B);
    Chain<PT> ch;
    chain_load(a, chain, g, ch);
    const double un = chain_unorm(ch, g, s);
    const m2 Pt = chain_product(ch, g, s);
    if (chain < a.n_chains && g.lt == 0) {
        ChainCtrl* cc = a.ctrl + chain;
        cc->d = un / (2.0 * ch.n) - 1.0;
        cc->L_re = 0.5 * (Pt.a.re + Pt.d.re);
        cc->L_im = 0.5 * (Pt.a.im + Pt.d.im);
    }
}

// links per thread, and threads per chain: the smallest power of two T with
// PT T >= n
int chain_per_thread(int n) { return n <= kChainShortMax ? kChainShortPT : kChainLongPT; }

int chain_threads(int n)
{
    const int pt = chain_per_thread(n);
    int T = 1;
    while (T * pt < n) T *= 2;
    return T;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers: chains of up to 128 links in 64-thread workgroups (64 / T chains
// each, two links per thread), longer ones in 256-thread workgroups (256 / T
// chains each; two links per thread up to 512 links, four above)

#define CHAIN_CASE(KERNEL, TT, PTT, ...)                                                                \
    case TT * 8 + PTT: {                                                                                \
        constexpr int B = TT <= 64 ? 64 : 256;                                                          \
        hipLaunchKernelGGL((KERNEL<B, TT, PTT>), dim3((a.n_chains + B / TT - 1) / (B / TT)), dim3(B), 0,  \
                           st, __VA_ARGS__);                                                            \
        break;                                                                                          \
    }

// one kernel instance per chain geometry (T, PT): the loops over the chain's
// threads and over a thread's links unroll
#define CHAIN_LAUNCH(KERNEL, ...)                                                                       \
    do {                                                                                                \
        switch (chain_threads(a.n) * 8 + chain_per_thread(a.n)) {                                       \
            CHAIN_CASE(KERNEL, 1, 2, __VA_ARGS__)                                                       \
            CHAIN_CASE(KERNEL, 2, 2, __VA_ARGS__)                                                       \
            CHAIN_CASE(KERNEL, 4, 2, __VA_ARGS__)                                                       \
            CHAIN_CASE(KERNEL, 8, 2, __VA_ARGS__)                                                       \
            CHAIN_CASE(KERNEL, 16, 2, __VA_ARGS__)                                                      \
            CHAIN_CASE(KERNEL, 32, 2, __VA_ARGS__)                                                      \
            CHAIN_CASE(KERNEL, 64, 2, __VA_ARGS__)                                                      \
            CHAIN_CASE(KERNEL, 128, 2, __VA_ARGS__)                                                     \
            CHAIN_CASE(KERNEL, 256, 2, __VA_ARGS__)                                                     \
            CHAIN_CASE(KERNEL, 256, 4, __VA_ARGS__)                                                     \
            default: return hipErrorInvalidValue;                                                       \
        }                                                                                               \
    } while (0)

hipError_t chain_launch_init(const ChainArgs& a, double sx, double sy, hipStream_t st)
{
    const size_t links = (size_t)a.n * a.n_chains;
    hipLaunchKernelGGL(k_chain_init, dim3((unsigned)((links + 255) / 256)), dim3(256), 0, st, a, sx, sy);
    return hipGetLastError();
}

hipError_t chain_launch_run(const ChainArgs& a, int n_steps, hipStream_t st)
{
    CHAIN_LAUNCH(k_chain_run, a, n_steps);
    return hipGetLastError();
}

hipError_t chain_launch_drift(const ChainArgs& a, hipStream_t st)
{
    CHAIN_LAUNCH(k_chain_drift, a);
    return hipGetLastError();
}

hipError_t chain_launch_cool(const ChainArgs& a, hipStream_t st)
{
    CHAIN_LAUNCH(k_chain_cool, a);
    return hipGetLastError();
}

hipError_t chain_launch_measure(const ChainArgs& a, hipStream_t st)
{
    CHAIN_LAUNCH(k_chain_measure, a);
    return hipGetLastError();
}

}  // namespace clgc
