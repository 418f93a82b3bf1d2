// su3.hpp -- 3x3 complex matrix arithmetic for SL(3,C) links on gfx950.
//
// Everything is plain VALU code in the working precision R (double or
// float): a product is 27 complex multiply-adds (108 FMAs), the inverse of
// a unit-determinant matrix is its adjugate, and the exponential of a
// traceless matrix uses the Cayley-Hamilton relation A^3 = s A + t 1
// (s = Tr(A^2)/2, t = det A), so that exp(A) = f0 + f1 A + f2 A^2 with the
// three coefficients summed as a Horner series in the scalars s, t.
#pragma once
#include <hip/hip_runtime.h>

namespace clgc {

template <typename R>
struct cx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> cmk(R re, R im) { return cx<R>{re, im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b)
{
    return {fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
template <typename R>
__device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
// a + b * c
template <typename R>
__device__ __forceinline__ cx<R> cfma(cx<R> b, cx<R> c, cx<R> a)
{
    return {fma(b.re, c.re, fma(-b.im, c.im, a.re)), fma(b.re, c.im, fma(b.im, c.re, a.im))};
}
template <typename R>
__device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
template <typename R>
__device__ __forceinline__ R norm2(cx<R> a) { return fma(a.re, a.re, a.im * a.im); }

template <typename R>
struct mat3 {
    cx<R> e[3][3];
};

template <typename R>
__device__ __forceinline__ mat3<R> m_zero()
{
    mat3<R> r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) r.e[i][j] = {R(0), R(0)};
    return r;
}

template <typename R>
__device__ __forceinline__ mat3<R> m_id()
{
    mat3<R> r = m_zero<R>();
    r.e[0][0].re = r.e[1][1].re = r.e[2][2].re = R(1);
    return r;
}

template <typename R>
__device__ __forceinline__ mat3<R> operator*(const mat3<R>& a, const mat3<R>& b)
{
    mat3<R> r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<R> s = a.e[i][0] * b.e[0][j];
            s = cfma(a.e[i][1], b.e[1][j], s);
            s = cfma(a.e[i][2], b.e[2][j], s);
            r.e[i][j] = s;
        }
    return r;
}

// acc += a * b
template <typename R>
__device__ __forceinline__ void m_mac(mat3<R>& acc, const mat3<R>& a, const mat3<R>& b)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<R> s = acc.e[i][j];
            s = cfma(a.e[i][0], b.e[0][j], s);
            s = cfma(a.e[i][1], b.e[1][j], s);
            s = cfma(a.e[i][2], b.e[2][j], s);
            acc.e[i][j] = s;
        }
}

// acc += c * m   (complex scalar c)
template <typename R>
__device__ __forceinline__ void m_axpy(mat3<R>& acc, cx<R> c, const mat3<R>& m)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) acc.e[i][j] = cfma(c, m.e[i][j], acc.e[i][j]);
}

template <typename R>
__device__ __forceinline__ mat3<R> operator+(const mat3<R>& a, const mat3<R>& b)
{
    mat3<R> r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) r.e[i][j] = a.e[i][j] + b.e[i][j];
    return r;
}

template <typename R>
__device__ __forceinline__ mat3<R> operator-(const mat3<R>& a, const mat3<R>& b)
{
    mat3<R> r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) r.e[i][j] = a.e[i][j] - b.e[i][j];
    return r;
}

template <typename R>
__device__ __forceinline__ mat3<R> m_scale(const mat3<R>& a, cx<R> c)
{
    mat3<R> r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) r.e[i][j] = c * a.e[i][j];
    return r;
}

// a times the purely imaginary scalar i c (c real): two products per entry
template <typename R>
__device__ __forceinline__ mat3<R> m_scale_i(const mat3<R>& a, R c)
{
    mat3<R> r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) r.e[i][j] = {-c * a.e[i][j].im, c * a.e[i][j].re};
    return r;
}

// a c for a complex c that is often real (a real theta): two products per
// entry when Im c = 0, the full complex product otherwise (c uniform across
// the wavefront, so the branch does not diverge)
template <typename R>
__device__ __forceinline__ mat3<R> m_scale_z(const mat3<R>& a, cx<R> c)
{
    mat3<R> r;
    if (c.im == R(0)) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) r.e[i][j] = {c.re * a.e[i][j].re, c.re * a.e[i][j].im};
    } else {
        r = m_scale(a, c);
    }
    return r;
}

// acc += i c m (c real): two fused multiply-adds per entry
template <typename R>
__device__ __forceinline__ void m_axpy_i(mat3<R>& acc, R c, const mat3<R>& m)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            acc.e[i][j] = {fma(-c, m.e[i][j].im, acc.e[i][j].re), fma(c, m.e[i][j].re, acc.e[i][j].im)};
}

template <typename R>
__device__ __forceinline__ cx<R> m_tr(const mat3<R>& a) { return a.e[0][0] + a.e[1][1] + a.e[2][2]; }

// Tr(a b) without forming the product
template <typename R>
__device__ __forceinline__ cx<R> m_trmul(const mat3<R>& a, const mat3<R>& b)
{
    cx<R> s = {R(0), R(0)};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) s = cfma(a.e[i][k], b.e[k][i], s);
    return s;
}

// Tr(a a^dagger) = sum |a_ij|^2
template <typename R>
__device__ __forceinline__ R m_norm2(const mat3<R>& a)
{
    R s = R(0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) s += norm2(a.e[i][j]);
    return s;
}

template <typename R>
__device__ __forceinline__ cx<R> m_det(const mat3<R>& a)
{
    cx<R> c0 = a.e[1][1] * a.e[2][2] - a.e[1][2] * a.e[2][1];
    cx<R> c1 = a.e[1][2] * a.e[2][0] - a.e[1][0] * a.e[2][2];
    cx<R> c2 = a.e[1][0] * a.e[2][1] - a.e[1][1] * a.e[2][0];
    return a.e[0][0] * c0 + a.e[0][1] * c1 + a.e[0][2] * c2;
}

// Adjugate: a * adj(a) = det(a) 1; the inverse on SL(3,C).
template <typename R>
__device__ __forceinline__ mat3<R> m_adj(const mat3<R>& a)
{
    mat3<R> r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int r0 = (j + 1) % 3, r1 = (j + 2) % 3, c0 = (i + 1) % 3, c1 = (i + 2) % 3;
            r.e[i][j] = a.e[r0][c0] * a.e[r1][c1] - a.e[r0][c1] * a.e[r1][c0];
        }
    return r;
}

// Traceless part M - Tr(M)/3.
template <typename R>
__device__ __forceinline__ mat3<R> m_traceless(mat3<R> a)
{
    cx<R> t = R(1.0 / 3.0) * m_tr(a);
#pragma unroll
    for (int i = 0; i < 3; ++i) a.e[i][i] = a.e[i][i] - t;
    return a;
}

template <typename R>
__device__ __forceinline__ mat3<R> m_dag(const mat3<R>& a)
{
    mat3<R> r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) r.e[i][j] = conj(a.e[j][i]);
    return r;
}

template <typename R>
__device__ __forceinline__ mat3<R> m_cast_from(const mat3<double>& a)
{
    mat3<R> r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) r.e[i][j] = {R(a.e[i][j].re), R(a.e[i][j].im)};
    return r;
}

template <typename R>
__device__ __forceinline__ mat3<double> m_to_double(const mat3<R>& a)
{
    mat3<double> r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) r.e[i][j] = {double(a.e[i][j].re), double(a.e[i][j].im)};
    return r;
}

// Number of Taylor terms that make the truncation error of exp(A), ||A||_F <= 1,
// fall below the working precision: 1/20! ~ 4e-19, 1/12! ~ 2e-9.
template <typename R> struct exp_terms { static constexpr int n = 20; };
template <> struct exp_terms<float> { static constexpr int n = 12; };

// Coefficients (f0, f1, f2) of exp(A) = f0 + f1 A + f2 A^2 for traceless A with
// A^3 = s A + t: Horner evaluation of sum_n A^n / n! in the basis (1, A, A^2),
// where multiplication by A maps (x, y, z) -> (t z, x + s z, y).
template <typename R>
__device__ __forceinline__ void ch_exp_coeffs(cx<R> s, cx<R> t, cx<R>& f0, cx<R>& f1, cx<R>& f2)
{
    cx<R> x = {R(1), R(0)}, y = {R(0), R(0)}, z = {R(0), R(0)};
#pragma unroll
    for (int n = exp_terms<R>::n; n >= 1; --n) {
        const R inv = R(1) / R(n);
        cx<R> nx = t * z;
        cx<R> ny = cfma(s, z, x);
        cx<R> nz = y;
        x = cmk(fma(inv, nx.re, R(1)), inv * nx.im);
        y = inv * ny;
        z = inv * nz;
    }
    f0 = x;
    f1 = y;
    f2 = z;
}

// exp(A) for a traceless 3x3 complex A.  A is first scaled by 2^-k so that
// ||A||_F <= 1 and the result squared k times.
template <typename R>
__device__ __forceinline__ mat3<R> m_exp_traceless(mat3<R> A)
{
    R fro2 = m_norm2(A);
    int k = 0;
    if (fro2 > R(1)) {
        // smallest k with fro2 / 4^k <= 1; a non-finite norm (a runaway, flagged
        // by the caller's reduction) takes no squarings: converting its infinite
        // log to int would give a loop of 2^31 squarings
        const R lk = R(0.5) * log2(fro2);
        k = lk < R(1100) ? (int)ceil(lk) : 0;
        const R sc = ldexp(R(1), -k);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) A.e[i][j] = sc * A.e[i][j];
    }
    mat3<R> A2 = A * A;
    cx<R> s = R(0.5) * m_tr(A2);
    cx<R> t = m_det(A);
    cx<R> f0, f1, f2;
    ch_exp_coeffs(s, t, f0, f1, f2);
    mat3<R> r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) r.e[i][j] = cfma(f2, A2.e[i][j], f1 * A.e[i][j]);
#pragma unroll
    for (int i = 0; i < 3; ++i) r.e[i][i] = r.e[i][i] + f0;
    for (int i = 0; i < k; ++i) r = r * r;
    return r;
}

// ---------------------------------------------------------------------------
// Hermitian 3x3 matrices (cooling): 3 real diagonal + 3 complex upper entries.

template <typename R>
struct herm3 {
    R d0, d1, d2;
    cx<R> u01, u02, u12;
};

template <typename R>
__device__ __forceinline__ herm3<R> h_zero()
{
    return {R(0), R(0), R(0), {R(0), R(0)}, {R(0), R(0)}, {R(0), R(0)}};
}

// acc += U U^dagger
template <typename R>
__device__ __forceinline__ void h_add_uudag(herm3<R>& h, const mat3<R>& u)
{
    h.d0 += norm2(u.e[0][0]) + norm2(u.e[0][1]) + norm2(u.e[0][2]);
    h.d1 += norm2(u.e[1][0]) + norm2(u.e[1][1]) + norm2(u.e[1][2]);
    h.d2 += norm2(u.e[2][0]) + norm2(u.e[2][1]) + norm2(u.e[2][2]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        h.u01 = cfma(u.e[0][k], conj(u.e[1][k]), h.u01);
        h.u02 = cfma(u.e[0][k], conj(u.e[2][k]), h.u02);
        h.u12 = cfma(u.e[1][k], conj(u.e[2][k]), h.u12);
    }
}

// acc -= U^dagger U
template <typename R>
__device__ __forceinline__ void h_sub_udagu(herm3<R>& h, const mat3<R>& u)
{
    h.d0 -= norm2(u.e[0][0]) + norm2(u.e[1][0]) + norm2(u.e[2][0]);
    h.d1 -= norm2(u.e[0][1]) + norm2(u.e[1][1]) + norm2(u.e[2][1]);
    h.d2 -= norm2(u.e[0][2]) + norm2(u.e[1][2]) + norm2(u.e[2][2]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        // (U^dagger U)_{ij} = sum_k conj(U_ki) U_kj
        h.u01 = h.u01 - conj(u.e[k][0]) * u.e[k][1];
        h.u02 = h.u02 - conj(u.e[k][0]) * u.e[k][2];
        h.u12 = h.u12 - conj(u.e[k][1]) * u.e[k][2];
    }
}

template <typename R>
__device__ __forceinline__ mat3<R> h_full(const herm3<R>& h)
{
    mat3<R> m;
    m.e[0][0] = {h.d0, R(0)};
    m.e[1][1] = {h.d1, R(0)};
    m.e[2][2] = {h.d2, R(0)};
    m.e[0][1] = h.u01;
    m.e[0][2] = h.u02;
    m.e[1][2] = h.u12;
    m.e[1][0] = conj(h.u01);
    m.e[2][0] = conj(h.u02);
    m.e[2][1] = conj(h.u12);
    return m;
}

}  // namespace clgc
