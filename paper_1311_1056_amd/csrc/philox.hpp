// philox.hpp -- counter-based Gaussian noise for the Langevin update.
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11): ten rounds of the 4x32 S-box with multipliers
// 0xD2511F53, 0xCD9E8D57, the two key words bumped by 0x9E3779B9 and
// 0xBB67AE85 between rounds.  The counter of a draw is
// (4*site + mu, step, draw, stream tag) with the lexicographic site, and the key
// is the 64-bit run seed, so every number is a pure function of where and when
// it is drawn: independent of layout, launch shape and batching.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace clgc {

struct u32x4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit product gives both halves (a single multiply
        // instruction instead of separate low and high ones)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        c = u32x4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Two standard normals from one block of four words: two 53-bit uniforms in
// (0, 1) from (w0, w1) and (w2, w3), then Box-Muller.  The uniforms are built
// exactly in double; the transform runs in the working precision R (in float,
// ln u on the upper half goes through log1p(u - 1)).
template <typename R>
__device__ __forceinline__ void normal_pair(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                                            uint32_t c3, R& n0, R& n1)
{
    const u32x4 w = philox4x32_10(u32x4{c0, c1, c2, c3}, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double uA = fma((double)(w.x >> 5), 67108864.0, (double)(w.y >> 6) + 0.5) * 0x1p-53;
    const double uB = fma((double)(w.z >> 5), 67108864.0, (double)(w.w >> 6) + 0.5) * 0x1p-53;
    R r;
    if constexpr (sizeof(R) == sizeof(float)) {
        // rounding u to float near u = 1 would dominate ln u (its spacing there,
        // 6e-8, is comparable to 1 - u); u - 1 is exact in double, so log1p of
        // it keeps ln u to float accuracy on the upper half
        const float l = uA < 0.5 ? logf((float)uA) : log1pf((float)(uA - 1.0));
        r = sqrtf(-2.0f * l);
    } else {
        r = sqrt(R(-2) * log(R(uA)));
    }
    R s, c;
    if constexpr (sizeof(R) == sizeof(float)) sincospif(R(2) * R(uB), &s, &c);
    else sincospi(R(2) * R(uB), &s, &c);
    n0 = r * c;
    n1 = r * s;
}

enum : uint32_t { kStreamNoise = 0u, kStreamInit = 1u };

}  // namespace clgc
