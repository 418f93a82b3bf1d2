// reduce.hpp -- the butterfly of the wavefront reductions (sums and maxima
// whose result is the same bits in every lane).
//
// Stage s pairs each lane with stage_partner(s, lane) and combines the two
// values: xor 32 and xor 16 (lane shuffles), then the mirror within 16 lanes
// (l -> 15 - l in each row of 16, i.e. l ^ 15), the mirror within 8 (l ^ 7)
// and the two quad swaps (l ^ 2, l ^ 1), the last four as DPP moves in
// registers.  Every stage is an xor with a mask, the masks 32, 16, 15, 7, 2, 1
// span all six lane bits, and a + b == b + a (as fmax) bitwise: so after the
// stages a lane's value depends only on its group, every group member adds
// the same pairs in the same order, and each input enters exactly once.  A
// group of T lanes (T a power of two <= 64, aligned) takes the stages whose
// span is below T.  The host checks in the tests run these definitions.
#pragma once
#include <hip/hip_runtime.h>

namespace clgc {

constexpr int kButterflyStages = 6;

// the lane whose value lane `lane` combines with at stage s
__host__ __device__ constexpr int stage_partner(int s, int lane)
{
    return s == 0 ? lane ^ 32
         : s == 1 ? lane ^ 16
         : s == 2 ? (lane & ~15) | (15 - (lane & 15))
         : s == 3 ? (lane & ~7) | (7 - (lane & 7))
         : s == 4 ? lane ^ 2
                  : lane ^ 1;
}

// stage s runs in groups of more than stage_span(s) lanes (its pairs lie
// within aligned blocks of 2 stage_span(s) lanes)
__host__ __device__ constexpr int stage_span(int s) { return 32 >> s; }

// DPP controls of stages 2..5: row_mirror, row_half_mirror, quad_perm(2,3,0,1), quad_perm(1,0,3,2)
__host__ __device__ constexpr int stage_dpp_ctrl(int s) { return s == 2 ? 0x140 : s == 3 ? 0x141 : s == 4 ? 0x4E : 0xB1; }

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}

template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, true);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// the value of stage_partner(S, lane)
template <int S, typename V>
__device__ __forceinline__ V stage_move(V v)
{
    if constexpr (S < 2) return __shfl_xor(v, stage_span(S), 64);
    else return dpp_move<stage_dpp_ctrl(S)>(v);
}

template <bool MAX, typename V>
__device__ __forceinline__ V combine(V a, V b)
{
    return MAX ? fmax(a, b) : a + b;
}

// sum (or max) over aligned groups of T lanes, the same bits in every lane of a group
template <bool MAX, typename V>
__device__ __forceinline__ V group_reduce(V v, int T)
{
    if (T > stage_span(0)) v = combine<MAX>(v, stage_move<0>(v));
    if (T > stage_span(1)) v = combine<MAX>(v, stage_move<1>(v));
    if (T > stage_span(2)) v = combine<MAX>(v, stage_move<2>(v));
    if (T > stage_span(3)) v = combine<MAX>(v, stage_move<3>(v));
    if (T > stage_span(4)) v = combine<MAX>(v, stage_move<4>(v));
    if (T > stage_span(5)) v = combine<MAX>(v, stage_move<5>(v));
    return v;
}

}  // namespace clgc
