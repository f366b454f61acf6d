// Workgroup sums in a fixed order, for the reductions of the Krylov
// recurrence. Within a wave a butterfly: at every level a lane adds the value
// of its partner lane (pairs: lane bit 0, bit 1, mirror images within 8 and
// within 16 lanes, lane bit 4, lane bit 5), and the partner adds the same two
// values in the other order, so (addition being commutative) all 64 lanes
// end with the identical sum. The wave sums are then added in ascending wave
// order. Every workgroup that reduces the same array with the same thread
// count therefore holds bit-identical results.
#pragma once

#include <hip/hip_runtime.h>

namespace tdse {

// v of the partner lane under DPP control CTRL (a permutation within rows of
// 16 lanes), two 32-bit moves per double
template <int CTRL>
__device__ __forceinline__ double dpp_partner(double v) {
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(x & 0xffffffffll), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(x >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// v + v of the lane whose index differs in bit 4 (BIT = 4) or bit 5 (BIT =
// 5): the permlane swaps exchange whole 16- or 32-lane groups, so every lane
// adds the lower group's value and the upper group's value in that order
template <int BIT>
__device__ __forceinline__ double swap_add(double v) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
    unsigned l0, l1, h0, h1;
    if constexpr (BIT == 5) {
        auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        l0 = l[0], l1 = l[1], h0 = h[0], h1 = h[1];
    } else {
        auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        l0 = l[0], l1 = l[1], h0 = h[0], h1 = h[1];
    }
    return __longlong_as_double(((long long)h0 << 32) | l0) + __longlong_as_double(((long long)h1 << 32) | l1);
}

__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_partner<0xB1>(v);   // quad_perm(1,0,3,2): lane bit 0
    v += dpp_partner<0x4E>(v);   // quad_perm(2,3,0,1): lane bit 1
    v += dpp_partner<0x141>(v);  // row_half_mirror: lane i <-> 7 - i within 8 lanes
    v += dpp_partner<0x140>(v);  // row_mirror: lane i <-> 15 - i within 16 lanes
    v = swap_add<4>(v);
    return swap_add<5>(v);
}

// Workgroup barrier ordering LDS accesses only: global loads in flight stay
// in flight across it.
__device__ __forceinline__ void lds_only_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Sum of v over a workgroup of NT threads (NT a multiple of 64). red: NT / 64
// doubles of LDS, free again when the call returns.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *red) {
    static_assert(NT % 64 == 0, "whole waves");
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    lds_only_barrier();
    double s = red[0];
#pragma unroll
    for (int k = 1; k < NT / 64; ++k) s += red[k];
    lds_only_barrier();
    return s;
}

// Sum of p[0 .. count): thread t adds p[t], p[t + NT], ... in order, then
// block_sum.
template <int NT>
__device__ __forceinline__ double block_sum_array(const double *p, int count, double *red) {
    double v = 0.0;
    for (int k = threadIdx.x; k < count; k += NT) v += p[k];
    return block_sum<NT>(v, red);
}

}  // namespace tdse
