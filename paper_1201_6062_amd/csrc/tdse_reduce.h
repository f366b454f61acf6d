// Workgroup sums in a fixed order, for the reductions of the Krylov
// recurrence. Within a wave a butterfly over the lane-index bits: at every
// level a lane adds its partner's value to its own, and the partner adds the
// same two values in the other order, so (addition being commutative) all 64
// lanes end with the identical sum. The wave sums are then added in ascending
// wave order. Every workgroup that reduces the same array with the same
// thread count therefore holds bit-identical results.
#pragma once

#include <hip/hip_runtime.h>

namespace tdse {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
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
