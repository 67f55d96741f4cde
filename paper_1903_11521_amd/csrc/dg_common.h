// Small helpers shared by the element-kernel families.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

namespace dgk {

// B (volume basis) and Bf (face basis) of degree n
__host__ __device__ constexpr int nb3(int n) { return n < 0 ? 0 : (n + 1) * (n + 2) * (n + 3) / 6; }
__host__ __device__ constexpr int nb2(int n) { return (n + 1) * (n + 2) / 2; }

template <int I, int E, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < E) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, E>(f);
    }
}

// XCD-aware block order: the hardware deals consecutive workgroups round
// robin to the 8 XCDs; remapping makes each XCD (own L2) walk a contiguous
// range of elements, which keeps face neighbours in the same L2.
__device__ __forceinline__ int64_t logical_block()
{
    const int64_t nb = gridDim.x, b = blockIdx.x;
    const int64_t full = (nb >> 3) << 3;
    return b < full ? (b & 7) * (nb >> 3) + (b >> 3) : b;
}

}  // namespace dgk
