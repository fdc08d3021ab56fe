// Lane moves inside one wavefront (gfx950), shared by the sketch-pass kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gn {

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// The 32-bit word of lane `lane ^ LM` (LM a power of two below 64) by lane moves
// that stay out of LDS: DPP copies within a row (xor 4 as the mirror of eight lanes
// followed by the mirror of four) and the gfx950 row and half-wave swaps.
template <int LM>
__device__ __forceinline__ uint32_t xor_lane_u32(uint32_t v, int lane) {
  if constexpr (LM == 1) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);  // quad_perm 1,0,3,2
  } else if constexpr (LM == 2) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);  // quad_perm 2,3,0,1
  } else if constexpr (LM == 4) {
    const int m = __builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
    return (uint32_t)__builtin_amdgcn_mov_dpp(m, 0x1B, 0xF, 0xF, false);      // quad_perm 3,2,1,0
  } else if constexpr (LM == 8) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, false);  // row_ror:8
  } else if constexpr (LM == 16) {
    // odd rows of the first operand trade places with even rows of the second
    const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (lane & 16) ? (uint32_t)p[0] : (uint32_t)p[1];
  } else {
    // the upper half of the first operand trades places with the lower half of the second
    const auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (lane & 32) ? (uint32_t)p[0] : (uint32_t)p[1];
  }
}

template <int LM>
__device__ __forceinline__ float xor_lane(float v, int lane) {
  return __uint_as_float(xor_lane_u32<LM>(__float_as_uint(v), lane));
}
template <int LM>
__device__ __forceinline__ double xor_lane(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const uint32_t lo = xor_lane_u32<LM>((uint32_t)b, lane);
  const uint32_t hi = xor_lane_u32<LM>((uint32_t)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

}  // namespace gn
