// Wavefront helpers shared by the FP64 kernels that reduce on chip (the core
// QR and the Jacobi SVD): uniform reads of one lane's double, per-lane selects
// with constant lane masks, and a transposing sum of several values over the 64
// lanes of a wave.
#pragma once

#include <hip/hip_runtime.h>

namespace gn {

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Per-lane choice between two doubles with the lane mask as a constant SGPR
// pair: lanes whose bit is set take `hi`.  (Written as a plain select, the
// compiler merges the choice into a run-time index of the register array and
// expands it into a compare-and-select chain over every element.)
__device__ __forceinline__ double lane_select(double lo, double hi, unsigned long long lanes) {
  const unsigned long long a = (unsigned long long)__double_as_longlong(lo);
  const unsigned long long b = (unsigned long long)__double_as_longlong(hi);
  unsigned r0, r1;
  asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r0) : "v"((unsigned)a), "v"((unsigned)b), "s"(lanes));
  asm("v_cndmask_b32_e64 %0, %1, %2, %3"
      : "=v"(r1)
      : "v"((unsigned)(a >> 32)), "v"((unsigned)(b >> 32)), "s"(lanes));
  return __longlong_as_double((long long)(((unsigned long long)r1 << 32) | r0));
}

// Lanes whose lane-index bit `bit` is set.
__host__ __device__ constexpr unsigned long long lanes_with_bit(int bit) {
  unsigned long long m = 0;
  for (int l = 0; l < 64; ++l)
    if (l & bit) m |= 1ull << l;
  return m;
}

// Sum of a[0..NV) over the 64 lanes of a wave, spread over the lanes: halving
// exchanges (xor 32, 16, ...) leave each lane one slot, then full exchanges over
// the remaining lane bits.  Returns the lane's sum; *slot receives its index.
template <int NV>
__device__ __forceinline__ double wave_transpose_sum(double (&a)[NV], int lane, int* slot) {
  static_assert(NV >= 1 && NV <= 32 && (NV & (NV - 1)) == 0, "NV must be a power of two");
  int sl = 0;
  int mask = 32;
#pragma unroll
  for (int h = NV; h > 1; h >>= 1) {
    const bool up = (lane & mask) != 0;
    const unsigned long long lm = lanes_with_bit(mask);
#pragma unroll
    for (int i = 0; i < h / 2; ++i) {
      const double mine = lane_select(a[i], a[i + h / 2], lm);
      const double other = lane_select(a[i + h / 2], a[i], lm);
      a[i] = mine + __shfl_xor(other, mask, 64);
    }
    sl = 2 * sl + (up ? 1 : 0);
    mask >>= 1;
  }
  double v = a[0];
  for (; mask > 0; mask >>= 1) v += __shfl_xor(v, mask, 64);
  *slot = sl;
  return v;
}

}  // namespace gn
