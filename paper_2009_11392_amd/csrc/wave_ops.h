// Wavefront helpers shared by the FP64 kernels that reduce on chip (the core
// QR and the Jacobi SVD): uniform reads of one lane's double, per-lane selects
// with constant lane masks, DPP copies and lane swaps, and a transposing sum of
// several values over the 64 lanes of a wave.
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

// Lane moves within a wave (no LDS): a DPP copy of a double, and the gfx950 lane
// swaps.  swap_sum<true>(x, y): lanes 0..31 get x + x of the lane 32 above, lanes
// 32..63 get y + y of the lane 32 below (the upper half of x trades places with
// the lower half of y); swap_sum<false> does the same for the 16-lane rows, odd
// rows of x trading places with even rows of y.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

template <bool H32>
__device__ __forceinline__ double swap_sum(double x, double y) {
  const unsigned long long bx = (unsigned long long)__double_as_longlong(x);
  const unsigned long long by = (unsigned long long)__double_as_longlong(y);
  const unsigned xl = (unsigned)bx, xh = (unsigned)(bx >> 32);
  const unsigned yl = (unsigned)by, yh = (unsigned)(by >> 32);
  unsigned l0, l1, h0, h1;
  if constexpr (H32) {
    const auto l = __builtin_amdgcn_permlane32_swap(xl, yl, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(xh, yh, false, false);
    l0 = l[0];
    l1 = l[1];
    h0 = h[0];
    h1 = h[1];
  } else {
    const auto l = __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
    l0 = l[0];
    l1 = l[1];
    h0 = h[0];
    h1 = h[1];
  }
  const double x2 = __longlong_as_double((long long)(((unsigned long long)h0 << 32) | l0));
  const double y2 = __longlong_as_double((long long)(((unsigned long long)h1 << 32) | l1));
  return x2 + y2;
}

// One halving exchange over lane bit MASK (8, 4, 2 or 1) through a DPP pattern
// that pairs each lane with one whose MASK bit differs: the lane keeps a[i] or
// a[i + H] by its bit and adds the partner's copy of the same element.
template <int MASK, int CTRL, int NV>
__device__ __forceinline__ void dpp_halve(double (&a)[NV], int h) {
  const unsigned long long m = lanes_with_bit(MASK);
#pragma unroll
  for (int i = 0; i < NV / 2; ++i) {
    if (i >= h) break;
    const double mine = lane_select(a[i], a[i + h], m);
    const double other = lane_select(a[i + h], a[i], m);
    a[i] = mine + dpp_f64<CTRL>(other);
  }
}

// Sum of a[0..NV) over the 64 lanes of a wave, spread over the lanes: halving
// exchanges over lane bits 32, 16, 8, ... leave each lane one element index (its
// slot: the bits it kept, most significant first), then full sums over the
// remaining low lane bits.  The 32- and 16-lane exchanges are lane swaps, the
// others DPP patterns (row rotate by 8, the 8-lane mirror, quad permutes); a
// mirror pairs a lane with one differing in more than the bit being halved, which
// the later exchanges over the lower bits absorb.  Returns the lane's sum; *slot
// receives its index.
template <int NV>
__device__ __forceinline__ double wave_transpose_sum(double (&a)[NV], int lane, int* slot) {
  static_assert(NV >= 1 && NV <= 64 && (NV & (NV - 1)) == 0, "NV must be a power of two");
  int sl = 0, h = NV / 2;
  if constexpr (NV >= 2) {
#pragma unroll
    for (int i = 0; i < NV / 2; ++i) a[i] = swap_sum<true>(a[i], a[i + NV / 2]);
    sl = (lane >> 5) & 1;
    h >>= 1;
  }
  if constexpr (NV >= 4) {
#pragma unroll
    for (int i = 0; i < NV / 4; ++i) a[i] = swap_sum<false>(a[i], a[i + NV / 4]);
    sl = 2 * sl + ((lane >> 4) & 1);
    h >>= 1;
  }
  if constexpr (NV >= 8) {
    dpp_halve<8, 0x128>(a, h);  // row_ror 8: partner lane ^ 8
    sl = 2 * sl + ((lane >> 3) & 1);
    h >>= 1;
  }
  if constexpr (NV >= 16) {
    dpp_halve<4, 0x141>(a, h);  // row_half_mirror: partner 7 - (lane & 7)
    sl = 2 * sl + ((lane >> 2) & 1);
    h >>= 1;
  }
  if constexpr (NV >= 32) {
    dpp_halve<2, 0x4E>(a, h);  // quad_perm [2, 3, 0, 1]
    sl = 2 * sl + ((lane >> 1) & 1);
    h >>= 1;
  }
  if constexpr (NV >= 64) {
    dpp_halve<1, 0xB1>(a, h);  // quad_perm [1, 0, 3, 2]
    sl = 2 * sl + (lane & 1);
  }
  double v = a[0];
  if constexpr (NV < 2) v = swap_sum<true>(v, v);
  if constexpr (NV < 4) v = swap_sum<false>(v, v);
  if constexpr (NV < 8) v += dpp_f64<0x128>(v);
  if constexpr (NV < 16) v += dpp_f64<0x141>(v);
  if constexpr (NV < 32) v += dpp_f64<0x4E>(v);
  if constexpr (NV < 64) v += dpp_f64<0xB1>(v);
  *slot = sl;
  return v;
}

}  // namespace gn
