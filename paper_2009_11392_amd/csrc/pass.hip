// The sketch pass of GN (Algorithm 2.1, step 2): AX and Y^T A in one launch.
//
// In FP32 and BF16 modes one kernel launch carries both products: its grid
// interleaves the workgroups of the Y^T A contraction with those that form AX,
// eight at a time (one per XCD), so both streams of work run side by side.
//   * Y^T A, and AX for a Gaussian or user X, are dense contractions on the
//     matrix cores (gemm_tiles.h): FP32 v_mfma_f32_32x32x2_f32, or BF16
//     v_mfma_f32_32x32x16_bf16 with A's power-of-two block scales applied
//     exactly as tiles are staged; FP32 accumulation.
//   * AX for an SRHT X (Section 1: X = D H S) is not a contraction: every row of
//     A is sign-flipped, Walsh-Hadamard transformed and sampled.  A wave takes one
//     row at a time in 512-column chunks, 8 entries per lane; stages of width
//     1, 2, 4 run inside a lane and 8 .. 256 across lanes (xor shuffles); the
//     sampled columns are gathered from LDS and added with the sign of the outer
//     factor (-1)^popcount(chunk & (s >> 9)), since the Sylvester-ordered
//     H_{n'} = H_{n'/512} (x) H_512.
// FP64 mode (the parity mode) runs the same SRHT body and the FP64 strided GEMM
// as separate launches.
#include <type_traits>

#include "gemm_h16.h"
#include "gemm_tiles.h"
#include "lane_ops.h"

namespace gn {
namespace {

using namespace tiles;

constexpr int SR_CHUNK = 512;
constexpr int SR_MAX_WAVES = 16;

struct SrhtArgs {
  int64_t rows_per_wg;
  int64_t m, n, r;
  const void* A;
  int64_t lda;
  const float* scales;
  int64_t nsb;
  const int8_t* signs;
  const int32_t* idx;
  void* AX;
  int64_t ldax;
};

template <typename T>
__device__ __forceinline__ T flip_if(T v, uint32_t neg) {
  return neg ? -v : v;
}

// 8 consecutive entries A[i, j .. j+7] (zero beyond n) as float.
template <int MODE>
__device__ __forceinline__ void srht_load8(const SrhtArgs& a, int64_t i, int64_t j, float (&x)[8]) {
  if constexpr (MODE == GN_MODE_F32) {
    const float* row = reinterpret_cast<const float*>(a.A) + i * a.lda;
    if (j + 7 < a.n && (a.lda % 4 == 0)) {
      const f32x4 v0 = *reinterpret_cast<const f32x4*>(row + j);
      const f32x4 v1 = *reinterpret_cast<const f32x4*>(row + j + 4);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        x[e] = v0[e];
        x[4 + e] = v1[e];
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = (j + e < a.n) ? row[j + e] : 0.f;
    }
  } else {  // 16-bit with block scales; j is a multiple of 8, so one 128-column block
    constexpr bool F16 = (MODE == GN_MODE_F16_BS);
    const uint16_t* row = reinterpret_cast<const uint16_t*>(a.A) + i * a.lda;
    const float sc = (j < a.n) ? a.scales[(i >> 7) * a.nsb + (j >> 7)] : 0.f;
    if (j + 7 < a.n && (a.lda % 8 == 0)) {
      const u32x4 v = *reinterpret_cast<const u32x4*>(row + j);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        x[2 * e] = h16_to_f32<F16>((uint16_t)(v[e] & 0xffffu)) * sc;
        x[2 * e + 1] = h16_to_f32<F16>((uint16_t)(v[e] >> 16)) * sc;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = (j + e < a.n) ? h16_to_f32<F16>(row[j + e]) * sc : 0.f;
    }
  }
}

// Orders this wave's LDS accesses (a wave-scope fence): enough where a wave
// stores to and reads from LDS that no other wave touches.
// One Walsh-Hadamard stage across lanes: lane pairs (l, l ^ LM), the lower lane
// keeping the sum and the upper the difference (lower minus upper).
template <int LM, typename T>
__device__ __forceinline__ void srht_stage(T (&x)[8], int lane) {
  const bool upper = (lane & LM) != 0;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const T y = xor_lane<LM>(x[e], lane);
    x[e] = upper ? (y - x[e]) : (x[e] + y);
  }
}

// Rows [local * rows_per_wg, ...) of AX = A D H S.  Each wave owns one row at a
// time (rows advance by the number of waves per step); at most 16 waves.
template <typename T, int MODE, int RPL>
__device__ void srht_rows(const SrhtArgs& a, int64_t local, char* smem) {
  T(*slot)[SR_CHUNK] = reinterpret_cast<T(*)[SR_CHUNK]>(smem);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (int)(blockDim.x >> 6);
  const int64_t row_begin = local * a.rows_per_wg;
  if (row_begin >= a.m) return;
  const int64_t row_end = (row_begin + a.rows_per_wg < a.m) ? row_begin + a.rows_per_wg : a.m;
  int32_t s_lo[RPL], s_hi[RPL];
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int64_t c = lane + 64 * t;
    const int32_t sv = (c < a.r) ? a.idx[c] : 0;
    s_lo[t] = sv & (SR_CHUNK - 1);
    s_hi[t] = sv >> 9;
  }
  // one chunk's entries of row i (as loaded: float, or double in FP64 mode) and
  // their signs; the loop below keeps the next chunk's loads in flight while it
  // transforms the current one
  using L = typename std::conditional<MODE == GN_MODE_F64, double, float>::type;
  auto load_chunk = [&](int64_t i, int64_t j0, L (&xl)[8], uint64_t& sg) {
    const int64_t j = j0 + 8 * lane;
    if constexpr (MODE == GN_MODE_F64) {
      const double* row = reinterpret_cast<const double*>(a.A) + i * a.lda;
#pragma unroll
      for (int e = 0; e < 8; ++e) xl[e] = (j + e < a.n) ? row[j + e] : 0.0;
    } else {
      srht_load8<MODE>(a, i, j, xl);
    }
    sg = 0;
    if (j + 7 < a.n) {
      sg = *reinterpret_cast<const uint64_t*>(a.signs + j);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (j + e < a.n) sg |= (uint64_t)(uint8_t)a.signs[j + e] << (8 * e);
    }
  };
  for (int64_t ib = row_begin; ib < row_end; ib += nw) {
    const int64_t i = ib + wave;
    const bool active = i < row_end;
    T acc[RPL];
#pragma unroll
    for (int t = 0; t < RPL; ++t) acc[t] = (T)0;
    // one chunk: sign flips, H_512, and the sampled columns added with the sign of
    // the outer factor
    auto process = [&](const L (&xl)[8], uint64_t sg, int64_t j0) {
      T x[8];
      if (active) {
        // D: Rademacher sign flips (entries beyond n are already zero)
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = flip_if((T)xl[e], (uint32_t)((sg >> (8 * e + 7)) & 1u));
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = (T)0;
      }
      // H_512: widths 1, 2, 4 inside the lane
#pragma unroll
      for (int h = 1; h < 8; h <<= 1)
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if ((e & h) == 0) {
            const T u = x[e], v = x[e | h];
            x[e] = u + v;
            x[e | h] = u - v;
          }
      // widths 8 .. 256 across lanes (lane xor 1 .. 32)
      srht_stage<1>(x, lane);
      srht_stage<2>(x, lane);
      srht_stage<4>(x, lane);
      srht_stage<8>(x, lane);
      srht_stage<16>(x, lane);
      srht_stage<32>(x, lane);
#pragma unroll
      for (int e = 0; e < 8; ++e) slot[wave][8 * lane + e] = x[e];
      // the slot is this wave's own: its LDS operations complete in order, so
      // ordering within the wave is enough (no workgroup barrier, waves drift)
      wave_lds_fence();
      const uint32_t chunk = (uint32_t)(j0 >> 9);
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const T v = slot[wave][s_lo[t]];
        acc[t] += flip_if(v, (uint32_t)(__popc(chunk & (uint32_t)s_hi[t]) & 1));
      }
      wave_lds_fence();  // the gathers are done before the next chunk's stores
    };
    // the next chunk's loads are in flight while this one is transformed
    L xn[8];
    uint64_t sgn = 0;
    if (active) load_chunk(i, 0, xn, sgn);
    for (int64_t j0 = 0; j0 < a.n; j0 += SR_CHUNK) {
      L xc[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) xc[e] = xn[e];
      const uint64_t sc = sgn;
      if (active && j0 + SR_CHUNK < a.n) load_chunk(i, j0 + SR_CHUNK, xn, sgn);
      process(xc, sc, j0);
    }
    if (active) {
      T* out = reinterpret_cast<T*>(a.AX) + i * a.ldax;
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int64_t c = lane + 64 * t;
        if (c < a.r) out[c] = acc[t];
      }
    }
  }
}

constexpr size_t SR_SMEM_F32 = SR_MAX_WAVES * SR_CHUNK * sizeof(float);
constexpr size_t SR_SMEM_F64 = 4 * SR_CHUNK * sizeof(double);  // launched with 4 waves
constexpr size_t smax(size_t a, size_t b) { return a > b ? a : b; }

// ------------------------------------------------------------------ fused kernels
// Which family a workgroup belongs to: interleaved (family_split) or, with
// srht_first, the SRHT rows occupy the first gS groups of the grid.
__device__ __forceinline__ bool take_first(int64_t gFirst, int64_t gSecond, int first_then_second,
                                           int64_t& local) {
  if (!first_then_second) return family_split(gFirst, gSecond, local);
  const int64_t g = (int64_t)blockIdx.x >> 3, x = (int64_t)blockIdx.x & 7;
  if (g < gFirst) {
    local = g * 8 + x;
    return true;
  }
  local = (g - gFirst) * 8 + x;
  return false;
}

// FP32: Y^T A reads Y (m x rl, row-major) and A both m/n-contiguous; AX reads A
// k-contiguous and X (n x r, row-major) n-contiguous.
template <class CF, bool VEC>
__global__ void __launch_bounds__(CF::T) pass_f32_gauss(GemmF32 yta, GemmF32 ax, int64_t gY,
                                                        int64_t gA) {
  __shared__ __attribute__((aligned(16))) char smem[smax(CF::template smem<false, false>(),
                                                         CF::template smem<true, false>())];
  int64_t local;
  if (family_split(gY, gA, local))
    f32_tile_cfg<CF, false, false, VEC>(yta, local, smem);
  else
    f32_tile_cfg<CF, true, false, VEC>(ax, local, smem);
}

// The same two families with K split into slices (blockIdx.y): slice s of Y^T A
// covers rows [s kslY, ...) of A, slice s of AX its columns [s kslA, ...); each
// writes its own partial (summed afterwards in slice order).  For problems with
// too few output tiles to fill the chip.
template <class CF, bool VEC>
__global__ void __launch_bounds__(CF::T) pass_f32_gauss_split(GemmF32 yta, GemmF32 ax, int64_t gY,
                                                              int64_t gA, int64_t kslY,
                                                              int64_t kslA, int64_t sY, int64_t sA,
                                                              float* partY, float* partA) {
  __shared__ __attribute__((aligned(16))) char smem[smax(CF::template smem<false, false>(),
                                                         CF::template smem<true, false>())];
  const int64_t sl = blockIdx.y;
  int64_t local;
  if (family_split(gY, gA, local)) {
    if (sl >= sY) return;
    const int64_t k0 = sl * kslY;
    GemmF32 g = yta;
    g.A = yta.A + k0 * yta.lda;  // Y (m x rl): A(i, k) = Y[k * rl + i]
    g.B = yta.B + k0 * yta.ldb;  // A (m x n):  B(k, j) = A[k * lda + j]
    g.K = (k0 + kslY < yta.K) ? kslY : yta.K - k0;
    g.D = partY + sl * yta.M * yta.N;
    g.ldd = yta.N;
    f32_tile_cfg<CF, false, false, VEC>(g, local, smem);
  } else {
    if (sl >= sA) return;
    const int64_t k0 = sl * kslA;
    GemmF32 g = ax;
    g.A = ax.A + k0;             // A (m x n):  A(i, k) = A[i * lda + k]
    g.B = ax.B + k0 * ax.ldb;    // X (n x r):  B(k, j) = X[k * r + j]
    g.K = (k0 + kslA < ax.K) ? kslA : ax.K - k0;
    g.D = partA + sl * ax.M * ax.N;
    g.ldd = ax.N;
    f32_tile_cfg<CF, true, false, VEC>(g, local, smem);
  }
}

template <class CF, int RPL, bool VEC>
__global__ void __launch_bounds__(CF::T) pass_f32_srht(GemmF32 yta, SrhtArgs sr, int64_t gY,
                                                       int64_t gS, int srht_first) {
  __shared__ __attribute__((aligned(16))) char smem[smax(CF::template smem<false, false>(),
                                                         SR_SMEM_F32)];
  int64_t local;
  if (take_first(gS, gY, srht_first, local))
    srht_rows<float, GN_MODE_F32, RPL>(sr, local, smem);
  else
    f32_tile_cfg<CF, false, false, VEC>(yta, local, smem);
}

template <class CF, bool F16>
__global__ void __launch_bounds__(CF::T) pass_bf16_gauss(GemmBF16 yta, GemmBF16 ax, int64_t gY,
                                                         int64_t gA) {
  __shared__ __attribute__((aligned(16))) char smem[CF::smem()];
  int64_t local;
  if (family_split(gY, gA, local))
    bf16_tile_cfg<CF, false, false, F16>(yta, local, smem);
  else
    bf16_tile_cfg<CF, true, true, F16>(ax, local, smem);
}

// One family of the pass on the large 16-bit tile (gemm_h16.h), one 256-thread
// workgroup per CU: Y^T A (AX_FAMILY false) or AX.  The two families run as two
// launches: in one launch, interleaved or one after the other, the pass took
// 19-20 ms at 32768^2, r = 2000, against 6.7 + 4.4 ms for the two alone.
template <bool F16, bool AX_FAMILY>
__global__ void __launch_bounds__(H16Big::T, 1) pass_h16_big(GemmBF16 g) {
  __shared__ __attribute__((aligned(16))) char smem[H16Big::smem()];
  h16_big_tile<AX_FAMILY, AX_FAMILY, F16>(g, blockIdx.x, smem);
}

template <class CF, int RPL, bool F16>
__global__ void __launch_bounds__(CF::T) pass_bf16_srht(GemmBF16 yta, SrhtArgs sr, int64_t gY,
                                                        int64_t gS, int srht_first) {
  __shared__ __attribute__((aligned(16))) char smem[smax(CF::smem(), SR_SMEM_F32)];
  int64_t local;
  if (take_first(gS, gY, srht_first, local))
    srht_rows<float, F16 ? GN_MODE_F16_BS : GN_MODE_BF16_BS, RPL>(sr, local, smem);
  else
    bf16_tile_cfg<CF, false, false, F16>(yta, local, smem);
}

template <int RPL>
__global__ void __launch_bounds__(256) pass_f64_srht(SrhtArgs sr) {
  __shared__ __attribute__((aligned(16))) char smem[SR_SMEM_F64];
  srht_rows<double, GN_MODE_F64, RPL>(sr, blockIdx.x, smem);
}

// B D H S for the rows of a row-major FP32 matrix B: the SRHT applied from the
// right exactly as the pass applies it to A, with the transform and the sums in
// FP64.  Gives the core matrix as (Y^T A) X for an SRHT X (Section 2.3's cost
// model: a transform of the r + l rows of Y^T A instead of a product over m).
template <int RPL>
__global__ void __launch_bounds__(256) srht_right_f64(SrhtArgs sr) {
  __shared__ __attribute__((aligned(16))) char smem[SR_SMEM_F64];
  srht_rows<double, GN_MODE_F32, RPL>(sr, blockIdx.x, smem);
}

int srht_rpl(int64_t r) {
  const int64_t q = cdiv(r, 64);
  return q <= 1 ? 1 : q <= 2 ? 2 : q <= 4 ? 4 : q <= 8 ? 8 : q <= 16 ? 16 : q <= 32 ? 32 : 0;
}

#define GN_RPL_SWITCH(RPL_VAL, CALL) \
  switch (RPL_VAL) {                 \
    case 1: CALL(1); break;          \
    case 2: CALL(2); break;          \
    case 4: CALL(4); break;          \
    case 8: CALL(8); break;          \
    case 16: CALL(16); break;        \
    case 32: CALL(32); break;        \
    default: return GN_ERR_UNSUPPORTED; \
  }

// Production FP32 schedule: SRHT rows first (they are HBM-bound and short),
// then the Y^T A tiles; 16 rows per SRHT workgroup.
constexpr int kSrhtFirst = 1;
constexpr int64_t kSrhtRows = 16;

// FP32 pass with tile configuration CF: one launch, SRHT rows or the AX tiles as
// the second family.
template <class CF>
gn_status launch_f32_cfg(bool srht, int srht_first, int64_t rows_per_wg, int64_t m, int64_t n,
                         int64_t r, int64_t rl, const float* A, int64_t lda, const float* X,
                         const float* Y, SrhtArgs sr, float* AX, int64_t ldax, float* YtA,
                         int64_t ldya, hipStream_t s) {
  GemmF32 yta{rl, n, m, Y, rl, A, lda, YtA, ldya, 1};
  const int64_t gY = cdiv(cdiv(rl, CF::BM) * cdiv(n, CF::BN), 8);
  bool vec = (lda % 4 == 0) && (rl % 4 == 0) && ((uintptr_t)A % 16 == 0) && ((uintptr_t)Y % 16 == 0);
  if (srht) {
    sr.rows_per_wg = rows_per_wg;
    const int64_t gS = cdiv(cdiv(m, rows_per_wg), 8);
    const dim3 grid((unsigned)(8 * (gY + gS)));
    const int rpl = srht_rpl(r);
#define GN_F32S(R)                                                                            \
  if (vec)                                                                                    \
    pass_f32_srht<CF, R, true><<<grid, dim3(CF::T), 0, s>>>(yta, sr, gY, gS, srht_first);      \
  else                                                                                        \
    pass_f32_srht<CF, R, false><<<grid, dim3(CF::T), 0, s>>>(yta, sr, gY, gS, srht_first)
    GN_RPL_SWITCH(rpl, GN_F32S)
#undef GN_F32S
  } else {
    GemmF32 ax{m, r, n, A, lda, X, r, AX, ldax, 0};
    const int64_t gA = cdiv(cdiv(m, CF::BM) * cdiv(r, CF::BN), 8);
    vec = vec && (r % 4 == 0) && ((uintptr_t)X % 16 == 0);
    const dim3 grid((unsigned)(8 * (gY + gA)));
    if (vec)
      pass_f32_gauss<CF, true><<<grid, dim3(CF::T), 0, s>>>(yta, ax, gY, gA);
    else
      pass_f32_gauss<CF, false><<<grid, dim3(CF::T), 0, s>>>(yta, ax, gY, gA);
  }
  GN_LAUNCH_CHECK();
  return GN_OK;
}

// FP32 Gaussian pass for r and r + l up to 512 and 768: tiles of 64 sketch rows
// (Y^T A) or columns (AX) by 256, four waves of 64 x 64 each, so the narrow side
// is padded to 64 instead of 256 (at 32768^2, r = 16, l = 8 the 256 x 256 tile
// did ten times the useful matrix-core work) and the many small tiles fill the
// CUs evenly where the 256 x 256 tiles leave a partial last round (r = 256, 384,
// 512 at 32768^2: 384, 640, 640 large tiles on 256 CUs).  Above that the large
// tile's higher reuse wins.
using F32NarrowY = F32Cfg<64, 256, 16, 1, 4, 32>;   // Y^T A: rl x n
using F32NarrowA = F32Cfg<256, 64, 16, 4, 1, 32>;   // AX:    m x r
static_assert(F32NarrowY::T == F32NarrowA::T, "one workgroup size for both families");
constexpr int64_t kNarrowMaxR = 512, kNarrowMaxRL = 768, kNarrowMinTiles = 128;

int64_t f32_narrow_tiles(int64_t m, int64_t n, int64_t r, int64_t rl) {
  return cdiv(rl, F32NarrowY::BM) * cdiv(n, F32NarrowY::BN) +
         cdiv(m, F32NarrowA::BM) * cdiv(r, F32NarrowA::BN);
}
bool use_f32_narrow_tiles(int64_t m, int64_t n, int64_t r, int64_t rl) {
  return r <= kNarrowMaxR && rl <= kNarrowMaxRL && f32_narrow_tiles(m, n, r, rl) >= kNarrowMinTiles;
}

// K split into slices (blockIdx.y) so that about three workgroups run per CU:
// slice s of Y^T A covers rows [s kslY, ...) of A and slice s of AX its columns
// [s kslA, ...), each writing its own partial, summed afterwards in slice order.
struct NarrowSplit {
  int64_t sY, kslY, sA, kslA;
  size_t bytes;  // partials (0: one slice)
};
NarrowSplit narrow_split(int64_t tiles, int64_t m, int64_t n, int64_t r, int64_t rl,
                         int64_t kgran, size_t elem) {
  int64_t sl = cdiv(768, tiles);
  if (sl > 16) sl = 16;
  NarrowSplit ns{1, m, 1, n, 0};
  if (sl <= 1) return ns;
  ns.kslY = cdiv(cdiv(m, sl), kgran) * kgran;
  ns.kslA = cdiv(cdiv(n, sl), kgran) * kgran;
  if (ns.kslY < 1024 || ns.kslA < 1024) return NarrowSplit{1, m, 1, n, 0};
  ns.sY = cdiv(m, ns.kslY);
  ns.sA = cdiv(n, ns.kslA);
  ns.bytes = align_up((size_t)ns.sY * rl * n * elem) + align_up((size_t)ns.sA * m * r * elem);
  return ns;
}

template <bool VEC>
__global__ void __launch_bounds__(F32NarrowY::T) pass_f32_gauss_nt(GemmF32 yta, GemmF32 ax,
                                                                   int64_t gY, int64_t gA,
                                                                   NarrowSplit ns, float* partY,
                                                                   float* partA) {
  __shared__ __attribute__((aligned(16))) char smem[smax(
      F32NarrowY::template smem<false, false>(), F32NarrowA::template smem<true, false>())];
  const int64_t sl = blockIdx.y;
  int64_t local;
  if (family_split(gY, gA, local)) {
    if (sl >= ns.sY) return;
    GemmF32 g = yta;
    if (partY) {
      const int64_t k0 = sl * ns.kslY;
      g.A = yta.A + k0 * yta.lda;  // Y (m x rl): A(i, k) = Y[k * rl + i]
      g.B = yta.B + k0 * yta.ldb;  // A (m x n):  B(k, j) = A[k * lda + j]
      g.K = (k0 + ns.kslY < yta.K) ? ns.kslY : yta.K - k0;
      g.D = partY + sl * yta.M * yta.N;
      g.ldd = yta.N;
    }
    f32_tile_cfg<F32NarrowY, false, false, VEC>(g, local, smem);
  } else {
    if (sl >= ns.sA) return;
    GemmF32 g = ax;
    if (partA) {
      const int64_t k0 = sl * ns.kslA;
      g.A = ax.A + k0;             // A (m x n):  A(i, k) = A[i * lda + k]
      g.B = ax.B + k0 * ax.ldb;    // X (n x r):  B(k, j) = X[k * r + j]
      g.K = (k0 + ns.kslA < ax.K) ? ns.kslA : ax.K - k0;
      g.D = partA + sl * ax.M * ax.N;
      g.ldd = ax.N;
    }
    f32_tile_cfg<F32NarrowA, true, false, VEC>(g, local, smem);
  }
}

NarrowSplit f32_narrow_split(int64_t m, int64_t n, int64_t r, int64_t rl) {
  return narrow_split(f32_narrow_tiles(m, n, r, rl), m, n, r, rl, F32NarrowY::BK, sizeof(float));
}

gn_status launch_f32_gauss_nt(int64_t m, int64_t n, int64_t r, int64_t rl, const float* A,
                              int64_t lda, const float* X, const float* Y, float* AX,
                              int64_t ldax, float* YtA, int64_t ldya, void* ws, size_t ws_bytes,
                              hipStream_t s) {
  GemmF32 yta{rl, n, m, Y, rl, A, lda, YtA, ldya, 1};
  GemmF32 ax{m, r, n, A, lda, X, r, AX, ldax, 0};
  const int64_t gY = cdiv(cdiv(rl, F32NarrowY::BM) * cdiv(n, F32NarrowY::BN), 8);
  const int64_t gA = cdiv(cdiv(m, F32NarrowA::BM) * cdiv(r, F32NarrowA::BN), 8);
  const bool vec = (lda % 4 == 0) && (rl % 4 == 0) && (r % 4 == 0) && ((uintptr_t)A % 16 == 0) &&
                   ((uintptr_t)Y % 16 == 0) && ((uintptr_t)X % 16 == 0);
  NarrowSplit ns = f32_narrow_split(m, n, r, rl);
  if (ns.bytes == 0 || !ws || ws_bytes < ns.bytes) ns = NarrowSplit{1, m, 1, n, 0};
  float* partY = ns.bytes ? (float*)ws : nullptr;
  float* partA = ns.bytes ? (float*)((char*)ws + align_up((size_t)ns.sY * rl * n * 4)) : nullptr;
  const int64_t sl = ns.sY > ns.sA ? ns.sY : ns.sA;
  const dim3 grid((unsigned)(8 * (gY + gA)), (unsigned)sl);
  if (vec)
    pass_f32_gauss_nt<true><<<grid, dim3(F32NarrowY::T), 0, s>>>(yta, ax, gY, gA, ns, partY, partA);
  else
    pass_f32_gauss_nt<false><<<grid, dim3(F32NarrowY::T), 0, s>>>(yta, ax, gY, gA, ns, partY,
                                                                  partA);
  GN_LAUNCH_CHECK();
  if (!ns.bytes) return GN_OK;
  GN_TRY(launch_splitk_sum_f32(partY, ns.sY, rl, n, YtA, ldya, s));
  return launch_splitk_sum_f32(partA, ns.sA, m, r, AX, ldax, s);
}

struct PassSplit {
  int64_t sY, kslY, sA, kslA;
  size_t bytes;
};
PassSplit pass_split(int64_t m, int64_t n, int64_t r, int64_t rl) {
  const int64_t tY = cdiv(rl, F32Pass::BM) * cdiv(n, F32Pass::BN);
  const int64_t tA = cdiv(m, F32Pass::BM) * cdiv(r, F32Pass::BN);
  const SplitK sk = f32_split2(tY, m, tA, n);
  PassSplit ps{1, m, 1, n, 0};
  if (sk.kslice == 0) return ps;
  ps.kslY = sk.kslice;
  ps.sY = cdiv(m, ps.kslY);
  ps.kslA = sk.kslice;
  ps.sA = cdiv(n, ps.kslA);
  ps.bytes = align_up((size_t)ps.sY * rl * n * sizeof(float)) +
             align_up((size_t)ps.sA * m * r * sizeof(float));
  return ps;
}

// FP32 Gaussian pass split along K (pass_split), then the slice sums.
gn_status launch_f32_split(const PassSplit& ps, int64_t m, int64_t n, int64_t r, int64_t rl,
                           const float* A, int64_t lda, const float* X, const float* Y, float* AX,
                           int64_t ldax, float* YtA, int64_t ldya, char* ws, hipStream_t s) {
  using CF = F32Pass;
  float* partY = (float*)ws;
  float* partA = (float*)(ws + align_up((size_t)ps.sY * rl * n * sizeof(float)));
  GemmF32 yta{rl, n, m, Y, rl, A, lda, YtA, ldya, 1};
  GemmF32 ax{m, r, n, A, lda, X, r, AX, ldax, 0};
  const int64_t gY = cdiv(cdiv(rl, CF::BM) * cdiv(n, CF::BN), 8);
  const int64_t gA = cdiv(cdiv(m, CF::BM) * cdiv(r, CF::BN), 8);
  const bool vec = (lda % 4 == 0) && (rl % 4 == 0) && (r % 4 == 0) && ((uintptr_t)A % 16 == 0) &&
                   ((uintptr_t)Y % 16 == 0) && ((uintptr_t)X % 16 == 0);
  const int64_t sl = ps.sY > ps.sA ? ps.sY : ps.sA;
  const dim3 grid((unsigned)(8 * (gY + gA)), (unsigned)sl);
  if (vec)
    pass_f32_gauss_split<CF, true><<<grid, dim3(CF::T), 0, s>>>(yta, ax, gY, gA, ps.kslY, ps.kslA,
                                                                ps.sY, ps.sA, partY, partA);
  else
    pass_f32_gauss_split<CF, false><<<grid, dim3(CF::T), 0, s>>>(yta, ax, gY, gA, ps.kslY,
                                                                 ps.kslA, ps.sY, ps.sA, partY,
                                                                 partA);
  GN_LAUNCH_CHECK();
  GN_TRY(launch_splitk_sum_f32(partY, ps.sY, rl, n, YtA, ldya, s));
  return launch_splitk_sum_f32(partA, ps.sA, m, r, AX, ldax, s);
}

// 16-bit Gaussian pass for small r and r + l (at most 64 and 96): the general
// 16-bit tile with 64 sketch rows (Y^T A) or columns (AX) by 256, four waves of
// 64 x 64 each, K staged 32 deep (the large tile padded r + l = 24 to 256).
constexpr int64_t kH16NarrowMaxR = 64, kH16NarrowMaxRL = 96;
using H16NarrowY = BF16Cfg<64, 256, 32, 1, 4>;
using H16NarrowA = BF16Cfg<256, 64, 32, 4, 1>;
static_assert(H16NarrowY::T == H16NarrowA::T, "one workgroup size for both families");

template <bool F16>
__global__ void __launch_bounds__(H16NarrowY::T) pass_bf16_gauss_nt(GemmBF16 yta, GemmBF16 ax,
                                                                    int64_t gY, int64_t gA,
                                                                    NarrowSplit ns, float* partY,
                                                                    float* partA) {
  __shared__ __attribute__((aligned(16))) char smem[smax(H16NarrowY::smem(), H16NarrowA::smem())];
  const int64_t sl = blockIdx.y;
  int64_t local;
  // K slices are multiples of 128, so a slice starts on a block-scale boundary
  if (family_split(gY, gA, local)) {
    if (sl >= ns.sY) return;
    GemmBF16 g = yta;
    if (partY) {
      const int64_t k0 = sl * ns.kslY;
      g.A = yta.A + k0;                   // Y^T (rl x m, k-contiguous)
      g.B = yta.B + k0 * yta.ldb;         // the matrix, row k0 on
      g.scales = yta.scales + (k0 >> 7) * yta.nsb;
      g.K = (k0 + ns.kslY < yta.K) ? ns.kslY : yta.K - k0;
      g.D = partY + sl * yta.M * yta.N;
      g.ldd = yta.N;
    }
    bf16_tile_cfg<H16NarrowY, false, false, F16>(g, local, smem);
  } else {
    if (sl >= ns.sA) return;
    GemmBF16 g = ax;
    if (partA) {
      const int64_t k0 = sl * ns.kslA;
      g.A = ax.A + k0;                    // the matrix, column k0 on
      g.B = ax.B + k0;                    // X^T (r x n, k-contiguous)
      g.scales = ax.scales + (k0 >> 7);
      g.K = (k0 + ns.kslA < ax.K) ? ns.kslA : ax.K - k0;
      g.D = partA + sl * ax.M * ax.N;
      g.ldd = ax.N;
    }
    bf16_tile_cfg<H16NarrowA, true, true, F16>(g, local, smem);
  }
}

int64_t h16_narrow_tiles(int64_t m, int64_t n, int64_t r, int64_t rl) {
  return cdiv(rl, H16NarrowY::BM) * cdiv(n, H16NarrowY::BN) +
         cdiv(m, H16NarrowA::BM) * cdiv(r, H16NarrowA::BN);
}
// (at r = 128, r + l = 192 the large tile was as fast: 1.91 against 2.02 ms at 32768^2)
bool use_h16_narrow_tiles(int64_t m, int64_t n, int64_t r, int64_t rl) {
  return r <= kH16NarrowMaxR && rl <= kH16NarrowMaxRL &&
         h16_narrow_tiles(m, n, r, rl) >= kNarrowMinTiles;
}
NarrowSplit h16_narrow_split(int64_t m, int64_t n, int64_t r, int64_t rl) {
  return narrow_split(h16_narrow_tiles(m, n, r, rl), m, n, r, rl, 128, sizeof(float));
}

// BF16 / binary16 (F16) pass with tile configuration CF (sketches stored
// transposed: Xt r x n, Yt rl x m).
template <class CF, bool F16>
gn_status launch_bf16_cfg(bool srht, int srht_first, int64_t rows_per_wg, int64_t m, int64_t n,
                          int64_t r, int64_t rl, const uint16_t* A, int64_t lda,
                          const float* scales, const uint16_t* Xt, const uint16_t* Yt, SrhtArgs sr,
                          float* AX, int64_t ldax, float* YtA, int64_t ldya, hipStream_t s,
                          void* ws, size_t ws_bytes) {
  const int64_t nsb = cdiv(n, 128);
  const bool vec_y = (lda % 8 == 0) && (m % 8 == 0) && ((uintptr_t)A % 16 == 0) &&
                     ((uintptr_t)Yt % 16 == 0);
  GemmBF16 yta{rl, n, m, Yt, m, A, lda, scales, nsb, YtA, ldya, 1, vec_y ? 1 : 0};
  const int64_t gY = cdiv(cdiv(rl, CF::BM) * cdiv(n, CF::BN), 8);
  if (srht) {
    sr.rows_per_wg = rows_per_wg;
    const int64_t gS = cdiv(cdiv(m, rows_per_wg), 8);
    const dim3 grid((unsigned)(8 * (gY + gS)));
    const int rpl = srht_rpl(r);
#define GN_BFS(R) pass_bf16_srht<CF, R, F16><<<grid, dim3(CF::T), 0, s>>>(yta, sr, gY, gS, srht_first)
    GN_RPL_SWITCH(rpl, GN_BFS)
#undef GN_BFS
  } else {
    const bool vec_x = (lda % 8 == 0) && (n % 8 == 0) && ((uintptr_t)A % 16 == 0) &&
                       ((uintptr_t)Xt % 16 == 0);
    GemmBF16 ax{m, r, n, A, lda, Xt, n, scales, nsb, AX, ldax, 0, vec_x ? 1 : 0};
    if (use_h16_narrow_tiles(m, n, r, rl)) {
      const int64_t gYn = cdiv(cdiv(rl, H16NarrowY::BM) * cdiv(n, H16NarrowY::BN), 8);
      const int64_t gAn = cdiv(cdiv(m, H16NarrowA::BM) * cdiv(r, H16NarrowA::BN), 8);
      NarrowSplit ns = h16_narrow_split(m, n, r, rl);
      if (ns.bytes == 0 || !ws || ws_bytes < ns.bytes) ns = NarrowSplit{1, m, 1, n, 0};
      float* partY = ns.bytes ? (float*)ws : nullptr;
      float* partA = ns.bytes ? (float*)((char*)ws + align_up((size_t)ns.sY * rl * n * 4)) : nullptr;
      const int64_t sl = ns.sY > ns.sA ? ns.sY : ns.sA;
      pass_bf16_gauss_nt<F16><<<dim3((unsigned)(8 * (gYn + gAn)), (unsigned)sl),
                                dim3(H16NarrowY::T), 0, s>>>(yta, ax, gYn, gAn, ns, partY, partA);
      GN_LAUNCH_CHECK();
      if (!ns.bytes) return GN_OK;
      GN_TRY(launch_splitk_sum_f32(partY, ns.sY, rl, n, YtA, ldya, s));
      return launch_splitk_sum_f32(partA, ns.sA, m, r, AX, ldax, s);
    }
    if (h16_big_eligible(yta, false) && h16_big_eligible(ax, true)) {
      const int64_t tY = cdiv(rl, H16Big::BM) * cdiv(n, H16Big::BN);
      const int64_t tA = cdiv(m, H16Big::BM) * cdiv(r, H16Big::BN);
      pass_h16_big<F16, false><<<dim3((unsigned)(8 * cdiv(tY, 8))), dim3(H16Big::T), 0, s>>>(yta);
      GN_LAUNCH_CHECK();
      pass_h16_big<F16, true><<<dim3((unsigned)(8 * cdiv(tA, 8))), dim3(H16Big::T), 0, s>>>(ax);
      GN_LAUNCH_CHECK();
      return GN_OK;
    }
    const int64_t gA = cdiv(cdiv(m, CF::BM) * cdiv(r, CF::BN), 8);
    pass_bf16_gauss<CF, F16><<<dim3((unsigned)(8 * (gY + gA))), dim3(CF::T), 0, s>>>(yta, ax, gY,
                                                                                       gA);
  }
  GN_LAUNCH_CHECK();
  return GN_OK;
}

}  // namespace

gn_status launch_pass(int32_t mode, int32_t kind_x, int64_t m, int64_t n, int64_t r, int64_t rl,
                      const void* A, int64_t lda, const float* scales, const void* Xs,
                      const int8_t* signs, const int32_t* idx, const void* Ys, void* AX,
                      int64_t ldax, void* YtA, int64_t ldya, hipStream_t s, void* split_ws,
                      size_t split_bytes) {
  // F64 / F32: Xs = X (n x r, ld r), Ys = Y (m x rl, ld rl).
  // BF16:      Xs = X^T (r x n, ld n), Ys = Y^T (rl x m, ld m).
  const void* Xt = Xs;
  const void* Yt = Ys;
  const bool srht = (kind_x == GN_SKETCH_SRHT);
  const int64_t nsb = cdiv(n, 128);
  SrhtArgs sr{16, m, n, r, A, lda, scales, nsb, signs, idx, AX, ldax};
  const int rpl = srht ? srht_rpl(r) : 1;

  if (mode == GN_MODE_F64) {
    if (srht) {
      const dim3 grid((unsigned)cdiv(m, sr.rows_per_wg));
#define GN_F64S(R) pass_f64_srht<R><<<grid, dim3(256), 0, s>>>(sr)
      GN_RPL_SWITCH(rpl, GN_F64S)
#undef GN_F64S
      GN_LAUNCH_CHECK();
    } else {
      // products with few output tiles split K through the workspace (slice sums in order)
      GN_TRY(launch_dgemm(m, r, n, 1.0, MatRef{A, GN_DT_F64, lda, 1}, MatRef{Xs, GN_DT_F64, r, 1},
                          0.0, (double*)AX, ldax, 1, nullptr, false, s, nullptr, 0, true,
                          (double*)split_ws, split_bytes));
    }
    return launch_dgemm(rl, n, m, 1.0, MatRef{Ys, GN_DT_F64, 1, rl}, MatRef{A, GN_DT_F64, lda, 1},
                        0.0, (double*)YtA, ldya, 1, nullptr, false, s, nullptr, 0, true,
                        (double*)split_ws, split_bytes);
  }

  if (mode == GN_MODE_F32 && !srht) {
    if (rl <= 16) {
      const gn_status st = launch_f32_gauss_narrow(m, n, r, rl, (const float*)A, lda,
                                                   (const float*)Xs, (const float*)Ys, (float*)AX,
                                                   ldax, (float*)YtA, ldya, split_ws, split_bytes, s);
      if (st != GN_ERR_UNSUPPORTED) return st;
    }
    if (use_f32_narrow_tiles(m, n, r, rl))
      return launch_f32_gauss_nt(m, n, r, rl, (const float*)A, lda, (const float*)Xs,
                                 (const float*)Ys, (float*)AX, ldax, (float*)YtA, ldya, split_ws,
                                 split_bytes, s);
    const PassSplit ps = pass_split(m, n, r, rl);
    if (ps.bytes > 0 && split_ws && split_bytes >= ps.bytes)
      return launch_f32_split(ps, m, n, r, rl, (const float*)A, lda, (const float*)Xs,
                              (const float*)Ys, (float*)AX, ldax, (float*)YtA, ldya,
                              (char*)split_ws, s);
  }
  if (mode == GN_MODE_F32 && srht) {
    const gn_status st = launch_f32_srht_narrow(m, n, r, rl, (const float*)A, lda, (const float*)Ys,
                                                signs, idx, (float*)AX, ldax, (float*)YtA, ldya,
                                                split_ws, split_bytes, s);
    if (st != GN_ERR_UNSUPPORTED) return st;
  }
  if (mode == GN_MODE_F32)
    return launch_f32_cfg<F32Pass>(srht, kSrhtFirst, kSrhtRows, m, n, r, rl, (const float*)A, lda,
                                   (const float*)Xs, (const float*)Ys, sr, (float*)AX, ldax,
                                   (float*)YtA, ldya, s);

  if (mode == GN_MODE_F16_BS)
    return launch_bf16_cfg<BF16Pass, true>(srht, kSrhtFirst, kSrhtRows, m, n, r, rl,
                                           (const uint16_t*)A, lda, scales, (const uint16_t*)Xs,
                                           (const uint16_t*)Ys, sr, (float*)AX, ldax, (float*)YtA,
                                           ldya, s, split_ws, split_bytes);
  return launch_bf16_cfg<BF16Pass, false>(srht, kSrhtFirst, kSrhtRows, m, n, r, rl,
                                          (const uint16_t*)A, lda, scales, (const uint16_t*)Xs,
                                          (const uint16_t*)Ys, sr, (float*)AX, ldax, (float*)YtA,
                                          ldya, s, split_ws, split_bytes);
}

gn_status launch_srht_right(int64_t rows, int64_t n, int64_t r, const float* B, int64_t ldb,
                            const int8_t* signs, const int32_t* idx, double* out, int64_t ldo,
                            hipStream_t s) {
  if (rows <= 0) return GN_OK;
  // four waves, one row each
  const SrhtArgs sr{4, rows, n, r, B, ldb, nullptr, 0, signs, idx, out, ldo};
  const dim3 grid((unsigned)cdiv(rows, 4));
#define GN_SRR(R) srht_right_f64<R><<<grid, dim3(256), 0, s>>>(sr)
  GN_RPL_SWITCH(srht_rpl(r), GN_SRR);
#undef GN_SRR
  GN_LAUNCH_CHECK();
  return GN_OK;
}

size_t pass_split_ws_bytes(int32_t mode, int32_t kind_x, int64_t m, int64_t n, int64_t r,
                           int64_t rl) {
  if (mode == GN_MODE_BF16_BS || mode == GN_MODE_F16_BS)
    return (kind_x == GN_SKETCH_GAUSSIAN && use_h16_narrow_tiles(m, n, r, rl))
               ? h16_narrow_split(m, n, r, rl).bytes
               : 0;
  if (mode == GN_MODE_F64) {
    const size_t y = dgemm_split_ws_bytes(rl, n, m);
    const size_t x = (kind_x == GN_SKETCH_SRHT) ? 0 : dgemm_split_ws_bytes(m, r, n);
    return x > y ? x : y;
  }
  if (mode != GN_MODE_F32) return 0;
  if (kind_x == GN_SKETCH_SRHT) return narrow_srht_ws_bytes(m, n, r, rl);
  const size_t gb = narrow_gauss_ws_bytes(m, n, r, rl);
  if (gb) return gb;
  if (use_f32_narrow_tiles(m, n, r, rl)) return f32_narrow_split(m, n, r, rl).bytes;
  return pass_split(m, n, r, rl).bytes;
}

}  // namespace gn
