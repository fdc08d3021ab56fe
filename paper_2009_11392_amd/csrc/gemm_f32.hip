// FP32 matrix-core products outside the fused pass:
//   * the core product C = Y^T (AX) of the FP32 and BF16 modes (Section 5.1
//     order), split along K = m into slices summed in order in FP64;
//   * a plain FP32 GEMM D = A B with the pass's 256 x 256 tile, optionally split
//     along K when there are too few output tiles to fill the chip (slices
//     written to their own partials and summed in slice order, in FP64, then
//     rounded once: deterministic);
//   * the core product of the BF16 mode on the BF16 matrix cores (Y is stored as
//     bfloat16 values, AX split into two bfloat16 terms);
//   * bfloat16 -> float widening of user sketches.
#include "gn_internal.h"
#include "gemm_tiles.h"

namespace gn {
namespace {

using namespace tiles;

// Large cores take the pass's 256 x 256 tile (16 waves, one workgroup per CU),
// small ones a 128 x 128 tile (4 waves) that gives them more workgroups.
using CoreBig = F32Pass;
using CoreSmall = F32Cfg<128, 128, 16, 2, 2, 32>;

template <class CoreCfg, bool VEC>
__global__ void __launch_bounds__(CoreCfg::T) core_product_f32(GemmF32 g, int64_t kslice) {
  __shared__ __attribute__((aligned(16))) char smem[CoreCfg::template smem<false, false>()];
  const int64_t s = blockIdx.y;
  const int64_t k0 = s * kslice;
  GemmF32 gs = g;
  gs.A = g.A + k0 * g.lda;
  gs.B = g.B + k0 * g.ldb;
  gs.K = (k0 + kslice < g.K) ? kslice : g.K - k0;
  gs.D = g.D + s * g.M * g.N;
  if (gs.K <= 0) return;
  f32_tile_cfg<CoreCfg, false, false, VEC>(gs, blockIdx.x, smem);
}

// ------------------------------------------------------------------ BF16 core product
// In BF16 mode Y holds bfloat16 values, so C = Y^T (AX) runs on the BF16 matrix
// cores: AX (FP32) is split into two bfloat16 terms, AX = hi + lo with hi =
// bf16(AX) and lo = bf16(AX - hi) (16 significant bits: the representation error,
// below 2^-17 |AX|, is far under the BF16 pass's own), and C = Y^T hi + Y^T lo
// with FP32 accumulation, K = m split into slices; the 2 x slices partial
// products are summed in FP64 in a fixed order.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__global__ void __launch_bounds__(256) split_bf16x2(const float* __restrict__ AX, int64_t ldax,
                                                    int64_t m, int64_t r, uint16_t* __restrict__ hi,
                                                    uint16_t* __restrict__ lo) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= m * r) return;
  const int64_t i = e / r, j = e - i * r;
  const float x = AX[i * ldax + j];
  const uint16_t h = f32_to_bf16_rne(x);
  hi[e] = h;
  lo[e] = f32_to_bf16_rne(x - bf16_bits_to_f32(h));  // the difference is exact in FP32
}

__global__ void __launch_bounds__(256) fill_f32(float* p, int64_t n, float v) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) p[e] = v;
}

// slice blockIdx.y of K (length kslice), term blockIdx.z (0: hi, 1: lo) to
// partial + (2 slice + term) M N
template <bool F16>
__global__ void __launch_bounds__(BF16Pass::T) core_product_bf16(GemmBF16 g, int64_t kslice,
                                                                 const uint16_t* hi,
                                                                 const uint16_t* lo,
                                                                 float* partial) {
  __shared__ __attribute__((aligned(16))) char smem[BF16Pass::smem()];
  const int64_t sl = blockIdx.y, term = blockIdx.z;
  const int64_t k0 = sl * kslice;
  GemmBF16 gs = g;
  gs.K = (k0 + kslice < g.K) ? kslice : g.K - k0;
  if (gs.K <= 0) return;
  gs.A = g.A + k0;
  gs.B = (term ? lo : hi) + k0 * g.ldb;
  gs.D = partial + (2 * sl + term) * g.M * g.N;
  bf16_tile_cfg<BF16Pass, true, false, F16>(gs, blockIdx.x, smem);
}

// ------------------------------------------------------------------ FP16 core product
// In FP16 mode Y holds binary16 values: the same two-term product on the f16
// matrix cores, with each column j of AX first divided by s_j, the power of two
// just above its largest magnitude, so that hi = f16(AX / s) and lo =
// f16(AX / s - hi) stay in binary16's range (22 significant bits for entries
// within 2^-14 of the column's largest; smaller ones keep an absolute error
// below 2^-25 s_j, under the FP16 pass's own).  C = (Y^T hi + Y^T lo) diag(s),
// the factor exact.

// cmax[j] = bits of max_i |AX[i][j]| (non-negative floats order as integers;
// cmax starts at zero).  Block (column group of 64, row group of 1024).
__global__ void __launch_bounds__(256) colmax_abs(const float* __restrict__ AX, int64_t ldax,
                                                  int64_t m, int64_t r, uint32_t* cmax) {
  __shared__ float red[4][64];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * 64 + tx;
  const int64_t i0 = (int64_t)blockIdx.y * 1024;
  float mx = 0.f;
  if (j < r) {
    const int64_t i1 = (i0 + 1024 < m) ? i0 + 1024 : m;
    for (int64_t i = i0 + ty; i < i1; i += 4) mx = fmaxf(mx, fabsf(AX[i * ldax + j]));
  }
  red[ty][tx] = mx;
  __syncthreads();
  if (ty == 0 && j < r) {
    mx = fmaxf(fmaxf(red[0][tx], red[1][tx]), fmaxf(red[2][tx], red[3][tx]));
    atomicMax(cmax + j, __float_as_uint(mx));
  }
}

// s_j = 2^e with max |AX[:, j]| = f 2^e, f in [0.5, 1) (1 for a zero column)
__device__ __forceinline__ float col_scale(uint32_t bits) {
  const float mx = __uint_as_float(bits);
  if (!(mx > 0.f)) return 1.f;
  int e;
  frexpf(mx, &e);
  return ldexpf(1.f, e);
}

__global__ void __launch_bounds__(256) split_f16x2(const float* __restrict__ AX, int64_t ldax,
                                                   int64_t m, int64_t r, const uint32_t* cmax,
                                                   uint16_t* __restrict__ hi,
                                                   uint16_t* __restrict__ lo) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= m * r) return;
  const int64_t i = e / r, j = e - i * r;
  const float x = AX[i * ldax + j] * (1.f / col_scale(cmax[j]));  // exact: a power of two
  const _Float16 h = (_Float16)x;
  hi[e] = __builtin_bit_cast(uint16_t, h);
  lo[e] = __builtin_bit_cast(uint16_t, (_Float16)(x - (float)h));  // the difference is exact
}

__global__ void __launch_bounds__(256) core_product_sum2_scaled(const float* partial,
                                                                int64_t nslice, int64_t mn,
                                                                int64_t r, const uint32_t* cmax,
                                                                double* C) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= mn) return;
  double acc = 0.0;
  for (int64_t q = 0; q < nslice; ++q)
    acc += (double)partial[2 * q * mn + e] + (double)partial[(2 * q + 1) * mn + e];
  C[e] = acc * (double)col_scale(cmax[e % r]);
}

__global__ void __launch_bounds__(256) core_product_sum2(const float* partial, int64_t nslice,
                                                         int64_t mn, double* C) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= mn) return;
  double acc = 0.0;
  for (int64_t q = 0; q < nslice; ++q)
    acc += (double)partial[2 * q * mn + e] + (double)partial[(2 * q + 1) * mn + e];
  C[e] = acc;
}

__global__ void __launch_bounds__(256) core_product_sum(const float* partial, int64_t nslice,
                                                        int64_t mn, double* C) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= mn) return;
  double acc = 0.0;
  for (int64_t q = 0; q < nslice; ++q) acc += (double)partial[q * mn + e];
  C[e] = acc;
}

bool core_big(int64_t rl, int64_t r) {
  return cdiv(rl, CoreBig::BM) * cdiv(r, CoreBig::BN) >= 32;
}

// K slices.  256 x 256 tiles: the count (at most 16, slices at least 1024 long)
// that minimizes the rounds of one workgroup per CU times the slice length.
// 128 x 128 tiles: about 512 workgroups, slices at least 512 long.
int64_t core_slices(int64_t m, int64_t rl, int64_t r) {
  if (!core_big(rl, r)) {
    const int64_t tiles = cdiv(rl, CoreSmall::BM) * cdiv(r, CoreSmall::BN);
    int64_t sl = cdiv(512, tiles);
    if (sl > cdiv(m, 512)) sl = cdiv(m, 512);
    if (sl > 16) sl = 16;
    return sl < 1 ? 1 : sl;
  }
  const int64_t tiles = cdiv(rl, CoreBig::BM) * cdiv(r, CoreBig::BN);
  int64_t best = 1;
  double best_cost = (double)cdiv(tiles, 256) * (double)m;
  for (int64_t sl = 2; sl <= 16 && cdiv(m, sl) >= 1024; ++sl) {
    const double c = (double)cdiv(tiles * sl, 256) * (double)cdiv(m, sl);
    if (c < best_cost) {
      best_cost = c;
      best = sl;
    }
  }
  return best;
}

// D = A B; with `partial`, slice blockIdx.y of K (length kslice) goes to
// partial + slice * M * N (row stride N).
template <bool A_KC, bool B_KC, bool VEC>
__global__ void __launch_bounds__(F32Pass::T) gemm_f32_kernel(GemmF32 g, int64_t kslice,
                                                              float* partial) {
  __shared__ __attribute__((aligned(16))) char smem[F32Pass::smem<A_KC, B_KC>()];
  GemmF32 gs = g;
  if (partial) {
    const int64_t s = blockIdx.y, k0 = s * kslice;
    gs.A = A_KC ? g.A + k0 : g.A + k0 * g.lda;
    gs.B = B_KC ? g.B + k0 : g.B + k0 * g.ldb;
    gs.K = (k0 + kslice < g.K) ? kslice : g.K - k0;
    gs.D = partial + s * g.M * g.N;
    gs.ldd = g.N;
  }
  f32_tile_cfg<F32Pass, A_KC, B_KC, VEC>(gs, blockIdx.x, smem);
}

// D[i*ldd + j] = sum over slices (in order, FP64) of partial[s][i][j], rounded.
__global__ void __launch_bounds__(256) splitk_sum_f32(const float* partial, int64_t nslice,
                                                      int64_t M, int64_t N, float* D,
                                                      int64_t ldd) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * N) return;
  const int64_t i = e / N, j = e - i * N;
  double acc = 0.0;
  for (int64_t q = 0; q < nslice; ++q) acc += (double)partial[q * M * N + e];
  D[i * ldd + j] = (float)acc;
}

template <bool F16>
__global__ void __launch_bounds__(256) widen_h16_kernel(int64_t rows, int64_t cols,
                                                        const uint16_t* src, int64_t lds,
                                                        float* dst, int64_t ldd) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = e / cols, j = e - i * cols;
  dst[i * ldd + j] = h16_to_f32<F16>(src[i * lds + j]);
}

}  // namespace

// Common K slice for up to two product families (tiles1 with length K1, tiles2
// with K2) with few output tiles.  Cost model: workgroups run in waves of
// kSplitTargetWG (one per CU) and a workgroup's time grows with its slice
// length plus a fixed prologue/epilogue of about 256 K steps; the candidate
// slices are multiples of kSplitMinSlice.  kslice == 0: no split.
SplitK f32_split2(int64_t tiles1, int64_t K1, int64_t tiles2, int64_t K2) {
  SplitK best{1, 0};
  const int64_t tiles = tiles1 + tiles2;
  const int64_t Kmax = K1 > K2 ? K1 : K2;
  if (tiles >= kSplitMinTiles || Kmax < 2 * kSplitMinSlice) return best;
  auto cost = [&](int64_t wgs, int64_t klen) {
    return cdiv(wgs, kSplitTargetWG) * (klen + 256);
  };
  int64_t best_cost = cost(tiles, Kmax);  // unsplit
  for (int64_t ks = kSplitMinSlice; ks < Kmax; ks += kSplitMinSlice) {
    const int64_t wgs = tiles1 * cdiv(K1, ks) + tiles2 * cdiv(K2, ks);
    if (cdiv(K1, ks) > 32 || cdiv(K2, ks) > 32) continue;
    const int64_t c = cost(wgs, ks);
    if (c < best_cost) {
      best_cost = c;
      best.kslice = ks;
    }
  }
  best.slices = best.kslice ? cdiv(K1 > 0 ? K1 : 1, best.kslice) : 1;
  return best;
}

SplitK f32_split(int64_t tiles, int64_t K) {
  SplitK sk = f32_split2(tiles, K, 0, 0);
  if (sk.kslice == 0) return SplitK{1, K};
  sk.slices = cdiv(K, sk.kslice);
  return sk;
}

gn_status launch_splitk_sum_f32(const float* partial, int64_t nslice, int64_t M, int64_t N,
                                float* D, int64_t ldd, hipStream_t s) {
  if (M <= 0 || N <= 0) return GN_OK;
  splitk_sum_f32<<<dim3((unsigned)cdiv(M * N, 256)), dim3(256), 0, s>>>(partial, nslice, M, N, D,
                                                                        ldd);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

size_t core_product_ws_bytes(int64_t m, int64_t rl, int64_t r) {
  return align_up((size_t)core_slices(m, rl, r) * rl * r * sizeof(float));
}

// K slices of the BF16 core product: the 2 x tiles x slices workgroups (one
// 1024-thread workgroup per CU) run in rounds of 256, each of time ~ K / slices,
// so the count that minimizes rounds / slices (the fewest such slices), with
// slices at least 1024 long and a multiple of 128, at most 16.
struct Bf16CoreLayout {
  int64_t kslice, nslice, nsb;
  size_t hi, lo, ones, partial, cmax, total;
};
static Bf16CoreLayout bf16_core_layout(int64_t m, int64_t rl, int64_t r) {
  Bf16CoreLayout L{};
  const int64_t tiles = cdiv(rl, BF16Pass::BM) * cdiv(r, BF16Pass::BN);
  const int64_t max_sl = std::max<int64_t>(1, std::min<int64_t>(16, cdiv(m, 1024)));
  int64_t sl = 1;
  double best = 0.0;
  for (int64_t c = 1; c <= max_sl; ++c) {
    const double t = (double)cdiv(2 * tiles * c, 256) / (double)c;
    if (c == 1 || t < best - 1e-9) {
      best = t;
      sl = c;
    }
  }
  L.kslice = cdiv(cdiv(m, sl), 128) * 128;
  L.nslice = cdiv(m, L.kslice);
  L.nsb = L.kslice / 128;
  size_t off = 0;
  L.hi = off;
  off += align_up((size_t)m * r * 2);
  L.lo = off;
  off += align_up((size_t)m * r * 2);
  L.ones = off;
  off += align_up((size_t)cdiv(rl, 128) * L.nsb * 4);
  L.partial = off;
  off += align_up((size_t)2 * L.nslice * rl * r * 4);
  L.cmax = off;
  off += align_up((size_t)r * 4);
  L.total = off;
  return L;
}

size_t core_product_bf16_ws_bytes(int64_t m, int64_t rl, int64_t r) {
  return bf16_core_layout(m, rl, r).total;
}

gn_status launch_core_product_h16(int64_t m, int64_t rl, int64_t r, const uint16_t* Yt, bool f16,
                                  const float* AX, int64_t ldax, void* ws, double* C,
                                  hipStream_t s) {
  const Bf16CoreLayout L = bf16_core_layout(m, rl, r);
  char* base = (char*)ws;
  uint16_t* hi = (uint16_t*)(base + L.hi);
  uint16_t* lo = (uint16_t*)(base + L.lo);
  float* ones = (float*)(base + L.ones);
  float* partial = (float*)(base + L.partial);
  uint32_t* cmax = (uint32_t*)(base + L.cmax);
  if (f16) {
    fill_f32<<<dim3((unsigned)cdiv(r, 256)), dim3(256), 0, s>>>((float*)cmax, r, 0.0f);
    GN_LAUNCH_CHECK();
    colmax_abs<<<dim3((unsigned)cdiv(r, 64), (unsigned)cdiv(m, 1024)), dim3(256), 0, s>>>(
        AX, ldax, m, r, cmax);
    GN_LAUNCH_CHECK();
    split_f16x2<<<dim3((unsigned)cdiv(m * r, 256)), dim3(256), 0, s>>>(AX, ldax, m, r, cmax, hi,
                                                                        lo);
  } else {
    split_bf16x2<<<dim3((unsigned)cdiv(m * r, 256)), dim3(256), 0, s>>>(AX, ldax, m, r, hi, lo);
  }
  GN_LAUNCH_CHECK();
  const int64_t nones = cdiv(rl, 128) * L.nsb;
  fill_f32<<<dim3((unsigned)cdiv(nones, 256)), dim3(256), 0, s>>>(ones, nones, 1.0f);
  GN_LAUNCH_CHECK();
  // A = Y^T (rl x m, k-contiguous) with unit block scales, B = hi / lo (m x r)
  const int vec = (m % 8 == 0) && (r % 8 == 0) && ((uintptr_t)Yt % 16 == 0) ? 1 : 0;
  const GemmBF16 g{rl, r, m, Yt, m, hi, r, ones, L.nsb, partial, r, 1, vec};
  const int64_t tiles = cdiv(rl, BF16Pass::BM) * cdiv(r, BF16Pass::BN);
  const dim3 grid((unsigned)(8 * cdiv(tiles, 8)), (unsigned)L.nslice, 2u);
  if (f16)
    core_product_bf16<true><<<grid, dim3(BF16Pass::T), 0, s>>>(g, L.kslice, hi, lo, partial);
  else
    core_product_bf16<false><<<grid, dim3(BF16Pass::T), 0, s>>>(g, L.kslice, hi, lo, partial);
  GN_LAUNCH_CHECK();
  if (f16)
    core_product_sum2_scaled<<<dim3((unsigned)cdiv(rl * r, 256)), dim3(256), 0, s>>>(
        partial, L.nslice, rl * r, r, cmax, C);
  else
    core_product_sum2<<<dim3((unsigned)cdiv(rl * r, 256)), dim3(256), 0, s>>>(partial, L.nslice,
                                                                            rl * r, C);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

gn_status launch_core_product_f32(int64_t m, int64_t rl, int64_t r, const float* Y, int64_t ldy,
                                  const float* AX, int64_t ldax, float* partial, double* C,
                                  hipStream_t s) {
  const int64_t sl = core_slices(m, rl, r);
  GemmF32 g{rl, r, m, Y, ldy, AX, ldax, partial, r, 1};
  const bool vec = (ldy % 4 == 0) && (ldax % 4 == 0) && ((uintptr_t)Y % 16 == 0) &&
                   ((uintptr_t)AX % 16 == 0);
  if (core_big(rl, r)) {
    const int64_t kslice = cdiv(cdiv(m, sl), CoreBig::BK) * CoreBig::BK;
    const int64_t tiles = cdiv(rl, CoreBig::BM) * cdiv(r, CoreBig::BN);
    const dim3 grid((unsigned)(8 * cdiv(tiles, 8)), (unsigned)sl);
    if (vec)
      core_product_f32<CoreBig, true><<<grid, dim3(CoreBig::T), 0, s>>>(g, kslice);
    else
      core_product_f32<CoreBig, false><<<grid, dim3(CoreBig::T), 0, s>>>(g, kslice);
  } else {
    const int64_t kslice = cdiv(cdiv(m, sl), 16) * 16;
    const int64_t tiles = cdiv(rl, CoreSmall::BM) * cdiv(r, CoreSmall::BN);
    const dim3 grid((unsigned)(8 * cdiv(tiles, 8)), (unsigned)sl);
    if (vec)
      core_product_f32<CoreSmall, true><<<grid, dim3(CoreSmall::T), 0, s>>>(g, kslice);
    else
      core_product_f32<CoreSmall, false><<<grid, dim3(CoreSmall::T), 0, s>>>(g, kslice);
  }
  GN_LAUNCH_CHECK();
  core_product_sum<<<dim3((unsigned)cdiv(rl * r, 256)), dim3(256), 0, s>>>(partial, sl, rl * r, C);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

size_t gemm_f32_split_ws_bytes(int64_t M, int64_t N, int64_t K) {
  const SplitK sk = f32_split(cdiv(M, F32Pass::BM) * cdiv(N, F32Pass::BN), K);
  return sk.slices > 1 ? align_up((size_t)sk.slices * M * N * sizeof(float)) : 0;
}

gn_status launch_gemm_f32(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda, bool a_kc,
                          const float* B, int64_t ldb, bool b_kc, float* D, int64_t ldd,
                          hipStream_t s, float* split_ws, size_t split_bytes) {
  if (M <= 0 || N <= 0) return GN_OK;
  GemmF32 g{M, N, K, A, lda, B, ldb, D, ldd, 1};
  const int64_t tiles = cdiv(M, F32Pass::BM) * cdiv(N, F32Pass::BN);
  SplitK sk = f32_split(tiles, K);
  if (sk.slices > 1 && (!split_ws || split_bytes < (size_t)sk.slices * M * N * sizeof(float)))
    sk = SplitK{1, K};
  float* partial = sk.slices > 1 ? split_ws : nullptr;
  const dim3 grid((unsigned)(8 * cdiv(tiles, 8)), (unsigned)sk.slices);
  const bool vec = (lda % 4 == 0) && (ldb % 4 == 0) && ((uintptr_t)A % 16 == 0) &&
                   ((uintptr_t)B % 16 == 0);
#define GN_GEMM(AK, BK)                                                                          \
  if (vec)                                                                                       \
    gemm_f32_kernel<AK, BK, true><<<grid, dim3(F32Pass::T), 0, s>>>(g, sk.kslice, partial);      \
  else                                                                                           \
    gemm_f32_kernel<AK, BK, false><<<grid, dim3(F32Pass::T), 0, s>>>(g, sk.kslice, partial)
  if (a_kc && b_kc) {
    GN_GEMM(true, true);
  } else if (a_kc) {
    GN_GEMM(true, false);
  } else if (b_kc) {
    GN_GEMM(false, true);
  } else {
    GN_GEMM(false, false);
  }
#undef GN_GEMM
  GN_LAUNCH_CHECK();
  if (partial) return launch_splitk_sum_f32(partial, sk.slices, M, N, D, ldd, s);
  return GN_OK;
}

gn_status launch_widen_h16(int64_t rows, int64_t cols, const uint16_t* src, int64_t lds, bool f16,
                           float* dst, int64_t ldd, hipStream_t s) {
  const dim3 grid((unsigned)cdiv(rows * cols, 256)), block(256);
  if (f16)
    widen_h16_kernel<true><<<grid, block, 0, s>>>(rows, cols, src, lds, dst, ldd);
  else
    widen_h16_kernel<false><<<grid, block, 0, s>>>(rows, cols, src, lds, dst, ldd);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

}  // namespace gn
