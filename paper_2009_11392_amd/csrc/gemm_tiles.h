// Matrix-core tile bodies for the sketch pass (device functions; each fused
// pass kernel calls one of them per workgroup).
//
// FP32: v_mfma_f32_32x32x2_f32 or v_mfma_f32_16x16x4_f32, tile shape a template
// parameter (F32Cfg).  BF16: v_mfma_f32_32x32x16_bf16, 256 threads = 4 waves in
// 2 x 2, workgroup tile 128 x 128, wave tile 64 x 64 = 2 x 2 MFMA blocks.  K is
// staged through LDS double buffered; FP32 accumulation.
#pragma once

#include <type_traits>

#include "gn_internal.h"

namespace gn {
namespace tiles {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ workgroup scheduling
// Workgroups are dispatched round-robin over the 8 XCDs (blockIdx % 8).  A fused
// grid holds two families of work in groups of 8 consecutive workgroups; group g
// goes to family A when floor((g+1) gA / G) > floor(g gA / G), which spreads the
// gA groups of A evenly among all G = gA + gB groups.  `local` is the index of
// the workgroup within its family, with local % 8 equal to its XCD.
__device__ __forceinline__ bool family_split(int64_t gA, int64_t gB, int64_t& local) {
  const int64_t g = (int64_t)blockIdx.x >> 3, x = (int64_t)blockIdx.x & 7;
  const int64_t G = gA + gB;
  const int64_t before = (g * gA) / G, after = ((g + 1) * gA) / G;
  if (after > before) {
    local = before * 8 + x;
    return true;
  }
  local = (g - before) * 8 + x;
  return false;
}

// Tile of a family: each XCD owns a contiguous range of tiles, and consecutive
// tiles on one XCD share the operand panel named by the outer index (it is then
// read from HBM once and served from that XCD's L2 afterwards).
__device__ __forceinline__ bool xcd_tile(int64_t local, int64_t tiles_inner, int64_t tiles_outer,
                                         int64_t& ti, int64_t& to) {
  const int64_t total = tiles_inner * tiles_outer;
  const int64_t per = (total + 7) / 8;
  const int64_t t = (local & 7) * per + (local >> 3);
  if (t >= total) return false;
  ti = t % tiles_inner;
  to = t / tiles_inner;
  return true;
}


// ------------------------------------------------------------------ FP32
// D (M x N) = A (M x K) B (K x N), FP32 in, FP32 accumulation.
//   A_KC: A(i,k) = A[i*lda + k] (k-contiguous), else A[k*lda + i] (m-contiguous).
//   B_KC: B(k,j) = B[j*ldb + k] (k-contiguous), else B[k*ldb + j] (n-contiguous).
// LDS holds both operands k-major, S[k][row]: m/n-contiguous operands are
// stored with 16-byte writes, k-contiguous ones are transposed on the way in.
struct GemmF32 {
  int64_t M, N, K;
  const float* A;
  int64_t lda;
  const float* B;
  int64_t ldb;
  float* D;
  int64_t ldd;
  int inner_is_m;  // consecutive tiles walk M (share the B panel) or N (share A)
};

// Tile shape: BM x BN per workgroup of WM x WN waves, K staged BK deep, double
// buffered; MF = 32 (v_mfma_f32_32x32x2_f32) or 16 (v_mfma_f32_16x16x4_f32).
template <int BM_, int BN_, int BK_, int WM_, int WN_, int MF_>
struct F32Cfg {
  static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_, MF = MF_;
  static constexpr int T = 64 * WM * WN;
  static constexpr int TM = BM / WM, TN = BN / WN;      // wave tile
  static constexpr int FM = TM / MF, FN = TN / MF;      // MFMA blocks per wave
  static constexpr int KSTEP = (MF == 32) ? 2 : 4;
  static constexpr int NACC = (MF == 32) ? 16 : 4;
  template <bool KC>
  static constexpr int ld(int rows) { return rows + (KC ? 1 : 4); }
  template <bool A_KC, bool B_KC>
  static constexpr size_t smem() {
    return 2 * (size_t)BK * (ld<A_KC>(BM) + ld<B_KC>(BN)) * sizeof(float);
  }
};

// Global -> registers for one operand tile (ROWS x BK) of the K slab at k0.
template <int ROWS, int BK, int T, bool KC, bool VEC>
struct F32Stage {
  static constexpr int NV = ROWS * BK / 4 / T;  // float4 per thread
  static_assert(NV * 4 * T == ROWS * BK, "tile not divisible");
  f32x4 v[NV];
  __device__ __forceinline__ void load(const float* __restrict__ P, int64_t ld, int64_t rows,
                                       int64_t K, int64_t r0, int64_t k0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int e = threadIdx.x + T * q;
      int64_t row, k;
      if (KC) {
        row = r0 + e / (BK / 4);
        k = k0 + 4 * (e % (BK / 4));
      } else {
        k = k0 + e / (ROWS / 4);
        row = r0 + 4 * (e % (ROWS / 4));
      }
      f32x4 x = {0.f, 0.f, 0.f, 0.f};
      if (KC) {
        if (row < rows) {
          const float* src = P + row * ld + k;
          if (VEC && k + 3 < K) {
            x = *reinterpret_cast<const f32x4*>(src);
          } else {
#pragma unroll
            for (int t = 0; t < 4; ++t)
              if (k + t < K) x[t] = src[t];
          }
        }
      } else {
        if (k < K) {
          const float* src = P + k * ld + row;
          if (VEC && row + 3 < rows) {
            x = *reinterpret_cast<const f32x4*>(src);
          } else {
#pragma unroll
            for (int t = 0; t < 4; ++t)
              if (row + t < rows) x[t] = src[t];
          }
        }
      }
      v[q] = x;
    }
  }
  __device__ __forceinline__ void store(float* S) const {
    constexpr int LD = ROWS + (KC ? 1 : 4);
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int e = threadIdx.x + T * q;
      if (KC) {
        const int row = e / (BK / 4), k = 4 * (e % (BK / 4));
#pragma unroll
        for (int t = 0; t < 4; ++t) S[(k + t) * LD + row] = v[q][t];
      } else {
        const int k = e / (ROWS / 4), row = 4 * (e % (ROWS / 4));
        *reinterpret_cast<f32x4*>(S + k * LD + row) = v[q];
      }
    }
  }
};

// One BM x BN output tile at (i0, j0) of D = A B (the whole K range).
template <class CF, bool A_KC, bool B_KC, bool VEC>
__device__ void f32_tile_at(const GemmF32& g, int64_t i0, int64_t j0, char* smem) {
  constexpr int BM = CF::BM, BN = CF::BN, BK = CF::BK, MF = CF::MF;
  constexpr int LDA = CF::template ld<A_KC>(BM), LDB = CF::template ld<B_KC>(BN);
  typedef float accv __attribute__((ext_vector_type(CF::NACC)));
  float* sA = reinterpret_cast<float*>(smem);  // [2][BK * LDA]
  float* sB = sA + 2 * BK * LDA;               // [2][BK * LDB]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % CF::WM, wn = wave / CF::WM;
  const int li = lane % MF, lk = lane / MF;
  accv acc[CF::FM][CF::FN];
#pragma unroll
  for (int x = 0; x < CF::FM; ++x)
#pragma unroll
    for (int y = 0; y < CF::FN; ++y)
#pragma unroll
      for (int v = 0; v < CF::NACC; ++v) acc[x][y][v] = 0.f;

  F32Stage<BM, BK, CF::T, A_KC, VEC> sa;
  F32Stage<BN, BK, CF::T, B_KC, VEC> sb;
  const int64_t nk = cdiv_d(g.K, BK);
  sa.load(g.A, g.lda, g.M, g.K, i0, 0);
  sb.load(g.B, g.ldb, g.N, g.K, j0, 0);
  sa.store(sA);
  sb.store(sB);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) {
      sa.load(g.A, g.lda, g.M, g.K, i0, (kt + 1) * BK);
      sb.load(g.B, g.ldb, g.N, g.K, j0, (kt + 1) * BK);
    }
    const float* a_s = sA + cur * BK * LDA + wm * CF::TM + li;
    const float* b_s = sB + cur * BK * LDB + wn * CF::TN + li;
#pragma unroll
    for (int kk = 0; kk < BK; kk += CF::KSTEP) {
      float af[CF::FM], bf[CF::FN];
#pragma unroll
      for (int x = 0; x < CF::FM; ++x) af[x] = a_s[(kk + lk) * LDA + x * MF];
#pragma unroll
      for (int y = 0; y < CF::FN; ++y) bf[y] = b_s[(kk + lk) * LDB + y * MF];
#pragma unroll
      for (int x = 0; x < CF::FM; ++x)
#pragma unroll
        for (int y = 0; y < CF::FN; ++y) {
          if constexpr (MF == 32)
            acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[x], bf[y], acc[x][y], 0, 0, 0);
          else
            acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[x], bf[y], acc[x][y], 0, 0, 0);
        }
    }
    if (kt + 1 < nk) {
      sa.store(sA + (cur ^ 1) * BK * LDA);
      sb.store(sB + (cur ^ 1) * BK * LDB);
    }
    __syncthreads();
  }
  // accumulator layouts: 32x32 -- register v of lane l is row 8(v/4) + 4(l/32) + v%4;
  // 16x16 -- row 4(l/16) + v; column l % MF in both.
#pragma unroll
  for (int x = 0; x < CF::FM; ++x)
#pragma unroll
    for (int y = 0; y < CF::FN; ++y)
#pragma unroll
      for (int v = 0; v < CF::NACC; ++v) {
        const int rr = (MF == 32) ? (8 * (v >> 2) + 4 * lk + (v & 3)) : (4 * lk + v);
        const int64_t row = i0 + wm * CF::TM + x * MF + rr;
        const int64_t col = j0 + wn * CF::TN + y * MF + li;
        if (row < g.M && col < g.N) g.D[row * g.ldd + col] = acc[x][y][v];
      }
}

// The tile of XCD-mapped index `local` (tiles of one XCD walk the inner index).
template <class CF, bool A_KC, bool B_KC, bool VEC>
__device__ void f32_tile_cfg(const GemmF32& g, int64_t local, char* smem) {
  const int64_t tm_n = cdiv_d(g.M, CF::BM), tn_n = cdiv_d(g.N, CF::BN);
  int64_t tm, tn;
  if (g.inner_is_m) {
    if (!xcd_tile(local, tm_n, tn_n, tm, tn)) return;
  } else {
    if (!xcd_tile(local, tn_n, tm_n, tn, tm)) return;
  }
  f32_tile_at<CF, A_KC, B_KC, VEC>(g, tm * CF::BM, tn * CF::BN, smem);
}

// The production FP32 configuration of the sketch pass: 256 x 256 tiles, 16 waves
// (4 x 4, wave tile 64 x 64), K staged 32 deep.
using F32Pass = F32Cfg<256, 256, 32, 4, 4, 32>;

// ------------------------------------------------------------------ BF16 with block scales
// A(i,k) = PA[i*lda + k] (k-contiguous; the matrix A when A_IS_MAT, then scaled);
// B(k,j) = PB[j*ldb + k] when B_KC, else PB[k*ldb + j] (the matrix A, scaled).
// LDS holds both operands k-contiguous, S[row][k] (row stride BK + 8 bf16), the
// layout the bf16 MFMA fragments read with one 16-byte load per lane.
struct GemmBF16 {
  int64_t M, N, K;
  const uint16_t* A;
  int64_t lda;
  const uint16_t* B;
  int64_t ldb;
  const float* scales;  // 128 x 128 block scales of the matrix operand
  int64_t nsb;          // scale blocks per row of the matrix
  float* D;
  int64_t ldd;
  int inner_is_m;
  int vec;
};

template <int BM_, int BN_, int BK_, int WM_, int WN_>
struct BF16Cfg {
  static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_;
  static constexpr int T = 64 * WM * WN;
  static constexpr int TM = BM / WM, TN = BN / WN;
  static constexpr int FM = TM / 32, FN = TN / 32;
  static constexpr int LDK = BK + 8;
  static constexpr size_t smem() { return 2 * (size_t)(BM + BN) * LDK * sizeof(uint16_t); }
};

// Multiply two packed bfloat16 values by a power of two (exact).
__device__ __forceinline__ uint32_t scale_bf16x2(uint32_t w, float s) {
  const float lo = __uint_as_float(w << 16) * s;
  const float hi = __uint_as_float(w & 0xffff0000u) * s;
  return (__float_as_uint(lo) >> 16) | (__float_as_uint(hi) & 0xffff0000u);
}

// k-contiguous operand tile (ROWS x BK): 16-byte chunks straight into S[row][k].
// load() only issues the global loads (the prefetch of the next K slab); the
// block scale is applied in store(), after the current slab's MFMAs.
template <int ROWS, int BK, int T, bool SCALED>
struct BFStageKC {
  static constexpr int NV = ROWS * BK / 8 / T;
  static_assert(NV * 8 * T == ROWS * BK, "tile not divisible");
  u32x4 v[NV];
  float sc[SCALED ? NV : 1];
  __device__ __forceinline__ void load(const uint16_t* __restrict__ P, int64_t ld, int64_t rows,
                                       int64_t K, int64_t r0, int64_t k0,
                                       const float* __restrict__ scales, int64_t nsb, bool vec) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int e = threadIdx.x + T * q;
      const int64_t row = r0 + e / (BK / 8), k = k0 + 8 * (e % (BK / 8));
      u32x4 x = {0u, 0u, 0u, 0u};
      float s = 0.f;
      if (row < rows && k < K) {
        const uint16_t* src = P + row * ld + k;
        if (vec && k + 7 < K) {
          x = *reinterpret_cast<const u32x4*>(src);
        } else {
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const uint32_t b = (k + t < K) ? src[t] : 0u;
            x[t >> 1] |= b << (16 * (t & 1));
          }
        }
        if (SCALED) s = scales[(row >> 7) * nsb + (k >> 7)];
      }
      v[q] = x;
      if (SCALED) sc[q] = s;
    }
  }
  __device__ __forceinline__ void store(uint16_t* S) const {
    constexpr int LDK = BK + 8;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int e = threadIdx.x + T * q;
      const int row = e / (BK / 8), kc = 8 * (e % (BK / 8));
      u32x4 x = v[q];
      if (SCALED) {
#pragma unroll
        for (int t = 0; t < 4; ++t) x[t] = scale_bf16x2(x[t], sc[q]);
      }
      *reinterpret_cast<u32x4*>(S + row * LDK + kc) = x;
    }
  }
};

// n-contiguous matrix operand (BK x COLS, scaled) transposed into S[j][k]: a task
// reads rows k, k+1 at 8 consecutive j and writes eight (k, k+1) pairs.  As in
// BFStageKC, scaling happens in store().
template <int COLS, int BK, int T>
struct BFStageNC {
  static constexpr int TASKS = (BK / 2) * (COLS / 8);
  static constexpr int NT = (TASKS + T - 1) / T;
  u32x4 v0[NT], v1[NT];
  float sc[NT];
  __device__ __forceinline__ void load(const uint16_t* __restrict__ P, int64_t ld, int64_t cols,
                                       int64_t K, int64_t j0, int64_t k0,
                                       const float* __restrict__ scales, int64_t nsb, bool vec) {
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      const int task = threadIdx.x + T * q;
      v0[q] = u32x4{0u, 0u, 0u, 0u};
      v1[q] = u32x4{0u, 0u, 0u, 0u};
      sc[q] = 0.f;
      if (task >= TASKS) continue;
      // consecutive lanes take consecutive k-pairs: their (k, k+1) words land in
      // consecutive LDS banks in store() (a j-major order would put all lanes of
      // a wave in one bank, the row stride of 8 columns being a multiple of 128 B)
      const int kp = task % (BK / 2), jc = task / (BK / 2);
      const int64_t k = k0 + 2 * kp, j = j0 + 8 * jc;
      if (j >= cols || k >= K) continue;
      // k is even, so rows k and k+1 share one 128-row scale block
      sc[q] = scales[(k >> 7) * nsb + (j >> 7)];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int64_t kk = k + h;
        if (kk >= K) continue;
        const uint16_t* src = P + kk * ld + j;
        u32x4 x = {0u, 0u, 0u, 0u};
        if (vec && j + 7 < cols) {
          x = *reinterpret_cast<const u32x4*>(src);
        } else {
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const uint32_t b = (j + t < cols) ? src[t] : 0u;
            x[t >> 1] |= b << (16 * (t & 1));
          }
        }
        if (h == 0)
          v0[q] = x;
        else
          v1[q] = x;
      }
    }
  }
  __device__ __forceinline__ void store(uint16_t* S) const {
    constexpr int LDK = BK + 8;
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      const int task = threadIdx.x + T * q;
      if (task >= TASKS) continue;
      const int kp = task % (BK / 2), jc = task / (BK / 2);
      u32x4 a4 = v0[q], b4 = v1[q];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        a4[t] = scale_bf16x2(a4[t], sc[q]);
        b4[t] = scale_bf16x2(b4[t], sc[q]);
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const uint32_t a = (a4[t >> 1] >> (16 * (t & 1))) & 0xffffu;
        const uint32_t b = (b4[t >> 1] >> (16 * (t & 1))) & 0xffffu;
        *reinterpret_cast<uint32_t*>(S + (8 * jc + t) * LDK + 2 * kp) = a | (b << 16);
      }
    }
  }
};

template <class CF, bool A_IS_MAT, bool B_KC>
__device__ void bf16_tile_cfg(const GemmBF16& g, int64_t local, char* smem) {
  constexpr int BM = CF::BM, BN = CF::BN, BK = CF::BK, LDK = CF::LDK;
  uint16_t* sA = reinterpret_cast<uint16_t*>(smem);  // [2][BM * LDK]
  uint16_t* sB = sA + 2 * BM * LDK;                  // [2][BN * LDK]
  const int64_t tm_n = cdiv_d(g.M, BM), tn_n = cdiv_d(g.N, BN);
  int64_t tm, tn;
  if (g.inner_is_m) {
    if (!xcd_tile(local, tm_n, tn_n, tm, tn)) return;
  } else {
    if (!xcd_tile(local, tn_n, tm_n, tn, tm)) return;
  }
  const int64_t i0 = tm * BM, j0 = tn * BN;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % CF::WM, wn = wave / CF::WM;
  const int li = lane & 31, lk = lane >> 5;
  const bool vec = g.vec != 0;
  f32x16 acc[CF::FM][CF::FN];
#pragma unroll
  for (int x = 0; x < CF::FM; ++x)
#pragma unroll
    for (int y = 0; y < CF::FN; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[x][y][v] = 0.f;

  BFStageKC<BM, BK, CF::T, A_IS_MAT> sa;
  typedef typename std::conditional<B_KC, BFStageKC<BN, BK, CF::T, false>,
                                    BFStageNC<BN, BK, CF::T>>::type StageB;
  StageB sb;
  const int64_t nk = cdiv_d(g.K, BK);
  sa.load(g.A, g.lda, g.M, g.K, i0, 0, g.scales, g.nsb, vec);
  sb.load(g.B, g.ldb, g.N, g.K, j0, 0, g.scales, g.nsb, vec);
  sa.store(sA);
  sb.store(sB);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) {
      sa.load(g.A, g.lda, g.M, g.K, i0, (kt + 1) * BK, g.scales, g.nsb, vec);
      sb.load(g.B, g.ldb, g.N, g.K, j0, (kt + 1) * BK, g.scales, g.nsb, vec);
    }
    const uint16_t* a_s = sA + cur * BM * LDK + (wm * CF::TM + li) * LDK + 8 * lk;
    const uint16_t* b_s = sB + cur * BN * LDK + (wn * CF::TN + li) * LDK + 8 * lk;
#pragma unroll
    for (int ks = 0; ks < BK; ks += 16) {
      bf16x8 af[CF::FM], bfr[CF::FN];
#pragma unroll
      for (int x = 0; x < CF::FM; ++x)
        af[x] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(a_s + x * 32 * LDK + ks));
#pragma unroll
      for (int y = 0; y < CF::FN; ++y)
        bfr[y] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(b_s + y * 32 * LDK + ks));
#pragma unroll
      for (int x = 0; x < CF::FM; ++x)
#pragma unroll
        for (int y = 0; y < CF::FN; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[x], bfr[y], acc[x][y], 0, 0, 0);
    }
    if (kt + 1 < nk) {
      sa.store(sA + (cur ^ 1) * BM * LDK);
      sb.store(sB + (cur ^ 1) * BN * LDK);
    }
    __syncthreads();
  }
  // 32x32 accumulator: register v of lane l holds row 8(v/4) + 4(l/32) + v%4, column l%32.
#pragma unroll
  for (int x = 0; x < CF::FM; ++x)
#pragma unroll
    for (int y = 0; y < CF::FN; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = i0 + wm * CF::TM + x * 32 + 8 * (v >> 2) + 4 * lk + (v & 3);
        const int64_t col = j0 + wn * CF::TN + y * 32 + li;
        if (row < g.M && col < g.N) g.D[row * g.ldd + col] = acc[x][y][v];
      }
}

// The production BF16 configuration: 256 x 256 tiles, 16 waves of 64 x 64.
using BF16Pass = BF16Cfg<256, 256, 32, 4, 4>;

}  // namespace tiles
}  // namespace gn
