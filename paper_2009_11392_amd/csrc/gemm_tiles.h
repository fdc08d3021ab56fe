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
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
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

// The same with the tiles of each XCD visited in blocks of bi (inner) x bo
// (outer) tiles: the workgroups resident on one XCD at a time then cover a
// roughly square block of the output and share both operands' panels in its L2
// (the order within the XCD's range: block rows of bo outer tiles, blocks of bi
// inner tiles along them, inner index fastest inside a block; partial blocks at
// the edges).
__device__ __forceinline__ bool xcd_tile_blocked(int64_t local, int64_t tiles_inner,
                                                 int64_t tiles_outer, int64_t bi, int64_t bo,
                                                 int64_t& ti, int64_t& to) {
  const int64_t total = tiles_inner * tiles_outer;
  const int64_t per = (total + 7) / 8;
  const int64_t t = (local & 7) * per + (local >> 3);
  if (t >= total) return false;
  const int64_t row = t / (tiles_inner * bo), rem = t - row * tiles_inner * bo;
  const int64_t h = (tiles_outer - row * bo < bo) ? tiles_outer - row * bo : bo;
  const int64_t ib = rem / (bi * h), rem2 = rem - ib * bi * h;
  const int64_t w = (tiles_inner - ib * bi < bi) ? tiles_inner - ib * bi : bi;
  ti = ib * bi + rem2 % w;
  to = row * bo + rem2 / w;
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
// A(i,k) = PA[i*lda + k] (k-contiguous; the matrix A when A_IS_MAT);
// B(k,j) = PB[j*ldb + k] when B_KC, else PB[k*ldb + j] (the matrix A).
// The matrix operand is stored as bfloat16 values in [-1, 1] with one
// power-of-two scale per 128 x 128 block.  Tiles copy the stored values into LDS
// unchanged; the scale is applied to the accumulators instead: each wave's 64
// output rows (AX) or columns (Y^T A) lie in one scale block, so along K the
// accumulators are kept in units of the current K block's scale and multiplied
// by the ratio of consecutive scales at each 128-deep K block boundary, and by
// the last scale at the end.  Scaling by powers of two is exact, so the result
// equals the product of the scaled values.
// k-contiguous operands live in LDS as S[row][k] (row stride BK + 8), read with
// one 16-byte load per lane per MFMA fragment; the n-contiguous matrix operand
// of Y^T A lives as S[k][j] (row stride BN + 16), copied 16 bytes at a time and
// read with the transposing LDS load (ds_read_b64_tr_b16): in each group of 16
// lanes, lane 4a + b reads the 4 values at row k0 + a, columns c0 + 4b .. + 3,
// and lane i receives column c0 + i at rows k0 .. k0 + 3, which is the layout
// of the MFMA B fragment.
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
  static constexpr int LDN = BN + 16;
  static_assert(TM % 32 == 0 && TN % 32 == 0 && 128 % TM == 0 && 128 % TN == 0 && 128 % BK == 0,
                "a wave's rows and columns must lie in one 128 x 128 scale block");
  static constexpr size_t smem() {
    const size_t kc = 2 * (size_t)(BM + BN) * LDK;
    const size_t nc = 2 * (size_t)BM * LDK + 2 * (size_t)BK * LDN;
    return (kc > nc ? kc : nc) * sizeof(uint16_t);
  }
};

// 16-byte chunks of a row-major operand slab: ROWS rows of WIDTH elements
// starting at (r0, c0) of P, copied into S[row][c] (row stride LDS_).
template <int ROWS, int WIDTH, int T, int LDS_>
struct BFStage {
  static constexpr int NV = ROWS * WIDTH / 8 / T;
  static_assert(NV >= 1 && NV * 8 * T == ROWS * WIDTH, "tile not divisible");
  u32x4 v[NV];
  __device__ __forceinline__ void load(const uint16_t* __restrict__ P, int64_t ld, int64_t rows,
                                       int64_t cols, int64_t r0, int64_t c0, bool vec) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int e = threadIdx.x + T * q;
      const int64_t row = r0 + e / (WIDTH / 8), c = c0 + 8 * (e % (WIDTH / 8));
      u32x4 x = {0u, 0u, 0u, 0u};
      if (row < rows && c < cols) {
        const uint16_t* src = P + row * ld + c;
        if (vec && c + 7 < cols) {
          x = *reinterpret_cast<const u32x4*>(src);
        } else {
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const uint32_t b = (c + t < cols) ? src[t] : 0u;
            x[t >> 1] |= b << (16 * (t & 1));
          }
        }
      }
      v[q] = x;
    }
  }
  __device__ __forceinline__ void store(uint16_t* S) const {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int e = threadIdx.x + T * q;
      const int row = e / (WIDTH / 8), c = 8 * (e % (WIDTH / 8));
      *reinterpret_cast<u32x4*>(S + row * LDS_ + c) = v[q];
    }
  }
};

typedef short bf16x4_bits __attribute__((ext_vector_type(4)));

// Eight k-consecutive bfloat16 values of column `col` for the MFMA B fragment
// from S[k][j] (row stride LDN): two transposing loads of four rows each.
template <int LDN>
__device__ __forceinline__ bf16x8 bf16_frag_tr(const uint16_t* S, int k0, int c0, int lane) {
  const int g = lane >> 4, p = lane & 15, a = p >> 2, b = p & 3;
  const int row = k0 + 8 * (g >> 1) + a, col = c0 + 16 * (g & 1) + 4 * b;
  typedef __attribute__((address_space(3))) bf16x4_bits lds_v4;
  const bf16x4_bits h0 = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4*)(S + row * LDN + col));
  const bf16x4_bits h1 =
      __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4*)(S + (row + 4) * LDN + col));
  typedef short s8 __attribute__((ext_vector_type(8)));
  const s8 v = {h0[0], h0[1], h0[2], h0[3], h1[0], h1[1], h1[2], h1[3]};
  return __builtin_bit_cast(bf16x8, v);
}

// One 32 x 32 x 16 matrix-core step on 16-bit operands held as raw bits: bfloat16
// (F16 = false) or IEEE binary16, FP32 accumulation.
template <bool F16>
__device__ __forceinline__ f32x16 mfma_32x32x16(bf16x8 a, bf16x8 b, f32x16 c) {
  if constexpr (F16)
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                   __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// One BM x BN tile at (i0, j0).
template <class CF, bool A_IS_MAT, bool B_KC, bool F16 = false>
__device__ void bf16_tile_at(const GemmBF16& g, int64_t i0, int64_t j0, char* smem) {
  constexpr int BM = CF::BM, BN = CF::BN, BK = CF::BK, LDK = CF::LDK, LDN = CF::LDN;
  constexpr int SB = B_KC ? BN * LDK : BK * LDN;     // one B buffer
  uint16_t* sA = reinterpret_cast<uint16_t*>(smem);  // [2][BM * LDK]
  uint16_t* sB = sA + 2 * BM * LDK;                  // [2][SB]
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
  // the scale block of this wave's rows (AX) or columns (Y^T A), clamped at the edge
  const int64_t nkb = cdiv_d(g.K, 128);
  const int64_t obl = A_IS_MAT ? (i0 + wm * CF::TM) >> 7 : (j0 + wn * CF::TN) >> 7;
  const int64_t omax = A_IS_MAT ? cdiv_d(g.M, 128) - 1 : g.nsb - 1;
  const int64_t ob = obl < omax ? obl : omax;
  auto scale_of = [&](int64_t kb) -> float {
    return A_IS_MAT ? g.scales[ob * g.nsb + kb] : g.scales[kb * g.nsb + ob];
  };
  int64_t kb_cur = 0;
  float s_cur = scale_of(0);

  BFStage<BM, BK, CF::T, LDK> sa;
  typedef typename std::conditional<B_KC, BFStage<BN, BK, CF::T, LDK>,
                                    BFStage<BK, BN, CF::T, LDN>>::type StageB;
  StageB sb;
  const int64_t nk = cdiv_d(g.K, BK);
  // A: rows i0.., k 0..; B: rows j0.., k 0.. (k-contiguous) or rows k 0.., columns j0..
  sa.load(g.A, g.lda, g.M, g.K, i0, 0, vec);
  if (B_KC)
    sb.load(g.B, g.ldb, g.N, g.K, j0, 0, vec);
  else
    sb.load(g.B, g.ldb, g.K, g.N, 0, j0, vec);
  sa.store(sA);
  sb.store(sB);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) {
      const int64_t kn = (kt + 1) * BK;
      sa.load(g.A, g.lda, g.M, g.K, i0, kn, vec);
      if (B_KC)
        sb.load(g.B, g.ldb, g.N, g.K, j0, kn, vec);
      else
        sb.load(g.B, g.ldb, g.K, g.N, kn, j0, vec);
    }
    {
      const int64_t kb = (kt * BK) >> 7;
      if (kb != kb_cur) {
        const float s_new = scale_of(kb);
        const float ratio = s_cur / s_new;  // a power of two: exact
#pragma unroll
        for (int x = 0; x < CF::FM; ++x)
#pragma unroll
          for (int y = 0; y < CF::FN; ++y) acc[x][y] *= ratio;
        s_cur = s_new;
        kb_cur = kb;
      }
    }
    const uint16_t* a_s = sA + cur * BM * LDK + (wm * CF::TM + li) * LDK + 8 * lk;
    const uint16_t* b_base = sB + cur * SB;
#pragma unroll
    for (int ks = 0; ks < BK; ks += 16) {
      bf16x8 af[CF::FM], bfr[CF::FN];
#pragma unroll
      for (int x = 0; x < CF::FM; ++x)
        af[x] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(a_s + x * 32 * LDK + ks));
#pragma unroll
      for (int y = 0; y < CF::FN; ++y) {
        if (B_KC)
          bfr[y] = __builtin_bit_cast(
              bf16x8, *reinterpret_cast<const u32x4*>(b_base + (wn * CF::TN + y * 32 + li) * LDK +
                                                      8 * lk + ks));
        else
          bfr[y] = bf16_frag_tr<LDN>(b_base, ks, wn * CF::TN + y * 32, lane);
      }
#pragma unroll
      for (int x = 0; x < CF::FM; ++x)
#pragma unroll
        for (int y = 0; y < CF::FN; ++y)
          acc[x][y] = mfma_32x32x16<F16>(af[x], bfr[y], acc[x][y]);
    }
    if (kt + 1 < nk) {
      sa.store(sA + (cur ^ 1) * BM * LDK);
      sb.store(sB + (cur ^ 1) * SB);
    }
    __syncthreads();
  }
  (void)nkb;
  // 32x32 accumulator: register v of lane l holds row 8(v/4) + 4(l/32) + v%4, column l%32.
#pragma unroll
  for (int x = 0; x < CF::FM; ++x)
#pragma unroll
    for (int y = 0; y < CF::FN; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = i0 + wm * CF::TM + x * 32 + 8 * (v >> 2) + 4 * lk + (v & 3);
        const int64_t col = j0 + wn * CF::TN + y * 32 + li;
        if (row < g.M && col < g.N) g.D[row * g.ldd + col] = acc[x][y][v] * s_cur;
      }
}

// The tile of XCD-mapped index `local` (tiles of one XCD walk the inner index).
template <class CF, bool A_IS_MAT, bool B_KC, bool F16 = false>
__device__ void bf16_tile_cfg(const GemmBF16& g, int64_t local, char* smem) {
  const int64_t tm_n = cdiv_d(g.M, CF::BM), tn_n = cdiv_d(g.N, CF::BN);
  int64_t tm, tn;
  if (g.inner_is_m) {
    if (!xcd_tile(local, tm_n, tn_n, tm, tn)) return;
  } else {
    if (!xcd_tile(local, tn_n, tm_n, tn, tm)) return;
  }
  bf16_tile_at<CF, A_IS_MAT, B_KC, F16>(g, tm * CF::BM, tn * CF::BN, smem);
}

// The production BF16 configuration: 256 x 256 tiles, 16 waves of 64 x 64, K
// staged 64 deep (a 32-deep slab leaves too little MFMA work per wave to cover
// the next slab's global loads).
using BF16Pass = BF16Cfg<256, 256, 64, 4, 4>;

}  // namespace tiles
}  // namespace gn
