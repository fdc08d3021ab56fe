// Matrix-core tile bodies for the sketch pass (device functions; each fused
// pass kernel calls one of them per workgroup).
//
// FP32: v_mfma_f32_32x32x2_f32.  BF16: v_mfma_f32_32x32x16_bf16.  Both: 256
// threads = 4 waves in 2 x 2, workgroup tile 128 x 128, wave tile 64 x 64 = 2 x 2
// MFMA blocks, K staged through LDS double buffered, FP32 accumulation.  The
// 32 x 32 accumulator of lane l holds, in register v, row 8(v/4) + 4(l/32) + v%4
// and column l%32 of its block.
#pragma once

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

inline int64_t gemm_groups(int64_t M, int64_t N) {  // groups of 8 workgroups
  return cdiv(cdiv(M, 128) * cdiv(N, 128), 8);
}

constexpr int T_BM = 128, T_BN = 128;

// ------------------------------------------------------------------ FP32
// D (M x N) = A (M x K) B (K x N).  A_KC: A(i,k) = A[i*lda + k], else A[k*lda + i].
// B_KC: B(k,j) = B[j*ldb + k], else B[k*ldb + j].  LDS holds both operands k-major.
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

constexpr int F_BK = 16, F_LD = T_BM + 4;
constexpr size_t F_SMEM = 2 * 2 * F_BK * F_LD * sizeof(float);

template <bool KC, bool VEC>
__device__ __forceinline__ void f32_load(const float* __restrict__ P, int64_t ld, int64_t rows,
                                         int64_t K, int64_t r0, int64_t k0, f32x4 (&reg)[2]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = tid + 256 * q;
    int64_t row, k;
    if (KC) {
      row = r0 + (e >> 2);
      k = k0 + 4 * (e & 3);
    } else {
      k = k0 + (e >> 5);
      row = r0 + 4 * (e & 31);
    }
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
    if (KC) {
      if (row < rows) {
        const float* src = P + row * ld + k;
        if (VEC && k + 3 < K) {
          v = *reinterpret_cast<const f32x4*>(src);
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (k + t < K) v[t] = src[t];
        }
      }
    } else {
      if (k < K) {
        const float* src = P + k * ld + row;
        if (VEC && row + 3 < rows) {
          v = *reinterpret_cast<const f32x4*>(src);
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (row + t < rows) v[t] = src[t];
        }
      }
    }
    reg[q] = v;
  }
}

template <bool KC>
__device__ __forceinline__ void f32_store(float* S, const f32x4 (&reg)[2]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = tid + 256 * q;
    if (KC) {
      const int row = e >> 2, k = 4 * (e & 3);
#pragma unroll
      for (int t = 0; t < 4; ++t) S[(k + t) * F_LD + row] = reg[q][t];
    } else {
      const int k = e >> 5, row = 4 * (e & 31);
      *reinterpret_cast<f32x4*>(S + k * F_LD + row) = reg[q];
    }
  }
}

template <bool A_KC, bool B_KC, bool VEC>
__device__ void f32_tile(const GemmF32& g, int64_t local, char* smem) {
  float* sA = reinterpret_cast<float*>(smem);           // [2][F_BK * F_LD]
  float* sB = sA + 2 * F_BK * F_LD;                       // [2][F_BK * F_LD]
  const int64_t tm_n = cdiv_d(g.M, T_BM), tn_n = cdiv_d(g.N, T_BN);
  int64_t tm, tn;
  if (g.inner_is_m) {
    if (!xcd_tile(local, tm_n, tn_n, tm, tn)) return;
  } else {
    if (!xcd_tile(local, tn_n, tm_n, tn, tm)) return;
  }
  const int64_t i0 = tm * T_BM, j0 = tn * T_BN;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int li = lane & 31, lk = lane >> 5;
  f32x16 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[x][y][v] = 0.f;

  const int64_t nk = cdiv_d(g.K, F_BK);
  f32x4 ra[2], rb[2];
  f32_load<A_KC, VEC>(g.A, g.lda, g.M, g.K, i0, 0, ra);
  f32_load<B_KC, VEC>(g.B, g.ldb, g.N, g.K, j0, 0, rb);
  f32_store<A_KC>(sA, ra);
  f32_store<B_KC>(sB, rb);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) {
      f32_load<A_KC, VEC>(g.A, g.lda, g.M, g.K, i0, (kt + 1) * F_BK, ra);
      f32_load<B_KC, VEC>(g.B, g.ldb, g.N, g.K, j0, (kt + 1) * F_BK, rb);
    }
    const float* a_s = sA + cur * F_BK * F_LD;
    const float* b_s = sB + cur * F_BK * F_LD;
#pragma unroll
    for (int kk = 0; kk < F_BK; kk += 2) {
      const float a0 = a_s[(kk + lk) * F_LD + wm * 64 + li];
      const float a1 = a_s[(kk + lk) * F_LD + wm * 64 + 32 + li];
      const float b0 = b_s[(kk + lk) * F_LD + wn * 64 + li];
      const float b1 = b_s[(kk + lk) * F_LD + wn * 64 + 32 + li];
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
    }
    if (kt + 1 < nk) {
      f32_store<A_KC>(sA + (cur ^ 1) * F_BK * F_LD, ra);
      f32_store<B_KC>(sB + (cur ^ 1) * F_BK * F_LD, rb);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = i0 + wm * 64 + x * 32 + 8 * (v >> 2) + 4 * lk + (v & 3);
        const int64_t col = j0 + wn * 64 + y * 32 + li;
        if (row < g.M && col < g.N) g.D[row * g.ldd + col] = acc[x][y][v];
      }
}

// ------------------------------------------------------------------ BF16 with block scales
// A(i,k) = PA[i*lda + k] (k-contiguous; the matrix A when A_IS_MAT, then scaled);
// B(k,j) = PB[j*ldb + k] when B_KC, else PB[k*ldb + j] (the matrix A, scaled).
// LDS holds both operands k-contiguous, S[row][k], 40 bf16 per row.
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

constexpr int B_BK = 32, B_LD = B_BK + 8;
constexpr size_t B_SMEM = 2 * 2 * T_BM * B_LD * sizeof(uint16_t);

// Multiply two packed bfloat16 values by a power of two (exact).
__device__ __forceinline__ uint32_t scale_bf16x2(uint32_t w, float s) {
  const float lo = __uint_as_float(w << 16) * s;
  const float hi = __uint_as_float(w & 0xffff0000u) * s;
  return (__float_as_uint(lo) >> 16) | (__float_as_uint(hi) & 0xffff0000u);
}

template <bool SCALED>
__device__ __forceinline__ void bf_load_kc(const uint16_t* __restrict__ P, int64_t ld, int64_t rows,
                                           int64_t K, int64_t r0, int64_t k0,
                                           const float* __restrict__ scales, int64_t nsb, bool vec,
                                           u32x4 (&reg)[2]) {
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = threadIdx.x + 256 * q;
    const int64_t row = r0 + (e >> 2), k = k0 + 8 * (e & 3);
    u32x4 v = {0u, 0u, 0u, 0u};
    if (row < rows && k < K) {
      const uint16_t* src = P + row * ld + k;
      if (vec && k + 7 < K) {
        v = *reinterpret_cast<const u32x4*>(src);
      } else {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const uint32_t b = (k + t < K) ? src[t] : 0u;
          v[t >> 1] |= b << (16 * (t & 1));
        }
      }
      if (SCALED) {
        const float s = scales[(row >> 7) * nsb + (k >> 7)];
#pragma unroll
        for (int t = 0; t < 4; ++t) v[t] = scale_bf16x2(v[t], s);
      }
    }
    reg[q] = v;
  }
}

__device__ __forceinline__ void bf_store_kc(uint16_t* S, const u32x4 (&reg)[2]) {
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = threadIdx.x + 256 * q;
    const int row = e >> 2, kc = 8 * (e & 3);
    *reinterpret_cast<u32x4*>(S + row * B_LD + kc) = reg[q];
  }
}

// n-contiguous matrix operand: rows k, k+1 at 8 consecutive j per thread.
__device__ __forceinline__ void bf_load_nc(const uint16_t* __restrict__ P, int64_t ld, int64_t cols,
                                           int64_t K, int64_t j0, int64_t k0,
                                           const float* __restrict__ scales, int64_t nsb, bool vec,
                                           u32x4& r0, u32x4& r1) {
  const int kp = threadIdx.x >> 4, jc = threadIdx.x & 15;
  const int64_t k = k0 + 2 * kp, j = j0 + 8 * jc;
  r0 = u32x4{0u, 0u, 0u, 0u};
  r1 = u32x4{0u, 0u, 0u, 0u};
  if (j >= cols) return;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t kk = k + h;
    if (kk >= K) continue;
    const uint16_t* src = P + kk * ld + j;
    u32x4 v = {0u, 0u, 0u, 0u};
    if (vec && j + 7 < cols) {
      v = *reinterpret_cast<const u32x4*>(src);
    } else {
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const uint32_t b = (j + t < cols) ? src[t] : 0u;
        v[t >> 1] |= b << (16 * (t & 1));
      }
    }
    const float s = scales[(kk >> 7) * nsb + (j >> 7)];
#pragma unroll
    for (int t = 0; t < 4; ++t) v[t] = scale_bf16x2(v[t], s);
    if (h == 0)
      r0 = v;
    else
      r1 = v;
  }
}

__device__ __forceinline__ void bf_store_nc(uint16_t* S, const u32x4& r0, const u32x4& r1) {
  const int kp = threadIdx.x >> 4, jc = threadIdx.x & 15;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const uint32_t a = (r0[t >> 1] >> (16 * (t & 1))) & 0xffffu;
    const uint32_t b = (r1[t >> 1] >> (16 * (t & 1))) & 0xffffu;
    *reinterpret_cast<uint32_t*>(S + (8 * jc + t) * B_LD + 2 * kp) = a | (b << 16);
  }
}

__device__ __forceinline__ bf16x8 bf_frag(const uint16_t* S, int row, int k) {
  const u32x4 w = *reinterpret_cast<const u32x4*>(S + row * B_LD + k);
  return __builtin_bit_cast(bf16x8, w);
}

template <bool A_IS_MAT, bool B_KC>
__device__ void bf16_tile(const GemmBF16& g, int64_t local, char* smem) {
  uint16_t* sA = reinterpret_cast<uint16_t*>(smem);  // [2][T_BM * B_LD]
  uint16_t* sB = sA + 2 * T_BM * B_LD;                // [2][T_BN * B_LD]
  const int64_t tm_n = cdiv_d(g.M, T_BM), tn_n = cdiv_d(g.N, T_BN);
  int64_t tm, tn;
  if (g.inner_is_m) {
    if (!xcd_tile(local, tm_n, tn_n, tm, tn)) return;
  } else {
    if (!xcd_tile(local, tn_n, tm_n, tn, tm)) return;
  }
  const int64_t i0 = tm * T_BM, j0 = tn * T_BN;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int li = lane & 31, lk = lane >> 5;
  const bool vec = g.vec != 0;
  f32x16 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[x][y][v] = 0.f;

  const int64_t nk = cdiv_d(g.K, B_BK);
  u32x4 ra[2], rb[2], rn0, rn1;
  bf_load_kc<A_IS_MAT>(g.A, g.lda, g.M, g.K, i0, 0, g.scales, g.nsb, vec, ra);
  if (B_KC)
    bf_load_kc<false>(g.B, g.ldb, g.N, g.K, j0, 0, g.scales, g.nsb, vec, rb);
  else
    bf_load_nc(g.B, g.ldb, g.N, g.K, j0, 0, g.scales, g.nsb, vec, rn0, rn1);
  bf_store_kc(sA, ra);
  if (B_KC)
    bf_store_kc(sB, rb);
  else
    bf_store_nc(sB, rn0, rn1);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) {
      bf_load_kc<A_IS_MAT>(g.A, g.lda, g.M, g.K, i0, (kt + 1) * B_BK, g.scales, g.nsb, vec, ra);
      if (B_KC)
        bf_load_kc<false>(g.B, g.ldb, g.N, g.K, j0, (kt + 1) * B_BK, g.scales, g.nsb, vec, rb);
      else
        bf_load_nc(g.B, g.ldb, g.N, g.K, j0, (kt + 1) * B_BK, g.scales, g.nsb, vec, rn0, rn1);
    }
    const uint16_t* a_s = sA + cur * T_BM * B_LD;
    const uint16_t* b_s = sB + cur * T_BN * B_LD;
#pragma unroll
    for (int ks = 0; ks < B_BK; ks += 16) {
      const bf16x8 a0 = bf_frag(a_s, wm * 64 + li, ks + 8 * lk);
      const bf16x8 a1 = bf_frag(a_s, wm * 64 + 32 + li, ks + 8 * lk);
      const bf16x8 b0 = bf_frag(b_s, wn * 64 + li, ks + 8 * lk);
      const bf16x8 b1 = bf_frag(b_s, wn * 64 + 32 + li, ks + 8 * lk);
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc[1][1], 0, 0, 0);
    }
    if (kt + 1 < nk) {
      bf_store_kc(sA + (cur ^ 1) * T_BM * B_LD, ra);
      if (B_KC)
        bf_store_kc(sB + (cur ^ 1) * T_BN * B_LD, rb);
      else
        bf_store_nc(sB + (cur ^ 1) * T_BN * B_LD, rn0, rn1);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = i0 + wm * 64 + x * 32 + 8 * (v >> 2) + 4 * lk + (v & 3);
        const int64_t col = j0 + wn * 64 + y * 32 + li;
        if (row < g.M && col < g.N) g.D[row * g.ldd + col] = acc[x][y][v];
      }
}

}  // namespace tiles
}  // namespace gn
