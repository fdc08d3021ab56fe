// BF16 form of the sketch pass: A stored as bfloat16 with one power-of-two FP32
// scale per 128 x 128 block, X and Y bfloat16, products on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation.  Each block scale is applied
// to A's elements as they are staged into LDS; a power of two only moves the
// exponent, so scale * stored value is formed exactly.
#include "gn_internal.h"

namespace gn {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int B_BM = 128, B_BN = 128, B_BK = 32, B_LD = B_BK + 8;  // LDS row: 40 bf16 = 80 B

__device__ __forceinline__ bool xcd_tile_b(int64_t tiles_inner, int64_t tiles_outer, int64_t& ti,
                                           int64_t& to) {
  const int64_t total = tiles_inner * tiles_outer;
  const int64_t per = (total + 7) / 8;
  const int64_t wg = blockIdx.x;
  const int64_t t = (wg & 7) * per + (wg >> 3);
  if (t >= total) return false;
  ti = t % tiles_inner;
  to = t / tiles_inner;
  return true;
}

// Multiply two packed bfloat16 values by a power of two (exact).
__device__ __forceinline__ uint32_t scale_bf16x2(uint32_t w, float s) {
  const float lo = __uint_as_float(w << 16) * s;
  const float hi = __uint_as_float(w & 0xffff0000u) * s;
  return (__float_as_uint(lo) >> 16) | (__float_as_uint(hi) & 0xffff0000u);
}

// Stage a k-contiguous operand tile (128 rows x 32 k) into S[row][k].
// SCALED: the operand is A itself, row r / col k take scales[(r>>7)*nsb + (k>>7)].
template <bool SCALED>
__device__ __forceinline__ void load_kc(const uint16_t* __restrict__ P, int64_t ld, int64_t rows,
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

__device__ __forceinline__ void store_kc(uint16_t* S, const u32x4 (&reg)[2]) {
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = threadIdx.x + 256 * q;
    const int row = e >> 2, kc = 8 * (e & 3);
    *reinterpret_cast<u32x4*>(S + row * B_LD + kc) = reg[q];
  }
}

// Stage the n-contiguous operand A (B(k, j) = A[k*ld + j], 32 k x 128 j) into
// S[j][k]: each thread reads rows k, k+1 at 8 consecutive j and writes eight
// (k, k+1) pairs.
__device__ __forceinline__ void load_nc(const uint16_t* __restrict__ P, int64_t ld, int64_t cols,
                                        int64_t K, int64_t j0, int64_t k0,
                                        const float* __restrict__ scales, int64_t nsb, bool vec,
                                        u32x4 (&r0)[1], u32x4 (&r1)[1]) {
  const int kp = threadIdx.x >> 4, jc = threadIdx.x & 15;
  const int64_t k = k0 + 2 * kp, j = j0 + 8 * jc;
  u32x4 v0 = {0u, 0u, 0u, 0u}, v1 = {0u, 0u, 0u, 0u};
  if (j < cols) {
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
        v0 = v;
      else
        v1 = v;
    }
  }
  r0[0] = v0;
  r1[0] = v1;
}

__device__ __forceinline__ void store_nc(uint16_t* S, const u32x4 (&r0)[1], const u32x4 (&r1)[1]) {
  const int kp = threadIdx.x >> 4, jc = threadIdx.x & 15;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const uint32_t a = (r0[0][t >> 1] >> (16 * (t & 1))) & 0xffffu;
    const uint32_t b = (r1[0][t >> 1] >> (16 * (t & 1))) & 0xffffu;
    *reinterpret_cast<uint32_t*>(S + (8 * jc + t) * B_LD + 2 * kp) = a | (b << 16);
  }
}

__device__ __forceinline__ bf16x8 frag(const uint16_t* S, int row, int k) {
  const u32x4 w = *reinterpret_cast<const u32x4*>(S + row * B_LD + k);
  return __builtin_bit_cast(bf16x8, w);
}

// D (M x N) = A (M x K) * B (K x N) with
//   A(i, k) = PA[i*lda + k]                       (k-contiguous, scaled if A_IS_MAT)
//   B(k, j) = PB[j*ldb + k]  if B_KC (k-contiguous), else PB[k*ldb + j] (the matrix A)
template <bool A_IS_MAT, bool B_KC>
__global__ void __launch_bounds__(256) gemm_bf16_mfma(int64_t M, int64_t N, int64_t K,
                                                      const uint16_t* __restrict__ PA, int64_t lda,
                                                      const uint16_t* __restrict__ PB, int64_t ldb,
                                                      const float* __restrict__ scales, int64_t nsb,
                                                      float* __restrict__ D, int64_t ldd,
                                                      bool inner_is_m, bool vec) {
  __shared__ __attribute__((aligned(16))) uint16_t sA[2][B_BM * B_LD];
  __shared__ __attribute__((aligned(16))) uint16_t sB[2][B_BN * B_LD];
  const int64_t tm_n = (M + B_BM - 1) / B_BM, tn_n = (N + B_BN - 1) / B_BN;
  int64_t tm, tn;
  if (inner_is_m) {
    if (!xcd_tile_b(tm_n, tn_n, tm, tn)) return;
  } else {
    if (!xcd_tile_b(tn_n, tm_n, tn, tm)) return;
  }
  const int64_t i0 = tm * B_BM, j0 = tn * B_BN;
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

  const int64_t nk = (K + B_BK - 1) / B_BK;
  u32x4 ra[2], rb[2], rn0[1], rn1[1];
  load_kc<A_IS_MAT>(PA, lda, M, K, i0, 0, scales, nsb, vec, ra);
  if (B_KC)
    load_kc<false>(PB, ldb, N, K, j0, 0, scales, nsb, vec, rb);
  else
    load_nc(PB, ldb, N, K, j0, 0, scales, nsb, vec, rn0, rn1);
  store_kc(sA[0], ra);
  if (B_KC)
    store_kc(sB[0], rb);
  else
    store_nc(sB[0], rn0, rn1);
  __syncthreads();

  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) {
      load_kc<A_IS_MAT>(PA, lda, M, K, i0, (kt + 1) * B_BK, scales, nsb, vec, ra);
      if (B_KC)
        load_kc<false>(PB, ldb, N, K, j0, (kt + 1) * B_BK, scales, nsb, vec, rb);
      else
        load_nc(PB, ldb, N, K, j0, (kt + 1) * B_BK, scales, nsb, vec, rn0, rn1);
    }
    const uint16_t* a_s = sA[cur];
    const uint16_t* b_s = sB[cur];
#pragma unroll
    for (int ks = 0; ks < B_BK; ks += 16) {
      const bf16x8 a0 = frag(a_s, wm * 64 + li, ks + 8 * lk);
      const bf16x8 a1 = frag(a_s, wm * 64 + 32 + li, ks + 8 * lk);
      const bf16x8 b0 = frag(b_s, wn * 64 + li, ks + 8 * lk);
      const bf16x8 b1 = frag(b_s, wn * 64 + 32 + li, ks + 8 * lk);
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc[1][1], 0, 0, 0);
    }
    if (kt + 1 < nk) {
      store_kc(sA[cur ^ 1], ra);
      if (B_KC)
        store_kc(sB[cur ^ 1], rb);
      else
        store_nc(sB[cur ^ 1], rn0, rn1);
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
        if (row < M && col < N) D[row * ldd + col] = acc[x][y][v];
      }
}

}  // namespace

gn_status launch_pass_ax_bf16(int64_t m, int64_t n, int64_t r, const uint16_t* A, int64_t lda,
                              const float* scales, const uint16_t* Xt, int64_t ldxt, float* AX,
                              int64_t ldax, hipStream_t s) {
  const int64_t nsb = cdiv(n, 128);
  const int64_t tiles = cdiv(m, B_BM) * cdiv(r, B_BN);
  const bool vec = (lda % 8 == 0) && (ldxt % 8 == 0) && ((uintptr_t)A % 16 == 0) &&
                   ((uintptr_t)Xt % 16 == 0);
  gemm_bf16_mfma<true, true><<<dim3((unsigned)(8 * cdiv(tiles, 8))), dim3(256), 0, s>>>(
      m, r, n, A, lda, Xt, ldxt, scales, nsb, AX, ldax, /*inner_is_m=*/false, vec);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

gn_status launch_pass_yta_bf16(int64_t m, int64_t n, int64_t rl, const uint16_t* A, int64_t lda,
                               const float* scales, const uint16_t* Yt, int64_t ldyt, float* YtA,
                               int64_t ldya, hipStream_t s) {
  const int64_t nsb = cdiv(n, 128);
  const int64_t tiles = cdiv(rl, B_BM) * cdiv(n, B_BN);
  const bool vec = (lda % 8 == 0) && (ldyt % 8 == 0) && ((uintptr_t)A % 16 == 0) &&
                   ((uintptr_t)Yt % 16 == 0);
  gemm_bf16_mfma<false, false><<<dim3((unsigned)(8 * cdiv(tiles, 8))), dim3(256), 0, s>>>(
      rl, n, m, Yt, ldyt, A, lda, scales, nsb, YtA, ldya, /*inner_is_m=*/true, vec);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

}  // namespace gn
