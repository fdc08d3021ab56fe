// The sketch pass of GN (Algorithm 2.1, step 2): AX and Y^T A.
//
// * Gaussian sketches: the two products are dense contractions and run on the
//   matrix cores.  FP32 mode uses v_mfma_f32_32x32x2_f32 with FP32 accumulation;
//   BF16 mode uses v_mfma_f32_32x32x16_bf16 on bfloat16 operands with FP32
//   accumulation, the per-128x128-block power-of-two scales of A folded into
//   the staged tile exactly.  FP64 mode uses the FP64 strided GEMM (dgemm.hip).
// * SRHT X: AX = A D H S is a sign flip, a Walsh-Hadamard transform of every row
//   and a column sample (Section 1); it is computed per 512-column chunk with an
//   in-register / cross-lane FWHT and a signed gather of the sampled columns,
//   using H_{n'} = H_{n'/512} (x) H_512 (Sylvester ordering).
#include "gn_internal.h"

namespace gn {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Map a linear workgroup id to a tile so that the 8 XCDs (workgroups are
// dispatched round-robin over them) each own a contiguous range of tiles, and
// consecutive tiles on one XCD share the panel named by the outer index.
__device__ __forceinline__ bool xcd_tile(int64_t tiles_inner, int64_t tiles_outer, int64_t& ti,
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

// =============================================================================== FP32 MFMA GEMM
// D (M x N) = A (M x K) * B (K x N), FP32 in, FP32 accumulation.
//   A_KC: A(i,k) = A[i*lda + k]  (else A[k*lda + i])
//   B_KC: B(k,j) = B[j*ldb + k]  (else B[k*ldb + j])
// 256 threads = 4 waves in 2 x 2; workgroup tile 128 x 128; wave tile 64 x 64 =
// 2 x 2 blocks of v_mfma_f32_32x32x2_f32; K staged through LDS 16 at a time,
// double buffered.  LDS holds both operands k-major: S[k][row].
constexpr int F_BM = 128, F_BN = 128, F_BK = 16, F_LD = F_BM + 4;

template <bool KC, bool VEC>
__device__ __forceinline__ void f32_load_tile(const float* __restrict__ P, int64_t ld, int64_t rows,
                                              int64_t K, int64_t r0, int64_t k0, f32x4 (&reg)[2]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = tid + 256 * q;
    int64_t row, k;
    if (KC) {  // 128 rows x 16 k: four float4 per row
      row = r0 + (e >> 2);
      k = k0 + 4 * (e & 3);
    } else {   // 16 k x 128 rows: 32 float4 per k
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
__device__ __forceinline__ void f32_store_tile(float* S, const f32x4 (&reg)[2]) {
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
__global__ void __launch_bounds__(256) gemm_f32_mfma(int64_t M, int64_t N, int64_t K,
                                                     const float* __restrict__ A, int64_t lda,
                                                     const float* __restrict__ B, int64_t ldb,
                                                     float* __restrict__ D, int64_t ldd,
                                                     bool inner_is_m) {
  __shared__ __attribute__((aligned(16))) float sA[2][F_BK * F_LD];
  __shared__ __attribute__((aligned(16))) float sB[2][F_BK * F_LD];
  const int64_t tm_n = (M + F_BM - 1) / F_BM, tn_n = (N + F_BN - 1) / F_BN;
  int64_t tm, tn;
  if (inner_is_m) {
    if (!xcd_tile(tm_n, tn_n, tm, tn)) return;
  } else {
    if (!xcd_tile(tn_n, tm_n, tn, tm)) return;
  }
  const int64_t i0 = tm * F_BM, j0 = tn * F_BN;
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

  const int64_t nk = (K + F_BK - 1) / F_BK;
  f32x4 ra[2], rb[2];
  f32_load_tile<A_KC, VEC>(A, lda, M, K, i0, 0, ra);
  f32_load_tile<B_KC, VEC>(B, ldb, N, K, j0, 0, rb);
  f32_store_tile<A_KC>(sA[0], ra);
  f32_store_tile<B_KC>(sB[0], rb);
  __syncthreads();

  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) {
      f32_load_tile<A_KC, VEC>(A, lda, M, K, i0, (kt + 1) * F_BK, ra);
      f32_load_tile<B_KC, VEC>(B, ldb, N, K, j0, (kt + 1) * F_BK, rb);
    }
    const float* a_s = sA[cur];
    const float* b_s = sB[cur];
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
      f32_store_tile<A_KC>(sA[cur ^ 1], ra);
      f32_store_tile<B_KC>(sB[cur ^ 1], rb);
    }
    __syncthreads();
  }

  // 32x32 accumulator layout: register v of lane l holds row 8*(v/4) + 4*(l/32) + v%4,
  // column l%32 of the block.
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

template <bool A_KC, bool B_KC>
gn_status run_gemm_f32(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                       const float* B, int64_t ldb, float* D, int64_t ldd, bool inner_is_m,
                       hipStream_t s) {
  const int64_t tiles = cdiv(M, F_BM) * cdiv(N, F_BN);
  const int64_t grid = 8 * cdiv(tiles, 8);
  const bool vec = (lda % 4 == 0) && (ldb % 4 == 0) && ((uintptr_t)A % 16 == 0) &&
                   ((uintptr_t)B % 16 == 0);
  if (vec)
    gemm_f32_mfma<A_KC, B_KC, true>
        <<<dim3((unsigned)grid), dim3(256), 0, s>>>(M, N, K, A, lda, B, ldb, D, ldd, inner_is_m);
  else
    gemm_f32_mfma<A_KC, B_KC, false>
        <<<dim3((unsigned)grid), dim3(256), 0, s>>>(M, N, K, A, lda, B, ldb, D, ldd, inner_is_m);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

// =============================================================================== SRHT: FWHT + sample
// One wave per row of A at a time; each lane holds 8 consecutive entries of a
// 512-column chunk.  Transform stages 1, 2, 4 run inside a lane, 8 .. 256 across
// lanes (xor shuffles).  The transformed chunk goes to a per-wave LDS slot, from
// which each lane gathers the sampled columns it owns (c = lane + 64 t) and adds
// them with the sign (-1)^popcount(chunk & (s >> 9)) of the outer Hadamard factor.
constexpr int SR_CHUNK = 512;

template <typename T>
__device__ __forceinline__ T flip_if(T v, uint32_t neg) {
  return neg ? -v : v;
}

template <int MODE>
__device__ __forceinline__ void srht_load8(const void* A, int64_t lda, const float* scales,
                                           int64_t nsb, int64_t i, int64_t j, int64_t n,
                                           float (&x)[8]) {
  if constexpr (MODE == GN_MODE_F32) {
    const float* row = reinterpret_cast<const float*>(A) + i * lda;
    if (j + 7 < n && (lda % 4 == 0)) {
      const f32x4 v0 = *reinterpret_cast<const f32x4*>(row + j);
      const f32x4 v1 = *reinterpret_cast<const f32x4*>(row + j + 4);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        x[e] = v0[e];
        x[4 + e] = v1[e];
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = (j + e < n) ? row[j + e] : 0.f;
    }
  } else {  // BF16 with block scales
    const uint16_t* row = reinterpret_cast<const uint16_t*>(A) + i * lda;
    // j is a multiple of 8, so the 8 entries share one 128-column block; read its
    // scale only when the block exists (j < n).
    const float sc = (j < n) ? scales[(i >> 7) * nsb + (j >> 7)] : 0.f;
    if (j + 7 < n && (lda % 8 == 0)) {
      const u32x4 v = *reinterpret_cast<const u32x4*>(row + j);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        x[2 * e] = __uint_as_float(v[e] << 16) * sc;
        x[2 * e + 1] = __uint_as_float(v[e] & 0xffff0000u) * sc;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = (j + e < n) ? bf16_bits_to_f32(row[j + e]) * sc : 0.f;
    }
  }
}

template <typename T, int MODE, int RPL>
__global__ void __launch_bounds__(256) srht_pass(int64_t m, int64_t n, int64_t r,
                                                 const void* __restrict__ A, int64_t lda,
                                                 const float* __restrict__ scales,
                                                 const int8_t* __restrict__ signs,
                                                 const int32_t* __restrict__ idx,
                                                 T* __restrict__ AX, int64_t ldax,
                                                 int64_t rows_per_wg) {
  __shared__ T slot[4][SR_CHUNK];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nsb = (n + 127) >> 7;
  // sampled columns owned by this lane
  int32_t s_lo[RPL], s_hi[RPL];
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int64_t c = lane + 64 * t;
    const int32_t sv = (c < r) ? idx[c] : 0;
    s_lo[t] = sv & (SR_CHUNK - 1);
    s_hi[t] = sv >> 9;
  }
  const int64_t row_begin = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t row_end = (row_begin + rows_per_wg < m) ? row_begin + rows_per_wg : m;
  for (int64_t ib = row_begin; ib < row_end; ib += 4) {
    const int64_t i = ib + wave;
    const bool active = i < row_end;
    T acc[RPL];
#pragma unroll
    for (int t = 0; t < RPL; ++t) acc[t] = (T)0;
    for (int64_t j0 = 0; j0 < n; j0 += SR_CHUNK) {
      const int64_t j = j0 + 8 * lane;
      T x[8];
      if (active) {
        if constexpr (MODE == GN_MODE_F64) {
          const double* row = reinterpret_cast<const double*>(A) + i * lda;
#pragma unroll
          for (int e = 0; e < 8; ++e) x[e] = (j + e < n) ? row[j + e] : 0.0;
        } else {
          float xf[8];
          srht_load8<MODE>(A, lda, scales, nsb, i, j, n, xf);
#pragma unroll
          for (int e = 0; e < 8; ++e) x[e] = xf[e];
        }
        // D: Rademacher sign flip (entries beyond n are zero already)
        uint64_t sg = 0;
        if (j + 7 < n) {
          sg = *reinterpret_cast<const uint64_t*>(signs + j);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e)
            if (j + e < n) sg |= (uint64_t)(uint8_t)signs[j + e] << (8 * e);
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = flip_if(x[e], (uint32_t)((sg >> (8 * e + 7)) & 1u));
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = (T)0;
      }
      // H_512, in-lane stages (h = 1, 2, 4)
#pragma unroll
      for (int h = 1; h < 8; h <<= 1)
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if ((e & h) == 0) {
            const T a = x[e], b = x[e | h];
            x[e] = a + b;
            x[e | h] = a - b;
          }
      // cross-lane stages (h = 8 .. 256  <->  lane xor 1 .. 32)
#pragma unroll
      for (int lm = 1; lm < 64; lm <<= 1) {
        const bool upper = (lane & lm) != 0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const T y = __shfl_xor(x[e], lm, 64);
          x[e] = upper ? (y - x[e]) : (x[e] + y);
        }
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) slot[wave][8 * lane + e] = x[e];
      __syncthreads();
      const uint32_t chunk = (uint32_t)(j0 >> 9);
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const T v = slot[wave][s_lo[t]];
        acc[t] += flip_if(v, (uint32_t)(__popc(chunk & (uint32_t)s_hi[t]) & 1));
      }
      __syncthreads();
    }
    if (active) {
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int64_t c = lane + 64 * t;
        if (c < r) AX[i * ldax + c] = acc[t];
      }
    }
  }
}

template <typename T, int MODE>
gn_status run_srht(int64_t m, int64_t n, int64_t r, const void* A, int64_t lda,
                   const float* scales, const int8_t* signs, const int32_t* idx, T* AX,
                   int64_t ldax, hipStream_t s) {
  const int64_t rows_per_wg = 4;
  const dim3 grid((unsigned)cdiv(m, rows_per_wg)), block(256);
  const int rpl = (int)cdiv(r, 64);
#define GN_SRHT(R)                                                                   \
  srht_pass<T, MODE, R><<<grid, block, 0, s>>>(m, n, r, A, lda, scales, signs, idx, AX, \
                                               ldax, rows_per_wg)
  if (rpl <= 1)
    GN_SRHT(1);
  else if (rpl <= 2)
    GN_SRHT(2);
  else if (rpl <= 4)
    GN_SRHT(4);
  else if (rpl <= 8)
    GN_SRHT(8);
  else if (rpl <= 16)
    GN_SRHT(16);
  else if (rpl <= 32)
    GN_SRHT(32);
  else
    return GN_ERR_UNSUPPORTED;
#undef GN_SRHT
  GN_LAUNCH_CHECK();
  return GN_OK;
}

}  // namespace

// BF16 contraction lives in pass_bf16.hip.
gn_status launch_pass_ax_bf16(int64_t m, int64_t n, int64_t r, const uint16_t* A, int64_t lda,
                              const float* scales, const uint16_t* Xt, int64_t ldxt, float* AX,
                              int64_t ldax, hipStream_t s);
gn_status launch_pass_yta_bf16(int64_t m, int64_t n, int64_t rl, const uint16_t* A, int64_t lda,
                               const float* scales, const uint16_t* Yt, int64_t ldyt, float* YtA,
                               int64_t ldya, hipStream_t s);

gn_status launch_pass_ax(int32_t mode, int64_t m, int64_t n, int64_t r, const void* A, int64_t lda,
                         const float* scales, const void* Xt, int64_t ldxt, void* AX, int64_t ldax,
                         hipStream_t s) {
  if (mode == GN_MODE_F64) {
    MatRef a{A, GN_DT_F64, lda, 1};
    MatRef b{Xt, GN_DT_F64, 1, ldxt};  // B(k, j) = Xt[j*ldxt + k]
    return launch_dgemm(m, r, n, 1.0, a, b, 0.0, (double*)AX, ldax, 1, nullptr, false, s);
  }
  if (mode == GN_MODE_F32)
    return run_gemm_f32<true, true>(m, r, n, (const float*)A, lda, (const float*)Xt, ldxt,
                                    (float*)AX, ldax, /*inner_is_m=*/false, s);
  return launch_pass_ax_bf16(m, n, r, (const uint16_t*)A, lda, scales, (const uint16_t*)Xt, ldxt,
                             (float*)AX, ldax, s);
}

gn_status launch_pass_yta(int32_t mode, int64_t m, int64_t n, int64_t rl, const void* A,
                          int64_t lda, const float* scales, const void* Yt, int64_t ldyt, void* YtA,
                          int64_t ldya, hipStream_t s) {
  if (mode == GN_MODE_F64) {
    MatRef a{Yt, GN_DT_F64, ldyt, 1};
    MatRef b{A, GN_DT_F64, lda, 1};
    return launch_dgemm(rl, n, m, 1.0, a, b, 0.0, (double*)YtA, ldya, 1, nullptr, false, s);
  }
  if (mode == GN_MODE_F32)
    return run_gemm_f32<true, false>(rl, n, m, (const float*)Yt, ldyt, (const float*)A, lda,
                                     (float*)YtA, ldya, /*inner_is_m=*/true, s);
  return launch_pass_yta_bf16(m, n, rl, (const uint16_t*)A, lda, scales, (const uint16_t*)Yt, ldyt,
                              (float*)YtA, ldya, s);
}

gn_status launch_pass_srht(int32_t mode, int64_t m, int64_t n, int64_t r, const void* A, int64_t lda,
                           const float* scales, const int8_t* signs, const int32_t* idx, void* AX,
                           int64_t ldax, hipStream_t s) {
  if (mode == GN_MODE_F64)
    return run_srht<double, GN_MODE_F64>(m, n, r, A, lda, scales, signs, idx, (double*)AX, ldax, s);
  if (mode == GN_MODE_F32)
    return run_srht<float, GN_MODE_F32>(m, n, r, A, lda, scales, signs, idx, (float*)AX, ldax, s);
  return run_srht<float, GN_MODE_BF16_BS>(m, n, r, A, lda, scales, signs, idx, (float*)AX, ldax,
                                          s);
}

}  // namespace gn
