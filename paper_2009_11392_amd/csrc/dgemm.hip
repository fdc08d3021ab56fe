// FP64 strided GEMM for the core of GN and its factor products:
//   D (M x N) = alpha * A (M x K) * B (K x N) + beta * D,
// A and B given by element strides and stored as double, float or bfloat16
// (promoted to double exactly).  Also the tile-wise residual ||Ref - A B||_F^2
// with a fixed-order (deterministic) reduction.
//
// 256 threads, 64 x 64 output tile, each thread a 4 x 4 register block; K staged
// through LDS 16 at a time.  Global loads follow whichever stride is 1.
#include "gn_internal.h"

namespace gn {
namespace {

constexpr int D_BM = 64, D_BN = 64, D_BK = 16;

__device__ __forceinline__ double ld_elem(const void* p, int32_t dt, int64_t off) {
  if (dt == GN_DT_F64) return reinterpret_cast<const double*>(p)[off];
  if (dt == GN_DT_F32) return (double)reinterpret_cast<const float*>(p)[off];
  return (double)bf16_bits_to_f32(reinterpret_cast<const uint16_t*>(p)[off]);
}

struct DArgs {
  int64_t M, N, K;
  MatRef A, B;
  double alpha, beta;
  double* D;
  int64_t rsd, csd;
  const int32_t* kmask;
  int32_t mask_rows;
  const int32_t* gate;  // run only if (*gate < gate_n) == gate_trunc
  int64_t gate_n;
  int32_t gate_trunc;
};

__device__ __forceinline__ bool gated_off(const DArgs& g) {
  if (!g.gate) return false;
  const bool trunc = *g.gate < g.gate_n;
  return trunc != (g.gate_trunc != 0);
}

// Stage A(i0.., k0..) into sA[k][i] and B(k0.., j0..) into sB[k][j].
__device__ __forceinline__ void d_stage(const DArgs& g, int64_t i0, int64_t j0, int64_t k0,
                                        double (*sA)[D_BM + 1], double (*sB)[D_BN + 1]) {
  const int tid = threadIdx.x;
  const bool a_kc = (g.A.cs == 1);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = tid + 256 * q;
    int ii, kk;
    if (a_kc) {
      ii = e >> 4;
      kk = e & 15;
    } else {
      kk = e >> 6;
      ii = e & 63;
    }
    const int64_t i = i0 + ii, k = k0 + kk;
    sA[kk][ii] = (i < g.M && k < g.K) ? ld_elem(g.A.p, g.A.dtype, i * g.A.rs + k * g.A.cs) : 0.0;
  }
  const bool b_kc = (g.B.rs == 1);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = tid + 256 * q;
    int jj, kk;
    if (b_kc) {
      jj = e >> 4;
      kk = e & 15;
    } else {
      kk = e >> 6;
      jj = e & 63;
    }
    const int64_t j = j0 + jj, k = k0 + kk;
    sB[kk][jj] = (j < g.N && k < g.K) ? ld_elem(g.B.p, g.B.dtype, k * g.B.rs + j * g.B.cs) : 0.0;
  }
}

// acc[a][b] = sum_k A(i0 + ty + 16a, k) B(k, j0 + tx + 16b)
__device__ __forceinline__ void d_tile(const DArgs& g, int64_t i0, int64_t j0, double (&acc)[4][4]) {
  __shared__ double sA[D_BK][D_BM + 1];
  __shared__ double sB[D_BK][D_BN + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int64_t k0 = 0; k0 < g.K; k0 += D_BK) {
    __syncthreads();
    d_stage(g, i0, j0, k0, sA, sB);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < D_BK; ++kk) {
      double av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = sA[kk][ty + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = sB[kk][tx + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
    }
  }
}

__global__ void __launch_bounds__(256) dgemm_kernel(DArgs g) {
  if (gated_off(g)) return;
  const int64_t tn_n = (g.N + D_BN - 1) / D_BN;
  const int64_t i0 = (int64_t)(blockIdx.x / tn_n) * D_BM;
  const int64_t j0 = (int64_t)(blockIdx.x % tn_n) * D_BN;
  double acc[4][4];
  d_tile(g, i0, j0, acc);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int32_t kk = g.kmask ? *g.kmask : 0;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t i = i0 + ty + 16 * a, j = j0 + tx + 16 * b;
      if (i >= g.M || j >= g.N) continue;
      double* d = g.D + i * g.rsd + j * g.csd;
      double v = g.alpha * acc[a][b];
      if (g.beta != 0.0) v += g.beta * (*d);
      if (g.kmask && (g.mask_rows ? (i >= kk) : (j >= kk))) v = 0.0;
      *d = v;
    }
}

struct RArgs {
  MatRef ref;
  const float* ref_scales;  // bf16 reference: 128 x 128 block scales
  int64_t nsb;
  double* partial;
};

__global__ void __launch_bounds__(256) residual_kernel(DArgs g, RArgs rr) {
  const int64_t tn_n = (g.N + D_BN - 1) / D_BN;
  const int64_t i0 = (int64_t)(blockIdx.x / tn_n) * D_BM;
  const int64_t j0 = (int64_t)(blockIdx.x % tn_n) * D_BN;
  double acc[4][4];
  d_tile(g, i0, j0, acc);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double ss = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t i = i0 + ty + 16 * a, j = j0 + tx + 16 * b;
      if (i >= g.M || j >= g.N) continue;
      double ref = ld_elem(rr.ref.p, rr.ref.dtype, i * rr.ref.rs + j * rr.ref.cs);
      if (rr.ref.dtype == GN_DT_BF16) ref *= (double)rr.ref_scales[(i >> 7) * rr.nsb + (j >> 7)];
      const double d = ref - acc[a][b];
      ss = fma(d, d, ss);
    }
  // fixed-order block reduction
  __shared__ double red[256];
  red[threadIdx.x] = ss;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) rr.partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) reduce_partials(const double* partial, int64_t n, double* out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

}  // namespace

gn_status launch_dgemm(int64_t M, int64_t N, int64_t K, double alpha, MatRef A, MatRef B,
                       double beta, double* D, int64_t rsd, int64_t csd, const int32_t* kmask,
                       bool mask_rows, hipStream_t s, const int32_t* gate, int64_t gate_n,
                       bool gate_trunc) {
  if (M <= 0 || N <= 0) return GN_OK;
  DArgs g{M, N,          K,          A,   B,   alpha, beta, D, rsd, csd, kmask, mask_rows ? 1 : 0,
          gate, gate_n, gate_trunc ? 1 : 0};
  const int64_t tiles = cdiv(M, D_BM) * cdiv(N, D_BN);
  dgemm_kernel<<<dim3((unsigned)tiles), dim3(256), 0, s>>>(g);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

size_t residual_ws_bytes(int64_t M, int64_t N) {
  return align_up((size_t)(cdiv(M, D_BM) * cdiv(N, D_BN)) * sizeof(double));
}

gn_status launch_residual(int64_t M, int64_t N, int64_t K, MatRef Ref, const float* ref_scales,
                          MatRef A, MatRef B, double* partial, double* out, hipStream_t s) {
  const int64_t tiles = cdiv(M, D_BM) * cdiv(N, D_BN);
  DArgs g{M, N, K, A, B, 1.0, 0.0, nullptr, 0, 0, nullptr, 0, nullptr, 0, 0};
  RArgs rr{Ref, ref_scales, cdiv(N, 128), partial};
  residual_kernel<<<dim3((unsigned)tiles), dim3(256), 0, s>>>(g, rr);
  GN_LAUNCH_CHECK();
  reduce_partials<<<dim3(1), dim3(256), 0, s>>>(partial, tiles, out);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

}  // namespace gn
