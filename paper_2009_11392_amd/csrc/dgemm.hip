// FP64 strided GEMM for the core of GN and its factor products:
//   D (M x N) = alpha * A (M x K) * B (K x N) + beta * D,
// A and B given by element strides and stored as double, float or bfloat16
// (promoted to double exactly).  Also the tile-wise residual ||Ref - A B||_F^2
// with a fixed-order (deterministic) reduction.
//
// 256 threads = 4 waves in 2 x 2, 64 x 64 output tile, wave tile 32 x 32 = 2 x 2
// blocks of v_mfma_f64_16x16x4f64 (register v of lane l of a 16 x 16 block
// holds row l/16 + 4v, column l%16 -- measured on gfx950).  K is staged through LDS 16 at a time
// with the next slab prefetched into registers.  Global loads follow whichever
// stride is 1.  Products with few output tiles and a long K are split along K
// into fixed slices whose partial results are summed in slice order.
#include "gn_internal.h"

namespace gn {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

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
  void* D;              // double, or float when d_dtype == GN_DT_F32 (rounded to nearest)
  int64_t rsd, csd;
  const int32_t* kmask;
  int32_t mask_rows;
  const int32_t* gate;  // run only if (*gate < gate_n) == gate_trunc
  int64_t gate_n;
  int32_t gate_trunc;
  int32_t ksplit;       // > 1: slice s of K written to partial + s*M*N
  int64_t kslice;
  double* partial;
  int32_t d_dtype;
};

// D(i, j) = alpha * sum + beta * D(i, j), zeroed beyond the mask.
__device__ __forceinline__ void store_d(const DArgs& g, int64_t i, int64_t j, double sum,
                                        int32_t kk) {
  const int64_t off = i * g.rsd + j * g.csd;
  double val = g.alpha * sum;
  if (g.d_dtype == GN_DT_F32) {
    float* d = reinterpret_cast<float*>(g.D) + off;
    if (g.beta != 0.0) val += g.beta * (double)(*d);
    if (g.kmask && (g.mask_rows ? (i >= kk) : (j >= kk))) val = 0.0;
    *d = __double2float_rn(val);
  } else {
    double* d = reinterpret_cast<double*>(g.D) + off;
    if (g.beta != 0.0) val += g.beta * (*d);
    if (g.kmask && (g.mask_rows ? (i >= kk) : (j >= kk))) val = 0.0;
    *d = val;
  }
}

__device__ __forceinline__ bool gated_off(const DArgs& g) {
  if (!g.gate) return false;
  const bool trunc = *g.gate < g.gate_n;
  return trunc != (g.gate_trunc != 0);
}

struct DStage {
  double a[4], b[4];
  __device__ __forceinline__ void load(const DArgs& g, int64_t i0, int64_t j0, int64_t k0,
                                       int64_t kend) {
    const int tid = threadIdx.x;
    const bool a_kc = (g.A.cs == 1);
    const bool b_kc = (g.B.rs == 1);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int ii = a_kc ? (e >> 4) : (e & 63);
      const int kk = a_kc ? (e & 15) : (e >> 6);
      const int64_t i = i0 + ii, k = k0 + kk;
      a[q] = (i < g.M && k < kend) ? ld_elem(g.A.p, g.A.dtype, i * g.A.rs + k * g.A.cs) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int jj = b_kc ? (e >> 4) : (e & 63);
      const int kk = b_kc ? (e & 15) : (e >> 6);
      const int64_t j = j0 + jj, k = k0 + kk;
      b[q] = (j < g.N && k < kend) ? ld_elem(g.B.p, g.B.dtype, k * g.B.rs + j * g.B.cs) : 0.0;
    }
  }
  __device__ __forceinline__ void store(const DArgs& g, double (*sA)[D_BM + 1],
                                        double (*sB)[D_BN + 1]) const {
    const int tid = threadIdx.x;
    const bool a_kc = (g.A.cs == 1);
    const bool b_kc = (g.B.rs == 1);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int ii = a_kc ? (e >> 4) : (e & 63);
      const int kk = a_kc ? (e & 15) : (e >> 6);
      sA[kk][ii] = a[q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int jj = b_kc ? (e >> 4) : (e & 63);
      const int kk = b_kc ? (e & 15) : (e >> 6);
      sB[kk][jj] = b[q];
    }
  }
};

// acc[x][y] = the (x, y) 16 x 16 block of this wave over k in [kbeg, kend).
__device__ __forceinline__ void d_tile(const DArgs& g, int64_t i0, int64_t j0, int64_t kbeg,
                                       int64_t kend, f64x4 (&acc)[2][2]) {
  __shared__ double sA[2][D_BK][D_BM + 1];
  __shared__ double sB[2][D_BK][D_BN + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = f64x4{0.0, 0.0, 0.0, 0.0};
  if (kend <= kbeg) return;
  const int64_t nk = (kend - kbeg + D_BK - 1) / D_BK;
  DStage st;
  st.load(g, i0, j0, kbeg, kend);
  st.store(g, sA[0], sB[0]);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) st.load(g, i0, j0, kbeg + (kt + 1) * D_BK, kend);
#pragma unroll
    for (int kk = 0; kk < D_BK; kk += 4) {
      double a[2], b[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) a[x] = sA[cur][kk + lk][wm * 32 + x * 16 + li];
#pragma unroll
      for (int y = 0; y < 2; ++y) b[y] = sB[cur][kk + lk][wn * 32 + y * 16 + li];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
    }
    if (kt + 1 < nk) st.store(g, sA[cur ^ 1], sB[cur ^ 1]);
    __syncthreads();
  }
}

__device__ __forceinline__ void d_coord(int x, int y, int v, int64_t i0, int64_t j0, int64_t& i,
                                        int64_t& j) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  i = i0 + wm * 32 + x * 16 + (lane >> 4) + 4 * v;
  j = j0 + wn * 32 + y * 16 + (lane & 15);
}

__global__ void __launch_bounds__(256) dgemm_kernel(DArgs g) {
  if (gated_off(g)) return;
  const int64_t tn_n = (g.N + D_BN - 1) / D_BN;
  const int64_t tiles = ((g.M + D_BM - 1) / D_BM) * tn_n;
  const int64_t t = blockIdx.x % tiles, s = blockIdx.x / tiles;
  const int64_t i0 = (t / tn_n) * D_BM, j0 = (t % tn_n) * D_BN;
  const int64_t kbeg = s * g.kslice;
  const int64_t kend = (kbeg + g.kslice < g.K) ? kbeg + g.kslice : g.K;
  f64x4 acc[2][2];
  d_tile(g, i0, j0, kbeg, kend, acc);
  if (g.ksplit > 1) {
    double* P = g.partial + s * g.M * g.N;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          int64_t i, j;
          d_coord(x, y, v, i0, j0, i, j);
          if (i < g.M && j < g.N) P[i * g.N + j] = acc[x][y][v];
        }
    return;
  }
  const int32_t kk = g.kmask ? *g.kmask : 0;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int64_t i, j;
        d_coord(x, y, v, i0, j0, i, j);
        if (i >= g.M || j >= g.N) continue;
        store_d(g, i, j, acc[x][y][v], kk);
      }
}

// D = alpha * sum_s partial[s] + beta * D, slices summed in order.
__global__ void __launch_bounds__(256) dgemm_reduce(DArgs g) {
  if (gated_off(g)) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.M * g.N) return;
  const int64_t i = e / g.N, j = e - i * g.N;
  double s = 0.0;
  for (int q = 0; q < g.ksplit; ++q) s += g.partial[q * g.M * g.N + e];
  store_d(g, i, j, s, g.kmask ? *g.kmask : 0);
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
  f64x4 acc[2][2];
  d_tile(g, i0, j0, 0, g.K, acc);
  double ss = 0.0;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int64_t i, j;
        d_coord(x, y, v, i0, j0, i, j);
        if (i >= g.M || j >= g.N) continue;
        double ref = ld_elem(rr.ref.p, rr.ref.dtype, i * rr.ref.rs + j * rr.ref.cs);
        if (rr.ref.dtype == GN_DT_BF16) ref *= (double)rr.ref_scales[(i >> 7) * rr.nsb + (j >> 7)];
        const double d = ref - acc[x][y][v];
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

constexpr int64_t kTargetWG = 512;  // two workgroups per CU
constexpr int64_t kMinSlice = 64;   // slices of at least 64 (four staged K blocks)

}  // namespace

int32_t dgemm_split(int64_t M, int64_t N, int64_t K) {
  const int64_t tiles = cdiv(M, D_BM) * cdiv(N, D_BN);
  if (tiles >= kTargetWG || K < 2 * kMinSlice) return 1;
  int64_t s = cdiv(kTargetWG, tiles);
  const int64_t smax = K / kMinSlice;
  if (s > smax) s = smax;
  if (s > 32) s = 32;
  return (int32_t)(s < 1 ? 1 : s);
}

size_t dgemm_split_ws_bytes(int64_t M, int64_t N, int64_t K) {
  const int32_t s = dgemm_split(M, N, K);
  return s > 1 ? align_up((size_t)s * M * N * sizeof(double)) : 0;
}

gn_status launch_dgemm_to(int64_t M, int64_t N, int64_t K, double alpha, MatRef A, MatRef B,
                          double beta, void* D, int32_t d_dtype, int64_t rsd, int64_t csd,
                          const int32_t* kmask, bool mask_rows, hipStream_t s, const int32_t* gate,
                          int64_t gate_n, bool gate_trunc, double* split_ws,
                          size_t split_ws_bytes) {
  if (M <= 0 || N <= 0) return GN_OK;
  DArgs g{M,    N,          K,          A,   B,   alpha, beta, D, rsd, csd, kmask, mask_rows ? 1 : 0,
          gate, gate_n, gate_trunc ? 1 : 0, 1, K > 0 ? K : 1, nullptr, d_dtype};
  const int64_t tiles = cdiv(M, D_BM) * cdiv(N, D_BN);
  int32_t ks = split_ws ? dgemm_split(M, N, K) : 1;
  if (ks > 1 && split_ws_bytes < (size_t)ks * M * N * sizeof(double)) ks = 1;
  if (ks > 1) {
    g.ksplit = ks;
    g.kslice = cdiv(cdiv(K, ks), D_BK) * D_BK;
    g.partial = split_ws;
    dgemm_kernel<<<dim3((unsigned)(tiles * ks)), dim3(256), 0, s>>>(g);
    GN_LAUNCH_CHECK();
    dgemm_reduce<<<dim3((unsigned)cdiv(M * N, 256)), dim3(256), 0, s>>>(g);
    GN_LAUNCH_CHECK();
    return GN_OK;
  }
  dgemm_kernel<<<dim3((unsigned)tiles), dim3(256), 0, s>>>(g);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

gn_status launch_dgemm(int64_t M, int64_t N, int64_t K, double alpha, MatRef A, MatRef B,
                       double beta, double* D, int64_t rsd, int64_t csd, const int32_t* kmask,
                       bool mask_rows, hipStream_t s, const int32_t* gate, int64_t gate_n,
                       bool gate_trunc, double* split_ws, size_t split_ws_bytes) {
  return launch_dgemm_to(M, N, K, alpha, A, B, beta, D, GN_DT_F64, rsd, csd, kmask, mask_rows, s,
                         gate, gate_n, gate_trunc, split_ws, split_ws_bytes);
}

size_t residual_ws_bytes(int64_t M, int64_t N) {
  return align_up((size_t)(cdiv(M, D_BM) * cdiv(N, D_BN)) * sizeof(double));
}

gn_status launch_residual(int64_t M, int64_t N, int64_t K, MatRef Ref, const float* ref_scales,
                          MatRef A, MatRef B, double* partial, double* out, hipStream_t s) {
  const int64_t tiles = cdiv(M, D_BM) * cdiv(N, D_BN);
  DArgs g{M, N, K, A, B, 1.0, 0.0, nullptr, 0, 0, nullptr, 0, nullptr, 0, 0, 1, K, nullptr,
          GN_DT_F64};  // no D: the tiles feed the residual
  RArgs rr{Ref, ref_scales, cdiv(N, 128), partial};
  residual_kernel<<<dim3((unsigned)tiles), dim3(256), 0, s>>>(g, rr);
  GN_LAUNCH_CHECK();
  reduce_partials<<<dim3(1), dim3(256), 0, s>>>(partial, tiles, out);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

}  // namespace gn
