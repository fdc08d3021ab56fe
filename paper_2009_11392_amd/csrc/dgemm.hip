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
#include "wave_ops.h"

namespace gn {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int D_BM = 64, D_BN = 64, D_BK = 16;

__device__ __forceinline__ double ld_elem(const void* p, int32_t dt, int64_t off) {
  if (dt == GN_DT_F64) return reinterpret_cast<const double*>(p)[off];
  if (dt == GN_DT_F32) return (double)reinterpret_cast<const float*>(p)[off];
  if (dt == GN_DT_F16) return (double)f16_bits_to_f32(reinterpret_cast<const uint16_t*>(p)[off]);
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

// Products with a narrow right factor B (N <= NW_N columns: a block of a few
// right-hand sides), for which 64x64 MFMA tiles would leave most of the chip idle
// and most of each tile empty.  They are bound by the one read of A, so A streams
// through coalesced loads and is read once; B's rows are staged in LDS per K chunk.
// K is split into slices (blockIdx.y) summed afterwards in slice order by
// dgemm_reduce, so results do not depend on scheduling.
//  * dgemm_narrow, A k-contiguous (A.cs == 1): a 512-thread workgroup owns NW_RW
//    rows per wave, lanes along K; B's chunk is stored by columns so each lane
//    reads consecutive LDS words; a wave's NW_RW x NW_N sums finish in one
//    transposing wave sum.
//  * dgemm_narrow_t, A m-contiguous (A.rs == 1): one row per thread, lanes along
//    M, the chunk of B read by every lane at the same LDS address (broadcast).
constexpr int NW_N = 16, NW_RW = 2, NW_T = 512, NW_KC = 256;
constexpr int NT_T = 256, NT_KC = 16;

// A's entries in their stored type (FP64, FP32, or BF16 / binary16 widened to FP32
// exactly).
template <int DT> struct NwElem { using T = float; };
template <> struct NwElem<GN_DT_F64> { using T = double; };
template <int DT>
__device__ __forceinline__ typename NwElem<DT>::T nw_load(const void* p, int64_t off) {
  if constexpr (DT == GN_DT_F64) return reinterpret_cast<const double*>(p)[off];
  else if constexpr (DT == GN_DT_F32) return reinterpret_cast<const float*>(p)[off];
  else if constexpr (DT == GN_DT_F16) return f16_bits_to_f32(reinterpret_cast<const uint16_t*>(p)[off]);
  else return bf16_bits_to_f32(reinterpret_cast<const uint16_t*>(p)[off]);
}

// Workgroup barrier for LDS traffic only: waits for this wave's LDS operations,
// leaving its global loads in flight (__syncthreads waits for those as well).
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

__device__ __forceinline__ void nw_store(const DArgs& g, int64_t s, int64_t i, int64_t j, double v) {
  if (g.ksplit > 1)
    g.partial[s * g.M * g.N + i * g.N + j] = v;
  else
    store_d(g, i, j, v, g.kmask ? *g.kmask : 0);
}

// Loads below are unconditional, from clamped (in-range) indices, with values
// outside the operands replaced by zero only after the barrier: a predicated load
// compiles to a branch that waits for each load before issuing the next.
template <int DT>
__global__ void __launch_bounds__(NW_T) dgemm_narrow(DArgs g) {
  using E = typename NwElem<DT>::T;
  constexpr int kStage = NW_KC * NW_N / NW_T;  // B entries staged per thread
  __shared__ double Bs[NW_N][NW_KC + 1];
  if (gated_off(g)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t row0 = ((int64_t)blockIdx.x * (NW_T / 64) + wave) * NW_RW;
  const int64_t s = blockIdx.y;
  const int64_t kb = s * g.kslice;
  const int64_t ke = (kb + g.kslice < g.K) ? kb + g.kslice : g.K;
  const double* B = reinterpret_cast<const double*>(g.B.p);
  double bv[kStage];
  E a[NW_KC / 64][NW_RW];
  // chunk k0's loads: B's first, then A's (loads complete in order, so the staging
  // of B waits for B only)
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < kStage; ++q) {
      const int e = tid + q * NW_T, kk = e / NW_N, c = e % NW_N;
      const int64_t k = k0 + kk;
      const int64_t kc = k < ke ? k : ke - 1, cc = c < g.N ? c : g.N - 1;
      bv[q] = B[kc * g.B.rs + cc * g.B.cs];
    }
#pragma unroll
    for (int u = 0; u < NW_KC / 64; ++u)
#pragma unroll
      for (int rr = 0; rr < NW_RW; ++rr) {
        const int64_t row = row0 + rr, k = k0 + u * 64 + lane;
        const int64_t rc = row < g.M ? row : g.M - 1, kc = k < ke ? k : ke - 1;
        a[u][rr] = nw_load<DT>(g.A.p, rc * g.A.rs + kc);
      }
  };
  double acc[NW_RW * NW_N];
#pragma unroll
  for (int e = 0; e < NW_RW * NW_N; ++e) acc[e] = 0.0;
  load(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += NW_KC) {
    lds_barrier();  // every wave has read the previous chunk
    // entries outside the operands are zeroed here, past the barrier that no load
    // crosses, so the loads stay unconditional
#pragma unroll
    for (int q = 0; q < kStage; ++q) {
      const int e = tid + q * NW_T, kk = e / NW_N, c = e % NW_N;
      Bs[c][kk] = (k0 + kk < ke && c < g.N) ? bv[q] : 0.0;
    }
    lds_barrier();
    double av[NW_KC / 64][NW_RW];
#pragma unroll
    for (int u = 0; u < NW_KC / 64; ++u) {
      const bool kin = k0 + u * 64 + lane < ke;
#pragma unroll
      for (int rr = 0; rr < NW_RW; ++rr)
        av[u][rr] = (kin && row0 + rr < g.M) ? (double)a[u][rr] : 0.0;
    }
    load(k0 + NW_KC);  // the next chunk (clamped indices past the slice)
    asm volatile("" ::: "memory");  // keeps those loads ahead of this chunk's products
#pragma unroll
    for (int u = 0; u < NW_KC / 64; ++u) {
#pragma unroll
      for (int c = 0; c < NW_N; ++c) {
        const double b = Bs[c][u * 64 + lane];
#pragma unroll
        for (int rr = 0; rr < NW_RW; ++rr)
          acc[rr * NW_N + c] = fma(av[u][rr], b, acc[rr * NW_N + c]);
      }
    }
  }
  int slot;
  const double v = wave_transpose_sum<NW_RW * NW_N>(acc, lane, &slot);
  const int64_t row = row0 + slot / NW_N;
  const int c = slot % NW_N;
  if (row < g.M && c < g.N) nw_store(g, s, row, c, v);
}

template <int DT>
__global__ void __launch_bounds__(NT_T) dgemm_narrow_t(DArgs g) {
  using E = typename NwElem<DT>::T;
  constexpr int kStage = NT_KC * NW_N / NT_T;
  __shared__ double Bs[NT_KC][NW_N];
  if (gated_off(g)) return;
  const int tid = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * NT_T + tid;
  const int64_t ic = i < g.M ? i : g.M - 1;
  const int64_t s = blockIdx.y;
  const int64_t kb = s * g.kslice;
  const int64_t ke = (kb + g.kslice < g.K) ? kb + g.kslice : g.K;
  const double* B = reinterpret_cast<const double*>(g.B.p);
  double bv[kStage];
  E a[NT_KC];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < kStage; ++q) {
      const int e = tid + q * NT_T, kk = e / NW_N, c = e % NW_N;
      const int64_t k = k0 + kk;
      const int64_t kc = k < ke ? k : ke - 1, cc = c < g.N ? c : g.N - 1;
      bv[q] = B[kc * g.B.rs + cc * g.B.cs];
    }
#pragma unroll
    for (int kk = 0; kk < NT_KC; ++kk) {
      const int64_t k = k0 + kk, kc = k < ke ? k : ke - 1;
      a[kk] = nw_load<DT>(g.A.p, ic + kc * g.A.cs);
    }
  };
  double acc[NW_N];
#pragma unroll
  for (int c = 0; c < NW_N; ++c) acc[c] = 0.0;
  load(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += NT_KC) {
    lds_barrier();  // every wave has read the previous chunk
#pragma unroll
    for (int q = 0; q < kStage; ++q) {
      const int e = tid + q * NT_T, kk = e / NW_N, c = e % NW_N;
      Bs[kk][c] = (k0 + kk < ke && c < g.N) ? bv[q] : 0.0;
    }
    lds_barrier();
    double av[NT_KC];
#pragma unroll
    for (int kk = 0; kk < NT_KC; ++kk) av[kk] = (i < g.M && k0 + kk < ke) ? (double)a[kk] : 0.0;
    load(k0 + NT_KC);  // the next chunk (clamped indices past the slice)
    asm volatile("" ::: "memory");  // keeps those loads ahead of this chunk's products
#pragma unroll
    for (int kk = 0; kk < NT_KC; ++kk)
#pragma unroll
      for (int c = 0; c < NW_N; ++c) acc[c] = fma(av[kk], Bs[kk][c], acc[c]);
  }
  if (i >= g.M) return;
#pragma unroll
  for (int c = 0; c < NW_N; ++c)
    if (c < g.N) nw_store(g, s, i, c, acc[c]);
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
        if (rr.ref.dtype == GN_DT_BF16 || rr.ref.dtype == GN_DT_F16)
          ref *= (double)rr.ref_scales[(i >> 7) * rr.nsb + (j >> 7)];
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

// A product for the narrow kernels: one factor of at most NW_N columns (or rows),
// the other contiguous along K or along M, stored FP64, FP32 or BF16.
static bool narrow_eligible(int64_t M, int64_t N, int64_t K, const MatRef& A, const MatRef& B,
                     int32_t d_dtype) {
  if (K <= 0 || (d_dtype != GN_DT_F64 && d_dtype != GN_DT_F32)) return false;
  const MatRef& wide = N <= NW_N ? A : B;
  const MatRef& thin = N <= NW_N ? B : A;
  if (thin.dtype != GN_DT_F64) return false;
  if (wide.dtype != GN_DT_F64 && wide.dtype != GN_DT_F32 && wide.dtype != GN_DT_BF16 &&
      wide.dtype != GN_DT_F16)
    return false;
  if (N <= NW_N) return A.cs == 1 || A.rs == 1;
  if (M <= NW_N) return B.rs == 1 || B.cs == 1;  // B^T is k- or m-contiguous
  return false;
}

// K slices for the narrow kernels: about kTargetWG workgroups, slices of at least
// 2048 (k-contiguous) or 64 (m-contiguous) entries, at most 32.
static int64_t narrow_split(int64_t rb, int64_t K, bool kcont) {
  int64_t ks = cdiv(kTargetWG, rb);
  const int64_t kmax = kcont ? cdiv(K, 2048) : cdiv(K, 64);
  if (ks > kmax) ks = kmax;
  if (ks > 32) ks = 32;
  return ks < 1 ? 1 : ks;
}

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
  int64_t s = dgemm_split(M, N, K);
  if (N <= NW_N || M <= NW_N) {  // the narrow kernels' largest split, either layout
    const int64_t wide = N <= NW_N ? M : N;
    const int64_t a = narrow_split(cdiv(wide, (NW_T / 64) * NW_RW), K, true);
    const int64_t b = narrow_split(cdiv(wide, NT_T), K, false);
    if (a > s) s = a;
    if (b > s) s = b;
  }
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
  if (narrow_eligible(M, N, K, A, B, d_dtype)) {
    // a narrow left factor becomes a narrow right one: D^T = B^T A^T
    if (N > NW_N) {
      const MatRef At{B.p, B.dtype, B.cs, B.rs}, Bt{A.p, A.dtype, A.cs, A.rs};
      g.M = N;
      g.N = M;
      g.A = At;
      g.B = Bt;
      g.rsd = csd;
      g.csd = rsd;
      g.mask_rows = mask_rows ? 0 : 1;
    }
    const bool kcont = g.A.cs == 1;
    const int64_t rb = kcont ? cdiv(g.M, (NW_T / 64) * NW_RW) : cdiv(g.M, NT_T);
    int64_t ks = narrow_split(rb, K, kcont);
    if (ks > 1 && (!split_ws || split_ws_bytes < (size_t)ks * M * N * sizeof(double))) ks = 1;
    g.kslice = cdiv(cdiv(K, ks), 64) * 64;  // slices start on 64-entry boundaries
    ks = cdiv(K, g.kslice);
    g.ksplit = (int32_t)ks;
    g.partial = split_ws;
    const dim3 grid((unsigned)rb, (unsigned)ks);
    const int32_t dt = g.A.dtype;
    if (kcont) {
      if (dt == GN_DT_F64)
        dgemm_narrow<GN_DT_F64><<<grid, dim3(NW_T), 0, s>>>(g);
      else if (dt == GN_DT_F32)
        dgemm_narrow<GN_DT_F32><<<grid, dim3(NW_T), 0, s>>>(g);
      else if (dt == GN_DT_F16)
        dgemm_narrow<GN_DT_F16><<<grid, dim3(NW_T), 0, s>>>(g);
      else
        dgemm_narrow<GN_DT_BF16><<<grid, dim3(NW_T), 0, s>>>(g);
    } else {
      if (dt == GN_DT_F64)
        dgemm_narrow_t<GN_DT_F64><<<grid, dim3(NT_T), 0, s>>>(g);
      else if (dt == GN_DT_F32)
        dgemm_narrow_t<GN_DT_F32><<<grid, dim3(NT_T), 0, s>>>(g);
      else if (dt == GN_DT_F16)
        dgemm_narrow_t<GN_DT_F16><<<grid, dim3(NT_T), 0, s>>>(g);
      else
        dgemm_narrow_t<GN_DT_BF16><<<grid, dim3(NT_T), 0, s>>>(g);
    }
    GN_LAUNCH_CHECK();
    if (ks > 1) {
      dgemm_reduce<<<dim3((unsigned)cdiv(M * N, 256)), dim3(256), 0, s>>>(g);
      GN_LAUNCH_CHECK();
    }
    return GN_OK;
  }
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
