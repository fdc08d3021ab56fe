// On-device sketch generators: Philox4x32-10 Gaussians and SRHT signs / column
// sample (Section 1 and Section 3.1 of the paper: i.i.d. N(0,1) sketches, or the
// subsampled randomized Hadamard transform).
#include "gn_internal.h"

namespace gn {
namespace {

// ---------------------------------------------------------------- Box-Muller in FP64
// The map of two 53-bit uniforms to two standard normals, z = sqrt(-2 ln u1) (cos t,
// sin t) with t the double nearest 2 pi u2, evaluated for exactly this domain
// (u1 in [2^-53, 1], t in [0, 2 pi)) with a few FMAs: the generic library log, sin
// and cos spent most of the generator's time on their range checks and on
// reductions for arguments that never occur here.  The log, sine and cosine are
// each within about one ulp of the correctly rounded value; z is within 3 ulp of
// NumPy's log, cos and sin over a block of 4M values (measured).

// ln x for x in [2^-53, 1]: x = 2^e m with m in (sqrt(2)/2, sqrt(2)], f = m - 1
// (exact), s = f / (2 + f), ln m = 2 atanh(s) = f - (f^2/2 - s (f^2/2 + R)) with
// R = sum_k 2 s^(2k) / (2k + 1) (k = 1 .. 12: the first omitted term is below
// 2^-60 of ln m), and e ln 2 added through FMAs with ln 2 in two parts.
__device__ __forceinline__ double bm_log(double x) {
#pragma clang fp contract(off)
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  int e = (int)(b >> 52) - 1023;
  double m = __longlong_as_double((long long)((b & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
  if (m > 0x1.6a09e667f3bcdp+0) {
    m *= 0.5;
    e += 1;
  }
  const double f = m - 1.0;
  const double s = f / (2.0 + f);
  const double z = s * s;
  double p = 2.0 / 25.0;
  p = __builtin_fma(p, z, 2.0 / 23.0);
  p = __builtin_fma(p, z, 2.0 / 21.0);
  p = __builtin_fma(p, z, 2.0 / 19.0);
  p = __builtin_fma(p, z, 2.0 / 17.0);
  p = __builtin_fma(p, z, 2.0 / 15.0);
  p = __builtin_fma(p, z, 2.0 / 13.0);
  p = __builtin_fma(p, z, 2.0 / 11.0);
  p = __builtin_fma(p, z, 2.0 / 9.0);
  p = __builtin_fma(p, z, 2.0 / 7.0);
  p = __builtin_fma(p, z, 2.0 / 5.0);
  p = __builtin_fma(p, z, 2.0 / 3.0);
  const double R = z * p;
  const double hfsq = 0.5 * f * f;
  const double lm = f - (hfsq - s * (hfsq + R));
  const double de = (double)e;
  return __builtin_fma(de, 0x1.62e42fefa39efp-1, __builtin_fma(de, 0x1.abc9e3b39803fp-56, lm));
}

// sin t and cos t for t in [0, 2 pi): k = nearest integer to t / (pi/2), y = t - k pi/2
// with pi/2 in three parts (the products exact inside the FMAs, so y is accurate
// to far below its ulp even next to a multiple of pi/2), |y| <= pi/4, then the
// Taylor series of sin y to y^17 and of cos y to y^16 (omitted terms below 2^-60)
// and the quadrant of k.
__device__ __forceinline__ void bm_sincos(double t, double& sn, double& cs) {
#pragma clang fp contract(off)
  const double k = __builtin_rint(t * 0x1.45f306dc9c883p-1);
  double y = __builtin_fma(-k, 0x1.921fb54442d18p+0, t);
  y = __builtin_fma(-k, 0x1.1a62633145c07p-54, y);
  y = __builtin_fma(-k, -0x1.f1976b7ed8fbcp-110, y);
  const double z = y * y;
  double ps = 1.0 / 355687428096000.0;                // 1/17!
  ps = __builtin_fma(ps, z, -1.0 / 1307674368000.0);  // 1/15!
  ps = __builtin_fma(ps, z, 1.0 / 6227020800.0);      // 1/13!
  ps = __builtin_fma(ps, z, -1.0 / 39916800.0);       // 1/11!
  ps = __builtin_fma(ps, z, 1.0 / 362880.0);          // 1/9!
  ps = __builtin_fma(ps, z, -1.0 / 5040.0);           // 1/7!
  ps = __builtin_fma(ps, z, 1.0 / 120.0);             // 1/5!
  ps = __builtin_fma(ps, z, -1.0 / 6.0);              // 1/3!
  const double sy = __builtin_fma(y * z, ps, y);
  double pc = 1.0 / 20922789888000.0;                 // 1/16!
  pc = __builtin_fma(pc, z, -1.0 / 87178291200.0);    // 1/14!
  pc = __builtin_fma(pc, z, 1.0 / 479001600.0);       // 1/12!
  pc = __builtin_fma(pc, z, -1.0 / 3628800.0);        // 1/10!
  pc = __builtin_fma(pc, z, 1.0 / 40320.0);           // 1/8!
  pc = __builtin_fma(pc, z, -1.0 / 720.0);            // 1/6!
  pc = __builtin_fma(pc, z, 1.0 / 24.0);              // 1/4!
  pc = __builtin_fma(pc, z, -0.5);                    // 1/2!
  const double cy = __builtin_fma(z, pc, 1.0);
  const int q = ((int)k) & 3;
  sn = (q == 0) ? sy : (q == 1) ? cy : (q == 2) ? -sy : -cy;
  cs = (q == 0) ? cy : (q == 1) ? -sy : (q == 2) ? -cy : sy;
}

// Two standard normals from one Philox block: 53-bit uniforms u1 in (0,1],
// u2 in [0,1) and the Box-Muller map, all in double precision.
__device__ __forceinline__ void bm_normal_pair(U4 w, double& z0, double& z1) {
#pragma clang fp contract(off)
  const uint64_t ka = ((uint64_t)(w.a >> 5) << 26) | (uint64_t)(w.b >> 6);
  const uint64_t kb = ((uint64_t)(w.c >> 5) << 26) | (uint64_t)(w.d >> 6);
  const double u1 = 1.0 - (double)ka * 0x1.0p-53;
  const double u2 = (double)kb * 0x1.0p-53;
  const double rad = sqrt(-2.0 * bm_log(u1));
  double sn, cs;
  bm_sincos(6.283185307179586 * u2, sn, cs);
  z0 = rad * cs;
  z1 = rad * sn;
}

template <int DT>
__device__ __forceinline__ void store_elem(void* out, int64_t off, double z) {
  if constexpr (DT == GN_DT_F64) {
    reinterpret_cast<double*>(out)[off] = z;
  } else if constexpr (DT == GN_DT_F32) {
    reinterpret_cast<float*>(out)[off] = __double2float_rn(z);
  } else if constexpr (DT == kDtBf16AsF32) {
    reinterpret_cast<float*>(out)[off] = bf16_bits_to_f32(f64_to_bf16_bits(z));
  } else if constexpr (DT == kDtF16AsF32) {
    reinterpret_cast<float*>(out)[off] = f16_bits_to_f32(f64_to_f16_bits(z));
  } else if constexpr (DT == GN_DT_F16) {
    reinterpret_cast<uint16_t*>(out)[off] = f64_to_f16_bits(z);
  } else {
    reinterpret_cast<uint16_t*>(out)[off] = f64_to_bf16_bits(z);
  }
}

// Row-major output: consecutive threads take consecutive column pairs.
template <int DT>
__global__ void __launch_bounds__(256) gaussian_rowmajor(uint32_t k0, uint32_t k1, uint32_t sid,
                                                         int64_t row0, int64_t col0, int64_t rows,
                                                         int64_t cols, int64_t pair0, int64_t npairs,
                                                         void* out, int64_t ld) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * npairs) return;
  const int64_t i = t / npairs;
  const int64_t p = pair0 + (t - i * npairs);
  const U4 w = philox10(U4{(uint32_t)(row0 + i), (uint32_t)p, sid, 0u}, k0, k1);
  double z[2];
  bm_normal_pair(w, z[0], z[1]);
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int64_t j = 2 * p + e - col0;
    if (j >= 0 && j < cols) store_elem<DT>(out, i * ld + j, z[e]);
  }
}

// Transposed output out[j*ld + i]: consecutive threads take consecutive rows.
template <int DT>
__global__ void __launch_bounds__(256) gaussian_transposed(uint32_t k0, uint32_t k1, uint32_t sid,
                                                           int64_t row0, int64_t col0, int64_t rows,
                                                           int64_t cols, int64_t pair0,
                                                           int64_t npairs, void* out, int64_t ld) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * npairs) return;
  const int64_t pl = t / rows;
  const int64_t i = t - pl * rows;
  const int64_t p = pair0 + pl;
  const U4 w = philox10(U4{(uint32_t)(row0 + i), (uint32_t)p, sid, 0u}, k0, k1);
  double z[2];
  bm_normal_pair(w, z[0], z[1]);
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int64_t j = 2 * p + e - col0;
    if (j >= 0 && j < cols) store_elem<DT>(out, j * ld + i, z[e]);
  }
}

// Batched row-major Gaussian blocks: job blockIdx.z, grid-stride over its
// rows x column pairs (counter layout as gaussian_rowmajor with row0 = col0 = 0).
template <int DT>
__global__ void __launch_bounds__(256) gaussian_rowmajor_b(const GaussJob* __restrict__ jobs) {
  const GaussJob J = jobs[blockIdx.z];
  const uint32_t k0 = (uint32_t)(J.seed & 0xffffffffu), k1 = (uint32_t)(J.seed >> 32);
  const int64_t npairs = (J.cols + 1) >> 1;
  const int64_t total = J.rows * npairs;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t / npairs;
    const int64_t p = t - i * npairs;
    const U4 w = philox10(U4{(uint32_t)i, (uint32_t)p, (uint32_t)J.sid, 0u}, k0, k1);
    double z[2];
    bm_normal_pair(w, z[0], z[1]);
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int64_t j = 2 * p + e;
      if (j < J.cols) store_elem<DT>(J.out, i * J.ld + j, z[e]);
    }
  }
}

__global__ void __launch_bounds__(256) srht_signs_keys(uint32_t k0, uint32_t k1, int64_t npad,
                                                       int8_t* signs, uint64_t* keys) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= npad) return;
  // sign: top bit of word (j & 3) of block (j >> 2, 0, 3, 0)
  const U4 ws = philox10(U4{(uint32_t)(j >> 2), 0u, 3u, 0u}, k0, k1);
  const uint32_t wsel[4] = {ws.a, ws.b, ws.c, ws.d};
  signs[j] = (wsel[j & 3] >> 31) ? (int8_t)-1 : (int8_t)1;
  // key: words (2b, 2b+1), b = j & 1, of block (j >> 1, 0, 4, 0)
  const U4 wk = philox10(U4{(uint32_t)(j >> 1), 0u, 4u, 0u}, k0, k1);
  const uint32_t hi = (j & 1) ? wk.c : wk.a;
  const uint32_t lo = (j & 1) ? wk.d : wk.b;
  keys[j] = ((uint64_t)hi << 32) | (uint64_t)lo;
}

// The r smallest (key, j) pairs in ascending order: idx[rank] = j.  One
// workgroup: a histogram of the top kSelBits key bits finds the first bin at
// which the cumulative count reaches r; every key in a later bin is larger than
// the >= r keys before it, so only the keys of bins up to that one (about
// r + npad / 2^kSelBits for uniform keys) are compacted into cand_* and ranked
// against each other.  Ties between equal keys are broken by the index j, so
// the result does not depend on the order of the atomic compaction.
constexpr int kSelBits = 12, kSelBins = 1 << kSelBits, kSelT = 1024;
__global__ void __launch_bounds__(kSelT) srht_select(const uint64_t* keys, int64_t npad, int64_t r,
                                                     uint64_t* cand_k, int32_t* cand_j,
                                                     int32_t* idx) {
  __shared__ int hist[kSelBins];
  __shared__ uint64_t tk[kSelT];
  __shared__ int32_t tj[kSelT];
  __shared__ int s_bin, s_cnt;
  const int t = threadIdx.x;
  for (int b = t; b < kSelBins; b += kSelT) hist[b] = 0;
  if (t == 0) {
    s_cnt = 0;
    s_bin = kSelBins - 1;
  }
  __syncthreads();
  for (int64_t j = t; j < npad; j += kSelT) atomicAdd(&hist[(int)(keys[j] >> (64 - kSelBits))], 1);
  __syncthreads();
  if (t < 64) {  // wave 0: lane t owns bins [64 t, 64 t + 64)
    int own = 0;
    for (int q = 0; q < kSelBins / 64; ++q) own += hist[t * (kSelBins / 64) + q];
    int inc = own;
    for (int d = 1; d < 64; d <<= 1) {
      const int v = __shfl_up(inc, d, 64);
      if (t >= d) inc += v;
    }
    const int exc = inc - own;
    if (exc < r && inc >= r) {
      int c = exc, b = t * (kSelBins / 64);
      while (c + hist[b] < r) c += hist[b++];
      s_bin = b;
    }
  }
  __syncthreads();
  const int bsel = s_bin;
  for (int64_t j = t; j < npad; j += kSelT) {
    const uint64_t k = keys[j];
    if ((int)(k >> (64 - kSelBits)) <= bsel) {
      const int pos = atomicAdd(&s_cnt, 1);
      cand_k[pos] = k;
      cand_j[pos] = (int32_t)j;
    }
  }
  __syncthreads();
  const int c = s_cnt;
  for (int base = 0; base < c; base += kSelT) {
    const int me = base + t;
    const uint64_t kme = (me < c) ? cand_k[me] : ~0ull;
    const int32_t jme = (me < c) ? cand_j[me] : 0x7fffffff;
    int rank = 0;
    for (int t0 = 0; t0 < c; t0 += kSelT) {
      __syncthreads();
      if (t0 + t < c) {
        tk[t] = cand_k[t0 + t];
        tj[t] = cand_j[t0 + t];
      }
      __syncthreads();
      const int len = (c - t0 < kSelT) ? (c - t0) : kSelT;
      for (int q = 0; q < len; ++q) rank += (tk[q] < kme) || (tk[q] == kme && tj[q] < jme);
    }
    if (me < c && rank < r) idx[rank] = jme;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) transpose_kernel(const T* in, int64_t rows, int64_t cols,
                                                        int64_t ldi, T* out, int64_t ldo) {
  __shared__ T tile[32][33];
  const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int y = ty; y < 32; y += 8) {
    const int64_t rr = r0 + y, cc = c0 + tx;
    if (rr < rows && cc < cols) tile[y][tx] = in[rr * ldi + cc];
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int64_t cc = c0 + y, rr = r0 + tx;
    if (rr < rows && cc < cols) out[cc * ldo + rr] = tile[tx][y];
  }
}

}  // namespace

gn_status launch_gaussian(uint64_t seed, int32_t sid, int64_t row0, int64_t col0, int64_t rows,
                          int64_t cols, int32_t dtype, int32_t layout, void* out, int64_t ld,
                          hipStream_t s) {
  if (rows <= 0 || cols <= 0) return GN_OK;
  const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
  const int64_t pair0 = col0 >> 1, pair1 = (col0 + cols - 1) >> 1;
  const int64_t npairs = pair1 - pair0 + 1;
  const int64_t total = rows * npairs;
  const dim3 grid((unsigned)cdiv(total, 256)), block(256);
#define GN_GAUSS(DT)                                                                       \
  if (layout == 0)                                                                         \
    gaussian_rowmajor<DT><<<grid, block, 0, s>>>(k0, k1, (uint32_t)sid, row0, col0, rows,  \
                                                 cols, pair0, npairs, out, ld);            \
  else                                                                                     \
    gaussian_transposed<DT><<<grid, block, 0, s>>>(k0, k1, (uint32_t)sid, row0, col0, rows, \
                                                   cols, pair0, npairs, out, ld);
  if (dtype == GN_DT_F64) {
    GN_GAUSS(GN_DT_F64)
  } else if (dtype == GN_DT_F32) {
    GN_GAUSS(GN_DT_F32)
  } else if (dtype == kDtBf16AsF32) {
    GN_GAUSS(kDtBf16AsF32)
  } else if (dtype == kDtF16AsF32) {
    GN_GAUSS(kDtF16AsF32)
  } else if (dtype == GN_DT_F16) {
    GN_GAUSS(GN_DT_F16)
  } else {
    GN_GAUSS(GN_DT_BF16)
  }
#undef GN_GAUSS
  GN_LAUNCH_CHECK();
  return GN_OK;
}

// keys (npad u64) | candidate keys (npad u64) | candidate indices (npad i32)
gn_status launch_gaussian_batched(const GaussJob* jobs, int32_t count, int32_t dtype, hipStream_t s) {
  if (count <= 0) return GN_OK;
  const dim3 grid(256, 1, (unsigned)count), block(256);
  if (dtype == GN_DT_F64)
    gaussian_rowmajor_b<GN_DT_F64><<<grid, block, 0, s>>>(jobs);
  else if (dtype == GN_DT_F32)
    gaussian_rowmajor_b<GN_DT_F32><<<grid, block, 0, s>>>(jobs);
  else
    return GN_ERR_DTYPE;
  GN_LAUNCH_CHECK();
  return GN_OK;
}

size_t srht_ws_bytes(int64_t npad) {
  return 2 * align_up((size_t)npad * sizeof(uint64_t)) + align_up((size_t)npad * sizeof(int32_t));
}

gn_status launch_srht(uint64_t seed, int64_t npad, int64_t r, int8_t* signs, int32_t* idx,
                      uint64_t* keys_ws, hipStream_t s) {
  const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
  const dim3 grid((unsigned)cdiv(npad, 256)), block(256);
  srht_signs_keys<<<grid, block, 0, s>>>(k0, k1, npad, signs, keys_ws);
  GN_LAUNCH_CHECK();
  char* base = reinterpret_cast<char*>(keys_ws);
  const size_t kb = align_up((size_t)npad * sizeof(uint64_t));
  srht_select<<<1, kSelT, 0, s>>>(keys_ws, npad, r, reinterpret_cast<uint64_t*>(base + kb),
                                  reinterpret_cast<int32_t*>(base + 2 * kb), idx);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

gn_status launch_transpose(const void* in, int64_t rows, int64_t cols, int64_t ldi, int32_t dtype,
                           void* out, int64_t ldo, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return GN_OK;
  const dim3 grid((unsigned)cdiv(cols, 32), (unsigned)cdiv(rows, 32)), block(256);
  if (dtype == GN_DT_F64)
    transpose_kernel<double><<<grid, block, 0, s>>>((const double*)in, rows, cols, ldi,
                                                    (double*)out, ldo);
  else if (dtype == GN_DT_F32)
    transpose_kernel<float><<<grid, block, 0, s>>>((const float*)in, rows, cols, ldi,
                                                   (float*)out, ldo);
  else
    transpose_kernel<uint16_t><<<grid, block, 0, s>>>((const uint16_t*)in, rows, cols, ldi,
                                                      (uint16_t*)out, ldo);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

}  // namespace gn
