// 16-bit storage of A with one power-of-two scale per 128 x 128 block:
// s = 2^ceil(log2 max|a|) (1 for an all-zero block), stored value RNE(a / s) in
// bfloat16 or IEEE binary16.  Dividing by a power of two is exact, so for
// bfloat16 s * stored == RNE_bf16(a); for binary16 the scale also keeps the
// block's entries out of the binary16 subnormal range down to 2^-14 of its
// largest magnitude.
#include "gn_internal.h"

namespace gn {
namespace {

template <typename T, bool F16>
__global__ void __launch_bounds__(256) quant_h16_bs(int64_t m, int64_t n, const T* __restrict__ A,
                                                     int64_t lda, uint16_t* __restrict__ out,
                                                     int64_t ldo, float* __restrict__ scales) {
  const int64_t nsb = (n + 127) >> 7;
  const int64_t bi = blockIdx.x / nsb, bj = blockIdx.x - bi * nsb;
  const int64_t r0 = bi * 128, c0 = bj * 128;
  const int tid = threadIdx.x;
  double mx = 0.0;
  for (int e = tid; e < 128 * 128; e += 256) {
    const int64_t i = r0 + (e >> 7), j = c0 + (e & 127);
    if (i < m && j < n) mx = fmax(mx, fabs((double)A[i * lda + j]));
  }
  __shared__ double red[256];
  red[tid] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  mx = red[0];
  double sc = 1.0;
  if (mx > 0.0) {
    int e;
    const double f = frexp(mx, &e);  // mx = f * 2^e, f in [0.5, 1)
    sc = ldexp(1.0, (f == 0.5) ? e - 1 : e);
  }
  if (tid == 0) scales[bi * nsb + bj] = (float)sc;
  const double inv = 1.0 / sc;  // exact: sc is a power of two
  for (int e = tid; e < 128 * 128; e += 256) {
    const int64_t i = r0 + (e >> 7), j = c0 + (e & 127);
    if (i < m && j < n) {
      const double v = (double)A[i * lda + j] * inv;
      out[i * ldo + j] = F16 ? f64_to_f16_bits(v) : f64_to_bf16_bits(v);
    }
  }
}

}  // namespace

gn_status launch_quantize(int64_t m, int64_t n, const void* A, int64_t lda, int32_t dtype,
                          uint16_t* out, int64_t ldo, float* scales, hipStream_t s, bool f16) {
  const int64_t blocks = cdiv(m, 128) * cdiv(n, 128);
  const dim3 grid((unsigned)blocks), block(256);
  if (dtype == GN_DT_F64) {
    if (f16)
      quant_h16_bs<double, true><<<grid, block, 0, s>>>(m, n, (const double*)A, lda, out, ldo, scales);
    else
      quant_h16_bs<double, false><<<grid, block, 0, s>>>(m, n, (const double*)A, lda, out, ldo, scales);
  } else {
    if (f16)
      quant_h16_bs<float, true><<<grid, block, 0, s>>>(m, n, (const float*)A, lda, out, ldo, scales);
    else
      quant_h16_bs<float, false><<<grid, block, 0, s>>>(m, n, (const float*)A, lda, out, ldo, scales);
  }
  GN_LAUNCH_CHECK();
  return GN_OK;
}

}  // namespace gn
