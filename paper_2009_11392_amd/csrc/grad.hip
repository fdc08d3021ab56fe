// Small kernels of the reverse mode (the adjoint of A -> A_hat with the kept rank
// k held at its forward value) and of the sketch updates: the masked transpose
// that starts the explicit core pseudoinverse M = R_1^+ Q_1^T, and matrix
// accumulation.
#include "gn_internal.h"

namespace gn {
namespace {

// out (cols x rows, ld ldo) = src^T with rows >= k of out zeroed:
// out[i][j] = (i < k) ? src[j][i] : 0, src rows x cols (ld lds).
__global__ void __launch_bounds__(256) transpose_rows_masked(int64_t rows, int64_t cols,
                                                             const double* __restrict__ src,
                                                             int64_t lds, const int32_t* kdev,
                                                             double* __restrict__ out, int64_t ldo) {
  __shared__ double tile[32][33];
  const int32_t k = *kdev;
  const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int y = ty; y < 32; y += 8) {
    const int64_t rr = r0 + y, cc = c0 + tx;
    if (rr < rows && cc < cols) tile[y][tx] = src[rr * lds + cc];
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int64_t cc = c0 + y, rr = r0 + tx;  // out row cc, column rr
    if (rr < rows && cc < cols) out[cc * ldo + rr] = (cc < k) ? tile[tx][y] : 0.0;
  }
}

// Y += alpha X (rows x cols, FP64).
__global__ void __launch_bounds__(256) mat_axpy(int64_t rows, int64_t cols, double alpha,
                                                const double* __restrict__ X, int64_t ldx,
                                                double* __restrict__ Y, int64_t ldy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = e / cols, j = e - i * cols;
  Y[i * ldy + j] = fma(alpha, X[i * ldx + j], Y[i * ldy + j]);
}

// dst += src (rows x cols), FP64 or FP32 (dt).
__global__ void __launch_bounds__(256) mat_add(int64_t rows, int64_t cols, int32_t dt,
                                               const void* __restrict__ src, int64_t lds,
                                               void* __restrict__ dst, int64_t ldd) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = e / cols, j = e - i * cols;
  if (dt == GN_DT_F64)
    reinterpret_cast<double*>(dst)[i * ldd + j] += reinterpret_cast<const double*>(src)[i * lds + j];
  else
    reinterpret_cast<float*>(dst)[i * ldd + j] += reinterpret_cast<const float*>(src)[i * lds + j];
}

}  // namespace

gn_status launch_add(int64_t rows, int64_t cols, int32_t dt, const void* src, int64_t lds, void* dst,
                     int64_t ldd, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return GN_OK;
  if (dt != GN_DT_F64 && dt != GN_DT_F32) return GN_ERR_DTYPE;
  mat_add<<<dim3((unsigned)cdiv(rows * cols, 256)), dim3(256), 0, s>>>(rows, cols, dt, src, lds, dst,
                                                                       ldd);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

gn_status launch_transpose_rows_masked(int64_t rows, int64_t cols, const double* src, int64_t lds,
                                       const int32_t* k, double* out, int64_t ldo, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return GN_OK;
  const dim3 grid((unsigned)cdiv(cols, 32), (unsigned)cdiv(rows, 32)), block(256);
  transpose_rows_masked<<<grid, block, 0, s>>>(rows, cols, src, lds, k, out, ldo);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

gn_status launch_axpy(int64_t rows, int64_t cols, double alpha, const double* X, int64_t ldx,
                      double* Y, int64_t ldy, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return GN_OK;
  mat_axpy<<<dim3((unsigned)cdiv(rows * cols, 256)), dim3(256), 0, s>>>(rows, cols, alpha, X, ldx,
                                                                         Y, ldy);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

}  // namespace gn
