// Triangular solves with the GN core factor (Section 5.1: apply R^{-1} by
// substitution, never forming an inverse; Section 5.1.1: R_2^{-T} for the
// truncated core).  Solves X T = B in place for X (rows x r), with the
// triangle chosen on the device from the kept rank k:
//   right products (left = false): T = R (k == r) or T = R2^T (k < r);
//   left products  (left = true) : T = R^T (k == r) or T = R2 (k < r),
// the latter applied to a transposed view of the right-hand sides.
// Blocked by 64 columns: off-diagonal updates with the FP64 GEMM, diagonal
// blocks by one thread per row with the block of T and the 64 unknowns in LDS.
#include "gn_internal.h"

namespace gn {
namespace {

constexpr int TB = 64;

__global__ void __launch_bounds__(TB) trsm_diag(int64_t rows, int64_t r, const double* __restrict__ R,
                                                const double* __restrict__ R2, int64_t ldt,
                                                const int32_t* __restrict__ kdev, int want_trunc,
                                                int left, int r_only, double* __restrict__ X,
                                                int64_t rsx, int64_t csx, int64_t jb, int w) {
  const int32_t k = *kdev;
  const bool trunc = k < r;
  if (trunc != (want_trunc != 0)) return;
  const double* S = (trunc && !r_only) ? R2 : R;
  // R, R2 are upper; their transposes lower
  const bool trans = r_only ? (left != 0) : (left ? !trunc : trunc);
  const bool upper = !trans;
  const int64_t kk = trunc ? k : r;
  __shared__ double Ts[TB][TB + 1];
  __shared__ double Xs[TB][TB + 1];  // Xs[col][row]
  const int tid = threadIdx.x;
  for (int e = tid; e < TB * TB; e += TB) {
    const int t = e / TB, j = e - t * TB;
    double v = 0.0;
    if (t < w && j < w) v = trans ? S[(jb + j) * ldt + jb + t] : S[(jb + t) * ldt + jb + j];
    Ts[t][j] = v;
  }
  const int64_t row = (int64_t)blockIdx.x * TB + tid;
  for (int j = 0; j < w; ++j) Xs[j][tid] = (row < rows) ? X[row * rsx + (jb + j) * csx] : 0.0;
  __syncthreads();
  if (upper) {
    for (int j = 0; j < w; ++j) {
      if (jb + j >= kk) {
        Xs[j][tid] = 0.0;
        continue;
      }
      double x = Xs[j][tid];
      for (int t = 0; t < j; ++t) x = fma(-Xs[t][tid], Ts[t][j], x);
      Xs[j][tid] = x / Ts[j][j];
    }
  } else {
    for (int j = w - 1; j >= 0; --j) {
      if (jb + j >= kk) {
        Xs[j][tid] = 0.0;
        continue;
      }
      double x = Xs[j][tid];
      for (int t = j + 1; t < w; ++t)
        if (jb + t < kk) x = fma(-Xs[t][tid], Ts[t][j], x);
      Xs[j][tid] = x / Ts[j][j];
    }
  }
  if (row < rows)
    for (int j = 0; j < w; ++j) X[row * rsx + (jb + j) * csx] = Xs[j][tid];
}

}  // namespace

gn_status launch_trsm_core(int64_t rows, int64_t r, const double* R, const double* R2, int64_t ldt,
                           const int32_t* k, double* X, int64_t rsx, int64_t csx, bool left,
                           bool maybe_trunc, hipStream_t s, bool r_only) {
  if (rows <= 0) return GN_OK;
  const dim3 grid((unsigned)cdiv(rows, TB)), block(TB);
  const int64_t nblk = cdiv(r, TB);
  for (int want_trunc = 0; want_trunc <= (maybe_trunc ? 1 : 0); ++want_trunc) {
    const double* S = (want_trunc && !r_only) ? R2 : R;
    const bool trans = r_only ? left : (left ? !want_trunc : (bool)want_trunc);
    const bool upper = !trans;
    for (int64_t bi = 0; bi < nblk; ++bi) {
      const int64_t b = upper ? bi : (nblk - 1 - bi);
      const int64_t jb = b * TB;
      const int w = (int)((r - jb < TB) ? (r - jb) : TB);
      // off-diagonal update from the already solved columns
      const int64_t t0 = upper ? 0 : jb + w;
      const int64_t t1 = upper ? jb : r;
      if (t1 > t0) {
        MatRef xa{X + t0 * csx, GN_DT_F64, rsx, csx};
        MatRef tm = trans ? MatRef{S + jb * ldt + t0, GN_DT_F64, 1, ldt}
                          : MatRef{S + t0 * ldt + jb, GN_DT_F64, ldt, 1};
        GN_TRY(launch_dgemm(rows, w, t1 - t0, -1.0, xa, tm, 1.0, X + jb * csx, rsx, csx, nullptr,
                            false, s, k, r, want_trunc != 0));
      }
      trsm_diag<<<grid, block, 0, s>>>(rows, r, R, R2, ldt, k, want_trunc, left ? 1 : 0,
                                       r_only ? 1 : 0, X, rsx, csx, jb, w);
      GN_LAUNCH_CHECK();
    }
  }
  return GN_OK;
}

}  // namespace gn
