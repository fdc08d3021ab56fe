// Triangular solves with the GN core factor (Section 5.1: apply R^{-1} by
// substitution, never forming an inverse; Section 5.1.1: R_2^{-T} for the
// truncated core).  Solves X T = B in place for X (rows x r), with the
// triangle chosen on the device from the kept rank k:
//   right products (left = false): T = R (k == r) or T = R2^T (k < r);
//   left products  (left = true) : T = R^T (k == r) or T = R2 (k < r),
// the latter applied to a transposed view of the right-hand sides.
// Blocked by 64 columns: off-diagonal updates with the FP64 GEMM, diagonal
// blocks by one thread per row with the 64 unknowns in registers.
#include "gn_internal.h"

namespace gn {
namespace {

constexpr int TB = 64;

// Diagonal block [jb, jb + w) of X T = B: one thread per row of X holding its w
// unknowns in registers (indices are compile-time after unrolling), T's block
// read from LDS by broadcast, stored column-major (Tt[j][t] = T(t, j)) so that
// each unknown's dot product reads consecutive entries.  UPPER: T upper, forward
// substitution; else lower, backward (each dot product in four interleaved
// partial sums to shorten the dependency chain).  Columns at or beyond the kept size kk are
// set to zero.  The host picks UPPER from (left, truncated, r_only); the gate
// on the device kept rank makes the launch a no-op when it is the other case.
template <bool UPPER>
__global__ void __launch_bounds__(TB) trsm_diag(int64_t rows, int64_t r, const double* __restrict__ R,
                                                const double* __restrict__ R2, int64_t ldt,
                                                const int32_t* __restrict__ kdev, int want_trunc,
                                                int trans, int r_only, double* __restrict__ X,
                                                int64_t rsx, int64_t csx, int64_t jb, int w,
                                                int force_trunc) {
  const int32_t k = *kdev;
  const bool trunc = force_trunc || k < r;
  if (trunc != (want_trunc != 0)) return;
  const double* S = (trunc && !r_only) ? R2 : R;
  const int64_t kk = (k < r) ? k : r;
  __shared__ __attribute__((aligned(16))) double Tt[TB][TB + 2];
  const int tid = threadIdx.x;
  // consecutive threads read consecutive addresses of T's storage
#pragma unroll 16
  for (int q = 0; q < TB; ++q) {
    const int a = q, b = tid;  // a: outer index of the stored row, b: within it
    const int t = trans ? b : a, j = trans ? a : b;
    double v = 0.0;
    if (t < w && j < w) v = trans ? S[(jb + j) * ldt + jb + t] : S[(jb + t) * ldt + jb + j];
    Tt[j][t] = v;
  }
  const int64_t row = (int64_t)blockIdx.x * TB + tid;
  const bool rok = row < rows;
  double x[TB];
#pragma unroll
  for (int j = 0; j < TB; ++j) x[j] = (rok && j < w) ? X[row * rsx + (jb + j) * csx] : 0.0;
  __syncthreads();
  if (UPPER) {
#pragma unroll
    for (int j = 0; j < TB; ++j) {
      double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t = 0; t < j; ++t) a[t & 3] = fma(x[t], Tt[j][t], a[t & 3]);
      const double v = x[j] - ((a[0] + a[1]) + (a[2] + a[3]));
      x[j] = (j < w && jb + j < kk) ? v / Tt[j][j] : 0.0;
    }
  } else {
#pragma unroll
    for (int j = TB - 1; j >= 0; --j) {
      double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t = j + 1; t < TB; ++t) a[t & 3] = fma(x[t], Tt[j][t], a[t & 3]);
      const double v = x[j] - ((a[0] + a[1]) + (a[2] + a[3]));
      x[j] = (j < w && jb + j < kk) ? v / Tt[j][j] : 0.0;
    }
  }
  if (rok) {
#pragma unroll
    for (int j = 0; j < TB; ++j)
      if (j < w) X[row * rsx + (jb + j) * csx] = x[j];
  }
}

}  // namespace

gn_status launch_trsm_core(int64_t rows, int64_t r, const double* R, const double* R2, int64_t ldt,
                           const int32_t* k, double* X, int64_t rsx, int64_t csx, bool left,
                           bool maybe_trunc, hipStream_t s, bool r_only, bool force_trunc) {
  if (rows <= 0) return GN_OK;
  const dim3 grid((unsigned)cdiv(rows, TB)), block(TB);
  const int64_t nblk = cdiv(r, TB);
  // force_trunc: the core is in the factored pseudoinverse form whatever k is;
  // the gate of the off-diagonal products then compares k with r + 1.
  const int64_t gate_n = force_trunc ? r + 1 : r;
  for (int want_trunc = force_trunc ? 1 : 0; want_trunc <= (maybe_trunc || force_trunc ? 1 : 0);
       ++want_trunc) {
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
                            false, s, k, gate_n, want_trunc != 0));
      }
      if (upper)
        trsm_diag<true><<<grid, block, 0, s>>>(rows, r, R, R2, ldt, k, want_trunc, trans ? 1 : 0,
                                               r_only ? 1 : 0, X, rsx, csx, jb, w,
                                               force_trunc ? 1 : 0);
      else
        trsm_diag<false><<<grid, block, 0, s>>>(rows, r, R, R2, ldt, k, want_trunc, trans ? 1 : 0,
                                                r_only ? 1 : 0, X, rsx, csx, jb, w,
                                                force_trunc ? 1 : 0);
      GN_LAUNCH_CHECK();
    }
  }
  return GN_OK;
}

}  // namespace gn
