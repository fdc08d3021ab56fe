// Internal declarations shared by the libgn HIP sources (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/gn.h"

namespace gn {

// ---------------------------------------------------------------------------- errors
#define GN_LAUNCH_CHECK()                                 \
  do {                                                    \
    if (hipGetLastError() != hipSuccess) return GN_ERR_HIP; \
  } while (0)

#define GN_TRY(expr)                 \
  do {                               \
    gn_status s_ = (expr);           \
    if (s_ != GN_OK) return s_;      \
  } while (0)

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ __forceinline__ int64_t cdiv_d(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------------------- Philox4x32-10
// Counter-based generator of Salmon et al. (SC'11): ten rounds of two 32x32->64
// multiplies with Weyl-sequence key increments between rounds.
struct U4 {
  uint32_t a, b, c, d;
};

__device__ __forceinline__ U4 philox10(U4 ctr, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint32_t lo0 = 0xD2511F53u * ctr.a;
    const uint32_t hi0 = __umulhi(0xD2511F53u, ctr.a);
    const uint32_t lo1 = 0xCD9E8D57u * ctr.c;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, ctr.c);
    ctr = U4{hi1 ^ ctr.b ^ k0, lo1, hi0 ^ ctr.d ^ k1, lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return ctr;
}

// ---------------------------------------------------------------------------- bfloat16
// Round a double to bfloat16 (8 significant bits) to nearest, ties to even,
// straight from the FP64 bit pattern.  Valid for zero and for magnitudes in the
// bfloat16 normal range (all values this library rounds).
__device__ __forceinline__ uint16_t f64_to_bf16_bits(double x) {
  uint64_t u = (uint64_t)__double_as_longlong(x);
  const uint64_t keep_lsb = (u >> 45) & 1ull;
  u += (1ull << 44) - 1ull + keep_lsb;
  u &= ~((1ull << 45) - 1ull);
  const float f = (float)__longlong_as_double((long long)u);  // exact
  return (uint16_t)(__float_as_uint(f) >> 16);
}

__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) {
  return __uint_as_float((uint32_t)b << 16);
}

// ---------------------------------------------------------------------------- float16
// Round a double to IEEE binary16 to nearest, ties to even, in one step (no
// intermediate float rounding): |x| < 2^-14 is a multiple of the subnormal unit
// 2^-24 (the scaling by 2^24 is exact, rint rounds to even; 1024 units is the
// smallest normal, encoded by the same bits); otherwise x = f 2^e with f in
// [0.5, 1) keeps q = rint(f 2^11) in [1024, 2048] significant units, the carry
// of q = 2048 running into the exponent field.  65520 and above round to
// infinity, NaN stays NaN.
__device__ __forceinline__ uint16_t f64_to_f16_bits(double x) {
  const uint32_t sign = signbit(x) ? 0x8000u : 0u;
  if (isnan(x)) return (uint16_t)(sign | 0x7e00u);
  const double a = fabs(x);
  if (!(a < 65520.0)) return (uint16_t)(sign | 0x7c00u);
  if (a < 0x1.0p-14) return (uint16_t)(sign | (uint32_t)rint(a * 0x1.0p24));
  int e;
  const double f = frexp(a, &e);
  const uint32_t q = (uint32_t)rint(ldexp(f, 11));
  return (uint16_t)(sign | ((((uint32_t)(e + 14)) << 10) + (q - 1024u)));
}

__device__ __forceinline__ float f16_bits_to_f32(uint16_t b) {
  return (float)__builtin_bit_cast(_Float16, b);
}

// A 16-bit storage element as float: bfloat16 (F16 = false) or binary16.
template <bool F16>
__device__ __forceinline__ float h16_to_f32(uint16_t b) {
  if constexpr (F16)
    return f16_bits_to_f32(b);
  else
    return bf16_bits_to_f32(b);
}

// ---------------------------------------------------------------------------- element traits
template <typename T>
__device__ __forceinline__ double to_f64(T v);
template <>
__device__ __forceinline__ double to_f64<double>(double v) { return v; }
template <>
__device__ __forceinline__ double to_f64<float>(float v) { return (double)v; }
template <>
__device__ __forceinline__ double to_f64<uint16_t>(uint16_t v) { return (double)bf16_bits_to_f32(v); }

// Internal element types: bfloat16- or binary16-rounded values stored as float
// (the 16-bit sketch widened exactly, for the FP32 core product).
constexpr int32_t kDtBf16AsF32 = 100;
constexpr int32_t kDtF16AsF32 = 101;

inline size_t dtype_size(int32_t dt) {
  return dt == GN_DT_F64 ? 8
         : (dt == GN_DT_F32 || dt == kDtBf16AsF32 || dt == kDtF16AsF32) ? 4
                                                                           : 2;
}
inline bool is_h16_mode(int32_t mode) { return mode == GN_MODE_BF16_BS || mode == GN_MODE_F16_BS; }
inline int32_t sketch_dtype(int32_t mode) {
  return mode == GN_MODE_F64   ? GN_DT_F64
         : mode == GN_MODE_F32 ? GN_DT_F32
         : mode == GN_MODE_F16_BS ? GN_DT_F16
                                  : GN_DT_BF16;
}
inline int32_t accum_dtype(int32_t mode) { return mode == GN_MODE_F64 ? GN_DT_F64 : GN_DT_F32; }

inline int64_t next_pow2(int64_t n) {
  int64_t p = 1;
  while (p < n) p <<= 1;
  return p;
}

// ---------------------------------------------------------------------------- launchers
// sketch_gen.hip
gn_status launch_gaussian(uint64_t seed, int32_t stream_id, int64_t row0, int64_t col0,
                          int64_t rows, int64_t cols, int32_t dtype, int32_t layout, void* out,
                          int64_t ld, hipStream_t s);
gn_status launch_srht(uint64_t seed, int64_t npad, int64_t r, int8_t* signs, int32_t* idx,
                      uint64_t* keys_ws, hipStream_t s);
gn_status launch_transpose(const void* in, int64_t rows, int64_t cols, int64_t ldi, int32_t dtype,
                           void* out, int64_t ldo, hipStream_t s);
size_t srht_ws_bytes(int64_t npad);
// out (rows x r, FP64, ld ldo) = B D H S for B (rows x n, FP32, ld ldb), the SRHT
// with the signs and sampled columns of launch_srht, transformed in FP64.
gn_status launch_srht_right(int64_t rows, int64_t n, int64_t r, const float* B, int64_t ldb,
                            const int8_t* signs, const int32_t* idx, double* out, int64_t ldo,
                            hipStream_t s);
// Batched row-major Gaussian blocks (rows x cols from (0, 0), stream sid, seed)
// in GN_DT_F64 or GN_DT_F32.
struct GaussJob {
  uint64_t seed;
  int64_t sid;
  int64_t rows, cols;
  void* out;
  int64_t ld;
};
gn_status launch_gaussian_batched(const GaussJob* jobs, int32_t count, int32_t dtype, hipStream_t s);

// pass.hip : the sketch pass, AX (m x r) and Y^T A (rl x n) from one launch in
// FP32 and BF16 modes.  Xt is the transposed Gaussian or user sketch (r x n,
// ld n; unused for SRHT), Yt the transposed Y (rl x m, ld m); signs / idx the
// SRHT parameters (SRHT X only).
// split_ws (pass_split_ws_bytes) lets an FP32 Gaussian pass with few output
// tiles split K; without it (or too small) the pass runs unsplit.
gn_status launch_pass(int32_t mode, int32_t kind_x, int64_t m, int64_t n, int64_t r, int64_t rl,
                      const void* A, int64_t lda, const float* scales, const void* Xt,
                      const int8_t* signs, const int32_t* idx, const void* Yt, void* AX,
                      int64_t ldax, void* YtA, int64_t ldya, hipStream_t s,
                      void* split_ws = nullptr, size_t split_bytes = 0);
size_t pass_split_ws_bytes(int32_t mode, int32_t kind_x, int64_t m, int64_t n, int64_t r,
                           int64_t rl);

// K splitting of FP32 products with few output tiles: a slice length kslice (a
// multiple of kSplitMinSlice) chosen by a wave-quantized cost model.
struct SplitK {
  int64_t slices, kslice;
};
constexpr int64_t kSplitMinTiles = 192;  // at or above: no split
constexpr int64_t kSplitTargetWG = 256;  // one 1024-thread workgroup per CU
constexpr int64_t kSplitMinSlice = 512;
SplitK f32_split(int64_t tiles, int64_t K);
// Two families sharing one slice length (kslice == 0: no split).
SplitK f32_split2(int64_t tiles1, int64_t K1, int64_t tiles2, int64_t K2);
// D[i*ldd + j] = sum over nslice partials (each M x N, row stride N) in slice
// order in FP64, rounded to float.
// FP32 pass with an SRHT X when r + l <= 16, n % 4 == 0, n' >= 1024 and A is
// 16-byte aligned with lda % 4 == 0: one read of A (each wave one 256-column
// chunk: the order-256 Walsh-Hadamard transform and the Y^T A product on the
// matrix cores from the same registers), per-chunk and per-row-range partial
// sums in ws added in a fixed order.  GN_ERR_UNSUPPORTED (nothing enqueued)
// when the shape or ws (narrow_srht_ws_bytes) does not fit.
size_t narrow_srht_ws_bytes(int64_t m, int64_t n, int64_t r, int64_t rl);
gn_status launch_f32_srht_narrow(int64_t m, int64_t n, int64_t r, int64_t rl, const float* A,
                                 int64_t lda, const float* Y, const int8_t* signs,
                                 const int32_t* idx, float* AX, int64_t ldax, float* YtA,
                                 int64_t ldya, void* ws, size_t ws_bytes, hipStream_t s);

// The same single read of A for a Gaussian (dense) X, n x r with ld r, when
// r + l <= 16, n % 4 == 0, n >= 1024 and A is 16-byte aligned with lda % 4 == 0:
// Y^T A on the matrix cores as above, AX from the same loaded values staged
// through LDS (16 rows at a time) on the matrix cores; partials in ws
// (narrow_gauss_ws_bytes) added in a fixed order.  GN_ERR_UNSUPPORTED (nothing
// enqueued) when the shape or ws does not fit.
size_t narrow_gauss_ws_bytes(int64_t m, int64_t n, int64_t r, int64_t rl);
gn_status launch_f32_gauss_narrow(int64_t m, int64_t n, int64_t r, int64_t rl, const float* A,
                                  int64_t lda, const float* X, const float* Y, float* AX,
                                  int64_t ldax, float* YtA, int64_t ldya, void* ws,
                                  size_t ws_bytes, hipStream_t s);

gn_status launch_splitk_sum_f32(const float* partial, int64_t nslice, int64_t M, int64_t N,
                                float* D, int64_t ldd, hipStream_t s);

// C ((rl) x r, FP64, ld r) = Y^T (AX) on the FP32 matrix cores: Y m x rl (ld
// ldy), AX m x r (ld ldax), both float; K = m split into slices whose FP32
// partial products (core_product_ws_bytes) are summed in FP64 in slice order.
gn_status launch_core_product_f32(int64_t m, int64_t rl, int64_t r, const float* Y, int64_t ldy,
                                  const float* AX, int64_t ldax, float* partial, double* C,
                                  hipStream_t s);
size_t core_product_ws_bytes(int64_t m, int64_t rl, int64_t r);
// BF16 / FP16 modes: C (rl x r, FP64) = Y^T (AX) with Yt (rl x m, bfloat16 or
// binary16 bits (f16), ld m) on the 16-bit matrix cores, AX split into two terms
// of that format (for binary16 after each column is divided by a power of two);
// ws: core_product_bf16_ws_bytes.
gn_status launch_core_product_h16(int64_t m, int64_t rl, int64_t r, const uint16_t* Yt, bool f16,
                                  const float* AX, int64_t ldax, void* ws, double* C,
                                  hipStream_t s);
size_t core_product_bf16_ws_bytes(int64_t m, int64_t rl, int64_t r);
// D (M x N, FP32) = A (M x K) B (K x N), FP32 MFMA with FP32 accumulation.
// a_kc: A(i,k) = A[i*lda + k], else A[k*lda + i]; b_kc: B(k,j) = B[j*ldb + k],
// else B[k*ldb + j].  With split_ws (gemm_f32_split_ws_bytes) a product with few
// output tiles is split along K.
gn_status launch_gemm_f32(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda, bool a_kc,
                          const float* B, int64_t ldb, bool b_kc, float* D, int64_t ldd,
                          hipStream_t s, float* split_ws = nullptr, size_t split_bytes = 0);
size_t gemm_f32_split_ws_bytes(int64_t M, int64_t N, int64_t K);
// widen a bfloat16 (f16 = false) or binary16 matrix (rows x cols, ld lds) to
// float (ld ldd)
gn_status launch_widen_h16(int64_t rows, int64_t cols, const uint16_t* src, int64_t lds, bool f16,
                           float* dst, int64_t ldd, hipStream_t s);

// dgemm.hip : FP64 strided GEMM  D = alpha * op(A) op(B) + beta * D
struct MatRef {
  const void* p;
  int32_t dtype;   // gn_dtype of the stored elements
  int64_t rs, cs;  // element (i, j) at p[i*rs + j*cs]
};
// kmask: when non-null, rows (mask_rows) or columns (!mask_rows) of D with index
// >= *kmask are written as zero (used to zero factors beyond the kept rank).
// gate: when non-null the kernel does nothing unless (*gate < gate_n) == gate_trunc
// (launches that only matter for a truncated / untruncated core).
// split_ws: optional scratch for splitting a long K over more workgroups
// (dgemm_split_ws_bytes(M, N, K) bytes); the slices are summed in fixed order.
gn_status launch_dgemm(int64_t M, int64_t N, int64_t K, double alpha, MatRef A, MatRef B,
                       double beta, double* D, int64_t rsd, int64_t csd, const int32_t* kmask,
                       bool mask_rows, hipStream_t s, const int32_t* gate = nullptr,
                       int64_t gate_n = 0, bool gate_trunc = true, double* split_ws = nullptr,
                       size_t split_ws_bytes = 0);
size_t dgemm_split_ws_bytes(int64_t M, int64_t N, int64_t K);
// The same product with D stored as d_dtype (GN_DT_F64 or GN_DT_F32, rounded to
// nearest; beta * D is read in that dtype).
gn_status launch_dgemm_to(int64_t M, int64_t N, int64_t K, double alpha, MatRef A, MatRef B,
                          double beta, void* D, int32_t d_dtype, int64_t rsd, int64_t csd,
                          const int32_t* kmask, bool mask_rows, hipStream_t s,
                          const int32_t* gate = nullptr, int64_t gate_n = 0,
                          bool gate_trunc = true, double* split_ws = nullptr,
                          size_t split_ws_bytes = 0);
// Per-tile sums of (Ref - A*B)^2 written to partial[], then reduced in fixed order.
gn_status launch_residual(int64_t M, int64_t N, int64_t K, MatRef Ref, const float* ref_scales,
                          MatRef A, MatRef B, double* partial, double* out, hipStream_t s);
size_t residual_ws_bytes(int64_t M, int64_t N);

// qr.hip : Householder QR of an M x N FP64 matrix (M >= N, M <= 4096), in place
// (the factored matrix keeps R above and the reflectors below its diagonal).
// R (N x N, ld ldr, R_ii >= 0 after the sign fix) and the explicit Q (M x N,
// ld ldq) are written out.  When gate_k is non-null, every kernel returns
// immediately unless *gate_k < N (the second QR, needed only when truncated).
gn_status launch_qr(int64_t M, int64_t N, double* Aq, int64_t lda, double* Q, int64_t ldq,
                    double* R, int64_t ldr, double* ws, const int32_t* gate_k, hipStream_t s);
// launch_qr in two parts on possibly different streams: the factorization with R,
// then the explicit Q (which reads the factored matrix and the block reflectors'
// T factors kept in ws, so it must follow the first part, with the same ws).
gn_status launch_qr_factor(int64_t M, int64_t N, double* Aq, int64_t lda, double* R, int64_t ldr,
                           double* ws, const int32_t* gate_k, hipStream_t s);
gn_status launch_qr_form_q(int64_t M, int64_t N, const double* Aq, int64_t lda, double* Q,
                           int64_t ldq, double* ws, const int32_t* gate_k, hipStream_t s);
size_t qr_ws_bytes(int64_t M, int64_t N);

// Batched QR: job z factors C (M x N, M <= 512) in place, writes Q, R (R_ii >=
// 0) and uses T (qr_batch_t_bytes(N)) and Wp (qr_batch_wp_bytes(M, N)) as
// scratch; a job is skipped unless !gate || *gate < gate_n.
struct QrJob {
  int64_t M, N;
  double* C;
  int64_t ldc;
  double* Q;
  int64_t ldq;
  double* R;
  int64_t ldr;
  double* T;
  double* Wp;
  const int32_t* gate;
  int64_t gate_n;
};
size_t qr_batch_t_bytes(int64_t N);
size_t qr_batch_wp_bytes(int64_t M, int64_t N);
gn_status launch_qr_batched(const QrJob* jobs, int32_t count, int64_t maxM, int64_t maxN,
                            hipStream_t s);
// Batched truncation scan (k, status) and Z = [R[:k, :]^T, 0] (when k < r).
struct TruncJob {
  int64_t r;
  const double* R;
  int64_t ldr;
  double tau;
  int32_t* k;
  int32_t* status;
  double* Z;
  int64_t ldz;
};
gn_status launch_truncate_batched(const TruncJob* jobs, int32_t count, int64_t maxr,
                                  hipStream_t s);
// k = prefix count of |R_ii| >= tau; status flags; builds R[:k,:]^T (r x r,
// zero beyond column k) in Z.
gn_status launch_truncate(int64_t r, const double* R, int64_t ldr, double tau, int32_t* k,
                          int32_t* status, double* Z, int64_t ldz, hipStream_t s);

// trsm.hip : right-side triangular solves with the kept-rank factor.
// Solves Xo * T = B for Xo (rows x r) where T = R (upper, when *k == r) or
// T = R2^T (lower, when *k < r, only the leading k columns); columns >= k of
// Xo are zero.  B and Xo may alias.  side handled by strides.
// left = false: X T = B with T = R (k == r) or T = R2^T (k < r): X = B R^{-1} or
//               B R2^{-T}  (right-side products with the core pseudoinverse).
// left = true : X T = B with T = R^T (k == r) or T = R2 (k < r): the transpose
//               of R^{-1} B^T or R2^{-T} B^T (left-side products), on a
//               transposed view of the data.
// Columns >= k of X are zeroed when k < r.  Solved in place on X (rows x r).
// r_only = true: both cases use the leading kk x kk block of R (kk = r, or k
// when k < r), transposed when left: X R^{-1} or X R_11^{-T} on the kept columns.
gn_status launch_trsm_core(int64_t rows, int64_t r, const double* R, const double* R2, int64_t ldt,
                           const int32_t* k, double* X, int64_t rsx, int64_t csx, bool left,
                           bool maybe_trunc, hipStream_t s, bool r_only = false,
                           bool force_trunc = false);

// stabilize.hip : the other Section 5.1.1 stabilizations and the Section 5.1.2
// check.  R (r x r, ld ldr) and Q1 ((r+l) x r, ld r) are C's QR; the outputs
// follow gn_core_out for the method.  R may alias Rp.
size_t stabilize_ws_bytes(int32_t method, int64_t r);
gn_status launch_svd_core(int64_t r, int64_t rl, const double* R, int64_t ldr, const double* Q1,
                          double tau, int lift, int32_t* k, int32_t* status, double* Q1_out,
                          double* Q2, double* R2, void* ws, hipStream_t s);
gn_status launch_rrqr_core(int64_t r, int64_t rl, const double* R, int64_t ldr, const double* Q1,
                           double tau, int32_t* k, int32_t* status, double* Q1_out, double* Rp,
                           double* Q2, double* R2, void* ws, hipStream_t s);
gn_status launch_lift_diag(int64_t r, double* R, int64_t ldr, double tau, int32_t* k,
                           int32_t* status, hipStream_t s);
size_t power_ws_bytes(int64_t r, int32_t nv);
// X T = B for at most small_solve_max_rhs() right-hand sides (rows of X): the same
// triangle and gating as launch_trsm_core (left product: T = R^T, or R2 when
// truncated or forced; right product: T = R, or R2^T), solved with inverted 64 x 64
// diagonal blocks, one launch per block, the off-diagonal updates spread over
// workgroups.  launch_small_solve_prep (the block inverses and the transposed
// factor, from R, R2 and k only) must precede launch_small_solve on the same ws,
// possibly from another stream.  ws: small_solve_ws_bytes(r).
size_t small_solve_ws_bytes(int64_t r);
int64_t small_solve_max_rhs();
gn_status launch_small_solve_prep(int64_t r, const double* R, const double* R2, const int32_t* k,
                                  bool force, void* ws, hipStream_t s);
gn_status launch_small_solve(int64_t r, const double* R, const double* R2, const int32_t* k,
                             bool force, bool left, double* X, int64_t nrhs, int64_t rsx,
                             int64_t csx, void* ws, hipStream_t s);
// force_trunc: the core is in the factored form Q2 R2^{-T} Q1^T whatever k is.
gn_status launch_power_check(int64_t r, uint64_t seed, int32_t nv, int32_t iters,
                             const double* R, const double* R2, const int32_t* k, bool force_trunc,
                             double tau_d, int32_t* status, double* est_out, void* ws,
                             hipStream_t s);

// grad.hip : helpers of the reverse mode.
// out (cols x rows) = src^T with rows >= *k of out zeroed (src rows x cols).
gn_status launch_transpose_rows_masked(int64_t rows, int64_t cols, const double* src, int64_t lds,
                                       const int32_t* k, double* out, int64_t ldo, hipStream_t s);
// dst += src (rows x cols) in GN_DT_F64 or GN_DT_F32.
gn_status launch_add(int64_t rows, int64_t cols, int32_t dt, const void* src, int64_t lds, void* dst,
                     int64_t ldd, hipStream_t s);
// Y += alpha X (rows x cols, FP64).
gn_status launch_axpy(int64_t rows, int64_t cols, double alpha, const double* X, int64_t ldx,
                      double* Y, int64_t ldy, hipStream_t s);

// quant.hip
// f16: binary16 storage instead of bfloat16
gn_status launch_quantize(int64_t m, int64_t n, const void* A, int64_t lda, int32_t dtype,
                          uint16_t* out, int64_t ldo, float* scales, hipStream_t s, bool f16);

}  // namespace gn
