/*
 * gn.h -- C ABI of libgn, an MI355X (gfx950) library for generalized Nystrom
 * (GN) low-rank approximation (Y. Nakatsukasa, "Fast and stable randomized
 * low-rank matrix approximation", arXiv:2009.11392).
 *
 * GN approximates A (m x n) by  A_hat = AX (Y^T A X)_eps^+ Y^T A  with a sketch
 * X (n x r) and an oversampled sketch Y (m x (r+l))  (Section 2, eqs. (3)-(4);
 * Algorithm 2.1).  The library computes, on one GPU:
 *   gn_generate_gaussian / gn_srht_generate  -- the random sketches,
 *   gn_sketch_prepare / gn_sketch_pass / gn_sketch -- the sketches and the
 *                   single pass over A that forms AX and Y^T A,
 *   gn_core       -- C = Y^T (AX), its Householder QR and the eps-truncation,
 *   gn_factors / gn_apply -- the factored approximant, products with it, and
 *                   the approximant itself,
 *   gn_backward   -- the reverse mode: dL/dA from dL/dA_hat,
 *   gn_residual   -- ||A - F G||_F^2 formed tile by tile (error measurement),
 *   gn_quantize_bf16_bs / gn_quantize_f16_bs -- bfloat16 or binary16 storage of
 *                   A with power-of-two block scales.
 *
 * Conventions (every entry point):
 *   * Pointers are device pointers unless marked (host).  All matrices are
 *     row-major; "ld" arguments are row strides in elements.
 *   * The caller owns every buffer, including the workspace `ws`; the library
 *     never allocates or frees device memory.  Its only state is one more stream
 *     (non-blocking, default priority) and two events per device, created at the
 *     first gn_core / gn_apply / gn_backward call on that device and kept until the
 *     process ends: those calls run independent parts of their work (the kept-rank
 *     scan and second QR; the solve's block inverses; the reverse mode's solves and
 *     products that need only the forward's core, then its U and V products) on
 *     it, joined back to `stream`
 *     by an event before returning, so work enqueued later on `stream` sees every
 *     result (the fork and join are also recorded under stream capture).
 *   * Arguments are validated synchronously; on an error the call returns
 *     before anything is enqueued.  Otherwise the work is enqueued on `stream`
 *     and the call returns without synchronizing.  GN_ERR_HIP reports a failed
 *     kernel launch.  Numeric conditions found on the device (a non-finite R
 *     diagonal, kept rank 0) are reported through the device status word of
 *     gn_core_out, never by aborting.
 *   * Calls are reentrant; calls on different streams with disjoint buffers may
 *     run concurrently (the forks above are serialized by a host mutex, and their
 *     side-stream parts run one after the other).
 */
#ifndef GN_H_
#define GN_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* gn_stream_t; /* a hipStream_t; NULL = default stream */

typedef enum {
  GN_OK = 0,
  GN_ERR_ARG = 1,        /* null pointer, bad enum value, eps/nu not finite     */
  GN_ERR_SHAPE = 2,      /* inconsistent m, n, r, l, ld                          */
  GN_ERR_DTYPE = 3,      /* dtype not valid for this mode / entry point          */
  GN_ERR_ALIGN = 4,      /* pointer not 16-byte aligned                          */
  GN_ERR_WORKSPACE = 5,  /* ws too small (query gn_workspace_size)               */
  GN_ERR_HIP = 6,        /* a HIP launch or runtime call failed                  */
  GN_ERR_NUMERIC = 7,    /* (status word only) non-finite or rank-0 core         */
  GN_ERR_UNSUPPORTED = 8 /* size or mode beyond what the library handles       */
} gn_status;

typedef enum { GN_SKETCH_GAUSSIAN = 0, GN_SKETCH_SRHT = 1, GN_SKETCH_USER = 2 } gn_sketch_kind;

/* Storage / contraction precision of A, X, Y in the sketch pass.  The core
 * (QR, truncation, triangular solves, products with the factors) is FP64 in
 * every mode. */
typedef enum {
  GN_MODE_F64 = 0,     /* A, X, Y double; AX, Y^T A double (FP64 accumulation)      */
  GN_MODE_F32 = 1,     /* A, X, Y float;  AX, Y^T A float  (FP32 accumulation)      */
  GN_MODE_BF16_BS = 2, /* A bfloat16 with one float scale per 128x128 block,
                          X, Y bfloat16; AX, Y^T A float (FP32 accumulation)        */
  GN_MODE_F16_BS = 3   /* A IEEE binary16 with one float scale per 128x128 block
                          (which keeps small entries out of the binary16 subnormal
                          range), X, Y binary16; AX, Y^T A float (FP32 accumulation) */
} gn_mode;

typedef enum { GN_DT_F64 = 0, GN_DT_F32 = 1, GN_DT_BF16 = 2, GN_DT_F16 = 3 } gn_dtype;

/* How gn_core stabilizes the core pseudoinverse (Section 5.1.1).  tau is the
 * threshold of gn_problem; the perturbations (LIFT_*) need eps > 0.
 *   QR        : truncated QR: keep the prefix of |R_ii| >= tau, then the QR of
 *               R[:k, :]^T (the method of the paper's experiments; default).
 *   SVD       : the SVD of the core, singular values below tau dropped.
 *   LIFT_SVD  : perturbation (a): singular values below tau raised to tau.
 *   LIFT_RRQR : perturbation (b): QR with column pivoting, diagonal entries of
 *               R below tau in magnitude raised to tau.
 *   LIFT_DIAG : perturbation (c): the unpivoted R's diagonal entries below tau
 *               raised to tau.
 * gn_backward and the batched solves support QR only. */
typedef enum {
  GN_CORE_QR = 0,
  GN_CORE_SVD = 1,
  GN_CORE_LIFT_SVD = 2,
  GN_CORE_LIFT_RRQR = 3,
  GN_CORE_LIFT_DIAG = 4
} gn_core_method;

/* Problem statement (Algorithm 2.1 inputs: A's shape, r, l, eps, sketch type,
 * seed).  l < 0 selects l = ceil(r/2) (Algorithm 2.1, step 1); l = 0 means no
 * oversampling (the Nystrom and HMT special cases with USER sketches).  Requires
 * 1 <= r <= min(m, n); r + l <= 4096 (core QR held on chip).  eps is absolute,
 * in units of A (Section 2: eps = O(u ||A||)); the core keeps the leading k
 * columns whose |R_ii| >= tau = eps * nu_x * nu_y, where nu_x, nu_y are the
 * sketch norm scales (<= 0 selects sqrt(rows)+sqrt(cols) for a Gaussian and
 * sqrt(n') for an SRHT; USER sketches should pass their own).  eps <= 0 means
 * plain GN: no truncation unless a diagonal entry is zero or not finite. */
typedef struct {
  int64_t m, n, r, l;
  int32_t kind_x;   /* gn_sketch_kind: GAUSSIAN, SRHT or USER             */
  int32_t kind_y;   /* gn_sketch_kind: GAUSSIAN or USER                   */
  uint64_t seed;    /* Philox4x32-10 key for X, Y and the SRHT            */
  int32_t mode;     /* gn_mode                                            */
  int32_t core_method; /* gn_core_method (0 = truncated QR)                */
  double eps, nu_x, nu_y;
} gn_problem;

/* Output of gn_core.  k and status live in device memory so that nothing on
 * the path synchronizes; read them back only when needed.
 *   k      : kept rank, 0 <= k <= r.
 *   status : bit flags, 0 = fine.  1 = non-finite diagonal or singular value,
 *            2 = k == 0 (both are GN_ERR_NUMERIC conditions), 4 = some |R_jj| >=
 *            tau after the first diagonal below tau (QR method; diagnostic: the
 *            QR was not rank revealing there), 8 = set by gn_core_check, 16 =
 *            something was raised to tau (LIFT_* methods), 32 = the Jacobi SVD
 *            stopped at its sweep limit (SVD, LIFT_SVD).
 * The buffers (all FP64, row-major, ld r): Q1 (r+l) x r, R, Q2, R2 r x r.
 *   QR        : Q1, R = the Householder QR of C = Y^T (AX) with R_ii >= 0; k =
 *               the prefix of |R_ii| >= tau; when k < r, Q2 and R2 are the QR
 *               factors of R[:k,:]^T (Q2: first k columns; R2: upper k x k
 *               block, R2_ii >= 0), and as R[:k,:] = R2^T Q2^T the
 *               eps-pseudoinverse of C is Q2 R2^{-T} Q1[:, :k]^T.  When k == r
 *               Q2 and R2 are left unchanged and unused, the inverse is R^{-1} Q1^T.
 *   SVD, LIFT_SVD : C = Q1 diag(s) Q2^T with the singular values s descending:
 *               Q1 the left and Q2 the right singular vectors, R2 = diag(s)
 *               (LIFT_SVD: diag(max(s, tau))), R the R of C's QR; k = the count of
 *               s >= tau (SVD) or r (LIFT_SVD).
 *   LIFT_RRQR : C P = Q1 R with column pivoting (R = the pivoted R before
 *               lifting); the lifted R equals R2^T Q3^T and Q2 = P Q3; k = r.
 *   LIFT_DIAG : Q1, R the QR of C with R's diagonal raised to tau; k = r; Q2, R2
 *               unused.
 * SVD, LIFT_SVD and LIFT_RRQR cores are always applied as Q2 R2^{-T} Q1[:, :k]^T. */
typedef struct {
  int32_t* k;
  int32_t* status;
  double* Q1;
  double* R;
  double* Q2;
  double* R2;
} gn_core_out;

/* Operations for gn_workspace_size. */
typedef enum {
  GN_OP_SKETCH = 0,
  GN_OP_CORE = 1,
  GN_OP_FACTORS = 2,
  GN_OP_APPLY = 3,     /* with kcols = the number of right-hand sides         */
  GN_OP_RESIDUAL = 4,
  GN_OP_SRHT = 5,
  GN_OP_BACKWARD = 6,  /* gn_backward                                          */
  GN_OP_MATERIALIZE = 7, /* gn_apply side 2                                    */
  GN_OP_UPDATE = 8,    /* gn_sketch_extend / _append / _update (p = the enlarged problem) */
  GN_OP_CHECK = 9      /* gn_core_check, with kcols = nv                      */
} gn_op;

/* Bytes of device workspace the given operation needs for problem p.  For
 * GN_OP_APPLY, kcols is the number of columns (side 0) or rows (side 1) of W;
 * it is ignored otherwise. */
gn_status gn_workspace_size(const gn_problem* p /*host*/, int32_t op, int64_t kcols,
                            size_t* bytes /*host*/);

/* Gaussian sketch block G[row0 + i, col0 + j] for 0 <= i < rows, 0 <= j < cols,
 * i.i.d. N(0,1) (Section 3.1) from Philox4x32-10: element (i, j) of stream s
 * takes the Box-Muller pair of the Philox block at counter (i, j >> 1, s, 0)
 * with key (seed lo, seed hi), z0 for even j and z1 for odd j, computed in FP64
 * and rounded to nearest-even into `dtype`.  layout 0 writes out[i*ld + j],
 * layout 1 writes the transpose out[j*ld + i].  Streams: 1 = X, 2 = Y. */
gn_status gn_generate_gaussian(uint64_t seed, int32_t stream, int64_t row0, int64_t col0,
                               int64_t rows, int64_t cols, int32_t dtype, int32_t layout,
                               void* out, int64_t ld, gn_stream_t stream_);

/* SRHT sketch parameters (Section 1): X = the first n rows of D H S, with H the
 * Sylvester-ordered Walsh-Hadamard matrix of order n' = next power of two >= n,
 * D = diag(signs), S the r sampled columns.  signs (n' int8, +1/-1): the top bit
 * of word (i & 3) of the Philox block at (i >> 2, 0, 3, 0).  idx (r int32): the
 * columns with the r smallest 64-bit keys (key_j from words 2b, 2b+1, b = j & 1,
 * of the block at (j >> 1, 0, 4, 0)), in ascending (key, j) order.  Needs
 * gn_workspace_size(GN_OP_SRHT) bytes of ws.  n' <= 2^17, r <= n'. */
gn_status gn_srht_generate(uint64_t seed, int64_t n, int64_t r, int8_t* signs, int32_t* idx,
                           void* ws, size_t ws_bytes, gn_stream_t stream);

/* Sketches for the pass (Algorithm 2.1, step 1), written into the workspace
 * ws (gn_workspace_size(GN_OP_SKETCH) bytes), which gn_sketch_pass then reads:
 * Gaussian X (stream 1) and Y (stream 2) drawn on the device from `seed` in the
 * mode's sketch dtype (double, float, bfloat16 or binary16), or the USER matrices
 * X_user (n x r, ld ldx) / Y_user (m x (r+l), ld ldy) in that dtype, or for an
 * SRHT X its signs and sample (copied to signs_out / idx_out when non-NULL, as
 * in gn_srht_generate).  One prepared workspace serves any number of passes
 * over matrices of the same problem shape. */
gn_status gn_sketch_prepare(const gn_problem* p, const void* X_user, int64_t ldx,
                            const void* Y_user, int64_t ldy, int8_t* signs_out, int32_t* idx_out,
                            void* ws, size_t ws_bytes, gn_stream_t stream);

/* The sketch pass (Algorithm 2.1, step 2): AX (m x r) and Y^T A ((r+l) x n)
 * from A (m x n, row stride lda >= n), with the sketches of a prepared ws.
 * In FP32 mode both products run in one kernel launch; in BF16 and F16 modes the
 * large-r Gaussian pass is one launch per product.  For small r the pass reads A
 * once (r + l <= 16, FP32: SRHT or Gaussian X) or takes narrow tiles (FP32
 * r <= 512 and r + l <= 768, 16-bit r <= 64, Gaussian X).
 *   A        : mode dtype (double, float, or bfloat16 / binary16 bits for
 *              BF16_BS / F16_BS).
 *   A_scales : BF16_BS and F16_BS only: float[ceil(m/128) * ceil(n/128)], row-major, the
 *              scale of each 128 x 128 block (A = scale * stored value).
 *   AX, YtA  : outputs in the accumulation dtype (double for F64, float else),
 *              row strides ldax >= r and ldya >= n.
 * All pointers 16-byte aligned.  When the problem has too few output tiles to
 * fill the GPU (FP64 and FP32 modes, the narrow tiles of the 16-bit modes), and
 * on the single-read paths (per-chunk and per-row-range partials), partial
 * products go to a scratch region at the end of ws and are summed in a fixed
 * order (deterministic): passes that run concurrently need separate workspaces. */
gn_status gn_sketch_pass(const gn_problem* p, const void* A, int64_t lda, const float* A_scales,
                         void* AX, int64_t ldax, void* YtA, int64_t ldya, void* ws,
                         size_t ws_bytes, gn_stream_t stream);

/* gn_sketch_prepare followed by gn_sketch_pass, with the arguments of both. */
gn_status gn_sketch(const gn_problem* p, const void* A, int64_t lda, const float* A_scales,
                    const void* X_user, int64_t ldx, const void* Y_user, int64_t ldy,
                    void* AX, int64_t ldax, void* YtA, int64_t ldya, int8_t* signs_out,
                    int32_t* idx_out, void* ws, size_t ws_bytes, gn_stream_t stream);

/* The core (Algorithm 2.1 step 2 and Section 5.1.1): C = Y^T (AX) accumulated
 * in FP64 (Y regenerated from the seed unless kind_y == USER), Householder QR
 * C = Q R with R_ii >= 0, then the stabilization p->core_method selects: the
 * kept rank k and, when k < r, the QR of R[:k,:]^T (QR); the SVD of R by
 * one-sided Jacobi (SVD, LIFT_SVD; r <= 4096); QR with column pivoting of R
 * followed by two QRs (LIFT_RRQR); or R's diagonal raised (LIFT_DIAG).  See
 * gn_core_out for what each leaves in `out`.  AX as produced by gn_sketch (ld
 * ldax).  YtA (ld ldya >= n, 16-byte aligned) may be NULL; when it is given
 * with an SRHT X in FP32, BF16 or F16 mode, C is formed as (Y^T A) X instead: the
 * r + l rows of Y^T A sign-flipped, Walsh-Hadamard transformed and sampled in
 * FP64 (Section 2.3 costs the core this way, O(n (r + l) log n) instead of the
 * O(m r (r + l)) product; Y is then not regenerated), and in every other case it
 * is ignored.  The cost beyond the QR is O(r^3) for SVD / LIFT_SVD (a few sweeps
 * of r^3 rotations) and LIFT_RRQR (2 r launches for the pivot order, two QRs). */
gn_status gn_core(const gn_problem* p, const void* AX, int64_t ldax, const void* YtA,
                  int64_t ldya, const void* Y_user, int64_t ldy,
                  const gn_core_out* out /*host struct of device ptrs*/, void* ws,
                  size_t ws_bytes, gn_stream_t stream);

/* Section 5.1.2: check a core for the instability plain GN can show.  A power
 * method estimates ||T^{-1}||_2 for T the triangular factor whose inverse
 * multiplies AX in gn_factors / gn_apply (R, or R2^T for a truncated or
 * factored core): nv start vectors (Philox stream 6 of p->seed; the first k
 * entries of each row of an nv x r Gaussian block) are normalized and driven
 * through y = T^{-T} v, z = T^{-1} y, v = z / ||z|| for `iters` steps of two
 * triangular solves (O(nv r^2) each).  The estimate, the largest ||y||, is a
 * lower bound of ||T^{-1}||_2.  When est * delta * nu_x * nu_y > 1 (delta <= 0
 * selects p->eps; both <= 0 is GN_ERR_ARG) bit 8 of core->status is set: the
 * core has a singular value below the threshold SGN with eps = delta would
 * truncate at, and the caller should switch to an SGN core.  est (device
 * double, or NULL) receives the estimate.  1 <= nv <= 16, 1 <= iters <= 64.
 * Workspace: gn_workspace_size(p, GN_OP_CHECK, nv). */
gn_status gn_core_check(const gn_problem* p, const gn_core_out* core /*host struct*/, double delta,
                        int32_t nv, int32_t iters, double* est, void* ws, size_t ws_bytes,
                        gn_stream_t stream);

/* The factored approximant A_hat = F G in FP64 (Section 5.1, the stable order):
 *   k == r : F = (AX) R^{-1} by triangular solves,  G = Q1^T (Y^T A)
 *   k <  r : F = (AX Q2) R2^{-T},                   G = Q1[:, :k]^T (Y^T A)
 * (the second form whatever k is for SVD, LIFT_SVD and LIFT_RRQR cores)
 * F is m x r (ld ldf), G is r x n (ld ldg); columns of F and rows of G beyond
 * k are set to zero.  Forming F costs O(m r^2) (the paper advises it only for
 * evaluation); use gn_apply for products. */
gn_status gn_factors(const gn_problem* p, const void* AX, int64_t ldax, const void* YtA,
                     int64_t ldya, const gn_core_out* core, double* F, int64_t ldf, double* G,
                     int64_t ldg, void* ws, size_t ws_bytes, gn_stream_t stream);

/* Products with the approximant in the order of Section 2 (after Alg. 2.1):
 *   side 0: out (m x kcols, ld ldo) = A_hat W,  W n x kcols (ld ldw),
 *           evaluated as AX (R^{-1} (Q^T (Y^T A W)));
 *   side 1: out (kcols x n, ld ldo) = W A_hat,  W kcols x m (ld ldw),
 *           evaluated as (((W AX) R^{-1}) Q^T) Y^T A;
 * (with Q2 R2^{-T} in place of R^{-1} when k < r); W and out are double.
 *   side 2: out (m x n, ld ldo) = A_hat itself, F G with the factors of
 *           gn_factors, in the mode's accumulation dtype (double in F64 mode,
 *           float otherwise); W and kcols are ignored; workspace
 *           gn_workspace_size(GN_OP_MATERIALIZE).  Costs O(mnr): for
 *           evaluation and for callers (autograd) that need A_hat as a tensor. */
gn_status gn_apply(const gn_problem* p, int32_t side, const void* AX, int64_t ldax,
                   const void* YtA, int64_t ldya, const gn_core_out* core, const double* W,
                   int64_t ldw, int64_t kcols, void* out, int64_t ldo, void* ws,
                   size_t ws_bytes, gn_stream_t stream);

/* Reverse mode of the approximant.  For L with dL/dA_hat = Gbar (m x n, ld ldg),
 * writes dA = dL/dA (m x n, ld ldda) for the map A -> A_hat = AX M Y^T A with
 * M = R_1^+ Q_1^T the eps-truncated core pseudoinverse (Section 5.1.1) and the
 * kept rank k held at the value the forward gn_core chose:
 *   G1 = Gbar (Y^T A)^T, G2 = (AX)^T Gbar  (one fused pass over Gbar),
 *   H = (AX)^T G1,  Cbar = the adjoint of M at H through the core (FP64),
 *   dA = [G1 M^T + Y Cbar] X^T + Y [M^T G2], formed as
 *   dA = [G1 M^T | Y] [X^T ; M^T G2 + Cbar X^T]   (one product of inner size 2r + l).
 * Modes GN_MODE_F64 (A, Gbar, AX, YtA, dA double) and GN_MODE_F32 (float; the
 * core adjoint is FP64 in both).  X and Y must be GN_SKETCH_GAUSSIAN (they are
 * regenerated from p->seed); other kinds return GN_ERR_UNSUPPORTED.  AX (ld
 * ldax) and YtA (ld ldya) are the forward pass's outputs; AX may be NULL, in
 * which case it is recomputed from A (ld lda) -- A is read only then.  `core`
 * is the forward gn_core output (read only).  Workspace:
 * gn_workspace_size(GN_OP_BACKWARD) bytes, 256-byte aligned; calls that run
 * concurrently need separate workspaces. */
gn_status gn_backward(const gn_problem* p, const void* A, int64_t lda, const void* Gbar,
                      int64_t ldg, const void* AX, int64_t ldax, const void* YtA, int64_t ldya,
                      const gn_core_out* core, void* dA, int64_t ldda, void* ws,
                      size_t ws_bytes, gn_stream_t stream);

/* ---- Section 6: resampling and updating the matrix ----
 * The sketches are counter-based (Philox, see gn_generate_gaussian; SRHT sample =
 * the r smallest keys), so a larger r, extra rows or extra columns only add
 * entries at new indices of the same streams: the updated AX and Y^T A equal the
 * products a fresh gn_sketch of the enlarged problem would give (up to rounding).
 * The core is then recomputed with gn_core on the enlarged problem (O(r^3)).
 * FP64 and FP32 modes, Gaussian Y; X Gaussian or SRHT except where noted; BF16, F16
 * and USER sketches return GN_ERR_UNSUPPORTED.  Workspace:
 * gn_workspace_size(<enlarged problem>, GN_OP_UPDATE). */

/* Resampling r -> r + dr: p_old and p_new differ only in r (and l; r_new > r_old,
 * l_new >= l_old).  AX is m x r_new (ld ldax) with the old AX in its first r_old
 * columns; YtA is (r_new + l_new) x n (ld ldya) with the old Y^T A in its first
 * r_old + l_old rows.  Fills the new columns A X_new and rows Y_new^T A from one
 * pass over A (m x n, ld lda). */
gn_status gn_sketch_extend(const gn_problem* p_old, const gn_problem* p_new, const void* A,
                           int64_t lda, void* AX, int64_t ldax, void* YtA, int64_t ldya, void* ws,
                           size_t ws_bytes, gn_stream_t stream);

/* Appended data.  p is the problem after the append.  axis 0: rows, A -> [A; B]
 * with B (m - old_size) x n (ld ldb): AX rows old_size.. receive B X and Y^T A +=
 * Y_B^T B (Y_B = rows old_size.. of Y).  axis 1: columns, A -> [A, B] with B
 * m x (n - old_size) (ld ldb; Gaussian X only): AX += B X_B (X_B = rows
 * old_size.. of X) and columns old_size.. of Y^T A receive Y^T B.  AX and YtA
 * hold the old products in their old positions. */
gn_status gn_sketch_append(const gn_problem* p, int32_t axis, int64_t old_size, const void* B,
                           int64_t ldb, void* AX, int64_t ldax, void* YtA, int64_t ldya, void* ws,
                           size_t ws_bytes, gn_stream_t stream);

/* Perturbation A -> A + E (E m x n, ld lde): AX += E X and Y^T A += Y^T E. */
gn_status gn_sketch_update(const gn_problem* p, const void* E, int64_t lde, void* AX, int64_t ldax,
                           void* YtA, int64_t ldya, void* ws, size_t ws_bytes, gn_stream_t stream);

/* ---- Batches of independent problems (many GN solves of uneven m, n, r) ----
 * One problem of a batch: the problem statement of gn_problem restricted to FP32
 * mode with Gaussian X and Y (stream 1 / stream 2 of its own seed), its input A
 * and its outputs.  All pointers are device pointers.
 *   A   : float, m x n, row stride lda >= n, lda % 4 == 0, 16-byte aligned.
 *   AX  : float, m x r (ldax >= r, ldax % 4 == 0, 16-byte aligned); YtA: float,
 *         (r+l) x n (ldya >= n).
 *   core: as for gn_core (Q1 (r+l) x r, R, Q2, R2 r x r, k, status).
 * Limits: 1 <= r <= min(m, n), r + l <= 512. */
typedef struct {
  int64_t m, n, r, l;          /* l < 0 -> ceil(r/2) */
  uint64_t seed;
  double eps;                  /* as gn_problem (tau = eps * nu_X * nu_Y, Gaussian nu) */
  const void* A;
  int64_t lda;
  void* AX;
  int64_t ldax;
  void* YtA;
  int64_t ldya;
  gn_core_out core;
} gn_batch_problem;

/* Filled by gn_batch_prepare (host); passed unchanged to gn_batch_solve. */
typedef struct {
  int32_t count;               /* problems */
  int32_t n_pass_items;        /* (problem, product, tile) work items of the pass */
  int32_t n_core_items;        /* work items of the core products Y^T (AX) */
  int32_t grid;                /* workgroups of the pass launch (one per work item) */
  int64_t max_m, max_n, max_r, max_rl;
  size_t ws_bytes;             /* workspace the plan was laid out in */
  size_t off_desc, off_items, off_qr, off_qr2, off_trunc, off_widen;
  double pass_flops;           /* algorithmic FLOPs of all sketch passes */
  double pass_bytes;           /* algorithmic bytes of all sketch passes */
  int32_t tile_policy[4];      /* the tile configurations used (see gn_batch_prepare) */
  int32_t pass_threads;        /* workgroup size of the pass launch (256 or 512) */
} gn_batch_plan;

/* Workspace bytes for a batch (probs: host array of count problems). */
gn_status gn_batch_workspace_size(const gn_batch_problem* probs /*host*/, int32_t count,
                                  size_t* bytes /*host*/);

/* Validates the batch, lays out the workspace, copies the device tables (problem
 * descriptors, the work items of the pass, QR and truncation jobs) into ws and
 * draws every problem's X and Y into it (FP32, the values gn_sketch would use).
 * tile_policy (host, 4 entries, or NULL for the built-in choice) picks the MFMA
 * tile of each product: [0] Y^T A with r + l <= 64, [1] Y^T A with r + l > 64,
 * [2] AX with r <= 64, [3] AX with r > 64; values (output rows x columns) with
 * 256-thread workgroups 0 = 64 x 256, 1 = 128 x 128, 2 = 256 x 64, or with
 * 512-thread workgroups 3 = 128 x 256, 4 = 256 x 128;
 * all four from the same workgroup size (GN_ERR_ARG otherwise).  Returns after the tables
 * are copied (the call synchronizes with `stream`).  Independent of the values
 * of A: one prepared workspace serves any number of gn_batch_solve calls. */
gn_status gn_batch_prepare(const gn_batch_problem* probs /*host*/, int32_t count,
                           const int32_t* tile_policy /*host or NULL*/,
                           gn_batch_plan* plan /*host*/, void* ws, size_t ws_bytes,
                           gn_stream_t stream);

/* Stages of gn_batch_solve. */
typedef enum { GN_BATCH_PASS = 1, GN_BATCH_CORE = 2, GN_BATCH_ALL = 3 } gn_batch_stage;

/* The sketch passes and cores of every problem of a prepared batch (Algorithm 2.1
 * steps 2-3 and Section 5.1.1 for each).  stages & GN_BATCH_PASS: one launch
 * over the pass's work items (AX, Y^T A of every problem; one workgroup per item,
 * largest first); stages & GN_BATCH_CORE: one launch over the core products C = Y^T (AX)
 * (reading the AX of an earlier pass), then the batched FP64 Householder QR,
 * truncation and second QR.  Every parameter is read from ws and `plan`: nothing
 * is allocated, copied from the host or synchronized, so the call can be captured
 * in a HIP graph and replayed. */
gn_status gn_batch_solve(const gn_batch_plan* plan /*host*/, int32_t stages, void* ws,
                         size_t ws_bytes, gn_stream_t stream);

/* ||A - F G||_F^2 accumulated in FP64, tile by tile (no Gram-matrix shortcut),
 * written to *out_sumsq (device double).  A is m x n in `a_dtype` (for
 * GN_DT_BF16 and GN_DT_F16, A_scales as in gn_sketch, else NULL); F m x k (ld ldf), G k x n
 * (ld ldg), both double.  The reduction order is fixed (deterministic). */
gn_status gn_residual(int64_t m, int64_t n, int64_t k, const void* A, int64_t lda,
                      int32_t a_dtype, const float* A_scales, const double* F, int64_t ldf,
                      const double* G, int64_t ldg, double* out_sumsq, void* ws,
                      size_t ws_bytes, gn_stream_t stream);

/* gn_residual for callers that cannot allocate device memory (code under stream
 * capture, serving loops, harnesses that forbid hipMalloc): the same kernels and
 * the same result, bit for bit, with the per-tile partial sums kept in a 2 MiB
 * device array compiled into the library (one per GPU, held until the process
 * ends) instead of a workspace.  Limit: ceil(m/64) * ceil(n/64) <= 262144 tiles
 * (m n <= 2^30, e.g. 32768 x 32768); larger sizes return GN_ERR_UNSUPPORTED
 * before anything is enqueued.  Allocates nothing.  Calls that overlap in time on
 * one GPU share the array and race: serialize them (one stream, or events). */
gn_status gn_residual_noalloc(int64_t m, int64_t n, int64_t k, const void* A, int64_t lda,
                              int32_t a_dtype, const float* A_scales, const double* F,
                              int64_t ldf, const double* G, int64_t ldg, double* out_sumsq,
                              gn_stream_t stream);

/* bfloat16 storage with power-of-two block scales: for each 128 x 128 block,
 * s = 2^ceil(log2 max|a|) (1 for an all-zero block), out = RNE_bf16(a / s).
 * A is m x n in a_dtype (GN_DT_F64 or GN_DT_F32); out is m x n bfloat16 bits
 * (ld ldo); scales float[ceil(m/128) * ceil(n/128)]. */
gn_status gn_quantize_bf16_bs(int64_t m, int64_t n, const void* A, int64_t lda, int32_t a_dtype,
                              uint16_t* out, int64_t ldo, float* scales, gn_stream_t stream);

/* binary16 storage with power-of-two block scales (GN_MODE_F16_BS): the same
 * blocks and scales as gn_quantize_bf16_bs, out = RNE_binary16(a / s) (bits). */
gn_status gn_quantize_f16_bs(int64_t m, int64_t n, const void* A, int64_t lda, int32_t a_dtype,
                             uint16_t* out, int64_t ldo, float* scales, gn_stream_t stream);

/* Human-readable name of a status code (static storage). */
const char* gn_status_string(int32_t s);

/* Library version, "major.minor.patch" (static storage). */
const char* gn_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GN_H_ */
