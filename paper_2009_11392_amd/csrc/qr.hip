// Householder QR of the GN core C = Y^T (AX) in FP64 (Algorithm 2.1 step 2 and
// Section 5.1: QR without pivoting, which is rank revealing with high
// probability because X and Y are random), and the eps-truncation of
// Section 5.1.1.
//
// Blocked right-looking QR.  Each panel of nb columns is factored by one
// 512-thread workgroup holding the panel in registers (row t + 512 q of the panel
// in thread t).  A column step needs one workgroup reduction: the dots of the
// current column x with every panel column over the rows at and below the pivot,
// with the slot of x itself holding the squared norm strictly below the pivot;
// with the pivot row (passed through LDS) these give beta, tau, the dots
// v^T p_j = (x.p_j - beta p_j[c]) / (alpha - beta) used by the update of the
// columns to the right, and the same expression for the earlier reflectors
// (the y of the compact-WY recurrence for T, H_1 ... H_nb = I - V T V^T).
// Reductions are in a fixed order, so results do not depend on scheduling.
//
// A panel's block reflector is applied to the columns left in its outer block of
// QR_OB columns, C2 <- (I - V T^T V^T) C2, by one kernel per panel that sums
// W = V^T C2 on chip; each outer block's panels are merged into one block
// reflector (T from the panels' T's and V^T V), which FP64 matrix products apply
// to the trailing columns and, walking the outer blocks backwards from [I; 0], to
// the explicit Q with Q2 <- (I - V T V^T) Q2.  The batched form (many small
// problems, one panel width at a time) updates with two kernels over
// (128-row chunk) x (64-column group) tiles: partial W = V^T D per chunk, then W
// summed over chunks in chunk order, multiplied by T^T (or T) and subtracted.
#include "gn_internal.h"
#include "wave_ops.h"

#include <utility>
#include <vector>

namespace gn {
namespace {

constexpr int QP_T = 512;  // largest panel workgroup (and the batched panel's)
constexpr int QR_MAXROWS = 4096;
constexpr int QR_NB = 16;  // largest panel width

// sqrt(s) and 1/b for s, b in the normal range with |result| normal: the hardware
// approximation refined by Newton steps (to within a few ulp).
__device__ __forceinline__ double qr_sqrt_nr(double s) {
  const double y = __builtin_amdgcn_rsq(s);
  double g = s * y, h = 0.5 * y;
  const double r = fma(-h, g, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, s);
  return fma(d, h, g);
}
__device__ __forceinline__ double qr_rcp_nr(double b) {
  double y = __builtin_amdgcn_rcp(b);
  double e = fma(-b, y, 1.0);
  y = fma(y, e, y);
  e = fma(-b, y, 1.0);
  return fma(y, e, y);
}

// One column step of the panel, c a compile-time column index: every register
// array is indexed by constants, and only row c's thread and the rows above the
// pivot (all in the first register row, c < NB) need run-time predicates.
template <int RPT, int NB, int NT, int c>
__device__ __forceinline__ void qr_column(double (&p)[RPT][NB], int t, int lane, int wave,
                                          double (*part)[NT / 64][NB], double (*prow)[NB],
                                          double (*T)[NB + 1]) {
  constexpr int buf = c & 1;
  constexpr int kLowBits = 64 / NB;  // lanes sharing a reduction slot
  double x[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) x[q] = p[q][c];
  // slot cc: x . p_cc over rows >= c; slot c: |x|^2 over rows > c.  Rows of
  // register row q >= 1 are >= NT > c.
  const double x_ge = (t >= c) ? x[0] : 0.0;
  const double x_gt = (t > c) ? x[0] : 0.0;
  double acc[NB];
#pragma unroll
  for (int cc = 0; cc < NB; ++cc) {
    double s = (cc == c ? x_gt : x_ge) * p[0][cc];
#pragma unroll
    for (int q = 1; q < RPT; ++q) s = fma(x[q], p[q][cc], s);
    acc[cc] = s;
  }
  if (t == c) {
#pragma unroll
    for (int cc = 0; cc < NB; ++cc) prow[buf][cc] = p[0][cc];
  }
  int slot;
  const double ws = wave_transpose_sum<NB>(acc, lane, &slot);
  if ((lane & (kLowBits - 1)) == 0) part[buf][wave][slot] = ws;
  __syncthreads();
  // lane l holds the total of slot l % NB (the waves' partials summed as a
  // balanced tree in a fixed order) and the pivot row's entry P_l; sigma and alpha
  // are made uniform
  const int sl = lane % NB;
  double pw[NT / 64];
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) pw[w] = part[buf][w][sl];
#pragma unroll
  for (int h = NT / 128; h >= 1; h >>= 1)
#pragma unroll
    for (int w = 0; w < h; ++w) pw[w] += pw[w + h];
  const double tot = pw[0];
  const double Pl = prow[buf][sl];
  const double sigma = readlane_f64(tot, c), alpha = prow[buf][c];
  // beta = -sign(alpha) ||x(c:)||, tau = (beta - alpha) / beta, scale = 1 / (alpha - beta),
  // rb = 1 / beta.  In the normal range the square root and the reciprocals are
  // refined hardware approximations (a few-ulp error, like any Householder
  // implementation's reflector), keeping the chain of dependent operations short;
  // elsewhere they are the correctly rounded operations.
  double beta = alpha, tau = 0.0, scale = 0.0, rb = 0.0;
  if (sigma != 0.0) {
    const double s2 = fma(alpha, alpha, sigma);
    if (s2 >= 0x1p-960 && s2 <= 0x1p960) {
      const double nrm = qr_sqrt_nr(s2);
      beta = (alpha >= 0.0) ? -nrm : nrm;
      rb = qr_rcp_nr(beta);
      scale = qr_rcp_nr(alpha - beta);
      tau = (beta - alpha) * rb;
    } else {
      const double nrm = sqrt(s2);
      beta = (alpha >= 0.0) ? -nrm : nrm;
      rb = 1.0 / beta;
      tau = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
  }
  // tw_j = -tau v^T p_j = -tau scale (x.p_j - beta p_j[c]) = x.p_j / beta - p_j[c]
  // (since -tau scale = 1 / beta), one j per lane, then made uniform: the update of
  // the columns right of c and, for j < c, the y of the T recurrence
  const double twl = (tau != 0.0) ? fma(tot, rb, -Pl) : 0.0;
  double tw[NB];
#pragma unroll
  for (int cc = 0; cc < NB; ++cc) tw[cc] = readlane_f64(twl, cc);
  // apply H_c to the columns right of c; store v and R_cc = beta in column c
  const double v0 = (t > c) ? x[0] * scale : (t == c ? 1.0 : 0.0);
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const double v = (q == 0) ? v0 : x[q] * scale;
#pragma unroll
    for (int cc = c + 1; cc < NB; ++cc) p[q][cc] = fma(tw[cc], v, p[q][cc]);
  }
  if (tau != 0.0) {
    p[0][c] = (t > c) ? v0 : (t == c ? beta : p[0][c]);
#pragma unroll
    for (int q = 1; q < RPT; ++q) p[q][c] = x[q] * scale;
  }
  // T(:, c) = [ -tau T(0:c, 0:c) y ; tau ]; thread t < c owns row t of T, whose
  // entries left of the diagonal are zero
  if (t < c) {
    double s = 0.0;
#pragma unroll
    for (int l = 0; l < c; ++l) s = fma(T[t][l], tw[l], s);
    T[t][c] = s;
  }
  if (t == c) T[c][c] = tau;
}

template <int RPT, int NB, int NT, int... Cs>
__device__ __forceinline__ void qr_columns(std::integer_sequence<int, Cs...>, int nbw,
                                           double (&p)[RPT][NB], int t, int lane, int wave,
                                           double (*part)[NT / 64][NB], double (*prow)[NB],
                                           double (*T)[NB + 1]) {
  // nbw is uniform: columns past the panel width are skipped by a scalar branch
  ((Cs < nbw ? (qr_column<RPT, NB, NT, Cs>(p, t, lane, wave, part, prow, T), 0) : 0), ...);
}

template <int RPT, int NB, int NT>
__device__ __forceinline__ void qr_panel_body(double* __restrict__ C, int64_t ldc, int64_t M,
                                              int64_t j0, int nbw, double* __restrict__ Tout) {
  __shared__ double part[2][NT / 64][NB];
  __shared__ double prow[2][NB];
  __shared__ double T[NB][NB + 1];
  // the panel moves between memory and the thread-per-row registers through LDS,
  // NT rows at a time: in memory consecutive lanes take consecutive columns of a
  // row (a wave covers 64 / NB whole rows, one cache line each) instead of one row
  // per lane (64 lines per instruction).  Register row q first holds the thread's
  // share of that row-contiguous layout, is exchanged through LDS, then holds the
  // thread's own row.  LDS rows are padded to NB + 1 doubles so that a thread's
  // own row is read without bank conflicts.
  __shared__ double stage[NT][NB + 1];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t Mp = M - j0;
  constexpr int kRowsPerPass = NT / NB;  // rows covered by one load of every thread
  const int cr = t / NB, ccol = t % NB;  // row offset and column of the thread's elements
  const bool col_ok = ccol < nbw;
  double p[RPT][NB];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t r0 = (int64_t)NT * q + cr;
    const double* src = C + (j0 + r0) * ldc + j0 + ccol;
#pragma unroll
    for (int k = 0; k < NB; ++k)
      p[q][k] = (col_ok && r0 + kRowsPerPass * k < Mp) ? src[(int64_t)kRowsPerPass * k * ldc] : 0.0;
#pragma unroll
    for (int k = 0; k < NB; ++k) stage[cr + kRowsPerPass * k][ccol] = p[q][k];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NB; ++c) p[q][c] = stage[t][c];
    __syncthreads();
  }
  if (t < NB) {
    for (int l = 0; l < NB; ++l) T[t][l] = 0.0;  // row t of T is only touched by thread t
  }
  qr_columns<RPT, NB, NT>(std::make_integer_sequence<int, NB>{}, nbw, p, t, lane, wave, part, prow,
                          T);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
#pragma unroll
    for (int c = 0; c < NB; ++c) stage[t][c] = p[q][c];
    __syncthreads();
    const int64_t r0 = (int64_t)NT * q + cr;
    double* dst = C + (j0 + r0) * ldc + j0 + ccol;
#pragma unroll
    for (int k = 0; k < NB; ++k)
      if (col_ok && r0 + kRowsPerPass * k < Mp)
        dst[(int64_t)kRowsPerPass * k * ldc] = stage[cr + kRowsPerPass * k][ccol];
    __syncthreads();
  }
  for (int e = t; e < NB * NB; e += NT) Tout[(e / NB) * QR_NB + (e % NB)] = T[e / NB][e % NB];  // stride QR_NB
}

template <int RPT, int NB, int NT>
__global__ void __launch_bounds__(NT) qr_panel(double* __restrict__ C, int64_t ldc, int64_t M,
                                                 int64_t j0, int nbw, double* __restrict__ Tout,
                                                 const int32_t* gate, int64_t gate_n) {
  if (gate && *gate >= gate_n) return;
  qr_panel_body<RPT, NB, NT>(C, ldc, M, j0, nbw, Tout);
}

// Batched: job blockIdx.z, panel of width 16 at column j0 (every job has at most
// QP_T rows, so one row per thread).
__global__ void __launch_bounds__(QP_T) qr_panel_b(const QrJob* __restrict__ jobs, int64_t j0) {
  const QrJob J = jobs[blockIdx.z];
  if (J.gate && *J.gate >= J.gate_n) return;
  if (j0 >= J.N) return;
  const int nbw = (int)((J.N - j0 < QR_NB) ? (J.N - j0) : QR_NB);
  qr_panel_body<1, QR_NB, QP_T>(J.C, J.ldc, J.M, j0, nbw, J.T + (j0 / QR_NB) * QR_NB * QR_NB);
}

// Block-reflector update of D[j0 + i, col0 + j] (0 <= i < M - j0, 0 <= j < ncols)
// by the panel at (j0, j0) of Cp (width nbw, unit-lower reflectors below the
// diagonal).  Stage 1: Wp[chunk][c][j] = sum over the chunk's rows of V[i][c] D[i][j].
constexpr int QU_CH = 128;  // rows per chunk
constexpr int QU_CG = 64;   // target columns per workgroup

__device__ __forceinline__ void qr_stage_v(double (*sV)[QR_NB + 1], const double* Cp, int64_t ldc,
                                           int64_t j0, int nbw, int64_t Mp, int64_t r0) {
  for (int e = threadIdx.x; e < QU_CH * QR_NB; e += blockDim.x) {
    const int rr = e / QR_NB, c = e % QR_NB;
    const int64_t row = r0 + rr;
    double v = 0.0;
    if (row < Mp && c < nbw) v = (row < c) ? 0.0 : (row == c ? 1.0 : Cp[(j0 + row) * ldc + j0 + c]);
    sV[rr][c] = v;
  }
}

__device__ __forceinline__ void qr_upd_w_body(const double* __restrict__ Cp, int64_t ldc,
                                              int64_t M, int64_t j0, int nbw,
                                              const double* __restrict__ D, int64_t ldd,
                                              int64_t col0, int64_t ncols,
                                              double* __restrict__ Wp, int64_t chunk,
                                              int64_t grp) {
  __shared__ double sV[QU_CH][QR_NB + 1];
  __shared__ double red[4][QR_NB][QU_CG + 1];
  const int tid = threadIdx.x, j = tid & 63, wq = tid >> 6;
  const int64_t Mp = M - j0;
  const int64_t r0 = chunk * QU_CH;
  const int64_t jg = grp * QU_CG + j;
  const bool jok = jg < ncols;
  double d[QU_CH / 4];
#pragma unroll
  for (int q = 0; q < QU_CH / 4; ++q) {
    const int64_t row = r0 + wq + 4 * q;
    d[q] = (jok && row < Mp) ? D[(j0 + row) * ldd + col0 + jg] : 0.0;
  }
  qr_stage_v(sV, Cp, ldc, j0, nbw, Mp, r0);
  __syncthreads();
  double acc[QR_NB];
#pragma unroll
  for (int c = 0; c < QR_NB; ++c) acc[c] = 0.0;
#pragma unroll
  for (int q = 0; q < QU_CH / 4; ++q)
#pragma unroll
    for (int c = 0; c < QR_NB; ++c) acc[c] = fma(sV[wq + 4 * q][c], d[q], acc[c]);
#pragma unroll
  for (int c = 0; c < QR_NB; ++c) red[wq][c][j] = acc[c];
  __syncthreads();
  // 256 threads: (c4 = tid / 64 -> slots 4 c4 .. 4 c4 + 3, column j)
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int c = 4 * wq + i;
    const double s = ((red[0][c][j] + red[1][c][j]) + red[2][c][j]) + red[3][c][j];
    if (jok) Wp[(chunk * QR_NB + c) * ncols + jg] = s;
  }
}


// Update of the columns left in the outer block (at most QR_OB - 16) by a panel,
// in two launches over (QI_CH-row chunk) x (16-column group) tiles: the chunk's
// V (QI_CH x 16) is staged in LDS once and D kept in registers (a thread owns one
// column and rows wq + 16 q), W_c = V_c^T D_c is summed over the 16 row groups in
// LDS in a fixed order; then every tile sums its group's partials in chunk order
// (all loads issued first), forms W2 = Top W (Top = T^T when trans, else T) and
// subtracts V_c W2 from its chunk.
constexpr int QI_CH = 128;                    // rows per chunk
constexpr int QI_RG = 16;                     // row groups: threads per column
constexpr int QI_RPT = QI_CH / QI_RG;         // rows per thread
constexpr int QI_MAXCH = QR_MAXROWS / QI_CH;  // chunks at the largest height

__device__ __forceinline__ void qi_stage_v(double (*sV)[QR_NB + 1], const double* __restrict__ Cp,
                                           int64_t ldc, int64_t j0, int nbw, int64_t Mp,
                                           int64_t r0) {
  for (int e = threadIdx.x; e < QI_CH * QR_NB; e += 256) {
    const int rr = e / QR_NB, c = e % QR_NB;
    const int64_t row = r0 + rr;
    double v = 0.0;
    if (row < Mp && c < nbw) v = (row < c) ? 0.0 : (row == c ? 1.0 : Cp[(j0 + row) * ldc + j0 + c]);
    sV[rr][c] = v;
  }
}

__global__ void __launch_bounds__(256) qr_iupd_w(const double* __restrict__ Cp, int64_t ldc,
                                                 int64_t M, int64_t j0, int nbw,
                                                 const double* __restrict__ D, int64_t ldd,
                                                 int64_t col0, int64_t ncols,
                                                 double* __restrict__ Wp, const int32_t* gate,
                                                 int64_t gate_n) {
  if (gate && *gate >= gate_n) return;
  __shared__ double sV[QI_CH][QR_NB + 1];
  __shared__ double red[QI_RG][QR_NB][QR_NB + 1];
  const int tid = threadIdx.x, j = tid & 15, wq = tid >> 4;
  const int64_t Mp = M - j0, r0 = (int64_t)blockIdx.x * QI_CH;
  const int64_t jg = (int64_t)blockIdx.y * QR_NB + j;
  const bool jok = jg < ncols;
  double d[QI_RPT];
#pragma unroll
  for (int q = 0; q < QI_RPT; ++q) {
    const int64_t row = r0 + wq + QI_RG * q;
    d[q] = (jok && row < Mp) ? D[(j0 + row) * ldd + col0 + jg] : 0.0;
  }
  qi_stage_v(sV, Cp, ldc, j0, nbw, Mp, r0);
  __syncthreads();
  double acc[QR_NB];
#pragma unroll
  for (int a = 0; a < QR_NB; ++a) acc[a] = 0.0;
#pragma unroll
  for (int q = 0; q < QI_RPT; ++q)
#pragma unroll
    for (int a = 0; a < QR_NB; ++a) acc[a] = fma(sV[wq + QI_RG * q][a], d[q], acc[a]);
#pragma unroll
  for (int a = 0; a < QR_NB; ++a) red[wq][a][j] = acc[a];
  __syncthreads();
  const int a = tid >> 4, jj = tid & 15;
  double sum = 0.0;
#pragma unroll
  for (int w = 0; w < QI_RG; ++w) sum += red[w][a][jj];
  const int64_t col = (int64_t)blockIdx.y * QR_NB + jj;
  if (col < ncols) Wp[((int64_t)blockIdx.x * QR_NB + a) * ncols + col] = sum;
}

__global__ void __launch_bounds__(256) qr_iupd_apply(const double* __restrict__ Cp, int64_t ldc,
                                                     int64_t M, int64_t j0, int nbw,
                                                     double* __restrict__ D, int64_t ldd,
                                                     int64_t col0, int64_t ncols,
                                                     const double* __restrict__ Wp, int nch,
                                                     const double* __restrict__ T, int trans,
                                                     const int32_t* gate, int64_t gate_n) {
  if (gate && *gate >= gate_n) return;
  __shared__ double sV[QI_CH][QR_NB + 1];
  __shared__ double sW[QR_NB][QR_NB + 1];
  __shared__ double sW2[QR_NB][QR_NB + 1];
  __shared__ double sT[QR_NB][QR_NB + 1];
  const int tid = threadIdx.x, j = tid & 15, wq = tid >> 4;
  const int64_t Mp = M - j0, r0 = (int64_t)blockIdx.x * QI_CH;
  const int64_t jg = (int64_t)blockIdx.y * QR_NB + j;
  const bool jok = jg < ncols;
  const int a = tid >> 4, jj = tid & 15;
  {  // W = sum of the group's partials in chunk order
    const int64_t col = (int64_t)blockIdx.y * QR_NB + jj;
    double v[QI_MAXCH];
#pragma unroll
    for (int c = 0; c < QI_MAXCH; ++c)
      v[c] = (c < nch && col < ncols) ? Wp[((int64_t)c * QR_NB + a) * ncols + col] : 0.0;
    double sum = 0.0;
#pragma unroll
    for (int c = 0; c < QI_MAXCH; ++c) sum += v[c];
    sW[a][jj] = sum;
    const double t = trans ? T[jj * QR_NB + a] : T[a * QR_NB + jj];
    sT[a][jj] = (a < nbw && jj < nbw) ? t : 0.0;
  }
  double d[QI_RPT];
#pragma unroll
  for (int q = 0; q < QI_RPT; ++q) {
    const int64_t row = r0 + wq + QI_RG * q;
    d[q] = (jok && row < Mp) ? D[(j0 + row) * ldd + col0 + jg] : 0.0;
  }
  qi_stage_v(sV, Cp, ldc, j0, nbw, Mp, r0);
  __syncthreads();
  {
    double sum = 0.0;
#pragma unroll
    for (int l = 0; l < QR_NB; ++l) sum = fma(sT[a][l], sW[l][jj], sum);
    sW2[a][jj] = sum;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < QI_RPT; ++q) {
    const int64_t row = r0 + wq + QI_RG * q;
    double sum = 0.0;
#pragma unroll
    for (int c = 0; c < QR_NB; ++c) sum = fma(sV[wq + QI_RG * q][c], sW2[c][j], sum);
    if (jok && row < Mp) D[(j0 + row) * ldd + col0 + jg] = d[q] - sum;
  }
}

// Batched update target of job J for the panel at j0: the trailing columns of C
// (phase 0) or the columns j0.. of Q (phase 1).  Returns false when this
// workgroup has nothing to do.
struct UpdTarget {
  double* D;
  int64_t ldd, col0, ncols, nch;
  int nbw;
};
__device__ __forceinline__ bool qr_upd_target(const QrJob& J, int64_t j0, int phase,
                                              UpdTarget& u) {
  if (J.gate && *J.gate >= J.gate_n) return false;
  if (j0 >= J.N) return false;
  u.nbw = (int)((J.N - j0 < QR_NB) ? (J.N - j0) : QR_NB);
  u.nch = (J.M - j0 + QU_CH - 1) / QU_CH;
  if (phase == 0) {
    u.D = J.C;
    u.ldd = J.ldc;
    u.col0 = j0 + u.nbw;
  } else {
    u.D = J.Q;
    u.ldd = J.ldq;
    u.col0 = j0;
  }
  u.ncols = J.N - u.col0;
  return u.ncols > 0 && (int64_t)blockIdx.x < u.nch && (int64_t)blockIdx.y * QU_CG < u.ncols;
}

__global__ void __launch_bounds__(256) qr_upd_w_b(const QrJob* __restrict__ jobs, int64_t j0,
                                                  int phase) {
  const QrJob J = jobs[blockIdx.z];
  UpdTarget u;
  if (!qr_upd_target(J, j0, phase, u)) return;
  qr_upd_w_body(J.C, J.ldc, J.M, j0, u.nbw, u.D, u.ldd, u.col0, u.ncols, J.Wp, blockIdx.x,
                blockIdx.y);
}

// Stage 2: W = sum over chunks of Wp (chunk order), W <- Top W (Top = T^T when
// trans, else T), D -= V W over this workgroup's chunk of rows.
__device__ __forceinline__ void qr_upd_apply_body(const double* __restrict__ Cp, int64_t ldc,
                                                  int64_t M, int64_t j0, int nbw,
                                                  double* __restrict__ D, int64_t ldd,
                                                  int64_t col0, int64_t ncols,
                                                  const double* __restrict__ Wp, int nchunks,
                                                  const double* __restrict__ T, int trans,
                                                  int64_t chunk, int64_t grp) {
  __shared__ double sV[QU_CH][QR_NB + 1];
  __shared__ double W[QR_NB][QU_CG + 1];
  __shared__ double sT[QR_NB][QR_NB + 1];
  const int tid = threadIdx.x, j = tid & 63, wq = tid >> 6;
  const int64_t Mp = M - j0;
  const int64_t r0 = chunk * QU_CH;
  const int64_t jg = grp * QU_CG + j;
  const bool jok = jg < ncols;
  double d[QU_CH / 4];
#pragma unroll
  for (int q = 0; q < QU_CH / 4; ++q) {
    const int64_t row = r0 + wq + 4 * q;
    d[q] = (jok && row < Mp) ? D[(j0 + row) * ldd + col0 + jg] : 0.0;
  }
  {  // sum over chunks in chunk order; loads issued four chunks at a time
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int ch = 0; ch < nchunks; ch += 4) {
      double v[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          v[u][i] = (jok && ch + u < nchunks)
                        ? Wp[((int64_t)(ch + u) * QR_NB + 4 * wq + i) * ncols + jg]
                        : 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int i = 0; i < 4; ++i) s[i] += v[u][i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) W[4 * wq + i][j] = s[i];
  }
  {
    const int c = tid / QR_NB, c2 = tid % QR_NB;  // 256 = 16 x 16
    const double v = trans ? T[c2 * QR_NB + c] : T[c * QR_NB + c2];
    sT[c][c2] = (c < nbw && c2 < nbw) ? v : 0.0;
  }
  qr_stage_v(sV, Cp, ldc, j0, nbw, Mp, r0);
  __syncthreads();
  double wt[QR_NB];
#pragma unroll
  for (int c = 0; c < QR_NB; ++c) {
    double s = 0.0;
#pragma unroll
    for (int c2 = 0; c2 < QR_NB; ++c2) s = fma(sT[c][c2], W[c2][j], s);
    wt[c] = s;
  }
#pragma unroll
  for (int q = 0; q < QU_CH / 4; ++q) {
    const int64_t row = r0 + wq + 4 * q;
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < QR_NB; ++c) s = fma(sV[wq + 4 * q][c], wt[c], s);
    if (jok && row < Mp) D[(j0 + row) * ldd + col0 + jg] = d[q] - s;
  }
}


__global__ void __launch_bounds__(256) qr_upd_apply_b(const QrJob* __restrict__ jobs, int64_t j0,
                                                      int phase) {
  const QrJob J = jobs[blockIdx.z];
  UpdTarget u;
  if (!qr_upd_target(J, j0, phase, u)) return;
  qr_upd_apply_body(J.C, J.ldc, J.M, j0, u.nbw, u.D, u.ldd, u.col0, u.ncols, J.Wp, (int)u.nch,
                    J.T + (j0 / QR_NB) * QR_NB * QR_NB, phase == 0 ? 1 : 0, blockIdx.x,
                    blockIdx.y);
}

__device__ __forceinline__ void qr_init_q_body(double* Q, int64_t ldq, int64_t M, int64_t N) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * N) return;
  const int64_t i = e / N, j = e - i * N;
  Q[i * ldq + j] = (i == j) ? 1.0 : 0.0;
}

__global__ void __launch_bounds__(256) qr_init_q(double* Q, int64_t ldq, int64_t M, int64_t N,
                                                 const int32_t* gate, int64_t gate_n) {
  if (gate && *gate >= gate_n) return;
  qr_init_q_body(Q, ldq, M, N);
}

__global__ void __launch_bounds__(256) qr_init_q_b(const QrJob* __restrict__ jobs) {
  const QrJob J = jobs[blockIdx.z];
  if (J.gate && *J.gate >= J.gate_n) return;
  qr_init_q_body(J.Q, J.ldq, J.M, J.N);
}

// R_ii >= 0: flip row i of R and column i of Q where the Householder diagonal is
// negative; copy the upper triangle of the factored matrix into R.
__device__ __forceinline__ void qr_signfix_body(const double* C, int64_t ldc, double* Q,
                                                int64_t ldq, double* R, int64_t ldr, int64_t M,
                                                int64_t N) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < M * N) {
    const int64_t i = e / N, j = e - i * N;
    if (C[j * ldc + j] < 0.0) Q[i * ldq + j] = -Q[i * ldq + j];
  }
  if (e < N * N) {
    const int64_t i = e / N, j = e - i * N;
    const double sg = (C[i * ldc + i] < 0.0) ? -1.0 : 1.0;
    R[i * ldr + j] = (j >= i) ? sg * C[i * ldc + j] : 0.0;
  }
}

__global__ void __launch_bounds__(256) qr_signfix(const double* C, int64_t ldc, double* Q,
                                                  int64_t ldq, double* R, int64_t ldr, int64_t M,
                                                  int64_t N, const int32_t* gate, int64_t gate_n) {
  if (gate && *gate >= gate_n) return;
  qr_signfix_body(C, ldc, Q, ldq, R, ldr, M, N);
}

__global__ void __launch_bounds__(256) qr_signfix_b(const QrJob* __restrict__ jobs) {
  const QrJob J = jobs[blockIdx.z];
  if (J.gate && *J.gate >= J.gate_n) return;
  qr_signfix_body(J.C, J.ldc, J.Q, J.ldq, J.R, J.ldr, J.M, J.N);
}

// The two halves of qr_signfix as separate launches: R (upper triangle of the
// factored matrix, row i scaled by the sign of its Householder diagonal) as soon
// as the factorization ends, and the column signs of Q once Q is formed.
__global__ void __launch_bounds__(256) qr_extract_r(const double* C, int64_t ldc, double* R,
                                                    int64_t ldr, int64_t N, const int32_t* gate,
                                                    int64_t gate_n) {
  if (gate && *gate >= gate_n) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * N) return;
  const int64_t i = e / N, j = e - i * N;
  const double sg = (C[i * ldc + i] < 0.0) ? -1.0 : 1.0;
  R[i * ldr + j] = (j >= i) ? sg * C[i * ldc + j] : 0.0;
}

__global__ void __launch_bounds__(256) qr_sign_q(const double* C, int64_t ldc, double* Q,
                                                 int64_t ldq, int64_t M, int64_t N,
                                                 const int32_t* gate, int64_t gate_n) {
  if (gate && *gate >= gate_n) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * N) return;
  const int64_t i = e / N, j = e - i * N;
  if (C[j * ldc + j] < 0.0) Q[i * ldq + j] = -Q[i * ldq + j];
}

// Kept rank: k = first i whose diagonal fails the keep test (|R_ii| >= tau, or
// |R_ii| > 0 when tau <= 0; non-finite always fails); status flags.
__device__ __forceinline__ void trunc_scan_body(int64_t r, const double* R, int64_t ldr,
                                                double tau, int32_t* kout, int32_t* status) {
  __shared__ int64_t s_first[256];
  __shared__ int s_flag[256];
  int64_t first = r;
  int nonfinite = 0;
  for (int64_t i = threadIdx.x; i < r; i += 256) {
    const double d = R[i * ldr + i];
    const bool fin = isfinite(d);
    const double a = fabs(d);
    const bool keep = fin && ((tau > 0.0) ? (a >= tau) : (a > 0.0));
    if (!fin) nonfinite = 1;
    if (!keep && i < first) first = i;
  }
  s_first[threadIdx.x] = first;
  s_flag[threadIdx.x] = nonfinite;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s_first[threadIdx.x] = min(s_first[threadIdx.x], s_first[threadIdx.x + w]);
      s_flag[threadIdx.x] |= s_flag[threadIdx.x + w];
    }
    __syncthreads();
  }
  const int64_t k = s_first[0];
  const int nf = s_flag[0];
  __syncthreads();
  // non-monotone: a diagonal that passes the test after the first failing one
  int nm = 0;
  for (int64_t i = k + 1 + threadIdx.x; i < r; i += 256) {
    const double d = R[i * ldr + i];
    const double a = fabs(d);
    if (isfinite(d) && ((tau > 0.0) ? (a >= tau) : (a > 0.0))) nm = 1;
  }
  s_flag[threadIdx.x] = nm;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s_flag[threadIdx.x] |= s_flag[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *kout = (int32_t)k;
    *status = (nf ? 1 : 0) | (k == 0 ? 2 : 0) | (s_flag[0] ? 4 : 0);
  }
}

__global__ void __launch_bounds__(256) trunc_scan(int64_t r, const double* R, int64_t ldr, double tau,
                                                  int32_t* kout, int32_t* status) {
  trunc_scan_body(r, R, ldr, tau, kout, status);
}

__global__ void __launch_bounds__(256) trunc_scan_b(const TruncJob* __restrict__ jobs) {
  const TruncJob J = jobs[blockIdx.z];
  trunc_scan_body(J.r, J.R, J.ldr, J.tau, J.k, J.status);
}

// Z (r x r) = [R[:k, :]^T, 0]: the matrix whose leading k columns are factored
// by the second QR (Section 5.1.1).  Runs only when k < r.
__device__ __forceinline__ void build_z_body(int64_t r, const double* R, int64_t ldr,
                                             const int32_t* kdev, double* Z, int64_t ldz) {
  const int32_t k = *kdev;
  if (k >= r) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= r * r) return;
  const int64_t j = e / r, i = e - j * r;  // Z[j][i] = R[i][j] for i < k
  Z[j * ldz + i] = (i < k) ? R[i * ldr + j] : 0.0;
}

__global__ void __launch_bounds__(256) build_z(int64_t r, const double* R, int64_t ldr,
                                               const int32_t* kdev, double* Z, int64_t ldz) {
  build_z_body(r, R, ldr, kdev, Z, ldz);
}

__global__ void __launch_bounds__(256) build_z_b(const TruncJob* __restrict__ jobs) {
  const TruncJob J = jobs[blockIdx.z];
  build_z_body(J.r, J.R, J.ldr, J.k, J.Z, J.ldz);
}

// ---------------------------------------------------------------------------- outer blocks
// Panels are grouped into outer blocks of QR_OB columns: inside a block the
// panel updates touch only the block's columns; the block's reflectors are then
// applied to the trailing columns (and, walking back, to Q) as one block
// reflector I - V T V^T by the FP64 MFMA kernels below.
constexpr int QR_OB = 64;

// Vb ((M - J0) x QR_OB, row-major) and Vt (its transpose, ld M - J0): the block's
// unit lower trapezoidal reflectors, zero past the block width w.
__global__ void __launch_bounds__(256) qr_build_v(const double* __restrict__ C, int64_t ldc,
                                                  int64_t M, int64_t J0, int w,
                                                  double* __restrict__ Vb, double* __restrict__ Vt,
                                                  const int32_t* gate, int64_t gate_n) {
  if (gate && *gate >= gate_n) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t Mp = M - J0;
  if (e >= Mp * QR_OB) return;
  {  // Vb: Mp x QR_OB, row-major
    const int64_t i = e / QR_OB;
    const int c = (int)(e - i * QR_OB);
    double v = 0.0;
    if (c < w) v = (i < c) ? 0.0 : (i == c ? 1.0 : C[(J0 + i) * ldc + J0 + c]);
    Vb[e] = v;
  }
  {  // Vt: QR_OB x Mp, row-major (V by columns)
    const int c = (int)(e / Mp);
    const int64_t i = e - (int64_t)c * Mp;
    double v = 0.0;
    if (c < w) v = (i < c) ? 0.0 : (i == c ? 1.0 : C[(J0 + i) * ldc + J0 + c]);
    Vt[e] = v;
  }
}

// The panels of one outer block (at most QR_OB / 8 of them).
// Outer-block reflector H = I - V T' V^T (V: Mp x QR_OB unit-lower, zero past the
// block width; T' = T^T when trans, else T) applied to an Mp x ncols target D,
// D <- D - V (T' (V^T D)), in three launches with FP64 MFMA
// (v_mfma_f64_16x16x4f64: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// register v of its result holds row l / 16 + 4 v, column l % 16):
//   qr_oupd_w     partial W_c = V_c^T D_c per QO_CH-row chunk c and QO_CG-column
//                 strip, the four waves each owning a 32 x 32 quarter;
//   qr_oupd_w2    per QO_CW columns, W = sum of the partials in chunk order (all
//                 loads issued first), W2 = T' W;
//   qr_oupd_apply per QO_CA-row chunk and strip, D_c -= V_c W2 with W2 staged in
//                 LDS, V read by columns (Vt) so that the operand loads are
//                 contiguous, and V and D loaded before the products.
typedef double qr_f64x4 __attribute__((ext_vector_type(4)));
constexpr int QO_CH = 128;  // rows per partial (at most QR_MAXROWS / QO_CH = 32 partials)
constexpr int QO_CG = 64;   // target columns per strip
constexpr int QO_CW = 16;   // target columns per W2 workgroup
constexpr int QO_CA = 128;  // rows per apply tile

__device__ __forceinline__ qr_f64x4 qr_mfma(double a, double b, qr_f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__global__ void __launch_bounds__(256) qr_oupd_w(const double* __restrict__ Vb, int64_t Mp,
                                                 const double* __restrict__ D, int64_t ldd,
                                                 int64_t ncols, double* __restrict__ Wp,
                                                 const int32_t* gate, int64_t gate_n) {
  if (gate && *gate >= gate_n) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * QO_CH;
  const int64_t c0 = (int64_t)blockIdx.y * QO_CG;
  qr_f64x4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = qr_f64x4{0.0, 0.0, 0.0, 0.0};
  // 16 rows of V and D per step; the next step's loads are issued before this
  // step's products, so every step after the first finds its operands loaded
  auto load = [&](int kb, double (&a)[4][2], double (&b)[4][2]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t row = r0 + kb + 4 * u + lk;
      const bool rin = row < Mp;
#pragma unroll
      for (int x = 0; x < 2; ++x) a[u][x] = rin ? Vb[row * QR_OB + wm * 32 + x * 16 + li] : 0.0;
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const int64_t col = c0 + wn * 32 + y * 16 + li;
        b[u][y] = (rin && col < ncols) ? D[row * ldd + col] : 0.0;
      }
    }
  };
  double a[2][4][2], b[2][4][2];
  load(0, a[0], b[0]);
#pragma unroll
  for (int st = 0; st < QO_CH / 16; ++st) {
    const int cur = st & 1;
    if (st + 1 < QO_CH / 16) load(16 * (st + 1), a[cur ^ 1], b[cur ^ 1]);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = qr_mfma(a[cur][u][x], b[cur][u][y], acc[x][y]);
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = wm * 32 + x * 16 + lk + 4 * v;
        const int64_t col = c0 + wn * 32 + y * 16 + li;
        if (col < ncols) Wp[((int64_t)blockIdx.x * QR_OB + a) * ncols + col] = acc[x][y][v];
      }
}

__global__ void __launch_bounds__(256) qr_oupd_w2(const double* __restrict__ Wp, int nch,
                                                  int64_t ncols, const double* __restrict__ T,
                                                  int trans, double* __restrict__ W2,
                                                  const int32_t* gate, int64_t gate_n) {
  if (gate && *gate >= gate_n) return;
  constexpr int kMaxCh = QR_MAXROWS / QO_CH;
  __shared__ double sT[QR_OB][QR_OB + 1];
  __shared__ double sW[QR_OB][QO_CW + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t c0 = (int64_t)blockIdx.x * QO_CW;
  // W (QR_OB x QO_CW) = sum of the partials in chunk order, every load issued first
#pragma unroll
  for (int q = 0; q < QR_OB * QO_CW / 256; ++q) {
    const int e = tid + 256 * q;
    const int a = e / QO_CW, b = e % QO_CW;
    const int64_t col = c0 + b;
    double v[kMaxCh];
#pragma unroll
    for (int c = 0; c < kMaxCh; ++c)
      v[c] = (c < nch && col < ncols) ? Wp[((int64_t)c * QR_OB + a) * ncols + col] : 0.0;
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < kMaxCh; ++c) acc += v[c];
    sW[a][b] = acc;
  }
  for (int e = tid; e < QR_OB * QR_OB; e += 256) {
    const int a = e / QR_OB, l = e % QR_OB;
    sT[a][l] = trans ? T[l * QR_OB + a] : T[a * QR_OB + l];
  }
  __syncthreads();
  // wave w: rows 16 w .. 16 w + 15 of W2 = T' W
  qr_f64x4 acc = qr_f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k0 = 0; k0 < QR_OB; k0 += 4)
    acc = qr_mfma(sT[16 * wave + li][k0 + lk], sW[k0 + lk][li], acc);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int a = 16 * wave + lk + 4 * v;
    const int64_t col = c0 + li;
    if (col < ncols) W2[(int64_t)a * ncols + col] = acc[v];
  }
}

__global__ void __launch_bounds__(256) qr_oupd_apply(const double* __restrict__ Vt, int64_t Mp,
                                                     double* __restrict__ D, int64_t ldd,
                                                     int64_t ncols, const double* __restrict__ W2,
                                                     const int32_t* gate, int64_t gate_n) {
  if (gate && *gate >= gate_n) return;
  __shared__ double sW[QR_OB][QO_CG + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * QO_CA + wave * (QO_CA / 4);  // 32 rows per wave
  const int64_t c0 = (int64_t)blockIdx.y * QO_CG;
  for (int e = tid; e < QR_OB * QO_CG; e += 256) {
    const int k = e / QO_CG, b = e % QO_CG;
    const int64_t col = c0 + b;
    sW[k][b] = (col < ncols) ? W2[(int64_t)k * ncols + col] : 0.0;
  }
  // this wave's V rows (all QR_OB columns) and its part of D, loaded before any use
  double a[QR_OB / 4][2];
#pragma unroll
  for (int ks = 0; ks < QR_OB / 4; ++ks)
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const int64_t row = r0 + x * 16 + li;
      a[ks][x] = (row < Mp) ? Vt[(int64_t)(4 * ks + lk) * Mp + row] : 0.0;
    }
  double d[2][4][4];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = r0 + x * 16 + lk + 4 * v;
        const int64_t col = c0 + y * 16 + li;
        d[x][y][v] = (row < Mp && col < ncols) ? D[row * ldd + col] : 0.0;
      }
  __syncthreads();
  qr_f64x4 acc[2][4];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = qr_f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ks = 0; ks < QR_OB / 4; ++ks) {
    double b[4];
#pragma unroll
    for (int y = 0; y < 4; ++y) b[y] = sW[4 * ks + lk][y * 16 + li];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[x][y] = qr_mfma(a[ks][x], b[y], acc[x][y]);
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = r0 + x * 16 + lk + 4 * v;
        const int64_t col = c0 + y * 16 + li;
        if (row < Mp && col < ncols) D[row * ldd + col] = d[x][y][v] - acc[x][y][v];
      }
}

// G = V^T V from its chunk partials, summed in chunk order (one entry per thread,
// every load issued first).
__global__ void __launch_bounds__(256) qr_sum_g(const double* __restrict__ Gp, int nch,
                                                double* __restrict__ G, const int32_t* gate,
                                                int64_t gate_n) {
  if (gate && *gate >= gate_n) return;
  constexpr int kMaxCh = QR_MAXROWS / QO_CH;
  const int e = blockIdx.x * 256 + threadIdx.x;  // < QR_OB * QR_OB
  double v[kMaxCh];
#pragma unroll
  for (int c = 0; c < kMaxCh; ++c) v[c] = (c < nch) ? Gp[(int64_t)c * QR_OB * QR_OB + e] : 0.0;
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < kMaxCh; ++c) acc += v[c];
  G[e] = acc;
}

struct OuterPanels {
  int count;
  int off[QR_OB / 8];    // first column within the block
  int width[QR_OB / 8];
  int tidx[QR_OB / 8];   // index of the panel's T in the T array
};

// T of the whole block (w x w, ld QR_OB, upper triangular) from the panels' T
// and G = Vb^T Vb, merging left to right: with T_a the block so far (columns
// 0..s) and T_b the next panel's, T = [T_a, -T_a G[0:s, b] T_b; 0, T_b]
// (the product of the two block reflectors).
__global__ void __launch_bounds__(256) qr_merge_t(const double* __restrict__ G,
                                                  const double* __restrict__ Tpanels,
                                                  OuterPanels op, int w,
                                                  double* __restrict__ Tout, const int32_t* gate,
                                                  int64_t gate_n) {
  if (gate && *gate >= gate_n) return;
  __shared__ double T[QR_OB][QR_OB + 1];
  __shared__ double Gs[QR_OB][QR_OB + 1];
  __shared__ double Y[QR_OB][QR_NB + 1];
  const int tid = threadIdx.x;
  // G and every panel's T loaded up front (all loads in flight at once)
  constexpr int kG = QR_OB * QR_OB / 256;
  double gv[kG];
#pragma unroll
  for (int q = 0; q < kG; ++q) gv[q] = G[tid + 256 * q];
  double tv[QR_OB / 8];
#pragma unroll
  for (int b = 0; b < QR_OB / 8; ++b) {
    const int wb = (b < op.count) ? op.width[b] : 0;
    tv[b] = (tid < wb * wb)
                ? Tpanels[(size_t)op.tidx[b] * QR_NB * QR_NB + (tid / wb) * QR_NB + tid % wb]
                : 0.0;
  }
#pragma unroll
  for (int q = 0; q < kG; ++q) {
    const int e = tid + 256 * q;
    T[e / QR_OB][e % QR_OB] = 0.0;
    Gs[e / QR_OB][e % QR_OB] = gv[q];
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < QR_OB / 8; ++b) {
    const int wb = (b < op.count) ? op.width[b] : 0;
    if (tid < wb * wb) T[op.off[b] + tid / wb][op.off[b] + tid % wb] = tv[b];
  }
  __syncthreads();
  // T[0:o, o:o+wb] = -T_a (V_a^T V_b) T_b for each later panel, in order; the dot
  // products are split over four partial sums
  for (int b = 1; b < op.count; ++b) {
    const int o = op.off[b], wb = op.width[b];
    // Y = T_a G[0:o, o:o+wb]   (o x wb)
    for (int e = tid; e < o * wb; e += 256) {
      const int i = e / wb, j = e % wb;
      double a4[4] = {0.0, 0.0, 0.0, 0.0};
      int l = i;
      for (; l + 3 < o; l += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) a4[u] = fma(T[i][l + u], Gs[l + u][o + j], a4[u]);
      }
      for (; l < o; ++l) a4[0] = fma(T[i][l], Gs[l][o + j], a4[0]);
      Y[i][j] = (a4[0] + a4[1]) + (a4[2] + a4[3]);
    }
    __syncthreads();
    // T[0:o, o:o+wb] = -Y T_b
    for (int e = tid; e < o * wb; e += 256) {
      const int i = e / wb, j = e % wb;
      double a4[4] = {0.0, 0.0, 0.0, 0.0};
      int l = 0;
      for (; l + 3 <= j; l += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) a4[u] = fma(Y[i][l + u], T[o + l + u][o + j], a4[u]);
      }
      for (; l <= j; ++l) a4[0] = fma(Y[i][l], T[o + l][o + j], a4[0]);
      T[i][o + j] = -((a4[0] + a4[1]) + (a4[2] + a4[3]));
    }
    __syncthreads();
  }
  for (int e = tid; e < QR_OB * QR_OB; e += 256) {
    const int i = e / QR_OB, j = e % QR_OB;
    Tout[e] = (i < w && j < w) ? T[i][j] : 0.0;
  }
}

// Panel width and rows per thread for the panel starting at j0 (Mp rows).
struct PanelShape {
  int nb, rpt;
};
inline PanelShape panel_shape(int64_t Mp) {
  const int rpt = (int)cdiv(Mp, QP_T);
  return PanelShape{rpt <= 5 ? 16 : 8, rpt};  // 6 x 16 doubles per thread would spill
}

gn_status run_panel(double* C, int64_t ldc, int64_t M, int64_t j0, int nbw, double* Tp,
                    const int32_t* gate, int64_t gate_n, hipStream_t s) {
  const PanelShape ps = panel_shape(M - j0);
  const dim3 g(1), b(QP_T);
#define GN_PANEL(R, NBV) qr_panel<R, NBV, QP_T><<<g, b, 0, s>>>(C, ldc, M, j0, nbw, Tp, gate, gate_n)
  switch (ps.rpt) {
    case 1: GN_PANEL(1, 16); break;
    case 2: GN_PANEL(2, 16); break;
    case 3: GN_PANEL(3, 16); break;
    case 4: GN_PANEL(4, 16); break;
    case 5: GN_PANEL(5, 16); break;
    case 6: GN_PANEL(6, 8); break;
    case 7: GN_PANEL(7, 8); break;
    case 8: GN_PANEL(8, 8); break;
    default: return GN_ERR_UNSUPPORTED;
  }
#undef GN_PANEL
  GN_LAUNCH_CHECK();
  return GN_OK;
}

gn_status run_update(const double* Cp, int64_t ldc, int64_t M, int64_t j0, int nbw, double* D,
                    int64_t ldd, int64_t col0, int64_t ncols, const double* Tp, int trans,
                    double* Wp, const int32_t* gate, int64_t gate_n, hipStream_t s) {
  if (ncols <= 0) return GN_OK;
  if (M - j0 > QR_MAXROWS) return GN_ERR_UNSUPPORTED;
  const int nch = (int)cdiv(M - j0, QI_CH);
  const dim3 g((unsigned)nch, (unsigned)cdiv(ncols, QR_NB)), b(256);
  qr_iupd_w<<<g, b, 0, s>>>(Cp, ldc, M, j0, nbw, D, ldd, col0, ncols, Wp, gate, gate_n);
  GN_LAUNCH_CHECK();
  qr_iupd_apply<<<g, b, 0, s>>>(Cp, ldc, M, j0, nbw, D, ldd, col0, ncols, Wp, nch, Tp, trans, gate,
                                gate_n);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

}  // namespace

// one nb x nb T per panel (panels are at least 8 wide)
static size_t qr_t_bytes(int64_t N) {
  return align_up((size_t)(cdiv(N, 8) + 1) * QR_NB * QR_NB * sizeof(double));
}
struct QrWs {
  size_t tin, wp, vb, vt, w2, part, g, tout, total;
};
static QrWs qr_ws_layout(int64_t M, int64_t N) {
  QrWs q{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  const int64_t nw = N > QR_OB ? N : QR_OB;  // widest target (the trailing columns, or V itself)
  q.tin = take(qr_t_bytes(N));
  q.wp = take((size_t)cdiv(M, QI_CH) * QR_NB * QR_OB * sizeof(double));  // inner updates
  q.vb = take((size_t)M * QR_OB * sizeof(double));
  q.vt = take((size_t)M * QR_OB * sizeof(double));
  q.w2 = take((size_t)QR_OB * nw * sizeof(double));
  // partial products V_c^T D_c, one per QO_CH-row chunk
  q.part = take((size_t)cdiv(M, QO_CH) * QR_OB * nw * sizeof(double));
  q.g = take((size_t)QR_OB * QR_OB * sizeof(double));
  q.tout = take((size_t)cdiv(N, QR_OB) * QR_OB * QR_OB * sizeof(double));
  q.total = off;
  return q;
}

size_t qr_ws_bytes(int64_t M, int64_t N) { return qr_ws_layout(M, N).total; }

// Two-level blocked Householder QR: panels (register kernel) inside outer blocks
// of QR_OB columns, panel updates restricted to the block, then one block
// reflector per outer block applied by FP64 MFMA products to the trailing
// columns; Q formed from [I; 0] by the outer blocks right to left.
namespace {
// Pointers into the QR workspace.
struct QrPtrs {
  double *Tin, *Wp, *Vb, *Vt, *W2, *part, *G, *Tout;
};
QrPtrs qr_ptrs(int64_t M, int64_t N, double* ws) {
  const QrWs L = qr_ws_layout(M, N);
  char* base = (char*)ws;
  return QrPtrs{(double*)(base + L.tin), (double*)(base + L.wp),   (double*)(base + L.vb),
                (double*)(base + L.vt),  (double*)(base + L.w2),   (double*)(base + L.part),
                (double*)(base + L.g),   (double*)(base + L.tout)};
}

// D <- (I - V T' V^T) D for an outer block (Mp rows of V), D with ncols columns.
gn_status qr_apply_block(const QrPtrs& w, int64_t Mp, double* D, int64_t ldd, int64_t ncols,
                         const double* Tb, int trans, const int32_t* gate_k, int64_t gate_n,
                         hipStream_t s) {
  if (ncols <= 0) return GN_OK;
  const unsigned nch = (unsigned)cdiv(Mp, QO_CH), nst = (unsigned)cdiv(ncols, QO_CG);
  qr_oupd_w<<<dim3(nch, nst), dim3(256), 0, s>>>(w.Vb, Mp, D, ldd, ncols, w.part, gate_k, gate_n);
  GN_LAUNCH_CHECK();
  qr_oupd_w2<<<dim3((unsigned)cdiv(ncols, QO_CW)), dim3(256), 0, s>>>(w.part, (int)nch, ncols, Tb,
                                                                       trans, w.W2, gate_k, gate_n);
  GN_LAUNCH_CHECK();
  qr_oupd_apply<<<dim3((unsigned)cdiv(Mp, QO_CA), nst), dim3(256), 0, s>>>(w.Vt, Mp, D, ldd, ncols,
                                                                          w.W2, gate_k, gate_n);
  GN_LAUNCH_CHECK();
  return GN_OK;
}
}  // namespace

gn_status launch_qr_factor(int64_t M, int64_t N, double* C, int64_t ldc, double* R, int64_t ldr,
                           double* ws, const int32_t* gate_k, hipStream_t s) {
  if (M < N || M > QR_MAXROWS || N < 1) return GN_ERR_UNSUPPORTED;
  const int64_t gate_n = N;
  const QrPtrs w = qr_ptrs(M, N, ws);
  const int64_t nob = cdiv(N, QR_OB);
  std::vector<OuterPanels> ops((size_t)nob);
  int pi = 0;
  // outer blocks left to right
  for (int64_t ob = 0; ob < nob; ++ob) {
    const int64_t J0 = ob * QR_OB, J1 = (J0 + QR_OB < N) ? J0 + QR_OB : N;
    const int nbo = (int)(J1 - J0);
    OuterPanels& op = ops[(size_t)ob];
    op.count = 0;
    for (int64_t j0 = J0; j0 < J1;) {
      const int nb = panel_shape(M - j0).nb;
      const int nbw = (int)((J1 - j0 < nb) ? (J1 - j0) : nb);
      double* Tp = w.Tin + (size_t)pi * QR_NB * QR_NB;
      GN_TRY(run_panel(C, ldc, M, j0, nbw, Tp, gate_k, gate_n, s));
      GN_TRY(run_update(C, ldc, M, j0, nbw, C, ldc, j0 + nbw, J1 - j0 - nbw, Tp, 1, w.Wp, gate_k,
                        gate_n, s));
      op.off[op.count] = (int)(j0 - J0);
      op.width[op.count] = nbw;
      op.tidx[op.count] = pi;
      ++op.count;
      ++pi;
      j0 += nbw;
    }
    const int64_t Mp = M - J0;
    qr_build_v<<<dim3((unsigned)cdiv(Mp * QR_OB, 256)), dim3(256), 0, s>>>(C, ldc, M, J0, nbo, w.Vb,
                                                                         w.Vt, gate_k, gate_n);
    GN_LAUNCH_CHECK();
    const unsigned nchg = (unsigned)cdiv(Mp, QO_CH);  // G = V^T V
    qr_oupd_w<<<dim3(nchg, 1), dim3(256), 0, s>>>(w.Vb, Mp, w.Vb, QR_OB, QR_OB, w.part, gate_k,
                                                  gate_n);
    GN_LAUNCH_CHECK();
    qr_sum_g<<<dim3(QR_OB * QR_OB / 256), dim3(256), 0, s>>>(w.part, (int)nchg, w.G, gate_k, gate_n);
    GN_LAUNCH_CHECK();
    double* Tb = w.Tout + (size_t)ob * QR_OB * QR_OB;
    qr_merge_t<<<dim3(1), dim3(256), 0, s>>>(w.G, w.Tin, op, nbo, Tb, gate_k, gate_n);
    GN_LAUNCH_CHECK();
    // C2 <- (I - V T^T V^T) C2 on the columns past the block
    GN_TRY(qr_apply_block(w, Mp, C + J0 * ldc + J1, ldc, N - J1, Tb, 1, gate_k, gate_n, s));
  }
  qr_extract_r<<<dim3((unsigned)cdiv(N * N, 256)), dim3(256), 0, s>>>(C, ldc, R, ldr, N, gate_k,
                                                                     gate_n);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

gn_status launch_qr_form_q(int64_t M, int64_t N, const double* C, int64_t ldc, double* Q,
                           int64_t ldq, double* ws, const int32_t* gate_k, hipStream_t s) {
  if (M < N || M > QR_MAXROWS || N < 1) return GN_ERR_UNSUPPORTED;
  const int64_t gate_n = N;
  const QrPtrs w = qr_ptrs(M, N, ws);
  const int64_t nob = cdiv(N, QR_OB);
  // start from [I; 0] and apply the outer blocks right to left,
  // Q2 <- (I - V T V^T) Q2 on rows and columns J0..
  qr_init_q<<<dim3((unsigned)cdiv(M * N, 256)), dim3(256), 0, s>>>(Q, ldq, M, N, gate_k, gate_n);
  GN_LAUNCH_CHECK();
  for (int64_t ob = nob - 1; ob >= 0; --ob) {
    const int64_t J0 = ob * QR_OB, J1 = (J0 + QR_OB < N) ? J0 + QR_OB : N;
    const int nbo = (int)(J1 - J0);
    const int64_t Mp = M - J0, nq = N - J0;
    qr_build_v<<<dim3((unsigned)cdiv(Mp * QR_OB, 256)), dim3(256), 0, s>>>(C, ldc, M, J0, nbo, w.Vb,
                                                                         w.Vt, gate_k, gate_n);
    GN_LAUNCH_CHECK();
    GN_TRY(qr_apply_block(w, Mp, Q + J0 * ldq + J0, ldq, nq, w.Tout + (size_t)ob * QR_OB * QR_OB, 0,
                          gate_k, gate_n, s));
  }
  qr_sign_q<<<dim3((unsigned)cdiv(M * N, 256)), dim3(256), 0, s>>>(C, ldc, Q, ldq, M, N, gate_k,
                                                                  gate_n);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

gn_status launch_qr(int64_t M, int64_t N, double* C, int64_t ldc, double* Q, int64_t ldq, double* R,
                    int64_t ldr, double* ws, const int32_t* gate_k, hipStream_t s) {
  GN_TRY(launch_qr_factor(M, N, C, ldc, R, ldr, ws, gate_k, s));
  return launch_qr_form_q(M, N, C, ldc, Q, ldq, ws, gate_k, s);
}

gn_status launch_truncate(int64_t r, const double* R, int64_t ldr, double tau, int32_t* k,
                          int32_t* status, double* Z, int64_t ldz, hipStream_t s) {
  trunc_scan<<<dim3(1), dim3(256), 0, s>>>(r, R, ldr, tau, k, status);
  GN_LAUNCH_CHECK();
  build_z<<<dim3((unsigned)cdiv(r * r, 256)), dim3(256), 0, s>>>(r, R, ldr, k, Z, ldz);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

size_t qr_batch_t_bytes(int64_t N) { return qr_t_bytes(N); }
size_t qr_batch_wp_bytes(int64_t M, int64_t N) {
  return align_up((size_t)cdiv(M, QU_CH) * QR_NB * N * sizeof(double));
}

gn_status launch_qr_batched(const QrJob* jobs, int32_t count, int64_t maxM, int64_t maxN,
                            hipStream_t s) {
  if (count <= 0 || maxN <= 0) return GN_OK;
  if (maxM > QP_T) return GN_ERR_UNSUPPORTED;
  const unsigned z = (unsigned)count;
  const int64_t np = cdiv(maxN, QR_NB);
  for (int64_t pi = 0; pi < np; ++pi) {
    const int64_t j0 = pi * QR_NB;
    qr_panel_b<<<dim3(1, 1, z), dim3(QP_T), 0, s>>>(jobs, j0);
    GN_LAUNCH_CHECK();
    const dim3 g((unsigned)cdiv(maxM - j0, QU_CH), (unsigned)cdiv(maxN - j0, QU_CG), z);
    qr_upd_w_b<<<g, dim3(256), 0, s>>>(jobs, j0, 0);
    GN_LAUNCH_CHECK();
    qr_upd_apply_b<<<g, dim3(256), 0, s>>>(jobs, j0, 0);
    GN_LAUNCH_CHECK();
  }
  qr_init_q_b<<<dim3((unsigned)cdiv(maxM * maxN, 256), 1, z), dim3(256), 0, s>>>(jobs);
  GN_LAUNCH_CHECK();
  for (int64_t pi = np - 1; pi >= 0; --pi) {
    const int64_t j0 = pi * QR_NB;
    const dim3 g((unsigned)cdiv(maxM - j0, QU_CH), (unsigned)cdiv(maxN - j0, QU_CG), z);
    qr_upd_w_b<<<g, dim3(256), 0, s>>>(jobs, j0, 1);
    GN_LAUNCH_CHECK();
    qr_upd_apply_b<<<g, dim3(256), 0, s>>>(jobs, j0, 1);
    GN_LAUNCH_CHECK();
  }
  qr_signfix_b<<<dim3((unsigned)cdiv(maxM * maxN, 256), 1, z), dim3(256), 0, s>>>(jobs);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

gn_status launch_truncate_batched(const TruncJob* jobs, int32_t count, int64_t maxr,
                                  hipStream_t s) {
  if (count <= 0) return GN_OK;
  trunc_scan_b<<<dim3(1, 1, (unsigned)count), dim3(256), 0, s>>>(jobs);
  GN_LAUNCH_CHECK();
  build_z_b<<<dim3((unsigned)cdiv(maxr * maxr, 256), 1, (unsigned)count), dim3(256), 0, s>>>(jobs);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

}  // namespace gn
