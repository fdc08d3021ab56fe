// Householder QR of the GN core C = Y^T (AX) in FP64 (Algorithm 2.1 step 2 and
// Section 5.1: QR without pivoting, which is rank revealing with high
// probability because X and Y are random), and the eps-truncation of
// Section 5.1.1.
//
// Blocked right-looking QR.  Each panel of nb columns is factored by one
// 512-thread workgroup holding the panel in registers (row t + 512 q of the panel
// in thread t), with fixed-order workgroup reductions for the column norms and
// the reflector dot products; it leaves R and the reflectors (below the
// diagonal, unit diagonal implicit) in place and writes the compact-WY factor T
// (H_1 ... H_nb = I - V T V^T).  One block-update kernel then applies the block
// reflector to the trailing columns, C2 <- (I - V T^T V^T) C2, and, walking the
// panels backwards, accumulates the explicit Q from [I; 0] with Q2 <- (I - V T V^T) Q2.
#include "gn_internal.h"

namespace gn {
namespace {

constexpr int QP_T = 512;
constexpr int QP_WAVES = QP_T / 64;
constexpr int QR_MAXROWS = 4096;
constexpr int QR_NB = 16;  // largest panel width

template <int NV>
__device__ __forceinline__ void qr_block_sum(double (&v)[NV], double* red /*[QP_WAVES][NV]*/,
                                             double* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double x = v[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    v[i] = x;
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[wave * NV + i] = v[i];
  }
  __syncthreads();
  if ((int)threadIdx.x < NV) {
    double s = 0.0;
    for (int w = 0; w < QP_WAVES; ++w) s += red[w * NV + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// The column loop runs at run time; register arrays are only ever indexed by
// compile-time constants (the current column is selected with predicated moves),
// so the panel stays in registers.
template <int RPT, int NB>
__global__ void __launch_bounds__(QP_T) qr_panel(double* __restrict__ C, int64_t ldc, int64_t M,
                                                 int64_t j0, int nbw, double* __restrict__ Tout,
                                                 const int32_t* gate, int64_t gate_n) {
  if (gate && *gate >= gate_n) return;
  __shared__ double red[QP_WAVES * NB];
  __shared__ double bc[NB];
  __shared__ double T[NB][NB];
  const int t = threadIdx.x;
  const int64_t Mp = M - j0;
  double p[RPT][NB];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t row = t + (int64_t)QP_T * q;
#pragma unroll
    for (int c = 0; c < NB; ++c)
      p[q][c] = (row < Mp && c < nbw) ? C[(j0 + row) * ldc + j0 + c] : 0.0;
  }
  if (t < NB * NB) T[t / NB][t % NB] = 0.0;
  __syncthreads();

#pragma unroll 1
  for (int c = 0; c < nbw; ++c) {
    // column c of this thread's rows
    double vr[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      double x = 0.0;
#pragma unroll
      for (int cc = 0; cc < NB; ++cc) x = (cc == c) ? p[q][cc] : x;
      vr[q] = x;
    }
    // squared norm below the pivot, and the pivot (row c lives in thread c, q = 0)
    double v2[2] = {0.0, 0.0};
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int64_t row = t + (int64_t)QP_T * q;
      if (row > c && row < Mp) v2[0] = fma(vr[q], vr[q], v2[0]);
    }
    if (t == c) v2[1] = vr[0];
    qr_block_sum<2>(v2, red, bc);
    const double sigma = bc[0], alpha = bc[1];
    double beta = alpha, tau = 0.0, scale = 0.0;
    if (sigma != 0.0) {
      const double nrm = sqrt(fma(alpha, alpha, sigma));
      beta = (alpha >= 0.0) ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    // reflector v (v_c = 1 implicit) below the pivot
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int64_t row = t + (int64_t)QP_T * q;
      if (row > c && row < Mp) {
        if (tau != 0.0) vr[q] *= scale;
      } else {
        vr[q] = (row == c) ? 1.0 : 0.0;
      }
    }
    // dots of v with every panel column over rows >= c (columns < c hold earlier
    // reflectors there: those dots are the y of the T recurrence)
    double d[NB];
#pragma unroll
    for (int cc = 0; cc < NB; ++cc) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < RPT; ++q) acc = fma(vr[q], p[q][cc], acc);
      d[cc] = acc;
    }
    qr_block_sum<NB>(d, red, bc);
    // apply H_c to the columns right of c; store v and R_cc = beta in column c
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int64_t row = t + (int64_t)QP_T * q;
#pragma unroll
      for (int cc = 0; cc < NB; ++cc) {
        if (cc > c) p[q][cc] = fma(-tau * bc[cc], vr[q], p[q][cc]);
        if (cc == c && row >= c) p[q][cc] = (row == c) ? beta : vr[q];
      }
    }
    // T(:, c) = [ -tau T(0:c, 0:c) y ; tau ],  y = bc[0:c]
    if (t < c) {
      double s = 0.0;
      for (int l = t; l < c; ++l) s = fma(T[t][l], bc[l], s);
      T[t][c] = -tau * s;
    }
    if (t == c) T[c][c] = tau;
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t row = t + (int64_t)QP_T * q;
    if (row >= Mp) continue;
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < nbw) C[(j0 + row) * ldc + j0 + c] = p[q][c];
  }
  if (t < NB * NB) Tout[(t / NB) * QR_NB + (t % NB)] = T[t / NB][t % NB];  // stride QR_NB
}

// D[j0 + i, col0 + j] for 0 <= i < M - j0, 0 <= j < ncols is replaced by
// (I - V Top V^T) D, V the unit-lower reflectors of the panel at (j0, j0) of Cp
// (width nbw) and Top = T^T (trans) or T.  One workgroup per 16 target columns:
// W = V^T D accumulated by 16 row groups, reduced in fixed order, W <- Top W,
// then D -= V W.  Panel rows are staged through LDS 256 at a time.
constexpr int QU_ROWS = 256;
constexpr int QU_RPG = QU_ROWS / 16;  // rows of a staged chunk per row group
__global__ void __launch_bounds__(256) qr_block_update(const double* __restrict__ Cp, int64_t ldc,
                                                       int64_t M, int64_t j0, int nbw,
                                                       double* __restrict__ D, int64_t ldd,
                                                       int64_t col0, int64_t ncols,
                                                       const double* __restrict__ T, int trans,
                                                       const int32_t* gate, int64_t gate_n) {
  if (gate && *gate >= gate_n) return;
  __shared__ double sV[QU_ROWS][QR_NB + 1];
  __shared__ double red[16][QR_NB][17];
  __shared__ double W[QR_NB][17];
  const int tid = threadIdx.x, col = tid & 15, grp = tid >> 4;
  const int64_t j = col0 + (int64_t)blockIdx.x * 16 + col;
  const bool jok = j < col0 + ncols;
  const int64_t Mp = M - j0;
  double w[QR_NB];
#pragma unroll
  for (int c = 0; c < QR_NB; ++c) w[c] = 0.0;

  // stage reflector rows r0 .. r0 + 255 of the panel (explicit unit-lower form)
  auto stage = [&](int64_t r0) {
    const int64_t row = r0 + tid;
#pragma unroll
    for (int c = 0; c < QR_NB; ++c) {
      double v = 0.0;
      if (row < Mp && c < nbw) v = (row < c) ? 0.0 : (row == c ? 1.0 : Cp[(j0 + row) * ldc + j0 + c]);
      sV[tid][c] = v;
    }
  };
  for (int64_t r0 = 0; r0 < Mp; r0 += QU_ROWS) {
    // this thread's 16 rows of the chunk: all loads issued before any use
    double x[QU_RPG];
#pragma unroll
    for (int q = 0; q < QU_RPG; ++q) {
      const int64_t row = r0 + grp + 16 * q;
      x[q] = (jok && row < Mp) ? D[(j0 + row) * ldd + j] : 0.0;
    }
    __syncthreads();
    stage(r0);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QU_RPG; ++q)
#pragma unroll
      for (int c = 0; c < QR_NB; ++c) w[c] = fma(sV[grp + 16 * q][c], x[q], w[c]);
  }
#pragma unroll
  for (int c = 0; c < QR_NB; ++c) red[grp][c][col] = w[c];
  __syncthreads();
  {  // fixed-order reduction over the 16 row groups, then W <- Top W
    const int c = grp;  // 16 x 16 threads: (c, col)
    double s = 0.0;
    for (int g2 = 0; g2 < 16; ++g2) s += red[g2][c][col];
    W[c][col] = s;
  }
  __syncthreads();
  double wt;
  {
    const int c = grp;
    double s = 0.0;
    for (int c2 = 0; c2 < nbw; ++c2) {
      const double top = trans ? T[c2 * QR_NB + c] : T[c * QR_NB + c2];
      s = fma(top, W[c2][col], s);
    }
    wt = (c < nbw) ? s : 0.0;
  }
  __syncthreads();
  W[grp][col] = wt;
  __syncthreads();
  double wc[QR_NB];
#pragma unroll
  for (int c = 0; c < QR_NB; ++c) wc[c] = W[c][col];
  // D -= V W
  for (int64_t r0 = 0; r0 < Mp; r0 += QU_ROWS) {
    double x[QU_RPG];
#pragma unroll
    for (int q = 0; q < QU_RPG; ++q) {
      const int64_t row = r0 + grp + 16 * q;
      x[q] = (jok && row < Mp) ? D[(j0 + row) * ldd + j] : 0.0;
    }
    __syncthreads();
    stage(r0);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QU_RPG; ++q) {
      const int64_t row = r0 + grp + 16 * q;
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < QR_NB; ++c) s = fma(sV[grp + 16 * q][c], wc[c], s);
      if (jok && row < Mp) D[(j0 + row) * ldd + j] = x[q] - s;
    }
  }
}

__global__ void __launch_bounds__(256) qr_init_q(double* Q, int64_t ldq, int64_t M, int64_t N,
                                                 const int32_t* gate, int64_t gate_n) {
  if (gate && *gate >= gate_n) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * N) return;
  const int64_t i = e / N, j = e - i * N;
  Q[i * ldq + j] = (i == j) ? 1.0 : 0.0;
}

// R_ii >= 0: flip row i of R and column i of Q where the Householder diagonal is
// negative; copy the upper triangle of the factored matrix into R.
__global__ void __launch_bounds__(256) qr_signfix(const double* C, int64_t ldc, double* Q,
                                                  int64_t ldq, double* R, int64_t ldr, int64_t M,
                                                  int64_t N, const int32_t* gate, int64_t gate_n) {
  if (gate && *gate >= gate_n) return;
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

// Kept rank: k = first i whose diagonal fails the keep test (|R_ii| >= tau, or
// |R_ii| > 0 when tau <= 0; non-finite always fails); status flags.
__global__ void __launch_bounds__(256) trunc_scan(int64_t r, const double* R, int64_t ldr, double tau,
                                                  int32_t* kout, int32_t* status) {
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

// Z (r x r) = [R[:k, :]^T, 0]: the matrix whose leading k columns are factored
// by the second QR (Section 5.1.1).  Runs only when k < r.
__global__ void __launch_bounds__(256) build_z(int64_t r, const double* R, int64_t ldr,
                                               const int32_t* kdev, double* Z, int64_t ldz) {
  const int32_t k = *kdev;
  if (k >= r) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= r * r) return;
  const int64_t j = e / r, i = e - j * r;  // Z[j][i] = R[i][j] for i < k
  Z[j * ldz + i] = (i < k) ? R[i * ldr + j] : 0.0;
}

// Panel width and rows per thread for the panel starting at j0 (Mp rows).
struct PanelShape {
  int nb, rpt;
};
inline PanelShape panel_shape(int64_t Mp) {
  const int rpt = (int)cdiv(Mp, QP_T);
  return PanelShape{rpt <= 4 ? 16 : 8, rpt};
}

gn_status run_panel(double* C, int64_t ldc, int64_t M, int64_t j0, int nbw, double* Tp,
                    const int32_t* gate, int64_t gate_n, hipStream_t s) {
  const PanelShape ps = panel_shape(M - j0);
  const dim3 g(1), b(QP_T);
#define GN_PANEL(R, NBV) qr_panel<R, NBV><<<g, b, 0, s>>>(C, ldc, M, j0, nbw, Tp, gate, gate_n)
  switch (ps.rpt) {
    case 1: GN_PANEL(1, 16); break;
    case 2: GN_PANEL(2, 16); break;
    case 3: GN_PANEL(3, 16); break;
    case 4: GN_PANEL(4, 16); break;
    case 5: GN_PANEL(5, 8); break;
    case 6: GN_PANEL(6, 8); break;
    case 7: GN_PANEL(7, 8); break;
    case 8: GN_PANEL(8, 8); break;
    default: return GN_ERR_UNSUPPORTED;
  }
#undef GN_PANEL
  GN_LAUNCH_CHECK();
  return GN_OK;
}

}  // namespace

size_t qr_ws_bytes(int64_t M, int64_t N) {
  // one nb x nb T per panel (panels are at least 8 wide)
  return align_up((size_t)(cdiv(N, 8) + 1) * QR_NB * QR_NB * sizeof(double));
}

gn_status launch_qr(int64_t M, int64_t N, double* C, int64_t ldc, double* Q, int64_t ldq, double* R,
                    int64_t ldr, double* ws, const int32_t* gate_k, hipStream_t s) {
  if (M < N || M > QR_MAXROWS || N < 1) return GN_ERR_UNSUPPORTED;
  const int64_t gate_n = N;
  int64_t starts[QR_MAXROWS];
  int widths[QR_MAXROWS];
  int np = 0;
  for (int64_t jj = 0; jj < N;) {
    const int nb = panel_shape(M - jj).nb;
    const int w = (int)((N - jj < nb) ? (N - jj) : nb);
    starts[np] = jj;
    widths[np] = w;
    ++np;
    jj += w;
  }
  // factor: panels left to right, each followed by the trailing update
  for (int pi = 0; pi < np; ++pi) {
    const int64_t j0 = starts[pi];
    const int nbw = widths[pi];
    double* Tp = ws + (size_t)pi * QR_NB * QR_NB;
    GN_TRY(run_panel(C, ldc, M, j0, nbw, Tp, gate_k, gate_n, s));
    const int64_t c0 = j0 + nbw, nt = N - c0;
    if (nt > 0) {
      qr_block_update<<<dim3((unsigned)cdiv(nt, 16)), dim3(256), 0, s>>>(
          C, ldc, M, j0, nbw, C, ldc, c0, nt, Tp, 1, gate_k, gate_n);
      GN_LAUNCH_CHECK();
    }
  }
  // explicit Q: start from [I; 0] and apply the block reflectors right to left
  qr_init_q<<<dim3((unsigned)cdiv(M * N, 256)), dim3(256), 0, s>>>(Q, ldq, M, N, gate_k, gate_n);
  GN_LAUNCH_CHECK();
  for (int pi = np - 1; pi >= 0; --pi) {
    const int64_t j0 = starts[pi];
    const double* Tp = ws + (size_t)pi * QR_NB * QR_NB;
    qr_block_update<<<dim3((unsigned)cdiv(N - j0, 16)), dim3(256), 0, s>>>(
        C, ldc, M, j0, widths[pi], Q, ldq, j0, N - j0, Tp, 0, gate_k, gate_n);
    GN_LAUNCH_CHECK();
  }
  qr_signfix<<<dim3((unsigned)cdiv(M * N, 256)), dim3(256), 0, s>>>(C, ldc, Q, ldq, R, ldr, M, N,
                                                                   gate_k, gate_n);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

gn_status launch_truncate(int64_t r, const double* R, int64_t ldr, double tau, int32_t* k,
                          int32_t* status, double* Z, int64_t ldz, hipStream_t s) {
  trunc_scan<<<dim3(1), dim3(256), 0, s>>>(r, R, ldr, tau, k, status);
  GN_LAUNCH_CHECK();
  build_z<<<dim3((unsigned)cdiv(r * r, 256)), dim3(256), 0, s>>>(r, R, ldr, k, Z, ldz);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

}  // namespace gn
