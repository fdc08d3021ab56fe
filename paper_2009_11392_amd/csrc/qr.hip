// Householder QR of the GN core C = Y^T (AX) in FP64 (Algorithm 2.1 step 2 and
// Section 5.1: QR without pivoting, which is rank revealing with high
// probability because X and Y are random), and the eps-truncation of
// Section 5.1.1.
//
// Blocked right-looking QR.  Each panel of nb columns is factored by one
// 1024-thread workgroup holding the panel in registers (row t + 1024 q of the
// panel in thread t), with fixed-order workgroup reductions for the column norms
// and the reflector dot products.  The panel kernel also forms the compact-WY
// factor T (H_1 ... H_nb = I - V T V^T) and the products V T^T and V T.  The
// trailing matrix is updated as C2 -= (V T^T) (V^T C2) and the explicit Q is
// accumulated backwards as Q2 -= (V T) (V^T Q2), both with the FP64 GEMM.
#include "gn_internal.h"

namespace gn {
namespace {

constexpr int QR_T = 1024;
constexpr int QR_WAVES = QR_T / 64;
constexpr int QR_MAXROWS = 4096;

template <int NV>
__device__ __forceinline__ void qr_block_sum(double (&v)[NV], double (*red)[NV], double* out) {
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
    for (int i = 0; i < NV; ++i) red[wave][i] = v[i];
  }
  __syncthreads();
  if ((int)threadIdx.x < NV) {
    double s = 0.0;
    for (int w = 0; w < QR_WAVES; ++w) s += red[w][threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

template <int RPT, int NB>
__global__ void __launch_bounds__(QR_T) qr_panel(double* __restrict__ C, int64_t ldc, int64_t M,
                                                 int64_t j0, int nbw, double* __restrict__ V,
                                                 double* __restrict__ VTt, double* __restrict__ VTn,
                                                 int64_t ldv, const int32_t* gate, int64_t gate_n) {
  if (gate && *gate >= gate_n) return;
  __shared__ double red[QR_WAVES][NB];
  __shared__ double bc[NB];
  __shared__ double T[NB][NB];
  const int t = threadIdx.x;
  const int64_t Mp = M - j0;
  double p[RPT][NB];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t row = t + (int64_t)QR_T * q;
#pragma unroll
    for (int c = 0; c < NB; ++c)
      p[q][c] = (row < Mp && c < nbw) ? C[(j0 + row) * ldc + j0 + c] : 0.0;
  }
  if (t < NB * NB) T[t / NB][t % NB] = 0.0;
  __syncthreads();

#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (c < nbw) {
      // squared norm of the column below the pivot, and the pivot itself
      double v2[2] = {0.0, 0.0};
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int64_t row = t + (int64_t)QR_T * q;
        if (row > c && row < Mp) v2[0] = fma(p[q][c], p[q][c], v2[0]);
      }
      if (t == c) v2[1] = p[0][c];
      qr_block_sum<2>(v2, reinterpret_cast<double(*)[2]>(&red[0][0]), bc);
      const double sigma = bc[0], alpha = bc[1];
      double beta = alpha, tau = 0.0, scale = 0.0;
      if (sigma != 0.0) {
        const double nrm = sqrt(fma(alpha, alpha, sigma));
        beta = (alpha >= 0.0) ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      __syncthreads();  // bc is reused below
      // reflector v (v_c = 1 implicit) stored below the pivot; R_cc = beta
      double vrow[RPT];
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int64_t row = t + (int64_t)QR_T * q;
        if (row > c && row < Mp) {
          if (tau != 0.0) p[q][c] *= scale;
          vrow[q] = p[q][c];
        } else {
          vrow[q] = (row == c) ? 1.0 : 0.0;
        }
      }
      // dots of v with every panel column over rows >= c
      double d[NB];
#pragma unroll
      for (int cc = 0; cc < NB; ++cc) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < RPT; ++q) s = fma(vrow[q], p[q][cc], s);
        d[cc] = s;
      }
      qr_block_sum<NB>(d, red, bc);
      // apply H_c to the columns right of c
#pragma unroll
      for (int cc = c + 1; cc < NB; ++cc) {
        const double w = tau * bc[cc];
#pragma unroll
        for (int q = 0; q < RPT; ++q) p[q][cc] = fma(-w, vrow[q], p[q][cc]);
      }
      if (t == c) p[0][c] = beta;
      // T(:, c) = [ -tau T(0:c, 0:c) y ; tau ],  y = V(:, 0:c)^T v
      if (t < c) {
        double s = 0.0;
        for (int l = t; l < c; ++l) s = fma(T[t][l], bc[l], s);
        T[t][c] = -tau * s;
      }
      if (t == c) T[c][c] = tau;
      __syncthreads();
    }
  }

  // write back: R (rows <= col) and reflectors (below) into C, explicit V, V T^T, V T
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t row = t + (int64_t)QR_T * q;
    if (row >= Mp) continue;
    double vv[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) vv[c] = (row < c) ? 0.0 : (row == c ? 1.0 : p[q][c]);
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      if (c >= nbw) continue;
      C[(j0 + row) * ldc + j0 + c] = p[q][c];
      V[(j0 + row) * ldv + j0 + c] = vv[c];
      double st = 0.0, sn = 0.0;
#pragma unroll
      for (int c2 = 0; c2 < NB; ++c2) {
        if (c2 >= nbw) continue;
        st = fma(vv[c2], T[c][c2], st);  // (V T^T)[row][c]
        sn = fma(vv[c2], T[c2][c], sn);  // (V T)[row][c]
      }
      VTt[(j0 + row) * ldv + j0 + c] = st;
      VTn[(j0 + row) * ldv + j0 + c] = sn;
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
  __shared__ int s_nonfinite[256];
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
  s_nonfinite[threadIdx.x] = nonfinite;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s_first[threadIdx.x] = min(s_first[threadIdx.x], s_first[threadIdx.x + w]);
      s_nonfinite[threadIdx.x] |= s_nonfinite[threadIdx.x + w];
    }
    __syncthreads();
  }
  const int64_t k = s_first[0];
  // non-monotone: a kept-size diagonal after the first failing one
  int nm = 0;
  for (int64_t i = k + 1 + threadIdx.x; i < r; i += 256) {
    const double d = R[i * ldr + i];
    const double a = fabs(d);
    if (isfinite(d) && ((tau > 0.0) ? (a >= tau) : (a > 0.0))) nm = 1;
  }
  __syncthreads();
  s_nonfinite[threadIdx.x] = nm;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s_nonfinite[threadIdx.x] |= s_nonfinite[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *kout = (int32_t)k;
    *status = (nonfinite ? 1 : 0) | (k == 0 ? 2 : 0) | (s_nonfinite[0] ? 4 : 0);
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

template <int RPT, int NB>
gn_status run_panel(double* C, int64_t ldc, int64_t M, int64_t j0, int nbw, double* V, double* VTt,
                    double* VTn, int64_t ldv, const int32_t* gate, int64_t gate_n, hipStream_t s) {
  qr_panel<RPT, NB><<<dim3(1), dim3(QR_T), 0, s>>>(C, ldc, M, j0, nbw, V, VTt, VTn, ldv, gate,
                                                   gate_n);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

inline int panel_width(int64_t Mp) { return Mp > 2048 ? 8 : 16; }

}  // namespace

size_t qr_ws_bytes(int64_t M, int64_t N) {
  return 3 * align_up((size_t)M * N * sizeof(double)) + align_up((size_t)16 * N * sizeof(double));
}

gn_status launch_qr(int64_t M, int64_t N, double* C, int64_t ldc, double* Q, int64_t ldq, double* R,
                    int64_t ldr, double* ws, const int32_t* gate_k, hipStream_t s) {
  if (M < N || M > QR_MAXROWS || N < 1) return GN_ERR_UNSUPPORTED;
  double* V = ws;
  double* VTt = V + align_up((size_t)M * N * sizeof(double)) / sizeof(double);
  double* VTn = VTt + align_up((size_t)M * N * sizeof(double)) / sizeof(double);
  double* W = VTn + align_up((size_t)M * N * sizeof(double)) / sizeof(double);
  const int64_t ldv = N, ldw = N;
  const int64_t gate_n = N;

  // factor: panels left to right
  int64_t j0 = 0;
  while (j0 < N) {
    const int64_t Mp = M - j0;
    const int nb = panel_width(Mp);
    const int nbw = (int)((N - j0 < nb) ? (N - j0) : nb);
    const int rpt = (int)cdiv(Mp, QR_T);
    if (rpt <= 1)
      GN_TRY((run_panel<1, 16>(C, ldc, M, j0, nbw, V, VTt, VTn, ldv, gate_k, gate_n, s)));
    else if (rpt <= 2)
      GN_TRY((run_panel<2, 16>(C, ldc, M, j0, nbw, V, VTt, VTn, ldv, gate_k, gate_n, s)));
    else if (rpt <= 3)
      GN_TRY((run_panel<3, 8>(C, ldc, M, j0, nbw, V, VTt, VTn, ldv, gate_k, gate_n, s)));
    else
      GN_TRY((run_panel<4, 8>(C, ldc, M, j0, nbw, V, VTt, VTn, ldv, gate_k, gate_n, s)));
    const int64_t Nt = N - j0 - nbw;
    if (Nt > 0) {
      // W = V_p^T C2  (nbw x Nt),  C2 = C[j0:, j0+nbw:]
      MatRef vt{V + j0 * ldv + j0, GN_DT_F64, 1, ldv};
      MatRef c2{C + j0 * ldc + j0 + nbw, GN_DT_F64, ldc, 1};
      GN_TRY(launch_dgemm(nbw, Nt, Mp, 1.0, vt, c2, 0.0, W, ldw, 1, nullptr, false, s, gate_k,
                          gate_n, true));
      // C2 -= (V T^T) W
      MatRef vtt{VTt + j0 * ldv + j0, GN_DT_F64, ldv, 1};
      MatRef w{W, GN_DT_F64, ldw, 1};
      GN_TRY(launch_dgemm(Mp, Nt, nbw, -1.0, vtt, w, 1.0, C + j0 * ldc + j0 + nbw, ldc, 1, nullptr,
                          false, s, gate_k, gate_n, true));
    }
    j0 += nbw;
  }

  // explicit Q: start from [I; 0] and apply the block reflectors right to left
  {
    const int64_t tot = M * N;
    qr_init_q<<<dim3((unsigned)cdiv(tot, 256)), dim3(256), 0, s>>>(Q, ldq, M, N, gate_k, gate_n);
    GN_LAUNCH_CHECK();
  }
  // recompute the panel boundaries and walk them backwards
  int64_t starts[QR_MAXROWS];
  int widths[QR_MAXROWS];
  int np = 0;
  for (int64_t jj = 0; jj < N;) {
    const int nb = panel_width(M - jj);
    const int w = (int)((N - jj < nb) ? (N - jj) : nb);
    starts[np] = jj;
    widths[np] = w;
    ++np;
    jj += w;
  }
  for (int pi = np - 1; pi >= 0; --pi) {
    const int64_t jp = starts[pi];
    const int nbw = widths[pi];
    const int64_t Mp = M - jp, Nq = N - jp;
    MatRef vt{V + jp * ldv + jp, GN_DT_F64, 1, ldv};
    MatRef q2{Q + jp * ldq + jp, GN_DT_F64, ldq, 1};
    GN_TRY(launch_dgemm(nbw, Nq, Mp, 1.0, vt, q2, 0.0, W, ldw, 1, nullptr, false, s, gate_k, gate_n,
                        true));
    MatRef vtn{VTn + jp * ldv + jp, GN_DT_F64, ldv, 1};
    MatRef w{W, GN_DT_F64, ldw, 1};
    GN_TRY(launch_dgemm(Mp, Nq, nbw, -1.0, vtn, w, 1.0, Q + jp * ldq + jp, ldq, 1, nullptr, false,
                        s, gate_k, gate_n, true));
  }
  {
    const int64_t tot = M * N;
    qr_signfix<<<dim3((unsigned)cdiv(tot, 256)), dim3(256), 0, s>>>(C, ldc, Q, ldq, R, ldr, M, N,
                                                                     gate_k, gate_n);
    GN_LAUNCH_CHECK();
  }
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
