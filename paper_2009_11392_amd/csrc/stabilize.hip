// The other stabilizations of the GN core (Section 5.1.1) and the power-method
// check of plain GN (Section 5.1.2), all in FP64.
//
// SVD route and perturbation (a).  After the Householder QR C = Q1 R, the SVD of
// R comes from one-sided (Hestenes) Jacobi on the rows of R: the vectors w_c =
// R[c, :] are rotated in pairs until mutually orthogonal, W J = [w'_c] with J
// orthogonal, so R^T J = U' Sigma and R = J Sigma U'^T, C = (Q1 J) Sigma U'^T.
// The rotation of a pair zeroes its inner product (Rutishauser's formulas) and
// is skipped when |w_p . w_q| <= sqrt(r) u ||w_p|| ||w_q||; one-sided Jacobi
// keeps the singular values accurate relative to the scale of each vector.
// Vectors are grouped in blocks of B; a launch pairs every block with one other
// (round robin over blocks, the circle method), so a sweep over all pairs takes
// nbe - 1 launches.  One 256-thread workgroup holds the 2B vectors of its pair
// in registers (element i of every vector in thread i mod 256) and runs B inner
// rounds of B disjoint pairs between the two blocks (the first launch of a sweep
// runs the full 2B - 1 rounds, which also covers the pairs inside each block).
// Each inner round needs one workgroup reduction of 3B dots; lane p then
// computes the rotation of pair p and every lane applies the B rotations to its
// elements.  The rotations are accumulated in a 2B x 2B matrix in LDS and applied
// to J once per launch.  A sweep in which no workgroup rotated sets the converged
// flag, after which every launch returns at once; the sweep count is bounded.
//
// Perturbation (b).  Householder QR with column pivoting (largest remaining
// column norm, lowest index on ties; norms recomputed at every step, not
// downdated) run on R, whose column norms are C's, gives the permutation P; the
// blocked QR of R P then gives R P = Q_R R_p, so C P = (Q1 Q_R) R_p.  R_p's small
// diagonal entries are raised to tau and the QR of the lifted R_p^T = Q3 R3 puts
// the inverse in the factored form of the truncated core: the core
// pseudoinverse is (P Q3) R3^{-T} (Q1 Q_R)^T.
//
// Perturbation (c).  R's diagonal (non-negative after the sign fix) raised to tau.
//
// Power-method check.  nv start vectors (Philox stream 6) are driven through
// y = T^{-T} v and z = T^{-1} y by the blocked triangular solves of the factor
// application, T being the factor whose inverse multiplies AX; the estimate is
// the largest ||y|| over unit iterates v.
#include "gn_internal.h"
#include "wave_ops.h"

#include <math.h>

#include <utility>

namespace gn {
namespace {

constexpr int JT = 256;      // threads of a Jacobi workgroup
constexpr int JW = JT / 64;  // its waves
constexpr int kMaxSweeps = 20;
constexpr int kSortMax = 4096;

constexpr int pow2_at_least(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Position q of a circle-method round robin over n players in round t.
__host__ __device__ constexpr int rr_pos(int q, int t, int n) {
  return q == 0 ? 0 : 1 + (q - 1 + t) % (n - 1);
}
// Pair p of inner round s over the 2B columns of a block pair: FULL covers every
// pair of the 2B columns in 2B - 1 rounds; otherwise only pairs across the two
// blocks, in B rounds.
template <int B, bool FULL>
__host__ __device__ constexpr int pair_a(int p, int s) {
  return FULL ? rr_pos(p, s, 2 * B) : p;
}
template <int B, bool FULL>
__host__ __device__ constexpr int pair_b(int p, int s) {
  return FULL ? rr_pos(2 * B - 1 - p, s, 2 * B) : B + (p + s) % B;
}

__device__ __forceinline__ void jacobi_rotation(double a, double b, double g, double tol, double& c,
                                                double& s, int& rot) {
  c = 1.0;
  s = 0.0;
  rot = 0;
  if (g != 0.0 && fabs(g) > tol * sqrt(a) * sqrt(b)) {
    const double zeta = (b - a) / (2.0 * g);
    const double az = fabs(zeta);
    double t = (az < 1e150) ? 1.0 / (az + sqrt(fma(az, az, 1.0))) : 0.5 / az;
    if (zeta < 0.0) t = -t;
    c = 1.0 / sqrt(fma(t, t, 1.0));
    s = c * t;
    rot = 1;
  }
}

template <int RPT, int B, bool FULL, int S>
__device__ __forceinline__ void jacobi_inner(double (&w)[RPT][2 * B],
                                             double (*part)[JW][pow2_at_least(3 * B)],
                                             double (*Gm)[2 * B + 1], int tid, int lane, int wave,
                                             double tol, int* rotated) {
  constexpr int NV = pow2_at_least(3 * B);
  constexpr int C2 = 2 * B;
  constexpr int buf = S & 1;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
#pragma unroll
  for (int p = 0; p < B; ++p) {
    const int a = pair_a<B, FULL>(p, S), b = pair_b<B, FULL>(p, S);
    double sa = 0.0, sb = 0.0, sg = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      sa = fma(w[q][a], w[q][a], sa);
      sb = fma(w[q][b], w[q][b], sb);
      sg = fma(w[q][a], w[q][b], sg);
    }
    acc[p] = sa;
    acc[B + p] = sb;
    acc[2 * B + p] = sg;
  }
  int slot;
  const double ws = wave_transpose_sum<NV>(acc, lane, &slot);
  constexpr int kLowBits = 64 / NV;
  if ((lane & (kLowBits - 1)) == 0) part[buf][wave][slot] = ws;
  __syncthreads();
  // lane p < B of every wave forms the rotation of pair p from the same sums
  double c = 1.0, s = 0.0;
  int rot = 0;
  if (lane < B) {
    double a = 0.0, b = 0.0, g = 0.0;
#pragma unroll
    for (int v = 0; v < JW; ++v) {
      a += part[buf][v][lane];
      b += part[buf][v][B + lane];
      g += part[buf][v][2 * B + lane];
    }
    jacobi_rotation(a, b, g, tol, c, s, rot);
  }
  if (rot && wave == 0) *rotated = 1;
#pragma unroll
  for (int p = 0; p < B; ++p) {
    const int a = pair_a<B, FULL>(p, S), b = pair_b<B, FULL>(p, S);
    const double cp = readlane_f64(c, p), sp = readlane_f64(s, p);
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const double wa = w[q][a], wb = w[q][b];
      w[q][a] = fma(cp, wa, -sp * wb);
      w[q][b] = fma(sp, wa, cp * wb);
    }
    if (tid < C2) {
      const double ga = Gm[tid][a], gb = Gm[tid][b];
      Gm[tid][a] = fma(cp, ga, -sp * gb);
      Gm[tid][b] = fma(sp, ga, cp * gb);
    }
  }
}

template <int RPT, int B, bool FULL, int... S>
__device__ __forceinline__ void jacobi_rounds(std::integer_sequence<int, S...>,
                                              double (&w)[RPT][2 * B],
                                              double (*part)[JW][pow2_at_least(3 * B)],
                                              double (*Gm)[2 * B + 1], int tid, int lane, int wave,
                                              double tol, int* rotated) {
  (jacobi_inner<RPT, B, FULL, S>(w, part, Gm, tid, lane, wave, tol, rotated), ...);
}

// One launch of a sweep: workgroup p takes blocks (rr_pos(p), rr_pos(nbe-1-p))
// of round t.  W and J hold vector c at [c*r, c*r + r).
template <int RPT, int B, bool FULL>
__global__ void __launch_bounds__(JT) jacobi_round(double* __restrict__ W, double* __restrict__ J,
                                                   int32_t* __restrict__ ctl, int64_t r, int nbe,
                                                   int t, int sweep, double tol) {
  if (ctl[0] != 0) return;  // converged in an earlier sweep
  constexpr int C2 = 2 * B;
  constexpr int NV = pow2_at_least(3 * B);
  __shared__ double part[2][JW][NV];
  __shared__ double Gm[C2][C2 + 1];
  __shared__ int rotated;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int p = blockIdx.x;
  const int bi = rr_pos(p, t, nbe), bj = rr_pos(nbe - 1 - p, t, nbe);
  int64_t col[C2];
#pragma unroll
  for (int c = 0; c < C2; ++c) col[c] = (c < B) ? (int64_t)bi * B + c : (int64_t)bj * B + (c - B);
  double w[RPT][C2];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t i = tid + (int64_t)q * JT;
#pragma unroll
    for (int c = 0; c < C2; ++c) w[q][c] = (i < r && col[c] < r) ? W[col[c] * r + i] : 0.0;
  }
  for (int e = tid; e < C2 * C2; e += JT) Gm[e / C2][e % C2] = (e / C2 == e % C2) ? 1.0 : 0.0;
  if (tid == 0) rotated = 0;
  __syncthreads();
  if (FULL)
    jacobi_rounds<RPT, B, FULL>(std::make_integer_sequence<int, C2 - 1>{}, w, part, Gm, tid, lane,
                                wave, tol, &rotated);
  else
    jacobi_rounds<RPT, B, FULL>(std::make_integer_sequence<int, B>{}, w, part, Gm, tid, lane, wave,
                                tol, &rotated);
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t i = tid + (int64_t)q * JT;
    if (i < r) {
#pragma unroll
      for (int c = 0; c < C2; ++c)
        if (col[c] < r) W[col[c] * r + i] = w[q][c];
    }
  }
  __syncthreads();
  // J[:, cols] <- J[:, cols] Gm
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t i = tid + (int64_t)q * JT;
    if (i < r) {
      double jr[C2];
#pragma unroll
      for (int c = 0; c < C2; ++c) jr[c] = (col[c] < r) ? J[col[c] * r + i] : 0.0;
#pragma unroll
      for (int c = 0; c < C2; ++c) {
        double o = 0.0;
#pragma unroll
        for (int d = 0; d < C2; ++d) o = fma(jr[d], Gm[d][c], o);
        if (col[c] < r) J[col[c] * r + i] = o;
      }
    }
  }
  if (tid == 0 && rotated) atomicAdd(&ctl[2 + sweep], 1);
}

// The same launch with one wave per pair: B waves, wave p holding element l +
// 64 q (q < E) of block I's vector p (wa) and of one block-J vector (wb).  In
// cross round s wave p pairs I_p with J_{(p+s) mod B}; after the round every
// wave passes its J vector to wave p - 1 through a double-buffered LDS ring, so
// a round needs one barrier and no workgroup reduction (the three dots are
// reduced inside the wave).  A FULL launch first runs the circle method inside
// each block with the 2B vectors in LDS (waves 0 .. B/2-1 on block I, the rest
// on block J).
// Sum over the 64 lanes, the same value in every lane: within each 16-lane row
// by lane swaps (xor 1, xor 2, then the 8- and 16-lane mirrors, each pairing
// lanes that hold disjoint partial sums), then the four row sums in a fixed order.
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

template <int E>
__device__ __forceinline__ void wave_dots(const double (&a)[E], const double (&b)[E], int lane,
                                          double& alpha, double& beta, double& gamma) {
  (void)lane;
  double s[3][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};  // two chains per dot
#pragma unroll
  for (int q = 0; q < E; ++q) {
    s[0][q & 1] = fma(a[q], a[q], s[0][q & 1]);
    s[1][q & 1] = fma(b[q], b[q], s[1][q & 1]);
    s[2][q & 1] = fma(a[q], b[q], s[2][q & 1]);
  }
  alpha = wave_sum_dpp(s[0][0] + s[0][1]);
  beta = wave_sum_dpp(s[1][0] + s[1][1]);
  gamma = wave_sum_dpp(s[2][0] + s[2][1]);
}

template <int E>
__device__ __forceinline__ void rotate_pair(double (&a)[E], double (&b)[E], double c, double s) {
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const double x = a[q], y = b[q];
    a[q] = fma(c, x, -s * y);
    b[q] = fma(s, x, c * y);
  }
}

template <int E, int B, bool FULL>
__global__ void __launch_bounds__(64 * B) jacobi_ring(double* __restrict__ W, double* __restrict__ J,
                                                      int32_t* __restrict__ ctl, int64_t r, int nbe,
                                                      int t, int sweep, double tol) {
  if (ctl[0] != 0) return;  // converged in an earlier sweep
  constexpr int C2 = 2 * B;
  __shared__ double ring[2][B][E * 64];
  __shared__ double Gm[C2][C2 + 1];
  __shared__ int rotated;
  const int tid = threadIdx.x, lane = tid & 63, p = tid >> 6;
  const int bi = rr_pos(blockIdx.x, t, nbe), bj = rr_pos(nbe - 1 - blockIdx.x, t, nbe);
  const int64_t colI = (int64_t)bi * B + p;
  double wa[E], wb[E];
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int64_t i = lane + 64 * q;
    wa[q] = (i < r && colI < r) ? W[colI * r + i] : 0.0;
    const int64_t cj = (int64_t)bj * B + p;
    wb[q] = (i < r && cj < r) ? W[cj * r + i] : 0.0;
  }
  for (int e = tid; e < C2 * C2; e += 64 * B) Gm[e / C2][e % C2] = (e / C2 == e % C2) ? 1.0 : 0.0;
  if (tid == 0) rotated = 0;
  int rot_any = 0;
  if (FULL) {
    // pairs inside each block: ring[0] holds block I, ring[1] block J
#pragma unroll
    for (int q = 0; q < E; ++q) {
      ring[0][p][lane + 64 * q] = wa[q];
      ring[1][p][lane + 64 * q] = wb[q];
    }
    __syncthreads();
    const int half = B / 2;
    const int blk = (p < half) ? 0 : 1, pq = p % half;
    for (int s2 = 0; s2 < B - 1; ++s2) {
      const int a = rr_pos(pq, s2, B), b = rr_pos(B - 1 - pq, s2, B);
      double xa[E], xb[E];
#pragma unroll
      for (int q = 0; q < E; ++q) {
        xa[q] = ring[blk][a][lane + 64 * q];
        xb[q] = ring[blk][b][lane + 64 * q];
      }
      double al, be, ga, c, sn;
      int rot;
      wave_dots<E>(xa, xb, lane, al, be, ga);
      jacobi_rotation(al, be, ga, tol, c, sn, rot);
      rot_any |= rot;
      rotate_pair<E>(xa, xb, c, sn);
#pragma unroll
      for (int q = 0; q < E; ++q) {
        ring[blk][a][lane + 64 * q] = xa[q];
        ring[blk][b][lane + 64 * q] = xb[q];
      }
      if (lane < C2) {
        const int ga_ = blk * B + a, gb_ = blk * B + b;
        const double g1 = Gm[lane][ga_], g2 = Gm[lane][gb_];
        Gm[lane][ga_] = fma(c, g1, -sn * g2);
        Gm[lane][gb_] = fma(sn, g1, c * g2);
      }
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < E; ++q) {
      wa[q] = ring[0][p][lane + 64 * q];
      wb[q] = ring[1][p][lane + 64 * q];
    }
    __syncthreads();
  }
  // cross rounds: wave p pairs I_p with J_{(p+s) mod B}
  for (int s2 = 0; s2 < B; ++s2) {
    const int jb = (p + s2) % B;
    double al, be, ga, c, sn;
    int rot;
    wave_dots<E>(wa, wb, lane, al, be, ga);
    jacobi_rotation(al, be, ga, tol, c, sn, rot);
    rot_any |= rot;
    rotate_pair<E>(wa, wb, c, sn);
    if (lane < C2) {
      const double g1 = Gm[lane][p], g2 = Gm[lane][B + jb];
      Gm[lane][p] = fma(c, g1, -sn * g2);
      Gm[lane][B + jb] = fma(sn, g1, c * g2);
    }
    if (s2 + 1 < B) {
      const int buf = s2 & 1;
#pragma unroll
      for (int q = 0; q < E; ++q) ring[buf][p][lane + 64 * q] = wb[q];
      __syncthreads();
      const int from = (p + 1) % B;
#pragma unroll
      for (int q = 0; q < E; ++q) wb[q] = ring[buf][from][lane + 64 * q];
    }
  }
  const int64_t cjf = (int64_t)bj * B + (p + B - 1) % B;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int64_t i = lane + 64 * q;
    if (i < r) {
      if (colI < r) W[colI * r + i] = wa[q];
      if (cjf < r) W[cjf * r + i] = wb[q];
    }
  }
  if (rot_any && lane == 0) rotated = 1;
  __syncthreads();
  // J[:, cols] <- J[:, cols] Gm, cols = block I then block J; each thread keeps
  // its rows of the 2B columns in registers and takes Gm one column at a time
  constexpr int JR = (E + B - 1) / B;  // rows per thread (r <= 64 E)
  int64_t col[C2];
#pragma unroll
  for (int c = 0; c < C2; ++c) col[c] = (c < B) ? (int64_t)bi * B + c : (int64_t)bj * B + (c - B);
  double jr[JR][C2];
#pragma unroll
  for (int q = 0; q < JR; ++q) {
    const int64_t i = tid + (int64_t)q * 64 * B;
#pragma unroll
    for (int c = 0; c < C2; ++c) jr[q][c] = (i < r && col[c] < r) ? J[col[c] * r + i] : 0.0;
  }
#pragma unroll
  for (int c = 0; c < C2; ++c) {
    double g[C2];
#pragma unroll
    for (int d = 0; d < C2; ++d) g[d] = Gm[d][c];
#pragma unroll
    for (int q = 0; q < JR; ++q) {
      const int64_t i = tid + (int64_t)q * 64 * B;
      double o = 0.0;
#pragma unroll
      for (int d = 0; d < C2; ++d) o = fma(jr[q][d], g[d], o);
      if (i < r && col[c] < r) J[col[c] * r + i] = o;
    }
  }
  if (tid == 0 && rotated) atomicAdd(&ctl[2 + sweep], 1);
}

__global__ void __launch_bounds__(64) jacobi_sweep_end(int32_t* ctl, int sweep) {
  if (threadIdx.x != 0 || ctl[0] != 0) return;
  ctl[1] = sweep + 1;
  if (ctl[2 + sweep] == 0) ctl[0] = 1;
}

// W = rows of R (vector c = R[c, :], zero below the diagonal), J = I, counters 0.
__global__ void __launch_bounds__(256) jacobi_init(const double* __restrict__ R, int64_t ldr,
                                                   int64_t r, double* __restrict__ W,
                                                   double* __restrict__ J, int32_t* ctl) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < 2 + kMaxSweeps) ctl[e] = 0;
  if (e >= r * r) return;
  const int64_t c = e / r, i = e - c * r;
  W[e] = (i >= c) ? R[c * ldr + i] : 0.0;
  J[e] = (i == c) ? 1.0 : 0.0;
}

// sigma[c] = ||W[c*r .. c*r + r)||, one wave per vector, fixed-order sums.
__global__ void __launch_bounds__(256) vec_norms(const double* __restrict__ W, int64_t r,
                                                 double* __restrict__ sigma) {
  const int lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= r) return;
  double s = 0.0;
  for (int64_t i = lane; i < r; i += 64) {
    const double x = W[c * r + i];
    s = fma(x, x, s);
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) sigma[c] = sqrt(s);
}

// Sort sigma descending (ties by index, NaN first), write perm and the sorted
// values, the kept rank and the status bits.  lift: perturbation (a) (k = r, bit
// 16 when something was raised); else the SVD truncation (k = count >= tau, or
// > 0 when tau <= 0).  Bit 32: Jacobi stopped at the sweep limit.
__global__ void __launch_bounds__(1024) svd_sort(const double* __restrict__ sigma, int64_t r,
                                                 double tau, int lift, const int32_t* ctl,
                                                 int32_t* __restrict__ perm,
                                                 double* __restrict__ sig_sorted, int32_t* kout,
                                                 int32_t* status) {
  __shared__ double key[kSortMax];
  __shared__ int idx[kSortMax];
  __shared__ int s_first, s_nf, s_low;
  const int tid = threadIdx.x;
  int n = 1;
  while (n < r) n <<= 1;
  for (int i = tid; i < n; i += 1024) {
    double v = (i < r) ? sigma[i] : -INFINITY;
    if (i < r && isnan(v)) v = INFINITY;
    key[i] = v;
    idx[i] = i;
  }
  if (tid == 0) {
    s_first = (int)r;
    s_nf = 0;
    s_low = 0;
  }
  __syncthreads();
  for (int size = 2; size <= n; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = tid; i < n; i += 1024) {
        const int j = i ^ stride;
        if (j > i) {
          const bool first_before = (key[i] > key[j]) || (key[i] == key[j] && idx[i] < idx[j]);
          const bool want = (i & size) == 0;  // this run in "comes before" order
          if (first_before != want) {
            const double tk = key[i];
            key[i] = key[j];
            key[j] = tk;
            const int ti = idx[i];
            idx[i] = idx[j];
            idx[j] = ti;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int j = tid; j < r; j += 1024) {
    const double v = sigma[idx[j]];
    perm[j] = idx[j];
    sig_sorted[j] = v;
    if (!isfinite(v)) atomicOr(&s_nf, 1);
    const bool keep = isfinite(v) && ((tau > 0.0) ? (v >= tau) : (v > 0.0));
    if (!keep) atomicMin(&s_first, j);
    if (lift && !(v >= tau)) atomicOr(&s_low, 1);
  }
  __syncthreads();
  if (tid == 0) {
    const int k = lift ? (int)r : s_first;
    *kout = k;
    *status = (s_nf ? 1 : 0) | (k == 0 ? 2 : 0) | (lift && s_low ? 16 : 0) | (ctl[0] == 0 ? 32 : 0);
  }
}

// dst[i*r + j] = src[perm[j]*r + i] (/ sig[j], or 0 when sig[j] == 0, if sig).
__global__ void __launch_bounds__(256) gather_transpose(const double* __restrict__ src,
                                                        const int32_t* __restrict__ perm,
                                                        const double* __restrict__ sig, int64_t r,
                                                        double* __restrict__ dst) {
  __shared__ double tile[32][33];
  const int64_t j0 = (int64_t)blockIdx.x * 32, i0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int y = ty; y < 32; y += 8) {
    const int64_t j = j0 + y, i = i0 + tx;
    double v = 0.0;
    if (j < r && i < r) {
      v = src[(int64_t)perm[j] * r + i];
      if (sig) {
        const double sv = sig[j];
        v = (sv != 0.0) ? v / sv : 0.0;
      }
    }
    tile[y][tx] = v;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int64_t i = i0 + y, j = j0 + tx;
    if (i < r && j < r) dst[i * r + j] = tile[tx][y];
  }
}

// R2 = diag(sig) (lift: diag(max(sig, tau))), zero elsewhere.
__global__ void __launch_bounds__(256) diag_matrix(const double* __restrict__ sig, int64_t r,
                                                   double tau, int lift, double* __restrict__ R2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= r * r) return;
  const int64_t i = e / r, j = e - i * r;
  double v = 0.0;
  if (i == j) {
    v = sig[i];
    if (lift && !(v >= tau)) v = tau;
  }
  R2[e] = v;
}

// ---------------------------------------------------------------------------- pivoted QR
// B = R (vector c = column c of R at B[c*r .. c*r + r)), perm = identity.
__global__ void __launch_bounds__(256) qrcp_init(const double* __restrict__ R, int64_t ldr,
                                                 int64_t r, double* __restrict__ Bc,
                                                 int32_t* __restrict__ perm) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < r) perm[e] = (int32_t)e;
  if (e >= r * r) return;
  const int64_t c = e / r, i = e - c * r;
  Bc[e] = R[i * ldr + c];
}

// One pivoting step in one launch.  Every workgroup finds the pivot p of step j
// (the largest norm among columns not pivoted before step j, lowest index on
// ties, NaN first), stages column p (rows j..r-1) in LDS with its squared norm
// below row j, and applies the reflector of column p to its own columns, one
// wave per column, writing their new trailing norms to nrm_out.  A wave loads its
// column (rows j..r-1, 64 per lane at most) into registers before the pivot is
// known, so the update and the recomputed norm take one pass.  The reflector is
// v = [1; x_p(j+1:) / (alpha - beta)], tau_h = (beta - alpha) / beta, and the
// scale is applied on the fly.  Column p itself is never written again (only the
// permutation is needed), and the pivot record is stamped with the step, so the
// launch has no write a concurrent workgroup reads.  Workgroup 0 records p.
constexpr int QCP_T = 256;
constexpr int QCP_COLS = QCP_T / 64;  // columns per workgroup, one per wave

__device__ __forceinline__ void argmax_take(double& v, int& i, double v2, int i2) {
  if (v2 > v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
}

template <int RPL>  // rows per lane: r <= 64 RPL
__global__ void __launch_bounds__(QCP_T) qrcp_step(double* __restrict__ Bc,
                                                   const double* __restrict__ nrm_in,
                                                   double* __restrict__ nrm_out,
                                                   int32_t* __restrict__ stamp,
                                                   int32_t* __restrict__ perm, int64_t r,
                                                   int64_t j) {
  __shared__ double sv[QCP_T / 64];
  __shared__ int si[QCP_T / 64];
  __shared__ double sred[QCP_T / 64];
  __shared__ double xp[4096];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // this wave's column, rows j..r-1, loaded first
  const int64_t c = (int64_t)blockIdx.x * QCP_COLS + wave;
  const bool live = c < r && stamp[c] >= j;
  double x[RPL];
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int64_t i = lane + 64 * q;
    x[q] = (live && i >= j && i < r) ? Bc[c * r + i] : 0.0;
  }
  // pivot: per-thread scan, wave argmax by shuffles, then the waves' results
  double best = -1.0;
  int bi = (int)r;
  for (int64_t cc = tid; cc < r; cc += QCP_T) {
    if (stamp[cc] < j) continue;  // pivoted at an earlier step
    double val = nrm_in[cc];
    if (isnan(val)) val = INFINITY;
    argmax_take(best, bi, val, (int)cc);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double v2 = __shfl_xor(best, off, 64);
    const int i2 = __shfl_xor(bi, off, 64);
    argmax_take(best, bi, v2, i2);
  }
  if (lane == 0) {
    sv[wave] = best;
    si[wave] = bi;
  }
  __syncthreads();
  best = sv[0];
  bi = si[0];
#pragma unroll
  for (int w = 1; w < QCP_T / 64; ++w) argmax_take(best, bi, sv[w], si[w]);
  const int64_t p = bi;
  if (blockIdx.x == 0 && tid == 0) {
    stamp[p] = (int32_t)j;
    perm[j] = (int32_t)p;
  }
  // column p, rows j..r-1, into LDS; its squared norm below row j
  double s2 = 0.0;
  for (int64_t i = j + tid; i < r; i += QCP_T) {
    const double e = Bc[p * r + i];
    xp[i - j] = e;
    if (i > j) s2 = fma(e, e, s2);
  }
  s2 = wave_sum_dpp(s2);
  if (lane == 0) sred[wave] = s2;
  __syncthreads();
  double sigma2 = 0.0;
#pragma unroll
  for (int w = 0; w < QCP_T / 64; ++w) sigma2 += sred[w];
  const double alpha = xp[0];
  double th = 0.0, scale = 0.0;
  if (sigma2 != 0.0) {
    const double beta = -copysign(sqrt(fma(alpha, alpha, sigma2)), alpha);
    th = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
  if (!live || c == p) return;  // wave-uniform: no barrier follows
  // v^T x = x_j + scale * sum_{i > j} x_p[i] x[i]
  double dot = 0.0, xj = 0.0;
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int64_t i = lane + 64 * q;
    if (i > j && i < r) dot = fma(xp[i - j], x[q], dot);
    if (i == j) xj = x[q];
  }
  dot = wave_sum_dpp(dot);
  xj = wave_sum_dpp(xj);  // the one lane holding row j
  const double tws = th * (xj + scale * dot) * scale;  // tau_h (v^T x) times the scale of v
  double n2 = 0.0;
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int64_t i = lane + 64 * q;
    if (i > j && i < r) {
      const double e = fma(-tws, xp[i - j], x[q]);
      Bc[c * r + i] = e;
      n2 = fma(e, e, n2);
    }
  }
  n2 = wave_sum_dpp(n2);
  if (lane == 0) nrm_out[c] = sqrt(n2);
}

// The last column is the one never pivoted.
__global__ void __launch_bounds__(256) qrcp_last(const int32_t* __restrict__ stamp,
                                                 int32_t* __restrict__ perm, int64_t r) {
  for (int64_t c = threadIdx.x; c < r; c += 256)
    if (stamp[c] >= r - 1) perm[r - 1] = (int32_t)c;
}

__global__ void __launch_bounds__(256) qrcp_stamp_init(int32_t* stamp, int64_t r) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < r) stamp[e] = (int32_t)r;
}

// Z[i*r + c] = R[i*ldr + perm[c]] (R with its columns permuted).
__global__ void __launch_bounds__(256) gather_cols(const double* __restrict__ R, int64_t ldr,
                                                   const int32_t* __restrict__ perm, int64_t r,
                                                   double* __restrict__ Z) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= r * r) return;
  const int64_t i = e / r, c = e - i * r;
  Z[e] = R[i * ldr + perm[c]];
}

__device__ __forceinline__ double lifted(double d, double tau) {
  return (fabs(d) < tau) ? ((d < 0.0) ? -tau : tau) : d;
}

// Z2 = (R_p with its small diagonal raised to tau)^T, row-major r x r.
__global__ void __launch_bounds__(256) lift_transpose(const double* __restrict__ Rp, int64_t r,
                                                      double tau, double* __restrict__ Z2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= r * r) return;
  const int64_t i = e / r, j = e - i * r;
  double v = 0.0;
  if (i == j)
    v = lifted(Rp[i * r + i], tau);
  else if (j < i)
    v = Rp[j * r + i];
  Z2[e] = v;
}

// k = r; status: 1 non-finite diagonal, 16 some |diagonal| < tau.  When
// in_place, the diagonal is raised to tau in R itself (perturbation (c)).
__global__ void __launch_bounds__(256) lift_scan(double* __restrict__ R, int64_t ldr, int64_t r,
                                                 double tau, int in_place, int32_t* kout,
                                                 int32_t* status) {
  __shared__ int s_nf, s_low;
  if (threadIdx.x == 0) {
    s_nf = 0;
    s_low = 0;
  }
  __syncthreads();
  for (int64_t i = threadIdx.x; i < r; i += 256) {
    const double d = R[i * ldr + i];
    if (!isfinite(d)) atomicOr(&s_nf, 1);
    if (fabs(d) < tau) {
      atomicOr(&s_low, 1);
      if (in_place) R[i * ldr + i] = lifted(d, tau);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    *kout = (int32_t)r;
    *status = (s_nf ? 1 : 0) | (s_low ? 16 : 0);
  }
}

// Q2[perm[j]*r + c] = Q3[j*r + c]  (Q2 = P Q3).
__global__ void __launch_bounds__(256) scatter_rows(const double* __restrict__ Q3,
                                                    const int32_t* __restrict__ perm, int64_t r,
                                                    double* __restrict__ Q2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= r * r) return;
  const int64_t j = e / r, c = e - j * r;
  Q2[(int64_t)perm[j] * r + c] = Q3[e];
}

// ---------------------------------------------------------------------------- power method
// Rows of V (nv x r): entries at or beyond the kept size zeroed, rows normalized
// to unit length; est = 0.  One wave per row.
__global__ void __launch_bounds__(1024) power_prep(double* __restrict__ V, int nv, int64_t r,
                                                   const int32_t* kdev, double* est) {
  const int lane = threadIdx.x & 63, row = threadIdx.x >> 6;
  const int64_t k = (*kdev < r) ? *kdev : r;
  if (threadIdx.x == 0) *est = 0.0;
  if (row >= nv) return;
  double* v = V + (int64_t)row * r;
  double s = 0.0;
  for (int64_t i = lane; i < r; i += 64) {
    if (i >= k) v[i] = 0.0;
    const double x = (i < k) ? v[i] : 0.0;
    s = fma(x, x, s);
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  const double inv = (s > 0.0) ? 1.0 / sqrt(s) : 0.0;
  for (int64_t i = lane; i < k; i += 64) v[i] *= inv;
}

// est = max(est, max_row ||row||); normalize: rows scaled to unit length.
__global__ void __launch_bounds__(1024) power_rows(double* __restrict__ V, int nv, int64_t r,
                                                   double* est, int normalize) {
  __shared__ double sn[16];
  const int lane = threadIdx.x & 63, row = threadIdx.x >> 6;
  double nr = 0.0;
  if (row < nv) {
    double* v = V + (int64_t)row * r;
    double s = 0.0;
    for (int64_t i = lane; i < r; i += 64) s = fma(v[i], v[i], s);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    nr = sqrt(s);
    if (normalize && nr > 0.0) {
      const double inv = 1.0 / nr;
      for (int64_t i = lane; i < r; i += 64) v[i] *= inv;
    }
  }
  if (normalize) return;
  if (lane == 0) sn[row] = nr;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = *est;
    for (int w = 0; w < nv; ++w) m = fmax(m, sn[w]);
    *est = m;
  }
}

__global__ void __launch_bounds__(64) power_flag(const double* est, double tau_d,
                                                 int32_t* status, double* est_out) {
  if (threadIdx.x != 0) return;
  const double e = *est;
  if (e * tau_d > 1.0 || isnan(e)) *status |= 8;
  if (est_out) *est_out = e;
}

// The check's solves in one workgroup.  U is the upper triangular factor the
// check solves with: R for a plain core, R2 for a truncated or factored one
// (k x k, ld r).  Its 64 x 64 diagonal blocks are inverted once (one thread per
// column, back substitution in LDS), U^T is copied once, and then a single
// launch runs every power step with the nv right-hand sides in LDS: a block of
// unknowns is the inverted diagonal block times its right-hand sides, then the
// later (forward) or earlier (backward) right-hand sides take the block's
// contribution, reading U's rows (forward) or U^T's rows (backward) coalesced.
constexpr int PB = 64;
constexpr int kPowerLds = 16384;  // doubles of right-hand sides held in LDS
constexpr int kPowerThreads = 512;

__device__ __forceinline__ const double* power_factor(const double* R, const double* R2,
                                                      int64_t r, const int32_t* kdev, int force,
                                                      int64_t& k, bool& use2) {
  k = (*kdev < r) ? *kdev : r;
  use2 = force || *kdev < r;
  return use2 ? R2 : R;
}

__global__ void __launch_bounds__(PB) power_block_inverse(const double* __restrict__ R,
                                                          const double* __restrict__ R2, int64_t r,
                                                          const int32_t* kdev, int force,
                                                          double* __restrict__ Dinv) {
  int64_t k;
  bool use2;
  const double* U = power_factor(R, R2, r, kdev, force, k, use2);
  const int64_t j0 = (int64_t)blockIdx.x * PB;
  if (j0 >= k) return;
  __shared__ double Bs[PB][PB + 1];
  __shared__ double Xs[PB][PB + 1];
  const int t = threadIdx.x;
  for (int i = 0; i < PB; ++i) {
    double v = (i == t) ? 1.0 : 0.0;  // identity beyond the kept size
    if (j0 + i < k && j0 + t < k) v = (t >= i) ? U[(j0 + i) * r + j0 + t] : 0.0;
    Bs[i][t] = v;
    Xs[i][t] = 0.0;
  }
  __syncthreads();
  // column t of the inverse: B x = e_t by back substitution (x_i = 0 for i > t)
  for (int i = t; i >= 0; --i) {
    double acc = (i == t) ? 1.0 : 0.0;
    for (int l = i + 1; l <= t; ++l) acc = fma(-Bs[i][l], Xs[l][t], acc);
    Xs[i][t] = acc / Bs[i][i];
  }
  for (int i = 0; i < PB; ++i) Dinv[(int64_t)blockIdx.x * PB * PB + i * PB + t] = Xs[i][t];
}

// Ut[i*r + j] = U[j*r + i] over the k x k block.
__global__ void __launch_bounds__(256) power_transpose(const double* __restrict__ R,
                                                       const double* __restrict__ R2, int64_t r,
                                                       const int32_t* kdev, int force,
                                                       double* __restrict__ Ut) {
  int64_t k;
  bool use2;
  const double* U = power_factor(R, R2, r, kdev, force, k, use2);
  __shared__ double tile[32][33];
  const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int y = ty; y < 32; y += 8) {
    const int64_t i = r0 + y, j = c0 + tx;
    tile[y][tx] = (i < k && j < k) ? U[i * r + j] : 0.0;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int64_t i = c0 + y, j = r0 + tx;  // Ut row i = U column i
    if (i < k && j < k) Ut[i * r + j] = tile[tx][y];
  }
}

// Row norms of X (nv x k in LDS, row v at v*kp, kp = k rounded up to a multiple
// of 64, the padding zero): one wave per row; optionally
// scales the rows to unit length; returns the largest norm (valid in thread 0
// after the call; every thread passes the barriers).
__device__ double power_norms(double* X, int nv, int64_t k, bool normalize, double* sn) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t kp = cdiv_d(k, PB) * PB;
  for (int v = wave; v < nv; v += kPowerThreads / 64) {
    double s = 0.0;
    for (int64_t i = lane; i < k; i += 64) s = fma(X[v * kp + i], X[v * kp + i], s);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    const double nr = sqrt(s);
    if (normalize && nr > 0.0) {
      const double inv = 1.0 / nr;
      for (int64_t i = lane; i < k; i += 64) X[v * kp + i] *= inv;
    }
    if (lane == 0) sn[v] = nr;
  }
  __syncthreads();
  double m = 0.0;
  if (threadIdx.x == 0)
    for (int v = 0; v < nv; ++v) m = fmax(m, sn[v]);
  return m;
}

// U^T x = b (forward) or U x = b (backward) for the nv rows of X in place.
template <bool FORWARD>
__device__ void power_solve(double* X, double* xtmp, int nv, int64_t k, int64_t r,
                            const double* U, const double* Ut, const double* Dinv) {
  const int tid = threadIdx.x;
  const int64_t kp = cdiv_d(k, PB) * PB;  // row stride of X
  const int nblk = (int)cdiv_d(k, PB);
  for (int s = 0; s < nblk; ++s) {
    const int b = FORWARD ? s : nblk - 1 - s;
    const int64_t j0 = (int64_t)b * PB;
    const int w = (int)((k - j0 < PB) ? (k - j0) : PB);
    const double* D = Dinv + (int64_t)b * PB * PB;
    // unknowns of the block: x = D^T b_blk (forward) or D b_blk (backward); D is
    // zero outside its upper triangle, so the sums run over the whole block with
    // the loads issued several at a time
    constexpr int VS = kPowerThreads / PB;  // vectors per pass over the block
    const int j = tid % PB;
#pragma unroll 1
    for (int v = tid / PB; v < nv; v += VS) {
      double acc = 0.0;
      if (j < w) {
        // rows of X are padded to a multiple of 64 with zeros, and D's entries
        // that pair with rows beyond the kept size are zero
        const double* xb = X + v * kp + j0;
#pragma unroll 1
        for (int u0 = 0; u0 < PB; u0 += 32) {
          double d[32];
#pragma unroll
          for (int u = 0; u < 32; ++u)
            d[u] = FORWARD ? D[(u0 + u) * PB + j] : D[j * PB + u0 + u];
          double xv[32];
#pragma unroll
          for (int u = 0; u < 32; ++u) xv[u] = xb[u0 + u];
          __builtin_amdgcn_sched_barrier(0);  // every LDS read issued before the first use
#pragma unroll
          for (int u = 0; u < 32; ++u) acc = fma(d[u], xv[u], acc);
        }
      }
      xtmp[v * PB + j] = acc;
    }
    __syncthreads();
    for (int v = tid / PB; v < nv; v += VS)
      if (j < w) X[v * kp + j0 + j] = xtmp[v * PB + j];
    __syncthreads();
    // the other right-hand sides take the block's contribution
    const int64_t c_lo = FORWARD ? j0 + w : 0, c_hi = FORWARD ? k : j0;
    const double* Ub = FORWARD ? U : Ut;
    for (int64_t c = c_lo + tid; c < c_hi; c += kPowerThreads) {
      // half of the block's column strip of U in flight at a time (zero beyond w)
#pragma unroll 1
      for (int t0 = 0; t0 < PB; t0 += 32) {
        double u[32];
#pragma unroll
        for (int t = 0; t < 32; ++t) u[t] = (t0 + t < w) ? Ub[(j0 + t0 + t) * r + c] : 0.0;
#pragma unroll 1
        for (int q = 0; q < nv; ++q) {
          const double* xq = X + q * kp + j0 + t0;
          double xv[32];
#pragma unroll
          for (int t = 0; t < 32; ++t) xv[t] = xq[t];
          __builtin_amdgcn_sched_barrier(0);  // every LDS read issued before the first use
          double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int t = 0; t < 32; ++t) a[t & 3] = fma(u[t], xv[t], a[t & 3]);
          X[q * kp + c] -= (a[0] + a[1]) + (a[2] + a[3]);
        }
      }
    }
    __syncthreads();
  }
}

// Every power step in one workgroup: v <- v / ||v||; y = T^{-T} v; est = max
// ||y||; z = T^{-1} y; v <- z / ||z||.  T = R (plain core): forward then
// backward; T = R2^T (truncated or factored core): backward then forward.
__global__ void __launch_bounds__(kPowerThreads) power_iterate(const double* __restrict__ R,
                                                      const double* __restrict__ R2, int64_t r,
                                                      const int32_t* kdev, int force,
                                                      const double* __restrict__ Dinv,
                                                      const double* __restrict__ Ut,
                                                      double* __restrict__ V, int nv, int iters,
                                                      double* est) {
  __shared__ double X[kPowerLds];
  __shared__ double xtmp[16 * PB];
  __shared__ double sn[16];
  int64_t k;
  bool use2;
  const double* U = power_factor(R, R2, r, kdev, force, k, use2);
  const int64_t kp = cdiv_d(k, PB) * PB;
  for (int64_t e = threadIdx.x; e < (int64_t)nv * kp; e += kPowerThreads) {
    const int64_t v = e / kp, i = e - v * kp;
    X[e] = (i < k) ? V[v * r + i] : 0.0;
  }
  __syncthreads();
  double best = 0.0;
  if (k > 0) {
    power_norms(X, nv, k, true, sn);
    for (int it = 0; it < iters; ++it) {
      if (use2)
        power_solve<false>(X, xtmp, nv, k, r, U, Ut, Dinv);
      else
        power_solve<true>(X, xtmp, nv, k, r, U, Ut, Dinv);
      best = fmax(best, power_norms(X, nv, k, false, sn));
      __syncthreads();
      if (use2)
        power_solve<true>(X, xtmp, nv, k, r, U, Ut, Dinv);
      else
        power_solve<false>(X, xtmp, nv, k, r, U, Ut, Dinv);
      power_norms(X, nv, k, true, sn);
      __syncthreads();
    }
  }
  for (int64_t e = threadIdx.x; e < (int64_t)nv * kp; e += kPowerThreads) {
    const int64_t v = e / kp, i = e - v * kp;
    if (i < k) V[v * r + i] = X[e];
  }
  if (threadIdx.x == 0) *est = best;
}

// Triangular solve for a few right-hand sides (the columns of a factored product),
// spread over workgroups with one launch per 64-row block of the factor, in the
// order the direction gives.  Right-hand side v is entry i of row v of Xg, i.e.
// Xg[v rsx + i csx].  The factor and the direction follow the kept rank on the
// device: U = R2 when truncated (or forced) and R otherwise; a left product
// solves U x = b with U = R and U^T x = b with U = R2, a right product the other
// way round.  In launch `step` every workgroup forms the block's unknowns x_b from
// the block's right-hand sides with the block's inverse (the same blocked
// substitution as the check), workgroup 0 stores them in S (v * r + i), and each
// workgroup subtracts their contribution from its own 64 of the right-hand-side
// rows still to be solved.  msolve_finish copies S back, zero at and beyond the
// kept size.
constexpr int MS_T = 256, MS_NV = 32;

__global__ void __launch_bounds__(MS_T) msolve_step(const double* __restrict__ R,
                                                    const double* __restrict__ R2, int64_t r,
                                                    const int32_t* kdev, int force, int left,
                                                    const double* __restrict__ Dinv,
                                                    const double* __restrict__ Ut,
                                                    double* __restrict__ Xg, int nrhs, int64_t rsx,
                                                    int64_t csx, double* __restrict__ S, int step) {
  __shared__ double rb[PB][MS_NV + 1];  // the block's right-hand sides, then its unknowns
  __shared__ double Ds[PB][PB + 1];     // the block's inverse
  int64_t k;
  bool use2;
  const double* U = power_factor(R, R2, r, kdev, force, k, use2);
  const bool fwd = left ? use2 : !use2;
  const int nblk = (int)cdiv_d(k, PB);
  if (step >= nblk) return;
  const int b = fwd ? step : nblk - 1 - step;
  const int64_t j0 = (int64_t)b * PB;
  const int w = (int)((k - j0 < PB) ? (k - j0) : PB);
  const int64_t c_lo = fwd ? j0 + w : 0, c_hi = fwd ? k : j0;
  const int64_t c0 = c_lo + (int64_t)blockIdx.x * PB;
  if (blockIdx.x > 0 && c0 >= c_hi) return;
  const int tid = threadIdx.x, j = tid % PB, grp = tid / PB;
  constexpr int NG = MS_T / PB;          // right-hand-side groups
  constexpr int NVT = MS_NV / NG;        // right-hand sides per thread
  // every global load first: this workgroup's strip of U (rows j0 .. j0 + w of the
  // factor, columns c0 + j; forward U[j0 + t][c], backward U[c][j0 + t] = Ut[j0 + t][c];
  // read in range, zeroed past w), the block's right-hand sides (zero past the
  // kept size) and the block's inverse (the identity past the kept size)
  const int64_t c = c0 + j;
  const int64_t cc = (c < c_hi) ? c : ((c_hi > 0) ? c_hi - 1 : 0);
  const double* Ub = fwd ? U : Ut;
  double u[PB];
#pragma unroll
  for (int t = 0; t < PB; ++t) u[t] = Ub[(j0 + (t < w ? t : w - 1)) * r + cc];
  for (int e = tid; e < PB * MS_NV; e += MS_T) {
    const int t = e / MS_NV, v = e % MS_NV;
    rb[t][v] = (t < w && v < nrhs) ? Xg[v * rsx + (j0 + t) * csx] : 0.0;
  }
  const double* D = Dinv + (int64_t)b * PB * PB;
  for (int e = tid; e < PB * PB; e += MS_T) Ds[e / PB][e % PB] = D[e];
  __syncthreads();
  // x_j = sum_u D[u][j] b_u (forward, D^T b) or sum_u D[j][u] b_u (backward)
  double x[NVT];
#pragma unroll
  for (int q = 0; q < NVT; ++q) {
    const int v = grp + NG * q;
    double a4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int uu = 0; uu < PB; ++uu)
      a4[uu & 3] = fma(fwd ? Ds[uu][j] : Ds[j][uu], rb[uu][v], a4[uu & 3]);
    x[q] = (a4[0] + a4[1]) + (a4[2] + a4[3]);
  }
  __syncthreads();  // every thread has read the right-hand sides
#pragma unroll
  for (int q = 0; q < NVT; ++q) rb[j][grp + NG * q] = x[q];
  __syncthreads();
  if (blockIdx.x == 0) {
    for (int e = tid; e < PB * MS_NV; e += MS_T) {
      const int t = e / MS_NV, v = e % MS_NV;
      if (t < w && v < nrhs) S[(int64_t)v * r + j0 + t] = rb[t][v];
    }
  }
  if (c0 >= c_hi) return;
  // rows c0 .. c0 + 63 of the remaining right-hand sides take the block's part:
  // forward  b_c -= sum_t U[j0 + t][c] x_t,  backward  b_c -= sum_t U[c][j0 + t] x_t
#pragma unroll
  for (int t = 0; t < PB; ++t) u[t] = (t < w) ? u[t] : 0.0;
  for (int v = grp; v < nrhs; v += NG) {
    double a4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < PB; ++t) a4[t & 3] = fma(u[t], rb[t][v], a4[t & 3]);
    if (c < c_hi) Xg[v * rsx + c * csx] -= (a4[0] + a4[1]) + (a4[2] + a4[3]);
  }
}

__global__ void __launch_bounds__(256) msolve_finish(int64_t r, const int32_t* kdev,
                                                     double* __restrict__ Xg, int nrhs,
                                                     int64_t rsx, int64_t csx,
                                                     const double* __restrict__ S) {
  const int64_t k = (*kdev < r) ? *kdev : r;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)nrhs * r) return;
  const int64_t v = e / r, i = e - v * r;
  Xg[v * rsx + i * csx] = (i < k) ? S[e] : 0.0;
}

// ---------------------------------------------------------------------------- Jacobi driver
template <int E, int B>
gn_status run_jacobi_ring(double* W, double* J, int32_t* ctl, int64_t r, double tol,
                          hipStream_t s) {
  const int nb = (int)cdiv(r, B);
  const int nbe = nb + (nb & 1);
  const dim3 grid((unsigned)(nbe / 2)), block(64 * B);
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    for (int t = 0; t < nbe - 1; ++t) {
      if (t == 0)
        jacobi_ring<E, B, true><<<grid, block, 0, s>>>(W, J, ctl, r, nbe, t, sweep, tol);
      else
        jacobi_ring<E, B, false><<<grid, block, 0, s>>>(W, J, ctl, r, nbe, t, sweep, tol);
      GN_LAUNCH_CHECK();
    }
    jacobi_sweep_end<<<dim3(1), dim3(64), 0, s>>>(ctl, sweep);
    GN_LAUNCH_CHECK();
  }
  return GN_OK;
}

template <int RPT, int B>
gn_status run_jacobi(double* W, double* J, int32_t* ctl, int64_t r, double tol, hipStream_t s) {
  const int nb = (int)cdiv(r, B);
  const int nbe = nb + (nb & 1);
  const dim3 grid((unsigned)(nbe / 2)), block(JT);
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    for (int t = 0; t < nbe - 1; ++t) {
      if (t == 0)
        jacobi_round<RPT, B, true><<<grid, block, 0, s>>>(W, J, ctl, r, nbe, t, sweep, tol);
      else
        jacobi_round<RPT, B, false><<<grid, block, 0, s>>>(W, J, ctl, r, nbe, t, sweep, tol);
      GN_LAUNCH_CHECK();
    }
    jacobi_sweep_end<<<dim3(1), dim3(64), 0, s>>>(ctl, sweep);
    GN_LAUNCH_CHECK();
  }
  return GN_OK;
}

struct SvdWs {
  size_t w, j, sig, sorted, perm, ctl, total;
};
SvdWs svd_ws(int64_t r) {
  SvdWs w{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  w.w = take((size_t)r * r * 8);
  w.j = take((size_t)r * r * 8);
  w.sig = take((size_t)r * 8);
  w.sorted = take((size_t)r * 8);
  w.perm = take((size_t)r * 4);
  w.ctl = take((size_t)(2 + kMaxSweeps) * 4);
  w.total = off;
  return w;
}

struct RrqrWs {
  size_t b, nrm, nrm2, stamp, perm, z, qr, z2, q3, qrws, total;
};
RrqrWs rrqr_ws(int64_t r) {
  RrqrWs w{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  w.b = take((size_t)r * r * 8);
  w.nrm = take((size_t)r * 8);
  w.nrm2 = take((size_t)r * 8);
  w.stamp = take((size_t)r * 4);
  w.perm = take((size_t)r * 4);
  w.z = take((size_t)r * r * 8);
  w.qr = take((size_t)r * r * 8);
  w.z2 = take((size_t)r * r * 8);
  w.q3 = take((size_t)r * r * 8);
  w.qrws = take(qr_ws_bytes(r, r));
  w.total = off;
  return w;
}

}  // namespace

size_t stabilize_ws_bytes(int32_t method, int64_t r) {
  if (method == GN_CORE_SVD || method == GN_CORE_LIFT_SVD) return svd_ws(r).total;
  if (method == GN_CORE_LIFT_RRQR) return rrqr_ws(r).total;
  return 0;
}

gn_status launch_svd_core(int64_t r, int64_t rl, const double* R, int64_t ldr, const double* Q1,
                          double tau, int lift, int32_t* k, int32_t* status, double* Q1_out,
                          double* Q2, double* R2, void* ws, hipStream_t s) {
  if (r < 1 || r > kSortMax) return GN_ERR_UNSUPPORTED;
  const SvdWs L = svd_ws(r);
  char* base = (char*)ws;
  double* W = (double*)(base + L.w);
  double* J = (double*)(base + L.j);
  double* sig = (double*)(base + L.sig);
  double* srt = (double*)(base + L.sorted);
  int32_t* perm = (int32_t*)(base + L.perm);
  int32_t* ctl = (int32_t*)(base + L.ctl);
  const int64_t nel = r * r > 2 + kMaxSweeps ? r * r : 2 + kMaxSweeps;
  jacobi_init<<<dim3((unsigned)cdiv(nel, 256)), dim3(256), 0, s>>>(R, ldr, r, W, J, ctl);
  GN_LAUNCH_CHECK();
  const double tol = sqrt((double)r) * 0x1.0p-53;
  if (r <= 256)
    GN_TRY((run_jacobi_ring<4, 8>(W, J, ctl, r, tol, s)));
  else if (r <= 512)
    GN_TRY((run_jacobi_ring<8, 8>(W, J, ctl, r, tol, s)));
  else if (r <= 1024)
    GN_TRY((run_jacobi_ring<16, 8>(W, J, ctl, r, tol, s)));
  else if (r <= 2048)
    GN_TRY((run_jacobi_ring<32, 4>(W, J, ctl, r, tol, s)));
  else
    GN_TRY((run_jacobi<16, 2>(W, J, ctl, r, tol, s)));
  vec_norms<<<dim3((unsigned)cdiv(r, 4)), dim3(256), 0, s>>>(W, r, sig);
  GN_LAUNCH_CHECK();
  svd_sort<<<dim3(1), dim3(1024), 0, s>>>(sig, r, tau, lift, ctl, perm, srt, k, status);
  GN_LAUNCH_CHECK();
  const dim3 tg((unsigned)cdiv(r, 32), (unsigned)cdiv(r, 32));
  // Q2 = U' (right singular vectors of C, sorted), then J's columns sorted into W
  gather_transpose<<<tg, dim3(256), 0, s>>>(W, perm, srt, r, Q2);
  GN_LAUNCH_CHECK();
  gather_transpose<<<tg, dim3(256), 0, s>>>(J, perm, nullptr, r, W);
  GN_LAUNCH_CHECK();
  diag_matrix<<<dim3((unsigned)cdiv(r * r, 256)), dim3(256), 0, s>>>(srt, r, tau, lift, R2);
  GN_LAUNCH_CHECK();
  // Q1_out = Q1 J (left singular vectors of C)
  GN_TRY(launch_dgemm(rl, r, r, 1.0, MatRef{Q1, GN_DT_F64, r, 1}, MatRef{W, GN_DT_F64, r, 1}, 0.0,
                      Q1_out, r, 1, nullptr, false, s));
  return GN_OK;
}

gn_status launch_rrqr_core(int64_t r, int64_t rl, const double* R, int64_t ldr, const double* Q1,
                           double tau, int32_t* k, int32_t* status, double* Q1_out, double* Rp,
                           double* Q2, double* R2, void* ws, hipStream_t s) {
  if (r > 4096) return GN_ERR_UNSUPPORTED;  // a column per wave in registers, column p in LDS
  const RrqrWs L = rrqr_ws(r);
  char* base = (char*)ws;
  double* Bc = (double*)(base + L.b);
  double* nrm = (double*)(base + L.nrm);
  int32_t* perm = (int32_t*)(base + L.perm);
  double* Z = (double*)(base + L.z);
  double* Qr = (double*)(base + L.qr);
  double* Z2 = (double*)(base + L.z2);
  double* Q3 = (double*)(base + L.q3);
  double* qws = (double*)(base + L.qrws);
  double* nrm2 = (double*)(base + L.nrm2);
  int32_t* stamp = (int32_t*)(base + L.stamp);
  qrcp_init<<<dim3((unsigned)cdiv(r * r, 256)), dim3(256), 0, s>>>(R, ldr, r, Bc, perm);
  GN_LAUNCH_CHECK();
  qrcp_stamp_init<<<dim3((unsigned)cdiv(r, 256)), dim3(256), 0, s>>>(stamp, r);
  GN_LAUNCH_CHECK();
  vec_norms<<<dim3((unsigned)cdiv(r, 4)), dim3(256), 0, s>>>(Bc, r, nrm);
  GN_LAUNCH_CHECK();
  for (int64_t j = 0; j + 1 < r; ++j) {
    const double* nin = (j & 1) ? nrm2 : nrm;
    double* nout = (j & 1) ? nrm : nrm2;
    const dim3 g((unsigned)cdiv(r, QCP_COLS)), b(QCP_T);
    if (r <= 1024)
      qrcp_step<16><<<g, b, 0, s>>>(Bc, nin, nout, stamp, perm, r, j);
    else if (r <= 2048)
      qrcp_step<32><<<g, b, 0, s>>>(Bc, nin, nout, stamp, perm, r, j);
    else
      qrcp_step<64><<<g, b, 0, s>>>(Bc, nin, nout, stamp, perm, r, j);
    GN_LAUNCH_CHECK();
  }
  qrcp_last<<<dim3(1), dim3(256), 0, s>>>(stamp, perm, r);
  GN_LAUNCH_CHECK();
  // R P = Q_R R_p by the blocked QR; C P = (Q1 Q_R) R_p
  gather_cols<<<dim3((unsigned)cdiv(r * r, 256)), dim3(256), 0, s>>>(R, ldr, perm, r, Z);
  GN_LAUNCH_CHECK();
  GN_TRY(launch_qr(r, r, Z, r, Qr, r, Rp, r, qws, nullptr, s));
  lift_scan<<<dim3(1), dim3(256), 0, s>>>(Rp, r, r, tau, 0, k, status);
  GN_LAUNCH_CHECK();
  lift_transpose<<<dim3((unsigned)cdiv(r * r, 256)), dim3(256), 0, s>>>(Rp, r, tau, Z2);
  GN_LAUNCH_CHECK();
  GN_TRY(launch_qr(r, r, Z2, r, Q3, r, R2, r, qws, nullptr, s));
  scatter_rows<<<dim3((unsigned)cdiv(r * r, 256)), dim3(256), 0, s>>>(Q3, perm, r, Q2);
  GN_LAUNCH_CHECK();
  GN_TRY(launch_dgemm(rl, r, r, 1.0, MatRef{Q1, GN_DT_F64, r, 1}, MatRef{Qr, GN_DT_F64, r, 1}, 0.0,
                      Q1_out, r, 1, nullptr, false, s));
  return GN_OK;
}

gn_status launch_lift_diag(int64_t r, double* R, int64_t ldr, double tau, int32_t* k,
                           int32_t* status, hipStream_t s) {
  lift_scan<<<dim3(1), dim3(256), 0, s>>>(R, ldr, r, tau, 1, k, status);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

size_t small_solve_ws_bytes(int64_t r) {
  return align_up((size_t)cdiv(r, PB) * PB * PB * 8) + align_up((size_t)r * r * 8) +
         align_up((size_t)MS_NV * r * 8);
}

int64_t small_solve_max_rhs() { return MS_NV; }

gn_status launch_small_solve_prep(int64_t r, const double* R, const double* R2, const int32_t* k,
                                  bool force, void* ws, hipStream_t s) {
  const size_t dbytes = align_up((size_t)cdiv(r, PB) * PB * PB * 8);
  double* Dinv = (double*)ws;
  double* Ut = (double*)((char*)ws + dbytes);
  power_block_inverse<<<dim3((unsigned)cdiv(r, PB)), dim3(PB), 0, s>>>(R, R2, r, k, force ? 1 : 0,
                                                                       Dinv);
  GN_LAUNCH_CHECK();
  power_transpose<<<dim3((unsigned)cdiv(r, 32), (unsigned)cdiv(r, 32)), dim3(256), 0, s>>>(
      R, R2, r, k, force ? 1 : 0, Ut);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

gn_status launch_small_solve(int64_t r, const double* R, const double* R2, const int32_t* k,
                             bool force, bool left, double* X, int64_t nrhs, int64_t rsx,
                             int64_t csx, void* ws, hipStream_t s) {
  if (nrhs <= 0) return GN_OK;
  if (nrhs > MS_NV) return GN_ERR_UNSUPPORTED;
  const size_t dbytes = align_up((size_t)cdiv(r, PB) * PB * PB * 8);
  const double* Dinv = (const double*)ws;
  const double* Ut = (const double*)((char*)ws + dbytes);
  double* S = (double*)((char*)ws + dbytes + align_up((size_t)r * r * 8));
  // one launch per block of the largest kept size; launches past the kept
  // size's blocks return at once
  const int nb = (int)cdiv(r, PB);
  for (int st = 0; st < nb; ++st) {
    msolve_step<<<dim3((unsigned)nb), dim3(MS_T), 0, s>>>(R, R2, r, k, force ? 1 : 0, left ? 1 : 0,
                                                          Dinv, Ut, X, (int)nrhs, rsx, csx, S, st);
    GN_LAUNCH_CHECK();
  }
  msolve_finish<<<dim3((unsigned)cdiv(nrhs * r, 256)), dim3(256), 0, s>>>(r, k, X, (int)nrhs, rsx,
                                                                        csx, S);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

size_t power_ws_bytes(int64_t r, int32_t nv) {
  return align_up((size_t)nv * r * 8) + 256 + align_up((size_t)cdiv(r, PB) * PB * PB * 8) +
         align_up((size_t)r * r * 8);
}

gn_status launch_power_check(int64_t r, uint64_t seed, int32_t nv, int32_t iters,
                             const double* R, const double* R2, const int32_t* k, bool force_trunc,
                             double tau_d, int32_t* status, double* est_out, void* ws,
                             hipStream_t s) {
  char* base = (char*)ws;
  double* V = (double*)base;
  double* est = (double*)(base + align_up((size_t)nv * r * 8));
  double* Dinv = (double*)(base + align_up((size_t)nv * r * 8) + 256);
  double* Ut = (double*)((char*)Dinv + align_up((size_t)cdiv(r, PB) * PB * PB * 8));
  GN_TRY(launch_gaussian(seed, 6, 0, 0, nv, r, GN_DT_F64, 0, V, r, s));
  power_prep<<<dim3(1), dim3(1024), 0, s>>>(V, nv, r, k, est);
  GN_LAUNCH_CHECK();
  if ((int64_t)nv * cdiv(r, PB) * PB <= kPowerLds) {
    const int f = force_trunc ? 1 : 0;
    power_block_inverse<<<dim3((unsigned)cdiv(r, PB)), dim3(PB), 0, s>>>(R, R2, r, k, f, Dinv);
    GN_LAUNCH_CHECK();
    power_transpose<<<dim3((unsigned)cdiv(r, 32), (unsigned)cdiv(r, 32)), dim3(256), 0, s>>>(
        R, R2, r, k, f, Ut);
    GN_LAUNCH_CHECK();
    power_iterate<<<dim3(1), dim3(kPowerThreads), 0, s>>>(R, R2, r, k, f, Dinv, Ut, V, nv, iters,
                                                          est);
    GN_LAUNCH_CHECK();
  } else {
    for (int it = 0; it < iters; ++it) {
      // y = T^{-T} v: the right-side solve X T = B (T = R, or R_2^T when truncated)
      GN_TRY(launch_trsm_core(nv, r, R, R2, r, k, V, r, 1, false, true, s, false, force_trunc));
      power_rows<<<dim3(1), dim3(1024), 0, s>>>(V, nv, r, est, 0);
      GN_LAUNCH_CHECK();
      // z = T^{-1} y: the transposed solve
      GN_TRY(launch_trsm_core(nv, r, R, R2, r, k, V, r, 1, true, true, s, false, force_trunc));
      power_rows<<<dim3(1), dim3(1024), 0, s>>>(V, nv, r, est, 1);
      GN_LAUNCH_CHECK();
    }
  }
  power_flag<<<dim3(1), dim3(64), 0, s>>>(est, tau_d, status, est_out);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

}  // namespace gn
