// FP32 sketch pass with an SRHT X for small r + l (at most 16): one read of A.
//
// FP32 pass with an SRHT X when r + l <= 16: HBM-bound (2(r+l) + log2 n' flops
// per 4-byte element of A lies far below the FP32 ridge), so A is read once and
// both products come out of the same registers.  Each wave owns one 256-column
// chunk of the padded matrix and a range of rows, 4 rows per step:
//   lane L = 16k + t holds row i0 + k, columns c*256 + 64g + 4t + q (g, q < 4);
//   Y^T A: v_mfma_f32_16x16x4_f32 with A's values as the first operand (its
//     row index is t, its K index k) and Y[i0 + k, t] as the second, so the
//     16 x 16 output block of (g, q) accumulates (Y^T A)[a, column(g, q, m)];
//   AX: the chunk times the signs, the order-256 Walsh-Hadamard transform
//     (bits 0-1 and 6-7 of the column inside the lane, bits 2-5 across the 16
//     lanes of a DPP row), the sampled positions idx_s mod 256 gathered from the
//     wave's LDS slot and multiplied by the sign of the outer Kronecker factor,
//     (-1)^popcount(c & (idx_s >> 8)) (H_n' = H_{n'/256} (x) H_256).
// Both results are partial sums (per row range for Y^T A, per chunk for AX)
// added afterwards in a fixed order.
#include "gn_internal.h"
#include "lane_ops.h"

namespace gn {
namespace {

typedef float nr_f32x4 __attribute__((ext_vector_type(4)));

constexpr int NR_CH = 256;       // columns per wave
constexpr int NR_WAVES = 4;      // waves (chunks) per workgroup
constexpr int NR_MAXRL = 16;     // r + l limit of this path

struct NarrowSrhtArgs {
  int64_t m, n, r, rl, rows_per_split;
  const float* A;
  int64_t lda;
  const float* Y;  // m x rl, ld rl
  const int8_t* signs;
  const int32_t* idx;
  float* partY;  // [splits][rl][n]
  float* partA;  // [chunks][m][r]
};

template <int LM>
__device__ __forceinline__ void nr_lane_stage(float (&x)[16], int lane) {
  const float sg = (lane & LM) ? -1.0f : 1.0f;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const float y = xor_lane<LM>(x[e], lane);
    x[e] = __builtin_fmaf(sg, x[e], y);  // lower lane: x + y, upper lane: y - x
  }
}

template <int B>
__device__ __forceinline__ void nr_reg_stage(float (&x)[16]) {
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    if (e & B) continue;
    const float a = x[e], b = x[e | B];
    x[e] = a + b;
    x[e | B] = a - b;
  }
}

__global__ void __launch_bounds__(64 * NR_WAVES) pass_f32_srht_narrow(NarrowSrhtArgs g) {
  __shared__ __attribute__((aligned(16))) float slot[NR_WAVES][4][NR_CH];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int t = lane & 15, k = lane >> 4;
  const int64_t c = (int64_t)blockIdx.x * NR_WAVES + w;
  const int64_t cb = c * NR_CH;
  const int64_t split = blockIdx.y;
  const int64_t i_begin = split * g.rows_per_split;
  const int64_t i_end = min(g.m, i_begin + g.rows_per_split);

  // per-lane constants: column signs (as sign-bit masks), validity of the 4-column
  // groups, the sampled position and outer sign of lane (k, s = t)
  uint32_t smask[16];
  bool cval[4];
#pragma unroll
  for (int gg = 0; gg < 4; ++gg) {
    const int64_t col = cb + 64 * gg + 4 * t;
    cval[gg] = col < g.n;  // n % 4 == 0: the whole group is inside A or outside
#pragma unroll
    for (int q = 0; q < 4; ++q)
      smask[4 * gg + q] = (g.signs[col + q] < 0) ? 0x80000000u : 0u;  // col + q < n'
  }
  const bool s_ok = t < g.r;
  const int id = g.idx[s_ok ? t : 0];
  const int lo = id & (NR_CH - 1);
  const float osg = (__builtin_popcountll((unsigned long long)(c & (int64_t)(id >> 8))) & 1) ? -1.0f : 1.0f;
  const bool a_ok = t < g.rl;
  const int64_t tcl = a_ok ? t : 0;

  nr_f32x4 acc[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = nr_f32x4{0.f, 0.f, 0.f, 0.f};

  // unconditional loads from clamped addresses (rows past the range, groups past
  // n and rows of Y past r + l are zeroed where the values are used, so no load
  // waits on a branch)
  auto load = [&](int64_t i0, nr_f32x4 (&v)[4], float& yb) {
    const int64_t i = i0 + k;
    const int64_t ic = i < i_end ? i : i_end - 1;
    const float* row = g.A + ic * g.lda;
#pragma unroll
    for (int gg = 0; gg < 4; ++gg) {
      const int64_t col = cval[gg] ? cb + 64 * gg + 4 * t : 0;
      v[gg] = *(const nr_f32x4*)(row + col);
    }
    yb = g.Y[ic * g.rl + tcl];
  };

  // one step: rows i0 .. i0 + 3 from registers v, yv
  auto step = [&](int64_t i0, const nr_f32x4 (&v)[4], float yv) {
    const bool rv = i0 + k < i_end;
    const float yb = (rv && a_ok) ? yv : 0.f;
    float x[16];
#pragma unroll
    for (int gg = 0; gg < 4; ++gg) {
      const bool ok = rv && cval[gg];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float a = ok ? v[gg][q] : 0.f;
        acc[4 * gg + q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, yb, acc[4 * gg + q], 0, 0, 0);
        x[4 * gg + q] = __uint_as_float(__float_as_uint(a) ^ smask[4 * gg + q]);
      }
    }
    nr_reg_stage<1>(x);
    nr_reg_stage<2>(x);
    nr_lane_stage<1>(x, lane);
    nr_lane_stage<2>(x, lane);
    nr_lane_stage<4>(x, lane);
    nr_lane_stage<8>(x, lane);
    nr_reg_stage<4>(x);
    nr_reg_stage<8>(x);
    wave_lds_fence();  // the previous step's gathers are done
#pragma unroll
    for (int gg = 0; gg < 4; ++gg)
      *(nr_f32x4*)&slot[w][k][64 * gg + 4 * t] =
          nr_f32x4{x[4 * gg], x[4 * gg + 1], x[4 * gg + 2], x[4 * gg + 3]};
    wave_lds_fence();
    const float sv = slot[w][k][lo] * osg;
    if (s_ok && rv) g.partA[(c * g.m + i0 + k) * g.r + t] = sv;
  };

  // loads run two steps ahead through three register buffers; the loop is
  // unrolled by three with no early exit (a step past the range is masked
  // entirely), so the buffers rotate without copies; rows past the range load
  // the last row again
  nr_f32x4 b0[4], b1[4], b2[4];
  float y0, y1, y2;
  load(i_begin, b0, y0);
  load(i_begin + 4, b1, y1);
  for (int64_t i0 = i_begin; i0 < i_end; i0 += 12) {
    load(i0 + 8, b2, y2);
    asm volatile("" ::: "memory");
    step(i0, b0, y0);
    load(i0 + 12, b0, y0);
    asm volatile("" ::: "memory");
    step(i0 + 4, b1, y1);
    load(i0 + 16, b1, y1);
    asm volatile("" ::: "memory");
    step(i0 + 8, b2, y2);
  }

  // the 16 x 16 blocks: lane L, register v holds output row 4(L >> 4) + v (the
  // column index m inside the group), column L & 15 (the row a of Y^T A)
  if (!a_ok) return;
  float* py = g.partY + (split * g.rl + t) * g.n;
#pragma unroll
  for (int gg = 0; gg < 4; ++gg) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t col = cb + 64 * gg + 4 * (4 * k + v) + q;
        if (col < g.n) py[col] = acc[4 * gg + q][v];
      }
    }
  }
}

struct NarrowSrhtPlan {
  int64_t chunks, splits, rows_per_split;
  size_t bytesY, bytes;
};
NarrowSrhtPlan narrow_srht_plan(int64_t m, int64_t n, int64_t r, int64_t rl) {
  NarrowSrhtPlan p{0, 0, 0, 0, 0};
  int64_t npad = 1;
  while (npad < n) npad <<= 1;
  if (m < 1 || rl > NR_MAXRL || r < 1 || n % 4 != 0 || npad < NR_CH * NR_WAVES) return p;
  p.chunks = npad / NR_CH;
  // about 4096 waves in all, whole 4-row steps per split
  const int64_t want = cdiv(4096, p.chunks);
  p.rows_per_split = 4 * cdiv(cdiv(m, want), 4);
  p.splits = cdiv(m, p.rows_per_split);
  p.bytesY = align_up((size_t)p.splits * rl * n * sizeof(float));
  p.bytes = p.bytesY + align_up((size_t)p.chunks * m * r * sizeof(float));
  return p;
}

// ---------------------------------------------------------------- Gaussian X
// The same single read of A for a dense X (n x r, r + l <= 16): Y^T A as above;
// AX from the same registers through LDS.  A wave stages four steps (16 rows x
// its 256 columns, rows padded to 260 floats so that the reads below hit 64
// distinct banks) and then runs 64 v_mfma_f32_16x16x4_f32 over the chunk's
// columns, four at a time, with the X values as the first operand (lane l:
// X[column 4 kb + l / 16][sketch column l % 16], held in registers for the
// whole row range since the wave keeps its chunk) and the staged A as the
// second (lane l: A[row l % 16][column 4 kb + l / 16]): register v of lane l
// is then AX[row l % 16][4 (l / 16) + v], the chunk's partial, added in order
// with the other chunks' afterwards.
constexpr int NG_LD = NR_CH + 4;

struct NarrowGaussArgs {
  int64_t m, n, r, rl, rows_per_split;
  const float* A;
  int64_t lda;
  const float* X;  // n x r, ld r
  const float* Y;  // m x rl, ld rl
  float* partY;    // [splits][rl][n]
  float* partA;    // [chunks][m][r]
};

__global__ void __launch_bounds__(64 * NR_WAVES) pass_f32_gauss_narrow(NarrowGaussArgs g) {
  __shared__ __attribute__((aligned(16))) float blk[NR_WAVES][16][NG_LD];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int t = lane & 15, k = lane >> 4;
  const int64_t c = (int64_t)blockIdx.x * NR_WAVES + w;
  const int64_t cb = c * NR_CH;
  const int64_t split = blockIdx.y;
  const int64_t i_begin = split * g.rows_per_split;
  const int64_t i_end = min(g.m, i_begin + g.rows_per_split);

  bool cval[4];
#pragma unroll
  for (int gg = 0; gg < 4; ++gg) cval[gg] = cb + 64 * gg + 4 * t < g.n;  // n % 4 == 0
  // this lane's X values: X[cb + 4 kb + k][t], zero past n and past r
  float xo[NR_CH / 4];
#pragma unroll
  for (int kb = 0; kb < NR_CH / 4; ++kb) {
    const int64_t col = cb + 4 * kb + k;
    xo[kb] = (col < g.n && t < g.r) ? g.X[col * g.r + t] : 0.f;
  }
  const bool a_ok = t < g.rl;
  const int64_t tcl = a_ok ? t : 0;

  nr_f32x4 acc[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = nr_f32x4{0.f, 0.f, 0.f, 0.f};

  auto load = [&](int64_t i0, nr_f32x4 (&v)[4], float& yb) {
    const int64_t i = i0 + k;
    const int64_t ic = i < i_end ? i : i_end - 1;
    const float* row = g.A + ic * g.lda;
#pragma unroll
    for (int gg = 0; gg < 4; ++gg) {
      const int64_t col = cval[gg] ? cb + 64 * gg + 4 * t : 0;
      v[gg] = *(const nr_f32x4*)(row + col);
    }
    yb = g.Y[ic * g.rl + tcl];
  };

  // AX of the staged block: rows blk_row0 .. blk_row0 + 15 (those below i_end)
  int nblk = 0;
  int64_t blk_row0 = i_begin;
  auto flush = [&]() {
    wave_lds_fence();  // the block's stores are visible to the wave
    nr_f32x4 d = nr_f32x4{0.f, 0.f, 0.f, 0.f};
    const float* br = &blk[w][t][k];
#pragma unroll
    for (int kb = 0; kb < NR_CH / 4; ++kb)
      d = __builtin_amdgcn_mfma_f32_16x16x4f32(xo[kb], br[4 * kb], d, 0, 0, 0);
    const int64_t row = blk_row0 + t;
    if (row < i_end && row < blk_row0 + 4 * nblk) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int jr = 4 * k + v;
        if (jr < g.r) g.partA[(c * g.m + row) * g.r + jr] = d[v];
      }
    }
    wave_lds_fence();  // the reads are done before the next block's stores
    nblk = 0;
  };

  auto step = [&](int64_t i0, const nr_f32x4 (&v)[4], float yv) {
    const bool rv = i0 + k < i_end;
    const float yb = (rv && a_ok) ? yv : 0.f;
    if (nblk == 0) blk_row0 = i0;
#pragma unroll
    for (int gg = 0; gg < 4; ++gg) {
      const bool ok = rv && cval[gg];
      nr_f32x4 a4;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float a = ok ? v[gg][q] : 0.f;
        acc[4 * gg + q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, yb, acc[4 * gg + q], 0, 0, 0);
        a4[q] = a;
      }
      *(nr_f32x4*)&blk[w][4 * nblk + k][64 * gg + 4 * t] = a4;
    }
    if (++nblk == 4) flush();
  };

  nr_f32x4 b0[4], b1[4], b2[4];
  float y0, y1, y2;
  load(i_begin, b0, y0);
  load(i_begin + 4, b1, y1);
  for (int64_t i0 = i_begin; i0 < i_end; i0 += 12) {
    load(i0 + 8, b2, y2);
    asm volatile("" ::: "memory");
    step(i0, b0, y0);
    load(i0 + 12, b0, y0);
    asm volatile("" ::: "memory");
    step(i0 + 4, b1, y1);
    load(i0 + 16, b1, y1);
    asm volatile("" ::: "memory");
    step(i0 + 8, b2, y2);
  }
  if (nblk > 0) flush();

  if (!a_ok) return;
  float* py = g.partY + (split * g.rl + t) * g.n;
#pragma unroll
  for (int gg = 0; gg < 4; ++gg) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t col = cb + 64 * gg + 4 * (4 * k + v) + q;
        if (col < g.n) py[col] = acc[4 * gg + q][v];
      }
    }
  }
}

struct NarrowGaussPlan {
  int64_t chunks, splits, rows_per_split;
  size_t bytesY, bytes;
};
NarrowGaussPlan narrow_gauss_plan(int64_t m, int64_t n, int64_t r, int64_t rl) {
  NarrowGaussPlan p{0, 0, 0, 0, 0};
  if (m < 1 || r < 1 || rl > NR_MAXRL || n % 4 != 0 || n < NR_CH * NR_WAVES) return p;
  p.chunks = NR_WAVES * cdiv(cdiv(n, NR_CH), NR_WAVES);
  const int64_t want = cdiv(4096, p.chunks);  // about 4096 waves in all
  p.rows_per_split = 16 * cdiv(cdiv(m, want), 16);
  p.splits = cdiv(m, p.rows_per_split);
  p.bytesY = align_up((size_t)p.splits * rl * n * sizeof(float));
  p.bytes = p.bytesY + align_up((size_t)p.chunks * m * r * sizeof(float));
  return p;
}

}  // namespace

size_t narrow_srht_ws_bytes(int64_t m, int64_t n, int64_t r, int64_t rl) {
  return narrow_srht_plan(m, n, r, rl).bytes;
}

gn_status launch_f32_srht_narrow(int64_t m, int64_t n, int64_t r, int64_t rl, const float* A,
                                 int64_t lda, const float* Y, const int8_t* signs,
                                 const int32_t* idx, float* AX, int64_t ldax, float* YtA,
                                 int64_t ldya, void* ws, size_t ws_bytes, hipStream_t s) {
  const NarrowSrhtPlan np = narrow_srht_plan(m, n, r, rl);
  if (np.bytes == 0 || !ws || ws_bytes < np.bytes || lda % 4 != 0 || (uintptr_t)A % 16 != 0)
    return GN_ERR_UNSUPPORTED;
  NarrowSrhtArgs g{m, n, r, rl, np.rows_per_split, A, lda, Y, signs, idx, (float*)ws,
                   (float*)((char*)ws + np.bytesY)};
  const dim3 grid((unsigned)(np.chunks / NR_WAVES), (unsigned)np.splits);
  pass_f32_srht_narrow<<<grid, dim3(64 * NR_WAVES), 0, s>>>(g);
  GN_LAUNCH_CHECK();
  GN_TRY(launch_splitk_sum_f32(g.partY, np.splits, rl, n, YtA, ldya, s));
  return launch_splitk_sum_f32(g.partA, np.chunks, m, r, AX, ldax, s);
}

}  // namespace gn

namespace gn {

size_t narrow_gauss_ws_bytes(int64_t m, int64_t n, int64_t r, int64_t rl) {
  return narrow_gauss_plan(m, n, r, rl).bytes;
}

gn_status launch_f32_gauss_narrow(int64_t m, int64_t n, int64_t r, int64_t rl, const float* A,
                                  int64_t lda, const float* X, const float* Y, float* AX,
                                  int64_t ldax, float* YtA, int64_t ldya, void* ws,
                                  size_t ws_bytes, hipStream_t s) {
  const NarrowGaussPlan np = narrow_gauss_plan(m, n, r, rl);
  if (np.bytes == 0 || !ws || ws_bytes < np.bytes || lda % 4 != 0 || (uintptr_t)A % 16 != 0)
    return GN_ERR_UNSUPPORTED;
  NarrowGaussArgs g{m, n, r, rl, np.rows_per_split, A, lda, X, Y, (float*)ws,
                    (float*)((char*)ws + np.bytesY)};
  const dim3 grid((unsigned)(np.chunks / NR_WAVES), (unsigned)np.splits);
  pass_f32_gauss_narrow<<<grid, dim3(64 * NR_WAVES), 0, s>>>(g);
  GN_LAUNCH_CHECK();
  GN_TRY(launch_splitk_sum_f32(g.partY, np.splits, rl, n, YtA, ldya, s));
  return launch_splitk_sum_f32(g.partA, np.chunks, m, r, AX, ldax, s);
}

}  // namespace gn
