// 16-bit matrix-core tile of the large sketch passes (bfloat16 or IEEE binary16
// operands, FP32 accumulation), one 256 x 256 output tile per workgroup of four
// waves.
//
// Each wave owns a 128 x 128 quarter of the tile: 4 x 4 blocks of the 32 x 32 x 16
// matrix-core instruction, 256 accumulators per lane (in the accumulation
// registers, one wave per SIMD).  With a 128 x 128 wave tile the operands a wave
// reads from LDS per 16-deep step (8 KB) feed 16 instructions (512 cycles), half
// of the CU's LDS read bandwidth when all four SIMDs run; a 64 x 64 wave tile
// needs all of it.
//
// K is staged 32 deep through a ring of four LDS stages (16 KB per operand per
// stage) filled by direct global -> LDS 16-byte loads, which go around the
// registers; the loads of stage t + 4 are issued while stage t is multiplied, so
// three stages (about 3000 cycles of matrix-core work) cover their latency.  The
// wait for a stage is an explicit vmcnt count plus a workgroup barrier without a
// memory fence (a fence would also wait for the loads of the later stages).
// Stages past the end of K load zeros, so every iteration has the same number of
// loads in flight; a k-contiguous chunk past K, and every row of the
// j-contiguous operand past K, is read from a zero block.
//
// LDS layouts: k-contiguous operand 256 rows x 32 k (64 bytes per row), the
// j-contiguous operand (the matrix in Y^T A) 32 k-rows x 256 columns, both
// XOR-swizzled at 16- or 32-byte granularity (h16_kc_swz, h16_jc_swz) so that
// the fragment reads below are free of bank conflicts.
// Direct-to-LDS loads write 1 KB per wave instruction to consecutive addresses
// (lane i at offset 16 i), so the swizzle is applied by choosing which global
// chunk each lane loads.
//
// Block scales (the matrix operand is stored as values in [-1, 1] with one
// power-of-two scale per 128 x 128 block): a wave's 128 output rows (AX) or
// columns (Y^T A) lie in one scale stripe; see h16_big_tile_at.
#pragma once

#include "gemm_tiles.h"

#include <type_traits>

namespace gn {
namespace tiles {

typedef __attribute__((address_space(3))) void lds_void;

// Sixteen zero bytes: the source of every chunk that lies past the end of K.
static __device__ __attribute__((aligned(16))) uint32_t g_h16_zero[4];

struct H16Big {
  static constexpr int BM = 256, BN = 256, BK = 32, NS = 4, T = 256;
  static constexpr int OP_ELEMS = 256 * BK;          // one operand, one stage (16 KB)
  static constexpr int STAGE_ELEMS = 2 * OP_ELEMS;   // both operands (32 KB)
  static constexpr size_t RING_BYTES = (size_t)NS * STAGE_ELEMS * sizeof(uint16_t);
  static constexpr int MAX_KB = 1024;                // scale blocks along K held in LDS
  static constexpr size_t smem() { return RING_BYTES + 2 * MAX_KB * sizeof(float); }
  static constexpr int LOADS = 8;                    // direct loads per thread per stage
};

// One direct global -> LDS 16-byte load per lane: lane i's 16 bytes from `src`
// land at LDS byte address lds + 16 i (lds wave-uniform, passed in M0, which is
// restored afterwards; one wait state after writing M0).  Written as inline
// assembly so that the compiler does not treat every later LDS read as
// depending on it (it would insert a wait for all loads in flight before the
// transposing reads); the stage barriers below order these loads explicitly.
// The instruction has no register result.
__device__ __forceinline__ void h16_dma16(uintptr_t src, uint32_t lds) {
  const uint32_t l = __builtin_amdgcn_readfirstlane(lds);
  uint32_t saved;
  asm volatile(
      "s_mov_b32 %0, m0\n\t"
      "s_mov_b32 m0, %2\n\t"
      "s_nop 0\n\t"
      "global_load_lds_dwordx4 %1, off\n\t"
      "s_mov_b32 m0, %0"
      : "=&s"(saved)
      : "v"(src), "s"(l)
      : "memory");
}

__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return (uint32_t)(uintptr_t)(lds_void*)p;
}

// Shapes the tile handles: K a multiple of 8 on k-contiguous operands, the
// j-contiguous operand's row length a multiple of 8 and at least 8, row strides
// multiples of 8 elements, 16-byte aligned bases.
__host__ __forceinline__ bool h16_big_eligible(const GemmBF16& g, bool b_kc) {
  const bool al = ((uintptr_t)g.A % 16 == 0) && ((uintptr_t)g.B % 16 == 0);
  if (!al || g.K % 8 != 0 || g.lda % 8 != 0 || g.ldb % 8 != 0) return false;
  if (!b_kc && (g.N % 8 != 0 || g.N < 8)) return false;
  return g.M >= 1 && g.N >= 1 && g.K >= 1;
}

// LDS swizzles.  k-contiguous operand: the 16-byte chunk c of row r sits in slot
// c ^ h16_kc_swz(r); rows r .. r + 7 (r a multiple of 8) take four different
// values for each row parity, and rows r .. r + 15 four different values for
// each r mod 4, so a 128-bit read of 32 rows at one chunk is free of bank
// conflicts whether the LDS serves 8 lanes (128 bytes) or 16 lanes (256 bytes)
// per cycle.  j-contiguous operand: the 32-byte granule g of k-row k sits at
// g ^ h16_jc_swz(k) with values 0, 3, 5, 6 for k mod 4 = 0 .. 3: distinct mod 4
// (the four rows a 16-lane group of a transposing read covers fall in four
// 32-byte bank groups of a 128-byte line) and distinct after halving (the eight
// row-granule pairs of 32 lanes fall in eight groups of a 256-byte line).
__device__ __forceinline__ int h16_kc_swz(int row) { return ((row >> 1) ^ (row >> 3)) & 3; }
__device__ __forceinline__ int h16_jc_swz(int kr) { return (0x6530 >> (4 * (kr & 3))) & 7; }

// The direct loads of one operand for every stage: each thread's four 16-byte
// chunks per stage, as running global addresses (advanced by one stage each
// time) and the K offset that decides whether a chunk is past the end of K.
//   k-contiguous operand (256 rows x 32 k per stage): chunk q of wave w holds
//     rows 16 (4w + q) + lane / 4 and, in slot lane % 4, the k-chunk
//     (lane % 4) ^ ((row / 2) % 4) of that row;
//   j-contiguous operand (32 k-rows x 256 columns per stage): chunk q holds
//     k-rows 2 (4w + q) + lane / 32, and in 16-byte slot lane % 32 the 32-byte
//     granule (slot / 2) ^ (k-row % 4) (its half slot % 2).
struct H16Dma {
  uintptr_t p[4];   // global address of each chunk at the current stage
  int64_t kof[4];   // its K index at stage 0 (valid while kof + k0 < K)
  int64_t step;     // address advance per stage, in bytes
};

__device__ __forceinline__ H16Dma h16_dma_kc_init(const uint16_t* P, int64_t ld, int64_t rows,
                                                  int64_t r0, int lane, int wave) {
  H16Dma d;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int row = (wave * 4 + q) * 16 + (lane >> 2);
    const int lc = (lane & 3) ^ h16_kc_swz(row);
    int64_t gr = r0 + row;
    gr = gr < rows ? gr : rows - 1;  // rows past the end: any valid row (outputs discarded)
    d.p[q] = (uintptr_t)(P + gr * ld + 8 * lc);
    d.kof[q] = 8 * lc;
  }
  d.step = (int64_t)H16Big::BK * (int64_t)sizeof(uint16_t);
  return d;
}

__device__ __forceinline__ H16Dma h16_dma_jc_init(const uint16_t* P, int64_t ld, int64_t N,
                                                  int64_t c0, int lane, int wave) {
  H16Dma d;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int kr = 2 * (wave * 4 + q) + (lane >> 5);
    const int slot = lane & 31;
    const int lg = (slot >> 1) ^ h16_jc_swz(kr);
    int64_t gc = c0 + 16 * lg + 8 * (slot & 1);
    gc = gc <= N - 8 ? gc : N - 8;  // columns past the end: any valid chunk (outputs discarded)
    d.p[q] = (uintptr_t)(P + (int64_t)kr * ld + gc);
    d.kof[q] = kr;
  }
  d.step = (int64_t)H16Big::BK * ld * (int64_t)sizeof(uint16_t);
  return d;
}

// MFMA operand fragment of a k-contiguous operand: 32 rows from rb, k from kk:
// lane l holds row rb + l % 32, k = kk + 8 (l / 32) .. + 7.
__device__ __forceinline__ bf16x8 h16_frag_kc(const uint16_t* S, int rb, int kk, int lane) {
  const int row = rb + (lane & 31);
  const int lc = (kk >> 3) + (lane >> 5);
  const int slot = lc ^ h16_kc_swz(row);
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(S + row * 32 + slot * 8));
}

// MFMA B fragment of the j-contiguous operand: lane l holds column cb + l % 32 at
// k = kk + 8 (l / 32) .. + 7, by two transposing reads of four k-rows each.
__device__ __forceinline__ bf16x8 h16_frag_jc(const uint16_t* S, int cb, int kk, int lane) {
  const int g = lane >> 4, p = lane & 15;
  const int kr = kk + 8 * (g >> 1) + (p >> 2);
  const int pg = ((cb >> 4) + (g & 1)) ^ h16_jc_swz(kr);
  const uint16_t* q = S + kr * 256 + pg * 16 + 4 * (p & 3);
  typedef __attribute__((address_space(3))) bf16x4_bits lds_v4;
  const bf16x4_bits h0 = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4*)q);
  const bf16x4_bits h1 = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4*)(q + 4 * 256));
  typedef short s8 __attribute__((ext_vector_type(8)));
  const s8 v = {h0[0], h0[1], h0[2], h0[3], h1[0], h1[1], h1[2], h1[3]};
  return __builtin_bit_cast(bf16x8, v);
}

// Workgroup barrier that waits for this thread's LDS reads and for all but the
// last N of its direct loads (the stages still in flight), without a fence.
template <int N>
__device__ __forceinline__ void h16_stage_barrier() {
  if constexpr (N == 16)
    asm volatile("s_waitcnt vmcnt(16) lgkmcnt(0)\n\ts_barrier" ::: "memory");
  else
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// One register (two values) of the non-matrix operand's fragment times f = 2^e
// (e <= 0, wave-uniform): for bfloat16 through float (the products stay bfloat16
// values, so taking their high halves is exact), for binary16 one packed
// multiply.
template <bool F16>
__device__ __forceinline__ uint32_t h16_scale_word(uint32_t w, float f) {
  if constexpr (F16) {
    typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, __builtin_bit_cast(f16x2, w) * (_Float16)f);
  } else {
    const float lo = __uint_as_float(w << 16) * f;
    const float hi = __uint_as_float(w & 0xffff0000u) * f;
    return __builtin_amdgcn_perm(__float_as_uint(hi), __float_as_uint(lo), 0x07060302u);
  }
}
template <bool F16>
__device__ __forceinline__ bf16x8 h16_scale_frag(bf16x8 v, float f) {
  u32x4 u = __builtin_bit_cast(u32x4, v);
#pragma unroll
  for (int i = 0; i < 4; ++i) u[i] = h16_scale_word<F16>(u[i], f);
  return __builtin_bit_cast(bf16x8, u);
}

// Largest and smallest entry of a stripe's block scales held in LDS (nkb
// values), reduced over the wave.
__device__ __forceinline__ void h16_stripe_range(const float* sc, int64_t nkb, int lane,
                                                 float& smax, float& smin) {
  float mx = 0.f, mn = 3.0e38f;
  for (int64_t kb = lane; kb < nkb; kb += 64) {
    const float v = sc[kb];
    mx = fmaxf(mx, v);
    mn = fminf(mn, v);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    mx = fmaxf(mx, __shfl_xor(mx, o));
    mn = fminf(mn, __shfl_xor(mn, o));
  }
  smax = mx;
  smin = mn;
}

// One 256 x 256 tile of D = A B at (i0, j0).
//   A(i, k) = PA[i lda + k]; A_IS_MAT: A is the block-scaled matrix (AX).
//   B(k, j) = PB[j ldb + k] when B_KC, else PB[k ldb + j] (the matrix: Y^T A).
// Block scales: the accumulators are kept in units of the largest scale s_ref
// of the wave's stripe; the contribution of a K block with scale s is taken with
// the non-matrix operand's fragments times s / s_ref, a power of two (exact for
// bfloat16 when s / s_ref >= 2^-32; binary16 values whose scaled magnitude falls
// below 2^-14 are rounded to the subnormal grid).  Tiles whose stripes span more
// than 2^32 (bfloat16) or 2^8 (binary16) between their largest and smallest
// scale take the general tile instead (which rescales the accumulators).
template <bool A_IS_MAT, bool B_KC, bool F16>
__device__ void h16_big_tile_at(const GemmBF16& g, int64_t i0, int64_t j0, char* smem) {
  using CF = H16Big;
  static_assert(CF::LOADS == 8 && CF::NS == 4, "the barrier counts assume 8 loads, 4 stages");
  uint16_t* ring = reinterpret_cast<uint16_t*>(smem);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int64_t nst = cdiv_d(g.K, CF::BK);
  const int64_t nkb = cdiv_d(g.K, 128);

  // the two scale stripes of the tile, copied to LDS after the ring (every wave
  // checks both, so the choice of path is the same in all four waves)
  const int64_t omax = A_IS_MAT ? cdiv_d(g.M, 128) - 1 : g.nsb - 1;
  const int64_t o0 = A_IS_MAT ? (i0 >> 7) : (j0 >> 7);
  const int64_t ob0 = o0 < omax ? o0 : omax, ob1 = o0 + 1 < omax ? o0 + 1 : omax;
  float* sc_lds = reinterpret_cast<float*>(smem + CF::RING_BYTES);  // [2][MAX_KB]
  const bool fits = nkb <= CF::MAX_KB;
  if (fits) {
    for (int64_t e = threadIdx.x; e < 2 * nkb; e += CF::T) {
      const int64_t st = e / nkb, kb = e - st * nkb, o = st ? ob1 : ob0;
      sc_lds[st * CF::MAX_KB + kb] = A_IS_MAT ? g.scales[o * g.nsb + kb] : g.scales[kb * g.nsb + o];
    }
  }
  __syncthreads();
  float mx0 = 1.f, mn0 = 0.f, mx1 = 1.f, mn1 = 0.f;
  if (fits) {
    h16_stripe_range(sc_lds, nkb, lane, mx0, mn0);
    h16_stripe_range(sc_lds + CF::MAX_KB, nkb, lane, mx1, mn1);
  }
  const float lim = F16 ? 0x1.0p-8f : 0x1.0p-32f;
  if (!(fits && mn0 >= lim * mx0 && mn1 >= lim * mx1)) {
    // wide scale range: the general 128 x 128 tile (4 waves), four times
    using Gen = BF16Cfg<128, 128, 64, 2, 2>;
    static_assert(Gen::T == CF::T && Gen::smem() <= CF::smem(), "general tile must fit");
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
      bf16_tile_at<Gen, A_IS_MAT, B_KC, F16>(g, i0 + 128 * (q & 1), j0 + 128 * (q >> 1), smem);
      __syncthreads();
    }
    return;
  }
  const int my = A_IS_MAT ? wm : wn;  // this wave's stripe
  const float s_ref = my ? mx1 : mx0, my_mn = my ? mn1 : mn0;
  const float inv_ref = 1.f / s_ref;  // exact: a power of two
  const float* my_sc = sc_lds + my * CF::MAX_KB;
  auto scale_of = [&](int64_t kb) -> float { return my_sc[kb]; };

  H16Dma da = h16_dma_kc_init(g.A, g.lda, g.M, i0, lane, wave);
  H16Dma db = B_KC ? h16_dma_kc_init(g.B, g.ldb, g.N, j0, lane, wave)
                   : h16_dma_jc_init(g.B, g.ldb, g.N, j0, lane, wave);
  const uint32_t ring_lds = lds_addr(smem);
  // Stage loads: issue_half(st, h) issues this thread's chunks h of stage st
  // (h = 0, 1: operand A; 2, 3: operand B; two chunks each), so that the eight
  // loads of a stage can be spread between the matrix-core instructions.
  // Stages are issued in order; past the end they load zeros.
  auto stage_k0 = [&](int64_t st) -> int64_t { return st < nst ? st * CF::BK : g.K; };
  auto stage_lds = [&](int64_t st) -> uint32_t {
    return ring_lds + (uint32_t)((st & (CF::NS - 1)) * CF::STAGE_ELEMS * 2);
  };
  const uintptr_t zero_src = (uintptr_t)g_h16_zero;  // read once (a relocated address)
  auto issue_half = [&](int64_t st, int h) {
    H16Dma& d = h < 2 ? da : db;
    const uint32_t base = stage_lds(st) + (h < 2 ? 0u : (uint32_t)(CF::OP_ELEMS * 2));
    const int64_t k0 = stage_k0(st);
#pragma unroll
    for (int q2 = 0; q2 < 2; ++q2) {
      const int q = 2 * (h & 1) + q2;
      const uintptr_t src = (d.kof[q] + k0 < g.K) ? d.p[q] : zero_src;
      h16_dma16(src, base + (uint32_t)((wave * 4 + q) * 1024));
      d.p[q] += d.step;
    }
  };
  auto frag_a = [&](int64_t st, int kk, int x) -> bf16x8 {
    const uint16_t* S = ring + (st & (CF::NS - 1)) * CF::STAGE_ELEMS;
    return h16_frag_kc(S, wm * 128 + 32 * x, kk, lane);
  };
  auto frag_b = [&](int64_t st, int kk, int y) -> bf16x8 {
    const uint16_t* S = ring + (st & (CF::NS - 1)) * CF::STAGE_ELEMS + CF::OP_ELEMS;
    if constexpr (B_KC)
      return h16_frag_kc(S, wn * 128 + 32 * y, kk, lane);
    else
      return h16_frag_jc(S, wn * 128 + 32 * y, kk, lane);
  };
  f32x16 acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[x][y][v] = 0.f;
  // The sketch operand (X, the B fragments, for AX; Y^T, the A fragments, for
  // Y^T A) carries the block scales: S[g] is its fragment g and O the other
  // operand's four.  A half stage's products are issued in four groups, group g
  // multiplying S[g] with O[0 .. 3].  When the wave's stripe holds more than one
  // scale, group g also scales the fragment that the following group needs, its
  // instructions placed between the group's matrix-core instructions so that they
  // issue while those execute.
  auto group = [&](auto scaled, int g, const bf16x8 (&S)[4], const bf16x8 (&O)[4], bf16x8& next,
                   float fn) {
    constexpr bool SC = decltype(scaled)::value;
    u32x4 nx = __builtin_bit_cast(u32x4, next);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      if constexpr (A_IS_MAT)
        acc[o][g] = mfma_32x32x16<F16>(O[o], S[g], acc[o][g]);
      else
        acc[g][o] = mfma_32x32x16<F16>(S[g], O[o], acc[g][o]);
      if constexpr (SC) {  // one register of `next` after each product, pinned there
        __builtin_amdgcn_sched_barrier(0);
        nx[o] = h16_scale_word<F16>(nx[o], fn);
        asm volatile("" : "+v"(nx[o]));  // computed here, not sunk to its use
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (SC) next = __builtin_bit_cast(bf16x8, nx);
  };

  // the K loop; `scaled` (std::true_type or std::false_type) says whether the
  // wave's stripe needs the scaling
  auto run = [&](auto scaled) {
    constexpr bool SC = decltype(scaled)::value;
    // prologue: stages 0 .. 3 in flight, stage 0 landed
#pragma unroll
    for (int st = 0; st < CF::NS; ++st)
#pragma unroll
      for (int h = 0; h < 4; ++h) issue_half(st, h);
    // f: the factor of the K block of the stage being multiplied; s_next: the
    // scale of the following K block
    float f = scale_of(0) * inv_ref;
    float s_next = nkb > 1 ? scale_of(1) : s_ref;
    asm volatile("s_waitcnt vmcnt(24)\n\ts_barrier" ::: "memory");
    bf16x8 fa0[4], fb0[4], fa1[4], fb1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      fb0[q] = frag_b(0, 0, q);
      fa0[q] = frag_a(0, 0, q);
    }
    bf16x8(&S0)[4] = A_IS_MAT ? fb0 : fa0;
    bf16x8(&O0)[4] = A_IS_MAT ? fa0 : fb0;
    bf16x8(&S1)[4] = A_IS_MAT ? fb1 : fa1;
    bf16x8(&O1)[4] = A_IS_MAT ? fa1 : fb1;
    if constexpr (SC) S0[0] = h16_scale_frag<F16>(S0[0], f);

    for (int64_t t = 0; t < nst; ++t) {
      // phase 1: the products of stage t's first 16-deep half, with the second
      // half's fragments read in between
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        fb1[x] = frag_b(t, 16, x);
        fa1[x] = frag_a(t, 16, x);
        group(scaled, x, S0, O0, x < 3 ? S0[x + 1] : S1[0], f);
      }
      h16_stage_barrier<16>();  // stage t + 1 landed; every wave is done with stage t
      float fn = f;
      if (((t + 1) & 3) == 0) {  // stage t + 1 starts a new 128-deep K block
        fn = s_next * inv_ref;
        const int64_t kb = ((t + 1) >> 2) + 1;
        if (kb < nkb) s_next = scale_of(kb);
      }
      // phase 2: the second half's products, with stage t + 4's loads and stage
      // t + 1's first-half fragments (B first: the next phase needs all of them
      // for its first group) issued in between; past the last stage the
      // fragments come from a zero stage and are not used
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        issue_half(t + CF::NS, x);
        if (x < 2) {
          fb0[2 * x] = frag_b(t + 1, 0, 2 * x);
          fb0[2 * x + 1] = frag_b(t + 1, 0, 2 * x + 1);
        } else {
          fa0[2 * x - 4] = frag_a(t + 1, 0, 2 * x - 4);
          fa0[2 * x - 3] = frag_a(t + 1, 0, 2 * x - 3);
        }
        group(scaled, x, S1, O1, x < 3 ? S1[x + 1] : S0[0], x < 3 ? f : fn);
      }
      f = fn;
    }
  };
  if (my_mn == s_ref)
    run(std::false_type{});
  else
    run(std::true_type{});
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // no load may land after the tile

  // 32 x 32 accumulator: register v of lane l holds row 8 (v / 4) + 4 (l / 32) + v % 4,
  // column l % 32
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = i0 + wm * 128 + x * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int64_t col = j0 + wn * 128 + y * 32 + (lane & 31);
        if (row < g.M && col < g.N) g.D[row * g.ldd + col] = acc[x][y][v] * s_ref;
      }
}

// The tile of XCD-mapped index `local` (tiles of one XCD walk the inner index).
template <bool A_IS_MAT, bool B_KC, bool F16>
__device__ void h16_big_tile(const GemmBF16& g, int64_t local, char* smem) {
  const int64_t tm_n = cdiv_d(g.M, H16Big::BM), tn_n = cdiv_d(g.N, H16Big::BN);
  int64_t tm, tn;
  if (g.inner_is_m) {
    if (!xcd_tile(local, tm_n, tn_n, tm, tn)) return;
  } else {
    if (!xcd_tile(local, tn_n, tm_n, tn, tm)) return;
  }
  h16_big_tile_at<A_IS_MAT, B_KC, F16>(g, tm * H16Big::BM, tn * H16Big::BN, smem);
}

}  // namespace tiles
}  // namespace gn
