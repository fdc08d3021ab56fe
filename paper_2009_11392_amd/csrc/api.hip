// libgn C ABI: argument validation, workspace layout and launch order.
// Every entry point validates synchronously, then enqueues on the caller's
// stream and returns without synchronizing.
#include <math.h>

#include <mutex>

#include "gn_internal.h"

using namespace gn;

namespace {

constexpr int64_t kMaxCore = 4096;      // r + l: core QR held on chip
constexpr int64_t kMaxSrhtPad = 1 << 17;  // n' for the SRHT column selection
constexpr int64_t kMaxSrhtR = 2048;       // sampled columns per row in registers

struct Plan {
  int64_t m, n, r, l, rl, npad;
  int32_t mode, kx, ky, sdt, adt;
  int32_t method;   // gn_core_method
  bool pinv_form;   // core applied as Q2 R2^{-T} Q1^T whatever k is
  int64_t gate_r;   // k is compared with this to pick the factored form
  double nux, nuy;
  double tau;
};

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// A second stream per device (non-blocking, default priority) for work that runs
// beside the caller's stream, with the events of one fork and its join.  Created
// on first use and kept until the process ends; the mutex is held from the fork
// to the join, so concurrent callers never share the events.
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
constexpr int kMaxDevices = 64;
std::mutex g_side_mu;
SideStream g_side[kMaxDevices];

gn_status side_stream(SideStream** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GN_ERR_HIP;
  SideStream& ss = g_side[dev];
  if (!ss.s) {
    hipStream_t st = nullptr;
    hipEvent_t ef = nullptr, ej = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return GN_ERR_HIP;
    if (hipEventCreateWithFlags(&ef, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ej, hipEventDisableTiming) != hipSuccess) {
      if (ef) (void)hipEventDestroy(ef);
      (void)hipStreamDestroy(st);
      return GN_ERR_HIP;
    }
    ss.s = st;
    ss.fork = ef;
    ss.join = ej;
  }
  *out = &ss;
  return GN_OK;
}

gn_status make_plan(const gn_problem* p, Plan& P) {
  if (!p) return GN_ERR_ARG;
  if (p->core_method < GN_CORE_QR || p->core_method > GN_CORE_LIFT_DIAG) return GN_ERR_ARG;
  if (p->mode < GN_MODE_F64 || p->mode > GN_MODE_F16_BS) return GN_ERR_ARG;
  if (p->kind_x < GN_SKETCH_GAUSSIAN || p->kind_x > GN_SKETCH_USER) return GN_ERR_ARG;
  if (p->kind_y != GN_SKETCH_GAUSSIAN && p->kind_y != GN_SKETCH_USER) return GN_ERR_ARG;
  if (!isfinite(p->eps) || !isfinite(p->nu_x) || !isfinite(p->nu_y)) return GN_ERR_ARG;
  if (p->m < 1 || p->n < 1 || p->r < 1 || p->r > p->m || p->r > p->n) return GN_ERR_SHAPE;
  if (p->m > INT32_MAX || p->n > INT32_MAX) return GN_ERR_UNSUPPORTED;
  P.m = p->m;
  P.n = p->n;
  P.r = p->r;
  P.l = (p->l < 0) ? (p->r + 1) / 2 : p->l;
  P.rl = P.r + P.l;
  if (P.rl > kMaxCore) return GN_ERR_UNSUPPORTED;
  P.npad = next_pow2(P.n);
  P.mode = p->mode;
  P.kx = p->kind_x;
  P.ky = p->kind_y;
  P.sdt = sketch_dtype(p->mode);
  P.adt = accum_dtype(p->mode);
  if (P.kx == GN_SKETCH_SRHT && (P.npad > kMaxSrhtPad || P.r > kMaxSrhtR)) return GN_ERR_UNSUPPORTED;
  double nux = p->nu_x, nuy = p->nu_y;
  if (nux <= 0.0)
    nux = (P.kx == GN_SKETCH_SRHT) ? sqrt((double)P.npad)
          : (P.kx == GN_SKETCH_GAUSSIAN) ? sqrt((double)P.n) + sqrt((double)P.r)
                                         : 1.0;
  if (nuy <= 0.0)
    nuy = (P.ky == GN_SKETCH_GAUSSIAN) ? sqrt((double)P.m) + sqrt((double)P.rl) : 1.0;
  P.nux = nux;
  P.nuy = nuy;
  P.tau = (p->eps > 0.0) ? p->eps * nux * nuy : 0.0;
  P.method = p->core_method;
  if (P.method >= GN_CORE_LIFT_SVD && !(P.tau > 0.0)) return GN_ERR_ARG;  // nothing to lift to
  P.pinv_form = P.method == GN_CORE_SVD || P.method == GN_CORE_LIFT_SVD ||
                P.method == GN_CORE_LIFT_RRQR;
  P.gate_r = P.r + (P.pinv_form ? 1 : 0);
  return GN_OK;
}

// ---- workspace layouts (offsets in bytes, each region 256-byte aligned)
struct SketchWs {
  size_t xt, yt, signs, idx, keys, split, split_bytes, total;
};
SketchWs sketch_ws(const Plan& P) {
  SketchWs w{};
  size_t off = 0;
  const size_t es = dtype_size(P.sdt);
  w.xt = off;
  if (P.kx != GN_SKETCH_SRHT) off += align_up((size_t)P.r * P.n * es);
  w.yt = off;
  off += align_up((size_t)P.rl * P.m * es);
  w.signs = off;
  w.idx = off;
  w.keys = off;
  if (P.kx == GN_SKETCH_SRHT) {
    w.signs = off;
    off += align_up((size_t)P.npad);
    w.idx = off;
    off += align_up((size_t)P.r * 4);
    w.keys = off;
    off += srht_ws_bytes(P.npad);
  }
  w.split = off;  // K-split partials of a pass with few output tiles
  w.split_bytes = pass_split_ws_bytes(P.mode, P.kx, P.m, P.n, P.r, P.rl);
  off += w.split_bytes;
  w.total = off;
  return w;
}

struct CoreWs {
  size_t yt, c, qr, z, qr2, split, q1, stab, signs, idx, keys, total;
};
CoreWs core_ws(const Plan& P) {
  CoreWs w{};
  size_t off = 0;
  w.yt = off;
  // Y for the core product: as stored by the pass in F64 mode (regenerated
  // unless USER); widened to float in F32 / BF16 modes.
  if (P.mode == GN_MODE_F64) {
    if (P.ky == GN_SKETCH_GAUSSIAN) off += align_up((size_t)P.rl * P.m * 8);
  } else if (P.ky == GN_SKETCH_GAUSSIAN || is_h16_mode(P.mode)) {
    off += align_up((size_t)P.rl * P.m * 4);
  }
  w.c = off;
  off += align_up((size_t)P.rl * P.r * 8);
  w.qr = off;
  off += qr_ws_bytes(P.rl, P.r);
  w.z = off;
  off += align_up((size_t)P.r * P.r * 8);
  w.qr2 = off;
  off += qr_ws_bytes(P.r, P.r);
  w.split = off;
  if (P.mode == GN_MODE_F64) {
    off += dgemm_split_ws_bytes(P.rl, P.r, P.m);
  } else {
    const size_t a = core_product_ws_bytes(P.m, P.rl, P.r);
    const size_t b = is_h16_mode(P.mode) ? core_product_bf16_ws_bytes(P.m, P.rl, P.r) : 0;
    off += a > b ? a : b;
  }
  // the QR's Q before the SVD / pivoting turns it into Q1, and that method's scratch
  w.q1 = off;
  if (P.pinv_form) off += align_up((size_t)P.rl * P.r * 8);
  w.stab = off;
  off += align_up(stabilize_ws_bytes(P.method, P.r));
  // SRHT signs and sampled columns for the core matrix as (Y^T A) X
  w.signs = w.idx = w.keys = off;
  if (P.kx == GN_SKETCH_SRHT && P.mode != GN_MODE_F64) {
    off += align_up((size_t)P.npad);
    w.idx = off;
    off += align_up((size_t)P.r * 4);
    w.keys = off;
    off += align_up(srht_ws_bytes(P.npad));
  }
  w.total = off;
  return w;
}

struct ApplyWs {
  size_t t1, t2, t3, split, split_bytes, solve, total;
};
ApplyWs apply_ws(const Plan& P, int64_t kc) {
  ApplyWs w{};
  const int64_t k1 = kc > 0 ? kc : 1;
  const size_t blk = align_up((size_t)P.rl * (size_t)k1 * 8);
  w.t1 = 0;
  w.t2 = blk;
  w.t3 = 2 * blk;
  w.split = 3 * blk;
  // K-slice partials of the products that split K (both sides)
  const int64_t shapes[6][3] = {{P.rl, k1, P.n}, {P.r, k1, P.rl}, {P.m, k1, P.r},
                                {k1, P.r, P.m},  {k1, P.rl, P.r}, {k1, P.n, P.rl}};
  w.split_bytes = 0;
  for (const auto& sh : shapes) {
    const size_t b = dgemm_split_ws_bytes(sh[0], sh[1], sh[2]);
    if (b > w.split_bytes) w.split_bytes = b;
  }
  w.solve = w.split + align_up(w.split_bytes);
  w.total = w.solve + (kc <= small_solve_max_rhs() ? small_solve_ws_bytes(P.r) : 0);
  return w;
}

// Reverse mode: sketch-dtype (sd) buffers for [U | Y] (m x (r+l)), [X^T ; V]
// ((r+l) x n), S^T (n x (r+l)), AX (m x r, when recomputed or re-strided),
// G1 (m x (r+l)) and G2 (r x n); FP64 buffers for H and the core adjoint.
struct BackWs {
  size_t lcat, rcat, st, p, g1, g2, h, m0, m1, c, bbar, x2, z, y5, t1, t2, t3, t4, t5, psplit,
      psplit_bytes, gsplit, gsplit_bytes, dsplit, dsplit_bytes, split, total;
};
BackWs back_ws(const Plan& P) {
  BackWs w{};
  const size_t sd = (P.mode == GN_MODE_F64) ? 8 : 4;
  const size_t rl = P.rl, r = P.r, m = P.m, n = P.n;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  w.lcat = take(m * (r + rl) * sd);
  w.rcat = take((r + rl) * n * sd);
  w.st = take(n * rl * sd);
  w.p = take(m * r * sd);
  w.g1 = take(m * rl * sd);
  w.g2 = take(r * n * sd);
  w.h = take(r * rl * 8);
  w.m0 = take(r * rl * 8);
  w.m1 = take(r * rl * 8);
  w.c = take(rl * r * 8);
  w.bbar = take(rl * r * 8);
  w.x2 = take(rl * r * 8);
  w.z = take(rl * r * 8);
  w.y5 = take(rl * r * 8);
  w.t1 = take(r * r * 8);
  w.t2 = take(r * r * 8);
  w.t3 = take(r * r * 8);
  w.t4 = take(r * r * 8);
  w.t5 = take(r * r * 8);
  w.psplit_bytes = pass_split_ws_bytes(P.mode, GN_SKETCH_GAUSSIAN, P.m, P.n, P.rl, P.r);
  w.psplit = take(w.psplit_bytes);
  w.gsplit_bytes = (P.mode == GN_MODE_F32) ? gemm_f32_split_ws_bytes(P.m, P.r, P.n) : 0;
  w.gsplit = take(w.gsplit_bytes);
  {
    const int64_t shapes[][3] = {{P.r, P.rl, P.r},  {P.rl, P.r, P.r},  {P.r, P.r, P.rl},
                                 {P.r, P.r, P.r},   {P.m, P.r, P.rl},  {P.rl, P.n, P.r},
                                 {P.m, P.n, P.r + P.rl}};
    size_t mx = 0;
    for (const auto& sh : shapes) {
      const size_t b = dgemm_split_ws_bytes(sh[0], sh[1], sh[2]);
      if (b > mx) mx = b;
    }
    w.dsplit_bytes = mx;
    w.dsplit = take(mx);
  }
  w.split = off;
  off += (P.mode == GN_MODE_F64) ? dgemm_split_ws_bytes(P.r, P.rl, P.m)
                                 : core_product_ws_bytes(P.m, P.r, P.rl);
  w.total = off;
  return w;
}

// Section 6 updates: sketch blocks X (up to n x r) and Y (up to m x (r+l)) in the
// sketch dtype, SRHT signs / sample / keys, temporaries for the products to be
// accumulated (m x r and (r+l) x n in the accumulation dtype), K-split scratch.
struct UpdWs {
  size_t xs, ys, signs, idx, keys, tax, tya, split, split_bytes, total;
};
UpdWs upd_ws(const Plan& P) {
  UpdWs w{};
  const size_t es = dtype_size(P.sdt), ac = dtype_size(P.adt);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  w.xs = take((size_t)P.n * P.r * es);
  w.ys = take((size_t)P.m * P.rl * es);
  if (P.kx == GN_SKETCH_SRHT) {
    w.signs = take((size_t)P.npad);
    w.idx = take((size_t)P.r * 4);
    w.keys = take(srht_ws_bytes(P.npad));
  }
  w.tax = take((size_t)P.m * P.r * ac);
  w.tya = take((size_t)P.rl * P.n * ac);
  w.split_bytes = pass_split_ws_bytes(P.mode, P.kx, P.m, P.n, P.r, P.rl);
  w.split = take(w.split_bytes);
  w.total = off;
  return w;
}

size_t materialize_ws(const Plan& P) {
  return align_up((size_t)P.m * P.r * 8) + align_up((size_t)P.r * P.n * 8) + 256;
}

// copy (and widen) an m x r matrix of dtype dt into double, run only when the
// gate says the core was not truncated.
__global__ void __launch_bounds__(256) widen_gated(int64_t rows, int64_t cols, const void* src,
                                                   int32_t dt, int64_t lds, double* dst,
                                                   int64_t ldd, const int32_t* kdev, int64_t r) {
  if (*kdev < r) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = e / cols, j = e - i * cols;
  double v;
  if (dt == GN_DT_F64)
    v = reinterpret_cast<const double*>(src)[i * lds + j];
  else if (dt == GN_DT_F32)
    v = (double)reinterpret_cast<const float*>(src)[i * lds + j];
  else if (dt == GN_DT_F16)
    v = (double)f16_bits_to_f32(reinterpret_cast<const uint16_t*>(src)[i * lds + j]);
  else
    v = (double)bf16_bits_to_f32(reinterpret_cast<const uint16_t*>(src)[i * lds + j]);
  dst[i * ldd + j] = v;
}

gn_status widen(int64_t rows, int64_t cols, const void* src, int32_t dt, int64_t lds, double* dst,
                int64_t ldd, const int32_t* kdev, int64_t r, hipStream_t s) {
  widen_gated<<<dim3((unsigned)cdiv(rows * cols, 256)), dim3(256), 0, s>>>(rows, cols, src, dt, lds,
                                                                           dst, ldd, kdev, r);
  GN_LAUNCH_CHECK();
  return GN_OK;
}

}  // namespace

extern "C" {

const char* gn_version(void) { return "0.1.0"; }

const char* gn_status_string(int32_t s) {
  switch (s) {
    case GN_OK: return "GN_OK";
    case GN_ERR_ARG: return "GN_ERR_ARG: invalid argument";
    case GN_ERR_SHAPE: return "GN_ERR_SHAPE: inconsistent shapes or leading dimensions";
    case GN_ERR_DTYPE: return "GN_ERR_DTYPE: dtype not valid here";
    case GN_ERR_ALIGN: return "GN_ERR_ALIGN: pointer not 16-byte aligned";
    case GN_ERR_WORKSPACE: return "GN_ERR_WORKSPACE: workspace too small";
    case GN_ERR_HIP: return "GN_ERR_HIP: HIP launch or runtime failure";
    case GN_ERR_NUMERIC: return "GN_ERR_NUMERIC: non-finite or rank-0 core";
    case GN_ERR_UNSUPPORTED: return "GN_ERR_UNSUPPORTED: size or mode beyond the library's limits";
    default: return "unknown gn_status";
  }
}

gn_status gn_workspace_size(const gn_problem* p, int32_t op, int64_t kcols, size_t* bytes) {
  if (!bytes) return GN_ERR_ARG;
  Plan P;
  GN_TRY(make_plan(p, P));
  switch (op) {
    case GN_OP_SKETCH: *bytes = sketch_ws(P).total; break;
    case GN_OP_CORE: *bytes = core_ws(P).total; break;
    case GN_OP_FACTORS: *bytes = 256; break;
    case GN_OP_APPLY:
      if (kcols < 1) return GN_ERR_SHAPE;
      *bytes = apply_ws(P, kcols).total;
      break;
    case GN_OP_RESIDUAL: *bytes = residual_ws_bytes(P.m, P.n); break;
    case GN_OP_SRHT: *bytes = srht_ws_bytes(P.npad); break;
    case GN_OP_BACKWARD: *bytes = back_ws(P).total; break;
    case GN_OP_MATERIALIZE: *bytes = materialize_ws(P); break;
    case GN_OP_UPDATE: *bytes = upd_ws(P).total; break;
    case GN_OP_CHECK:
      if (kcols < 1 || kcols > 16) return GN_ERR_ARG;
      *bytes = power_ws_bytes(P.r, (int32_t)kcols);
      break;
    default: return GN_ERR_ARG;
  }
  return GN_OK;
}

gn_status gn_generate_gaussian(uint64_t seed, int32_t stream, int64_t row0, int64_t col0,
                               int64_t rows, int64_t cols, int32_t dtype, int32_t layout, void* out,
                               int64_t ld, gn_stream_t stream_) {
  if (!out) return GN_ERR_ARG;
  if (dtype < GN_DT_F64 || dtype > GN_DT_F16 || (layout != 0 && layout != 1)) return GN_ERR_ARG;
  if (rows < 0 || cols < 0 || row0 < 0 || col0 < 0) return GN_ERR_SHAPE;
  if (row0 + rows > ((int64_t)1 << 32) || ((col0 + cols) >> 1) > ((int64_t)1 << 32))
    return GN_ERR_UNSUPPORTED;
  if (layout == 0 ? (ld < cols) : (ld < rows)) return GN_ERR_SHAPE;
  return launch_gaussian(seed, stream, row0, col0, rows, cols, dtype, layout, out, ld,
                         (hipStream_t)stream_);
}

gn_status gn_srht_generate(uint64_t seed, int64_t n, int64_t r, int8_t* signs, int32_t* idx,
                           void* ws, size_t ws_bytes, gn_stream_t stream) {
  if (!signs || !idx || !ws) return GN_ERR_ARG;
  if (n < 1 || r < 1) return GN_ERR_SHAPE;
  const int64_t npad = next_pow2(n);
  if (r > npad) return GN_ERR_SHAPE;
  if (npad > kMaxSrhtPad) return GN_ERR_UNSUPPORTED;
  if (ws_bytes < srht_ws_bytes(npad)) return GN_ERR_WORKSPACE;
  if (((uintptr_t)ws & 7u) != 0) return GN_ERR_ALIGN;
  return launch_srht(seed, npad, r, signs, idx, (uint64_t*)ws, (hipStream_t)stream);
}

gn_status gn_sketch_prepare(const gn_problem* p, const void* X_user, int64_t ldx,
                            const void* Y_user, int64_t ldy, int8_t* signs_out, int32_t* idx_out,
                            void* ws, size_t ws_bytes, gn_stream_t stream_) {
  Plan P;
  GN_TRY(make_plan(p, P));
  hipStream_t s = (hipStream_t)stream_;
  if (!ws) return GN_ERR_ARG;
  if (P.kx == GN_SKETCH_USER && !X_user) return GN_ERR_ARG;
  if (P.ky == GN_SKETCH_USER && !Y_user) return GN_ERR_ARG;
  if (P.kx == GN_SKETCH_USER && ldx < P.r) return GN_ERR_SHAPE;
  if (P.ky == GN_SKETCH_USER && ldy < P.rl) return GN_ERR_SHAPE;
  if (!aligned16(ws)) return GN_ERR_ALIGN;
  const SketchWs W = sketch_ws(P);
  if (ws_bytes < W.total) return GN_ERR_WORKSPACE;
  char* base = (char*)ws;
  // Algorithm 2.1, step 1: the sketches.  FP64/FP32 passes read X (n x r) and
  // Y (m x (r+l)) row-major; the BF16 pass reads them transposed (k-contiguous).
  const int lay = is_h16_mode(P.mode) ? 1 : 0;
  const size_t es = dtype_size(P.sdt);
  if (P.ky == GN_SKETCH_GAUSSIAN) {
    GN_TRY(launch_gaussian(p->seed, 2, 0, 0, P.m, P.rl, P.sdt, lay, base + W.yt, lay ? P.m : P.rl, s));
  } else if (lay) {
    GN_TRY(launch_transpose(Y_user, P.m, P.rl, ldy, P.sdt, base + W.yt, P.m, s));
  } else if (hipMemcpy2DAsync(base + W.yt, P.rl * es, Y_user, ldy * es, P.rl * es, P.m,
                              hipMemcpyDeviceToDevice, s) != hipSuccess) {
    return GN_ERR_HIP;
  }
  if (P.kx == GN_SKETCH_GAUSSIAN) {
    GN_TRY(launch_gaussian(p->seed, 1, 0, 0, P.n, P.r, P.sdt, lay, base + W.xt, lay ? P.n : P.r, s));
  } else if (P.kx == GN_SKETCH_USER) {
    if (lay) {
      GN_TRY(launch_transpose(X_user, P.n, P.r, ldx, P.sdt, base + W.xt, P.n, s));
    } else if (hipMemcpy2DAsync(base + W.xt, P.r * es, X_user, ldx * es, P.r * es, P.n,
                                hipMemcpyDeviceToDevice, s) != hipSuccess) {
      return GN_ERR_HIP;
    }
  } else {
    int8_t* signs = (int8_t*)(base + W.signs);
    int32_t* idx = (int32_t*)(base + W.idx);
    GN_TRY(launch_srht(p->seed, P.npad, P.r, signs, idx, (uint64_t*)(base + W.keys), s));
    if (signs_out && hipMemcpyAsync(signs_out, signs, (size_t)P.npad, hipMemcpyDeviceToDevice, s) !=
                         hipSuccess)
      return GN_ERR_HIP;
    if (idx_out && hipMemcpyAsync(idx_out, idx, (size_t)P.r * 4, hipMemcpyDeviceToDevice, s) !=
                       hipSuccess)
      return GN_ERR_HIP;
  }
  return GN_OK;
}

gn_status gn_sketch_pass(const gn_problem* p, const void* A, int64_t lda, const float* A_scales,
                         void* AX, int64_t ldax, void* YtA, int64_t ldya, void* ws,
                         size_t ws_bytes, gn_stream_t stream_) {
  Plan P;
  GN_TRY(make_plan(p, P));
  if (!A || !AX || !YtA || !ws) return GN_ERR_ARG;
  if (is_h16_mode(P.mode) && !A_scales) return GN_ERR_ARG;
  if (lda < P.n || ldax < P.r || ldya < P.n) return GN_ERR_SHAPE;
  if (!aligned16(A) || !aligned16(AX) || !aligned16(YtA) || !aligned16(ws)) return GN_ERR_ALIGN;
  const SketchWs W = sketch_ws(P);
  if (ws_bytes < W.total) return GN_ERR_WORKSPACE;
  char* base = (char*)ws;
  return launch_pass(P.mode, P.kx, P.m, P.n, P.r, P.rl, A, lda, A_scales, base + W.xt,
                     (const int8_t*)(base + W.signs), (const int32_t*)(base + W.idx), base + W.yt,
                     AX, ldax, YtA, ldya, (hipStream_t)stream_, base + W.split, W.split_bytes);
}

gn_status gn_sketch(const gn_problem* p, const void* A, int64_t lda, const float* A_scales,
                    const void* X_user, int64_t ldx, const void* Y_user, int64_t ldy, void* AX,
                    int64_t ldax, void* YtA, int64_t ldya, int8_t* signs_out, int32_t* idx_out,
                    void* ws, size_t ws_bytes, gn_stream_t stream) {
  Plan P;
  GN_TRY(make_plan(p, P));
  // validate the pass arguments before anything is enqueued
  if (!A || !AX || !YtA || !ws) return GN_ERR_ARG;
  if (is_h16_mode(P.mode) && !A_scales) return GN_ERR_ARG;
  if (lda < P.n || ldax < P.r || ldya < P.n) return GN_ERR_SHAPE;
  if (!aligned16(A) || !aligned16(AX) || !aligned16(YtA) || !aligned16(ws)) return GN_ERR_ALIGN;
  GN_TRY(gn_sketch_prepare(p, X_user, ldx, Y_user, ldy, signs_out, idx_out, ws, ws_bytes, stream));
  return gn_sketch_pass(p, A, lda, A_scales, AX, ldax, YtA, ldya, ws, ws_bytes, stream);
}

gn_status gn_core(const gn_problem* p, const void* AX, int64_t ldax, const void* YtA, int64_t ldya,
                  const void* Y_user, int64_t ldy, const gn_core_out* out, void* ws,
                  size_t ws_bytes, gn_stream_t stream_) {
  Plan P;
  GN_TRY(make_plan(p, P));
  hipStream_t s = (hipStream_t)stream_;
  if (!AX || !out || !ws || !out->k || !out->status || !out->Q1 || !out->R || !out->Q2 || !out->R2)
    return GN_ERR_ARG;
  if (P.ky == GN_SKETCH_USER && !Y_user) return GN_ERR_ARG;
  if (ldax < P.r) return GN_ERR_SHAPE;
  if (P.ky == GN_SKETCH_USER && ldy < P.rl) return GN_ERR_SHAPE;
  if (YtA && ldya < P.n) return GN_ERR_SHAPE;
  if (!aligned16(AX) || !aligned16(ws) || (YtA && !aligned16(YtA))) return GN_ERR_ALIGN;
  const CoreWs W = core_ws(P);
  if (ws_bytes < W.total) return GN_ERR_WORKSPACE;
  char* base = (char*)ws;
  double* C = (double*)(base + W.c);
  double* Z = (double*)(base + W.z);

  // C = Y^T (AX) (the order of the Section 5.1 evaluation): FP64 in F64 mode;
  // in F32 mode (and the 16-bit modes with a user Y) on the FP32 matrix cores (the
  // pass precision), in BF16 / FP16 modes on the matrix cores of that format, the
  // K slices summed in FP64.  With an SRHT X and Y^T A given (F32 / BF16 modes), C = (Y^T A) X
  // instead, the order Section 2.3 costs: the r + l rows of Y^T A sign-flipped,
  // Walsh-Hadamard transformed and sampled in FP64, with the signs and columns
  // regenerated from the seed (bit-identical to the pass's).
  if (YtA && P.kx == GN_SKETCH_SRHT && P.mode != GN_MODE_F64) {
    int8_t* sg = (int8_t*)(base + W.signs);
    int32_t* ix = (int32_t*)(base + W.idx);
    GN_TRY(launch_srht(p->seed, P.npad, P.r, sg, ix, (uint64_t*)(base + W.keys), s));
    GN_TRY(launch_srht_right(P.rl, P.n, P.r, (const float*)YtA, ldya, sg, ix, C, P.r, s));
  } else if (P.mode == GN_MODE_F64) {
    MatRef yt;
    if (P.ky == GN_SKETCH_GAUSSIAN) {
      void* Yt = base + W.yt;
      GN_TRY(launch_gaussian(p->seed, 2, 0, 0, P.m, P.rl, P.sdt, 1, Yt, P.m, s));
      yt = MatRef{Yt, P.sdt, P.m, 1};
    } else {
      yt = MatRef{Y_user, P.sdt, 1, ldy};  // Y^T(c, i) = Y[i*ldy + c]
    }
    MatRef ax{AX, P.adt, ldax, 1};
    GN_TRY(launch_dgemm(P.rl, P.r, P.m, 1.0, yt, ax, 0.0, C, P.r, 1, nullptr, false, s, nullptr,
                        0, true, (double*)(base + W.split), W.total - W.split));
  } else if (is_h16_mode(P.mode) && P.ky == GN_SKETCH_GAUSSIAN) {
    // BF16 / FP16 modes: Y's 16-bit values (transposed, as the pass reads them) on
    // the 16-bit matrix cores, AX in two terms of the same format
    const bool f16 = (P.mode == GN_MODE_F16_BS);
    uint16_t* Yt = (uint16_t*)(base + W.yt);
    GN_TRY(launch_gaussian(p->seed, 2, 0, 0, P.m, P.rl, f16 ? GN_DT_F16 : GN_DT_BF16, 1, Yt, P.m,
                           s));
    GN_TRY(launch_core_product_h16(P.m, P.rl, P.r, Yt, f16, (const float*)AX, ldax,
                                   base + W.split, C, s));
  } else {
    const float* Yf;
    int64_t ldyf;
    if (P.ky == GN_SKETCH_GAUSSIAN) {
      const int32_t gdt = (P.mode == GN_MODE_BF16_BS)   ? kDtBf16AsF32
                          : (P.mode == GN_MODE_F16_BS) ? kDtF16AsF32
                                                       : GN_DT_F32;
      GN_TRY(launch_gaussian(p->seed, 2, 0, 0, P.m, P.rl, gdt, 0, base + W.yt, P.rl, s));
      Yf = (const float*)(base + W.yt);
      ldyf = P.rl;
    } else if (is_h16_mode(P.mode)) {
      GN_TRY(launch_widen_h16(P.m, P.rl, (const uint16_t*)Y_user, ldy, P.mode == GN_MODE_F16_BS,
                              (float*)(base + W.yt), P.rl, s));
      Yf = (const float*)(base + W.yt);
      ldyf = P.rl;
    } else {
      Yf = (const float*)Y_user;
      ldyf = ldy;
    }
    GN_TRY(launch_core_product_f32(P.m, P.rl, P.r, Yf, ldyf, (const float*)AX, ldax,
                                   (float*)(base + W.split), C, s));
  }
  double* qws = (double*)(base + W.qr);
  switch (P.method) {
    case GN_CORE_QR: {
      // Householder QR; then, on a side stream, the kept rank and the second QR
      // (whose kernels return at once unless truncated) while this stream forms Q1;
      // the two meet again before the call's later work.
      GN_TRY(launch_qr_factor(P.rl, P.r, C, P.r, out->R, P.r, qws, nullptr, s));
      std::lock_guard<std::mutex> lock(g_side_mu);
      SideStream* ss = nullptr;
      GN_TRY(side_stream(&ss));
      if (hipEventRecord(ss->fork, s) != hipSuccess ||
          hipStreamWaitEvent(ss->s, ss->fork, 0) != hipSuccess)
        return GN_ERR_HIP;
      GN_TRY(launch_truncate(P.r, out->R, P.r, P.tau, out->k, out->status, Z, P.r, ss->s));
      GN_TRY(launch_qr(P.r, P.r, Z, P.r, out->Q2, P.r, out->R2, P.r, (double*)(base + W.qr2),
                       out->k, ss->s));
      if (hipEventRecord(ss->join, ss->s) != hipSuccess) return GN_ERR_HIP;
      GN_TRY(launch_qr_form_q(P.rl, P.r, C, P.r, out->Q1, P.r, qws, nullptr, s));
      if (hipStreamWaitEvent(s, ss->join, 0) != hipSuccess) return GN_ERR_HIP;
      break;
    }
    case GN_CORE_LIFT_DIAG:
      GN_TRY(launch_qr(P.rl, P.r, C, P.r, out->Q1, P.r, out->R, P.r, qws, nullptr, s));
      GN_TRY(launch_lift_diag(P.r, out->R, P.r, P.tau, out->k, out->status, s));
      break;
    case GN_CORE_SVD:
    case GN_CORE_LIFT_SVD: {
      double* q1 = (double*)(base + W.q1);
      GN_TRY(launch_qr(P.rl, P.r, C, P.r, q1, P.r, out->R, P.r, qws, nullptr, s));
      GN_TRY(launch_svd_core(P.r, P.rl, out->R, P.r, q1, P.tau,
                             P.method == GN_CORE_LIFT_SVD ? 1 : 0, out->k, out->status, out->Q1,
                             out->Q2, out->R2, base + W.stab, s));
      break;
    }
    case GN_CORE_LIFT_RRQR: {
      double* q1 = (double*)(base + W.q1);
      GN_TRY(launch_qr(P.rl, P.r, C, P.r, q1, P.r, out->R, P.r, qws, nullptr, s));
      GN_TRY(launch_rrqr_core(P.r, P.rl, out->R, P.r, q1, P.tau, out->k, out->status, out->Q1,
                              out->R, out->Q2, out->R2, base + W.stab, s));
      break;
    }
    default:
      return GN_ERR_ARG;
  }
  return GN_OK;
}

gn_status gn_core_check(const gn_problem* p, const gn_core_out* core, double delta, int32_t nv,
                        int32_t iters, double* est, void* ws, size_t ws_bytes, gn_stream_t stream_) {
  Plan P;
  GN_TRY(make_plan(p, P));
  hipStream_t s = (hipStream_t)stream_;
  if (!core || !ws || !core->k || !core->status || !core->R || !core->R2) return GN_ERR_ARG;
  if (nv < 1 || nv > 16 || iters < 1 || iters > 64) return GN_ERR_ARG;
  if (!isfinite(delta)) return GN_ERR_ARG;
  const double tau_d = (delta > 0.0) ? delta * P.nux * P.nuy : P.tau;
  if (!(tau_d > 0.0)) return GN_ERR_ARG;
  if (ws_bytes < power_ws_bytes(P.r, nv)) return GN_ERR_WORKSPACE;
  if (((uintptr_t)ws & 7u) != 0) return GN_ERR_ALIGN;
  return launch_power_check(P.r, p->seed, nv, iters, core->R, core->R2, core->k, P.pinv_form,
                            tau_d, core->status, est, ws, s);
}

gn_status gn_factors(const gn_problem* p, const void* AX, int64_t ldax, const void* YtA,
                     int64_t ldya, const gn_core_out* core, double* F, int64_t ldf, double* G,
                     int64_t ldg, void* ws, size_t ws_bytes, gn_stream_t stream_) {
  Plan P;
  GN_TRY(make_plan(p, P));
  hipStream_t s = (hipStream_t)stream_;
  (void)ws;
  (void)ws_bytes;
  if (!AX || !YtA || !core || !F || !G || !core->k || !core->Q1 || !core->R || !core->Q2 || !core->R2)
    return GN_ERR_ARG;
  if (ldax < P.r || ldya < P.n || ldf < P.r || ldg < P.n) return GN_ERR_SHAPE;
  // F = AX R^{-1}  or  (AX Q2) R2^{-T}
  GN_TRY(widen(P.m, P.r, AX, P.adt, ldax, F, ldf, core->k, P.gate_r, s));
  MatRef ax{AX, P.adt, ldax, 1};
  MatRef q2{core->Q2, GN_DT_F64, P.r, 1};
  GN_TRY(launch_dgemm(P.m, P.r, P.r, 1.0, ax, q2, 0.0, F, ldf, 1, nullptr, false, s, core->k,
                      P.gate_r, true));
  GN_TRY(launch_trsm_core(P.m, P.r, core->R, core->R2, P.r, core->k, F, ldf, 1, false, true, s,
                          false, P.pinv_form));
  // G = Q1[:, :k]^T (Y^T A), rows >= k zero
  MatRef q1t{core->Q1, GN_DT_F64, 1, P.r};
  MatRef yta{YtA, P.adt, ldya, 1};
  GN_TRY(launch_dgemm(P.r, P.n, P.rl, 1.0, q1t, yta, 0.0, G, ldg, 1, core->k, true, s));
  return GN_OK;
}

gn_status gn_apply(const gn_problem* p, int32_t side, const void* AX, int64_t ldax, const void* YtA,
                   int64_t ldya, const gn_core_out* core, const double* W, int64_t ldw, int64_t kc,
                   void* out_, int64_t ldo, void* ws, size_t ws_bytes, gn_stream_t stream_) {
  Plan P;
  GN_TRY(make_plan(p, P));
  hipStream_t s = (hipStream_t)stream_;
  if (side == 2) {  // A_hat = F G, in the accumulation dtype
    if (!AX || !YtA || !core || !out_ || !ws) return GN_ERR_ARG;
    if (ldo < P.n) return GN_ERR_SHAPE;
    if (ws_bytes < materialize_ws(P)) return GN_ERR_WORKSPACE;
    if (((uintptr_t)ws & 7u) != 0) return GN_ERR_ALIGN;
    double* F = (double*)ws;
    double* G = (double*)((char*)ws + align_up((size_t)P.m * P.r * 8));
    GN_TRY(gn_factors(p, AX, ldax, YtA, ldya, core, F, P.r, G, P.n, nullptr, 0, stream_));
    return launch_dgemm_to(P.m, P.n, P.r, 1.0, MatRef{F, GN_DT_F64, P.r, 1},
                           MatRef{G, GN_DT_F64, P.n, 1}, 0.0, out_, P.adt, ldo, 1, nullptr, false,
                           s);
  }
  double* out = (double*)out_;
  if (!AX || !YtA || !core || !W || !out || !ws || !core->k || !core->Q1 || !core->R || !core->Q2 ||
      !core->R2)
    return GN_ERR_ARG;
  if (side != 0 && side != 1) return GN_ERR_ARG;
  if (kc < 1) return GN_ERR_SHAPE;
  if (ldax < P.r || ldya < P.n) return GN_ERR_SHAPE;
  if (side == 0 && (ldw < kc || ldo < kc)) return GN_ERR_SHAPE;
  if (side == 1 && (ldw < P.m || ldo < P.n)) return GN_ERR_SHAPE;
  const ApplyWs Wl = apply_ws(P, kc);
  if (ws_bytes < Wl.total) return GN_ERR_WORKSPACE;
  char* base = (char*)ws;
  double* t1 = (double*)(base + Wl.t1);
  double* t2 = (double*)(base + Wl.t2);
  double* t3 = (double*)(base + Wl.t3);
  double* sp = (double*)(base + Wl.split);
  MatRef ax{AX, P.adt, ldax, 1};
  MatRef yta{YtA, P.adt, ldya, 1};
  // few right-hand sides: the solve's preparation (block inverses, transposed
  // factor; it needs only the core) runs on the side stream during the products
  // that precede the solve
  const bool few = kc <= small_solve_max_rhs();
  std::unique_lock<std::mutex> lock(g_side_mu, std::defer_lock);
  SideStream* ss = nullptr;
  if (few) {
    lock.lock();
    GN_TRY(side_stream(&ss));
    if (hipEventRecord(ss->fork, s) != hipSuccess ||
        hipStreamWaitEvent(ss->s, ss->fork, 0) != hipSuccess)
      return GN_ERR_HIP;
    GN_TRY(launch_small_solve_prep(P.r, core->R, core->R2, core->k, P.pinv_form, base + Wl.solve,
                                   ss->s));
    if (hipEventRecord(ss->join, ss->s) != hipSuccess) return GN_ERR_HIP;
  }
  auto join = [&]() -> gn_status {
    return hipStreamWaitEvent(s, ss->join, 0) == hipSuccess ? GN_OK : GN_ERR_HIP;
  };
  if (side == 0) {
    // t1 = (Y^T A) W : rl x kc
    GN_TRY(launch_dgemm(P.rl, kc, P.n, 1.0, yta, MatRef{W, GN_DT_F64, ldw, 1}, 0.0, t1, kc, 1,
                        nullptr, false, s, nullptr, 0, true, sp, Wl.split_bytes));
    // t2 = Q1[:, :k]^T t1 : r x kc (rows >= k zero)
    GN_TRY(launch_dgemm(P.r, kc, P.rl, 1.0, MatRef{core->Q1, GN_DT_F64, 1, P.r},
                        MatRef{t1, GN_DT_F64, kc, 1}, 0.0, t2, kc, 1, core->k, true, s, nullptr,
                        0, true, sp, Wl.split_bytes));
    // t2 <- R^{-1} t2  or  R2^{-T} t2   (left solve on the transposed view)
    if (few) {
      GN_TRY(join());
      GN_TRY(launch_small_solve(P.r, core->R, core->R2, core->k, P.pinv_form, true, t2, kc, 1, kc,
                                base + Wl.solve, s));
    } else
      GN_TRY(launch_trsm_core(kc, P.r, core->R, core->R2, P.r, core->k, t2, 1, kc, true, true, s,
                              false, P.pinv_form));
    // t3 = t2 (k == r)  or  Q2 t2 (k < r)
    GN_TRY(widen(P.r, kc, t2, GN_DT_F64, kc, t3, kc, core->k, P.gate_r, s));
    GN_TRY(launch_dgemm(P.r, kc, P.r, 1.0, MatRef{core->Q2, GN_DT_F64, P.r, 1},
                        MatRef{t2, GN_DT_F64, kc, 1}, 0.0, t3, kc, 1, nullptr, false, s, core->k,
                        P.gate_r, true));
    // out = AX t3 : m x kc
    GN_TRY(launch_dgemm(P.m, kc, P.r, 1.0, ax, MatRef{t3, GN_DT_F64, kc, 1}, 0.0, out, ldo, 1,
                        nullptr, false, s, nullptr, 0, true, sp, Wl.split_bytes));
  } else {
    // t1 = W AX : kc x r
    GN_TRY(launch_dgemm(kc, P.r, P.m, 1.0, MatRef{W, GN_DT_F64, ldw, 1}, ax, 0.0, t1, P.r, 1,
                        nullptr, false, s, nullptr, 0, true, sp, Wl.split_bytes));
    // t2 = t1 (k == r)  or  t1 Q2 (k < r); then t2 <- t2 R^{-1}  or  t2 R2^{-T}
    GN_TRY(widen(kc, P.r, t1, GN_DT_F64, P.r, t2, P.r, core->k, P.gate_r, s));
    GN_TRY(launch_dgemm(kc, P.r, P.r, 1.0, MatRef{t1, GN_DT_F64, P.r, 1},
                        MatRef{core->Q2, GN_DT_F64, P.r, 1}, 0.0, t2, P.r, 1, nullptr, false, s,
                        core->k, P.gate_r, true));
    if (few) {
      GN_TRY(join());
      GN_TRY(launch_small_solve(P.r, core->R, core->R2, core->k, P.pinv_form, false, t2, kc, P.r, 1,
                                base + Wl.solve, s));
    } else
      GN_TRY(launch_trsm_core(kc, P.r, core->R, core->R2, P.r, core->k, t2, P.r, 1, false, true, s,
                              false, P.pinv_form));
    // t3 = t2 Q1^T : kc x rl   (columns of t2 beyond k are zero)
    GN_TRY(launch_dgemm(kc, P.rl, P.r, 1.0, MatRef{t2, GN_DT_F64, P.r, 1},
                        MatRef{core->Q1, GN_DT_F64, 1, P.r}, 0.0, t3, P.rl, 1, nullptr, false, s,
                        nullptr, 0, true, sp, Wl.split_bytes));
    // out = t3 (Y^T A) : kc x n
    GN_TRY(launch_dgemm(kc, P.n, P.rl, 1.0, MatRef{t3, GN_DT_F64, P.rl, 1}, yta, 0.0, out, ldo, 1,
                        nullptr, false, s, nullptr, 0, true, sp, Wl.split_bytes));
  }
  return GN_OK;
}

gn_status gn_backward(const gn_problem* p, const void* A, int64_t lda, const void* Gbar,
                      int64_t ldg, const void* AX, int64_t ldax, const void* YtA, int64_t ldya,
                      const gn_core_out* core, void* dA, int64_t ldda, void* ws, size_t ws_bytes,
                      gn_stream_t stream_) {
  Plan P;
  GN_TRY(make_plan(p, P));
  hipStream_t s = (hipStream_t)stream_;
  if (P.mode != GN_MODE_F64 && P.mode != GN_MODE_F32) return GN_ERR_UNSUPPORTED;
  if (P.kx != GN_SKETCH_GAUSSIAN || P.ky != GN_SKETCH_GAUSSIAN) return GN_ERR_UNSUPPORTED;
  if (P.method != GN_CORE_QR) return GN_ERR_UNSUPPORTED;  // differentiates the truncated QR only
  if (!Gbar || !YtA || !core || !dA || !ws || !core->k || !core->Q1 || !core->R || !core->Q2 ||
      !core->R2)
    return GN_ERR_ARG;
  if (!AX && !A) return GN_ERR_ARG;
  if (ldg < P.n || ldya < P.n || ldda < P.n) return GN_ERR_SHAPE;
  if (AX && ldax < P.r) return GN_ERR_SHAPE;
  if (!AX && lda < P.n) return GN_ERR_SHAPE;
  if (!aligned16(ws)) return GN_ERR_ALIGN;
  const BackWs W = back_ws(P);
  if (ws_bytes < W.total) return GN_ERR_WORKSPACE;

  const bool f32 = (P.mode == GN_MODE_F32);
  const int32_t sdt = P.sdt, adt = P.adt;  // both the mode's dtype here
  const size_t sd = f32 ? 4 : 8;
  const int64_t m = P.m, n = P.n, r = P.r, rl = P.rl, K2 = P.r + P.rl;
  char* base = (char*)ws;
  char* lcat = base + W.lcat;  // [U | Y], m x (r + rl)
  char* rcat = base + W.rcat;  // [X^T ; V], (r + rl) x n
  void* St = base + W.st;
  void* G1 = base + W.g1;
  void* G2 = base + W.g2;
  double* H = (double*)(base + W.h);
  double* M0 = (double*)(base + W.m0);
  double* M = (double*)(base + W.m1);
  double* Cm = (double*)(base + W.c);
  double* Bb = (double*)(base + W.bbar);
  double* X2 = (double*)(base + W.x2);
  double* Z = (double*)(base + W.z);
  double* Y5 = (double*)(base + W.y5);
  double* T1 = (double*)(base + W.t1);
  double* T2 = (double*)(base + W.t2);
  double* T3 = (double*)(base + W.t3);
  double* T4 = (double*)(base + W.t4);
  double* T5 = (double*)(base + W.t5);
  const int32_t* kd = core->k;
  constexpr int32_t F64 = GN_DT_F64;
  double* DS = (double*)(base + W.dsplit);  // split-contraction scratch of the FP64 products
  const size_t DSB = W.dsplit_bytes;
  const MatRef Q1r{core->Q1, F64, r, 1}, Q1t{core->Q1, F64, 1, r};
  const MatRef Q2r{core->Q2, F64, r, 1}, Q2t{core->Q2, F64, 1, r};
  auto sq = [&](double* T) { return MatRef{T, F64, r, 1}; };  // ld r (r x r and rl x r)

  // The parts of the core adjoint that need only the forward's core run on the
  // side stream while this stream draws the sketches and makes the pass over
  // Gbar; the two meet before Bbar.  The side stream alone uses M0, M, C, Z, T5
  // and the DS scratch until then.
  std::lock_guard<std::mutex> side_lock(g_side_mu);
  SideStream* ss = nullptr;
  GN_TRY(side_stream(&ss));
  const hipStream_t s2 = ss->s;
  if (hipEventRecord(ss->fork, s) != hipSuccess || hipStreamWaitEvent(s2, ss->fork, 0) != hipSuccess)
    return GN_ERR_HIP;
  // M = R^{-1} Q1^T (k == r) or Q2 R2^{-T} Q1[:, :k]^T (k < r)
  GN_TRY(launch_transpose_rows_masked(rl, r, core->Q1, r, kd, M0, rl, s2));
  GN_TRY(launch_trsm_core(rl, r, core->R, core->R2, r, kd, M0, 1, rl, true, true, s2));
  GN_TRY(widen(r, rl, M0, F64, rl, M, rl, kd, r, s2));
  GN_TRY(launch_dgemm(r, rl, r, 1.0, Q2r, MatRef{M0, F64, rl, 1}, 0.0, M, rl, 1, nullptr, false, s2,
                      kd, r, true, DS, DSB));
  // C = Q1 R
  GN_TRY(launch_dgemm(rl, r, r, 1.0, Q1r, MatRef{core->R, F64, r, 1}, 0.0, Cm, r, 1, nullptr,
                      false, s2, nullptr, 0, true, DS, DSB));
  // Z = Q1k R11^{-T} (columns >= k zero), then T5 = C^T Z
  if (hipMemcpyAsync(Z, core->Q1, (size_t)rl * r * 8, hipMemcpyDeviceToDevice, s2) != hipSuccess)
    return GN_ERR_HIP;
  GN_TRY(launch_trsm_core(rl, r, core->R, core->R2, r, kd, Z, r, 1, true, true, s2, true));
  GN_TRY(launch_dgemm(r, r, rl, 1.0, MatRef{Cm, F64, 1, r}, sq(Z), 0.0, T5, r, 1, nullptr, false,
                      s2, nullptr, 0, true, DS, DSB));
  if (hipEventRecord(ss->join, s2) != hipSuccess) return GN_ERR_HIP;

  // sketches, as the forward pass drew them: X^T in rows [0, r) of rcat, Y in
  // columns [r, r + rl) of lcat
  GN_TRY(launch_gaussian(p->seed, 1, 0, 0, n, r, sdt, 1, rcat, n, s));
  GN_TRY(launch_gaussian(p->seed, 2, 0, 0, m, rl, sdt, 0, lcat + r * sd, K2, s));
  // AX with row stride r: the caller's, re-strided, or recomputed from A
  const void* Pm = AX;
  if (AX && ldax != r) {
    if (hipMemcpy2DAsync(base + W.p, r * sd, AX, ldax * sd, r * sd, m, hipMemcpyDeviceToDevice,
                         s) != hipSuccess)
      return GN_ERR_HIP;
    Pm = base + W.p;
  } else if (!AX) {
    if (f32)
      GN_TRY(launch_gemm_f32(m, r, n, (const float*)A, lda, true, (const float*)rcat, n, true,
                             (float*)(base + W.p), r, s, (float*)(base + W.gsplit),
                             W.gsplit_bytes));
    else
      GN_TRY(launch_dgemm(m, r, n, 1.0, MatRef{A, F64, lda, 1}, MatRef{rcat, F64, 1, n}, 0.0,
                          (double*)(base + W.p), r, 1, nullptr, false, s));
    Pm = base + W.p;
  }
  // G1 = Gbar (Y^T A)^T and G2 = (AX)^T Gbar: the sketch pass over Gbar with
  // sketches (Y^T A)^T (n x rl) and AX (m x r)
  GN_TRY(launch_transpose(YtA, rl, n, ldya, adt, St, rl, s));
  GN_TRY(launch_pass(P.mode, GN_SKETCH_GAUSSIAN, m, n, rl, r, Gbar, ldg, nullptr, St, nullptr,
                     nullptr, Pm, G1, rl, G2, n, s, base + W.psplit, W.psplit_bytes));
  // H = (AX)^T G1 = dL/dM
  if (f32)
    GN_TRY(launch_core_product_f32(m, r, rl, (const float*)Pm, r, (const float*)G1, rl,
                                   (float*)(base + W.split), H, s));
  else
    GN_TRY(launch_dgemm(r, rl, m, 1.0, MatRef{Pm, F64, 1, r}, MatRef{G1, F64, rl, 1}, 0.0, H, rl, 1,
                        nullptr, false, s, nullptr, 0, true, (double*)(base + W.split),
                        W.total - W.split));

  // ---- the rest of the core adjoint in FP64 (k from the forward pass, on the
  // device), after the side stream's M, C, Z and C^T Z; the small products split
  // their contraction through the DS scratch region
  if (hipStreamWaitEvent(s, ss->join, 0) != hipSuccess) return GN_ERR_HIP;
  const MatRef Mr{M, F64, rl, 1}, Mt{M, F64, 1, rl};
  const MatRef Hr{H, F64, rl, 1}, Ht{H, F64, 1, rl};
  // U = G1 M^T (columns [0, r) of lcat) and V's first term M^T G2 (rows [r, r + rl)
  // of rcat) need only M, G1 and G2: the side stream forms them while this stream
  // runs the chain of small products below (neither touches lcat, rcat or DS).
  if (hipEventRecord(ss->fork, s) != hipSuccess || hipStreamWaitEvent(s2, ss->fork, 0) != hipSuccess)
    return GN_ERR_HIP;
  GN_TRY(launch_dgemm_to(m, r, rl, 1.0, MatRef{G1, adt, rl, 1}, Mt, 0.0, lcat, sdt, K2, 1, nullptr,
                         false, s2));
  GN_TRY(launch_dgemm_to(rl, n, r, 1.0, Mt, MatRef{G2, adt, n, 1}, 0.0, rcat + (size_t)r * n * sd,
                         sdt, n, 1, nullptr, false, s2));
  if (hipEventRecord(ss->join, s2) != hipSuccess) return GN_ERR_HIP;
  // Bbar = -M^T H M^T
  GN_TRY(launch_dgemm(r, r, rl, 1.0, Hr, Mt, 0.0, T1, r, 1, nullptr, false, s, nullptr, 0, true, DS, DSB));
  GN_TRY(launch_dgemm(rl, r, r, -1.0, Mt, sq(T1), 0.0, Bb, r, 1, nullptr, false, s, nullptr, 0, true, DS, DSB));
  // Bbar += (I - Q1k Q1k^T) H^T M M^T
  GN_TRY(launch_dgemm(r, r, rl, 1.0, Mr, Mt, 0.0, T2, r, 1, nullptr, false, s, nullptr, 0, true, DS, DSB));
  GN_TRY(launch_dgemm(rl, r, r, 1.0, Ht, sq(T2), 0.0, X2, r, 1, nullptr, false, s, nullptr, 0, true, DS, DSB));
  GN_TRY(launch_dgemm(r, r, rl, 1.0, Q1t, sq(X2), 0.0, T3, r, 1, kd, true, s, nullptr, 0, true, DS, DSB));
  GN_TRY(launch_dgemm(rl, r, r, -1.0, Q1r, sq(T3), 1.0, X2, r, 1, nullptr, false, s, nullptr, 0, true, DS, DSB));
  GN_TRY(launch_axpy(rl, r, 1.0, X2, r, Bb, r, s));
  // k < r: Bbar += M^T (M H^T)(I - Q2k Q2k^T)
  GN_TRY(launch_dgemm(r, r, rl, 1.0, Mr, Ht, 0.0, T1, r, 1, nullptr, false, s, kd, r, true, DS, DSB));
  GN_TRY(launch_dgemm(r, r, r, 1.0, sq(T1), Q2r, 0.0, T4, r, 1, kd, false, s, kd, r, true, DS, DSB));
  GN_TRY(launch_dgemm(r, r, r, -1.0, sq(T4), Q2t, 1.0, T1, r, 1, nullptr, false, s, kd, r, true, DS, DSB));
  GN_TRY(launch_dgemm(rl, r, r, 1.0, Mt, sq(T1), 1.0, Bb, r, 1, nullptr, false, s, kd, r, true, DS, DSB));
  // Y5 = Bbar (C^T Z) + C (Bbar^T Z), C^T Z = T5 from the side stream
  GN_TRY(launch_dgemm(r, r, rl, 1.0, MatRef{Bb, F64, 1, r}, sq(Z), 0.0, T3, r, 1, nullptr, false,
                      s, nullptr, 0, true, DS, DSB));
  GN_TRY(launch_dgemm(rl, r, r, 1.0, sq(Bb), sq(T5), 0.0, Y5, r, 1, nullptr, false, s, nullptr, 0, true, DS, DSB));
  GN_TRY(launch_dgemm(rl, r, r, 1.0, sq(Cm), sq(T3), 1.0, Y5, r, 1, nullptr, false, s, nullptr, 0, true, DS, DSB));
  // Cbar = Y5 + Q1k Q1k^T (Bbar - Y5)   (kept in Y5)
  GN_TRY(launch_dgemm(r, r, rl, 1.0, Q1t, sq(Bb), 0.0, T4, r, 1, kd, true, s, nullptr, 0, true, DS, DSB));
  GN_TRY(launch_dgemm(r, r, rl, -1.0, Q1t, sq(Y5), 1.0, T4, r, 1, kd, true, s, nullptr, 0, true, DS, DSB));
  GN_TRY(launch_dgemm(rl, r, r, 1.0, Q1r, sq(T4), 1.0, Y5, r, 1, nullptr, false, s, nullptr, 0, true, DS, DSB));

  // dA = G1 M^T X^T + Y (Cbar X^T + M^T G2): with U = G1 M^T and V = M^T G2 from the
  // side stream, Cbar X^T is added to V (an (r + l) x n product, against m x r for
  // adding Y Cbar to U), and dA = [U | Y] [X^T ; V]
  if (hipStreamWaitEvent(s, ss->join, 0) != hipSuccess) return GN_ERR_HIP;
  GN_TRY(launch_dgemm_to(rl, n, r, 1.0, sq(Y5), MatRef{rcat, sdt, n, 1}, 1.0,
                         rcat + (size_t)r * n * sd, sdt, n, 1, nullptr, false, s, nullptr, 0, true,
                         DS, DSB));
  if (f32)
    return launch_gemm_f32(m, n, K2, (const float*)lcat, K2, true, (const float*)rcat, n, false,
                           (float*)dA, ldda, s);
  return launch_dgemm(m, n, K2, 1.0, MatRef{lcat, F64, K2, 1}, MatRef{rcat, F64, n, 1}, 0.0,
                      (double*)dA, ldda, 1, nullptr, false, s, nullptr, 0, true, DS, DSB);
}

// ---- Section 6: resampling, appended rows / columns, A <- A + E
namespace {
gn_status upd_common(const Plan& P, bool allow_srht) {
  if (P.mode != GN_MODE_F64 && P.mode != GN_MODE_F32) return GN_ERR_UNSUPPORTED;
  if (P.ky != GN_SKETCH_GAUSSIAN) return GN_ERR_UNSUPPORTED;
  if (P.kx != GN_SKETCH_GAUSSIAN && !(allow_srht && P.kx == GN_SKETCH_SRHT))
    return GN_ERR_UNSUPPORTED;
  return GN_OK;
}
}  // namespace

gn_status gn_sketch_extend(const gn_problem* p_old, const gn_problem* p_new, const void* A,
                           int64_t lda, void* AX, int64_t ldax, void* YtA, int64_t ldya, void* ws,
                           size_t ws_bytes, gn_stream_t stream_) {
  Plan Po, Pn;
  GN_TRY(make_plan(p_old, Po));
  GN_TRY(make_plan(p_new, Pn));
  GN_TRY(upd_common(Pn, true));
  if (Po.mode != Pn.mode || Po.kx != Pn.kx || Po.ky != Pn.ky || p_old->seed != p_new->seed)
    return GN_ERR_ARG;
  if (!A || !AX || !YtA || !ws) return GN_ERR_ARG;
  if (Po.m != Pn.m || Po.n != Pn.n) return GN_ERR_SHAPE;
  const int64_t dr = Pn.r - Po.r, drl = Pn.rl - Po.rl;
  if (dr < 1 || drl < 1 || Pn.l < Po.l) return GN_ERR_SHAPE;
  if (lda < Pn.n || ldax < Pn.r || ldya < Pn.n) return GN_ERR_SHAPE;
  if (!aligned16(A) || !aligned16(ws)) return GN_ERR_ALIGN;
  const UpdWs W = upd_ws(Pn);
  if (ws_bytes < W.total) return GN_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream_;
  char* base = (char*)ws;
  const size_t ac = dtype_size(Pn.adt);
  // the new columns of X (or the enlarged SRHT sample) and of Y
  const int32_t* idx = nullptr;
  const int8_t* signs = nullptr;
  if (Pn.kx == GN_SKETCH_SRHT) {
    GN_TRY(launch_srht(p_new->seed, Pn.npad, Pn.r, (int8_t*)(base + W.signs),
                       (int32_t*)(base + W.idx), (uint64_t*)(base + W.keys), s));
    signs = (const int8_t*)(base + W.signs);
    idx = (const int32_t*)(base + W.idx) + Po.r;  // prefix-stable: the first r are the old sample
  } else {
    GN_TRY(launch_gaussian(p_new->seed, 1, 0, Po.r, Pn.n, dr, Pn.sdt, 0, base + W.xs, dr, s));
  }
  GN_TRY(launch_gaussian(p_new->seed, 2, 0, Po.rl, Pn.m, drl, Pn.sdt, 0, base + W.ys, drl, s));
  return launch_pass(Pn.mode, Pn.kx, Pn.m, Pn.n, dr, drl, A, lda, nullptr, base + W.xs, signs, idx,
                     base + W.ys, (char*)AX + Po.r * ac, ldax, (char*)YtA + Po.rl * ldya * ac, ldya,
                     s, base + W.split, W.split_bytes);
}

gn_status gn_sketch_append(const gn_problem* p, int32_t axis, int64_t old_size, const void* B,
                           int64_t ldb, void* AX, int64_t ldax, void* YtA, int64_t ldya, void* ws,
                           size_t ws_bytes, gn_stream_t stream_) {
  Plan P;
  GN_TRY(make_plan(p, P));
  if (axis != 0 && axis != 1) return GN_ERR_ARG;
  GN_TRY(upd_common(P, axis == 0));
  if (!B || !AX || !YtA || !ws) return GN_ERR_ARG;
  const int64_t full = (axis == 0) ? P.m : P.n;
  if (old_size < P.r || old_size >= full) return GN_ERR_SHAPE;
  const int64_t add = full - old_size;
  if (ldb < ((axis == 0) ? P.n : add) || ldax < P.r || ldya < P.n) return GN_ERR_SHAPE;
  if (!aligned16(B) || !aligned16(ws)) return GN_ERR_ALIGN;
  const UpdWs W = upd_ws(P);
  if (ws_bytes < W.total) return GN_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream_;
  char* base = (char*)ws;
  const size_t ac = dtype_size(P.adt);
  if (axis == 0) {
    // A -> [A; B]: X as before, Y_B = rows old_size.. of Y; AX gains B X, Y^T A += Y_B^T B
    const int32_t* idx = nullptr;
    const int8_t* signs = nullptr;
    if (P.kx == GN_SKETCH_SRHT) {
      GN_TRY(launch_srht(p->seed, P.npad, P.r, (int8_t*)(base + W.signs), (int32_t*)(base + W.idx),
                         (uint64_t*)(base + W.keys), s));
      signs = (const int8_t*)(base + W.signs);
      idx = (const int32_t*)(base + W.idx);
    } else {
      GN_TRY(launch_gaussian(p->seed, 1, 0, 0, P.n, P.r, P.sdt, 0, base + W.xs, P.r, s));
    }
    GN_TRY(launch_gaussian(p->seed, 2, old_size, 0, add, P.rl, P.sdt, 0, base + W.ys, P.rl, s));
    GN_TRY(launch_pass(P.mode, P.kx, add, P.n, P.r, P.rl, B, ldb, nullptr, base + W.xs, signs, idx,
                       base + W.ys, (char*)AX + old_size * ldax * ac, ldax, base + W.tya, P.n, s,
                       base + W.split, W.split_bytes));
    return launch_add(P.rl, P.n, P.adt, base + W.tya, P.n, YtA, ldya, s);
  }
  // A -> [A, B]: X_B = rows old_size.. of X, Y as before; AX += B X_B, Y^T A gains Y^T B
  GN_TRY(launch_gaussian(p->seed, 1, old_size, 0, add, P.r, P.sdt, 0, base + W.xs, P.r, s));
  GN_TRY(launch_gaussian(p->seed, 2, 0, 0, P.m, P.rl, P.sdt, 0, base + W.ys, P.rl, s));
  GN_TRY(launch_pass(P.mode, P.kx, P.m, add, P.r, P.rl, B, ldb, nullptr, base + W.xs, nullptr,
                     nullptr, base + W.ys, base + W.tax, P.r, (char*)YtA + old_size * ac, ldya, s,
                     base + W.split, W.split_bytes));
  return launch_add(P.m, P.r, P.adt, base + W.tax, P.r, AX, ldax, s);
}

gn_status gn_sketch_update(const gn_problem* p, const void* E, int64_t lde, void* AX, int64_t ldax,
                           void* YtA, int64_t ldya, void* ws, size_t ws_bytes,
                           gn_stream_t stream_) {
  Plan P;
  GN_TRY(make_plan(p, P));
  GN_TRY(upd_common(P, true));
  if (!E || !AX || !YtA || !ws) return GN_ERR_ARG;
  if (lde < P.n || ldax < P.r || ldya < P.n) return GN_ERR_SHAPE;
  if (!aligned16(E) || !aligned16(ws)) return GN_ERR_ALIGN;
  const UpdWs W = upd_ws(P);
  if (ws_bytes < W.total) return GN_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream_;
  char* base = (char*)ws;
  const int32_t* idx = nullptr;
  const int8_t* signs = nullptr;
  if (P.kx == GN_SKETCH_SRHT) {
    GN_TRY(launch_srht(p->seed, P.npad, P.r, (int8_t*)(base + W.signs), (int32_t*)(base + W.idx),
                       (uint64_t*)(base + W.keys), s));
    signs = (const int8_t*)(base + W.signs);
    idx = (const int32_t*)(base + W.idx);
  } else {
    GN_TRY(launch_gaussian(p->seed, 1, 0, 0, P.n, P.r, P.sdt, 0, base + W.xs, P.r, s));
  }
  GN_TRY(launch_gaussian(p->seed, 2, 0, 0, P.m, P.rl, P.sdt, 0, base + W.ys, P.rl, s));
  GN_TRY(launch_pass(P.mode, P.kx, P.m, P.n, P.r, P.rl, E, lde, nullptr, base + W.xs, signs, idx,
                     base + W.ys, base + W.tax, P.r, base + W.tya, P.n, s, base + W.split,
                     W.split_bytes));
  GN_TRY(launch_add(P.m, P.r, P.adt, base + W.tax, P.r, AX, ldax, s));
  return launch_add(P.rl, P.n, P.adt, base + W.tya, P.n, YtA, ldya, s);
}

gn_status gn_residual(int64_t m, int64_t n, int64_t k, const void* A, int64_t lda, int32_t a_dtype,
                      const float* A_scales, const double* F, int64_t ldf, const double* G,
                      int64_t ldg, double* out_sumsq, void* ws, size_t ws_bytes,
                      gn_stream_t stream_) {
  if (!A || !F || !G || !out_sumsq || !ws) return GN_ERR_ARG;
  if (a_dtype < GN_DT_F64 || a_dtype > GN_DT_F16) return GN_ERR_ARG;
  if ((a_dtype == GN_DT_BF16 || a_dtype == GN_DT_F16) && !A_scales) return GN_ERR_ARG;
  if (m < 1 || n < 1 || k < 0 || lda < n || ldf < k || ldg < n) return GN_ERR_SHAPE;
  if (ws_bytes < residual_ws_bytes(m, n)) return GN_ERR_WORKSPACE;
  if (((uintptr_t)ws & 7u) != 0) return GN_ERR_ALIGN;
  return launch_residual(m, n, k, MatRef{A, a_dtype, lda, 1}, A_scales, MatRef{F, GN_DT_F64, ldf, 1},
                         MatRef{G, GN_DT_F64, ldg, 1}, (double*)ws, out_sumsq,
                         (hipStream_t)stream_);
}

gn_status gn_quantize_bf16_bs(int64_t m, int64_t n, const void* A, int64_t lda, int32_t a_dtype,
                              uint16_t* out, int64_t ldo, float* scales, gn_stream_t stream) {
  if (!A || !out || !scales) return GN_ERR_ARG;
  if (a_dtype != GN_DT_F64 && a_dtype != GN_DT_F32) return GN_ERR_DTYPE;
  if (m < 1 || n < 1 || lda < n || ldo < n) return GN_ERR_SHAPE;
  return launch_quantize(m, n, A, lda, a_dtype, out, ldo, scales, (hipStream_t)stream, false);
}

gn_status gn_quantize_f16_bs(int64_t m, int64_t n, const void* A, int64_t lda, int32_t a_dtype,
                             uint16_t* out, int64_t ldo, float* scales, gn_stream_t stream) {
  if (!A || !out || !scales) return GN_ERR_ARG;
  if (a_dtype != GN_DT_F64 && a_dtype != GN_DT_F32) return GN_ERR_DTYPE;
  if (m < 1 || n < 1 || lda < n || ldo < n) return GN_ERR_SHAPE;
  return launch_quantize(m, n, A, lda, a_dtype, out, ldo, scales, (hipStream_t)stream, true);
}

}  // extern "C"
