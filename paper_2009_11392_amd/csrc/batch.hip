// Batches of independent GN problems of uneven m, n, r (FP32 mode, Gaussian X and
// Y): Algorithm 2.1 steps 2-3 and the Section 5.1.1 truncation for every problem
// of a batch in a fixed, small number of launches.
//
// The sketch passes of all problems are one launch over a table of work items
// (problem, product, tile configuration, tile), one workgroup per item.  Each item is one
// output tile of Y^T A or AX on the FP32 matrix cores with one of three
// tile shapes (256 threads: 64 x 256, 128 x 128, 256 x 64; 512 threads: 128 x 256,
// 256 x 128), chosen per product from the size of its
// narrow side by a tile policy that the autotuner can replace);
// items are ordered by decreasing cost, so the dispatcher starts the largest
// first and hands the small ones to whichever CU frees up (no static round-robin,
// and no loop whose hoisted per-thread offsets of every tile shape stay live: the
// kernel fits three waves per SIMD).  The core products C = Y^T (AX) are a second launch of
// the same kernel, and the FP64 Householder QR, truncation scan and second QR run
// batched over the problems (one grid dimension per problem).  Every table lives
// in the workspace, so a solve is replayable inside a HIP graph.
#include <algorithm>
#include <cmath>
#include <vector>

#include "gemm_tiles.h"
#include "gn_internal.h"

namespace gn {
namespace {

using namespace tiles;

// Tile configurations (output rows x columns per workgroup; every wave owns a
// 64 x 64 block of 2 x 2 v_mfma_f32_32x32x2_f32 tiles, K staged 16 deep):
// 0-2 with 256 threads, 3-4 with 512 threads.
using BC0 = F32Cfg<64, 256, 16, 1, 4, 32>;
using BC1 = F32Cfg<128, 128, 16, 2, 2, 32>;
using BC2 = F32Cfg<256, 64, 16, 4, 1, 32>;
using BC3 = F32Cfg<128, 256, 16, 2, 4, 32>;
using BC4 = F32Cfg<256, 128, 16, 4, 2, 32>;
constexpr int kNumCfg = 5;
constexpr int kTileBM[kNumCfg] = {BC0::BM, BC1::BM, BC2::BM, BC3::BM, BC4::BM};
constexpr int kTileBN[kNumCfg] = {BC0::BN, BC1::BN, BC2::BN, BC3::BN, BC4::BN};
constexpr int kCfgThreads[kNumCfg] = {BC0::T, BC1::T, BC2::T, BC3::T, BC4::T};
constexpr int kCoreCfg = 1;  // the core products Y^T (AX) (a 256-thread launch)

constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }
template <class CF>
constexpr size_t cfg_smem() {
  return cmax(CF::template smem<false, false>(), CF::template smem<true, false>());
}
constexpr size_t kSmem256 = cmax(cmax(cfg_smem<BC0>(), cfg_smem<BC1>()), cfg_smem<BC2>());
constexpr size_t kSmem512 = cmax(cfg_smem<BC3>(), cfg_smem<BC4>());

constexpr int kMaxCoreRows = 512;   // r + l: one QR row per thread

struct BatchDesc {
  int64_t m, n, r, rl;
  const float* A;
  int64_t lda;
  const float* X;  // n x r, row stride ldx
  int64_t ldx;
  const float* Y;  // m x rl, row stride ldy
  int64_t ldy;
  float* AX;
  int64_t ldax;
  float* YtA;
  int64_t ldya;
  float* Cf;       // Y^T (AX), rl x r, FP32
  double* C;       // the same widened, factored in place by the QR
};

// fam 0: Y^T A (rl x n, K = m); fam 1: AX (m x r, K = n); fam 2: Y^T (AX) (rl x r, K = m)
struct PassItem {
  int32_t prob, fam, cfg, tm, tn, pad0, pad1, pad2;
};

template <class CF>
__device__ __forceinline__ void batch_tile(const GemmF32& g, int fam, int tm, int tn, char* smem) {
  if (fam == 1)
    f32_tile_at<CF, true, false, true>(g, (int64_t)tm * CF::BM, (int64_t)tn * CF::BN, smem);
  else
    f32_tile_at<CF, false, false, true>(g, (int64_t)tm * CF::BM, (int64_t)tn * CF::BN, smem);
}

// One work item per workgroup (item blockIdx.x).  The 256-thread instantiation
// takes 69 VGPRs and 64 accumulation registers (three waves per SIMD, three
// workgroups of 4 waves per CU), the 512-thread one 118 VGPRs (two waves per SIMD).
template <int NT, size_t SMEM>
__global__ void __launch_bounds__(NT) batch_pass(const BatchDesc* __restrict__ probs,
                                                 const PassItem* __restrict__ items,
                                                 int64_t n_items) {
  __shared__ __attribute__((aligned(16))) char smem[SMEM];
  const int64_t it = blockIdx.x;
  if (it >= n_items) return;
  const PassItem w = items[it];
  const BatchDesc d = probs[w.prob];
  GemmF32 g;
  if (w.fam == 0)
    g = GemmF32{d.rl, d.n, d.m, d.Y, d.ldy, d.A, d.lda, d.YtA, d.ldya, 1};
  else if (w.fam == 1)
    g = GemmF32{d.m, d.r, d.n, d.A, d.lda, d.X, d.ldx, d.AX, d.ldax, 0};
  else
    g = GemmF32{d.rl, d.r, d.m, d.Y, d.ldy, d.AX, d.ldax, d.Cf, d.r, 1};
  if constexpr (NT == 256) {
    if (w.cfg == 0)
      batch_tile<BC0>(g, w.fam, w.tm, w.tn, smem);
    else if (w.cfg == 1)
      batch_tile<BC1>(g, w.fam, w.tm, w.tn, smem);
    else
      batch_tile<BC2>(g, w.fam, w.tm, w.tn, smem);
  } else {
    if (w.cfg == 3)
      batch_tile<BC3>(g, w.fam, w.tm, w.tn, smem);
    else
      batch_tile<BC4>(g, w.fam, w.tm, w.tn, smem);
  }
}

// C = (double) Cf for every problem (job blockIdx.z).
__global__ void __launch_bounds__(256) batch_widen(const BatchDesc* __restrict__ probs) {
  const BatchDesc d = probs[blockIdx.z];
  const int64_t total = d.rl * d.r;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x)
    d.C[e] = (double)d.Cf[e];
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }
int64_t round4(int64_t x) { return (x + 3) / 4 * 4; }

struct Layout {
  // tables
  size_t desc, items, qr1, qr2, trunc, gauss, tables_end;
  // per-problem scratch, offsets of problem p at per[p]
  std::vector<size_t> x, y, cf, c, t1, wp1, z, t2, wp2;
  size_t total;
  int64_t n_pass, n_core;
};

int default_cfg(int slot) {
  static const int d[4] = {0, 1, 2, 1};
  return d[slot];
}

gn_status validate(const gn_batch_problem* probs, int32_t count) {
  if (!probs || count < 1) return GN_ERR_ARG;
  for (int32_t p = 0; p < count; ++p) {
    const gn_batch_problem& b = probs[p];
    if (!b.A || !b.AX || !b.YtA || !b.core.k || !b.core.status || !b.core.Q1 || !b.core.R ||
        !b.core.Q2 || !b.core.R2)
      return GN_ERR_ARG;
    if (!std::isfinite(b.eps)) return GN_ERR_ARG;
    if (b.m < 1 || b.n < 1 || b.r < 1 || b.r > b.m || b.r > b.n) return GN_ERR_SHAPE;
    const int64_t l = b.l < 0 ? (b.r + 1) / 2 : b.l;
    if (b.r + l > kMaxCoreRows) return GN_ERR_UNSUPPORTED;
    if (b.m > INT32_MAX || b.n > INT32_MAX) return GN_ERR_UNSUPPORTED;
    if (b.lda < b.n || b.ldax < b.r || b.ldya < b.n) return GN_ERR_SHAPE;
    if (b.lda % 4 != 0 || b.ldax % 4 != 0) return GN_ERR_ALIGN;
    if (!aligned16(b.A) || !aligned16(b.AX) || !aligned16(b.YtA)) return GN_ERR_ALIGN;
  }
  return GN_OK;
}

// Work items of one product: (rows x cols) output in tiles of configuration cfg.
void add_items(std::vector<PassItem>& v, std::vector<double>& cost, int32_t prob, int32_t fam,
               int32_t cfg, int64_t rows, int64_t cols, int64_t K) {
  const int64_t tm_n = cdiv(rows, kTileBM[cfg]), tn_n = cdiv(cols, kTileBN[cfg]);
  for (int64_t tm = 0; tm < tm_n; ++tm)
    for (int64_t tn = 0; tn < tn_n; ++tn) {
      v.push_back(PassItem{prob, fam, cfg, (int32_t)tm, (int32_t)tn, 0, 0, 0});
      cost.push_back((double)K * kTileBM[cfg] * kTileBN[cfg]);
    }
}

// Items of all problems in decreasing cost (ties by position), pass then core.
void build_items(const gn_batch_problem* probs, int32_t count, const int32_t* policy,
                 std::vector<PassItem>& items, int64_t& n_pass, int64_t& n_core) {
  std::vector<PassItem> pass, core;
  std::vector<double> cp, cc;
  for (int32_t p = 0; p < count; ++p) {
    const gn_batch_problem& b = probs[p];
    const int64_t l = b.l < 0 ? (b.r + 1) / 2 : b.l, rl = b.r + l;
    add_items(pass, cp, p, 0, policy[rl <= 64 ? 0 : 1], rl, b.n, b.m);
    add_items(pass, cp, p, 1, policy[b.r <= 64 ? 2 : 3], b.m, b.r, b.n);
    add_items(core, cc, p, 2, kCoreCfg, rl, b.r, b.m);
  }
  auto order = [](const std::vector<PassItem>& v, const std::vector<double>& c) {
    std::vector<size_t> idx(v.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return c[a] > c[b]; });
    std::vector<PassItem> out;
    out.reserve(v.size());
    for (size_t i : idx) out.push_back(v[i]);
    return out;
  };
  items = order(pass, cp);
  const std::vector<PassItem> co = order(core, cc);
  n_pass = (int64_t)items.size();
  n_core = (int64_t)co.size();
  items.insert(items.end(), co.begin(), co.end());
}

// Upper bound of the item count over every tile policy (the layout must not
// depend on the policy).
int64_t max_items(const gn_batch_problem* probs, int32_t count) {
  int64_t total = 0;
  for (int32_t p = 0; p < count; ++p) {
    const gn_batch_problem& b = probs[p];
    const int64_t l = b.l < 0 ? (b.r + 1) / 2 : b.l, rl = b.r + l;
    int64_t t0 = 0, t1 = 0;
    for (int c = 0; c < kNumCfg; ++c) {
      t0 = std::max(t0, cdiv(rl, kTileBM[c]) * cdiv(b.n, kTileBN[c]));
      t1 = std::max(t1, cdiv(b.m, kTileBM[c]) * cdiv(b.r, kTileBN[c]));
    }
    total += t0 + t1 + cdiv(rl, kTileBM[kCoreCfg]) * cdiv(b.r, kTileBN[kCoreCfg]);
  }
  return total;
}

Layout layout(const gn_batch_problem* probs, int32_t count) {
  const int64_t n_items = max_items(probs, count);
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  L.desc = take((size_t)count * sizeof(BatchDesc));
  L.items = take((size_t)n_items * sizeof(PassItem));
  L.qr1 = take((size_t)count * sizeof(QrJob));
  L.qr2 = take((size_t)count * sizeof(QrJob));
  L.trunc = take((size_t)count * sizeof(TruncJob));
  L.gauss = take((size_t)2 * count * sizeof(GaussJob));
  L.tables_end = off;
  for (int32_t p = 0; p < count; ++p) {
    const gn_batch_problem& b = probs[p];
    const int64_t l = b.l < 0 ? (b.r + 1) / 2 : b.l, rl = b.r + l;
    L.x.push_back(take((size_t)b.n * round4(b.r) * 4));
    L.y.push_back(take((size_t)b.m * round4(rl) * 4));
    L.cf.push_back(take((size_t)rl * b.r * 4));
    L.c.push_back(take((size_t)rl * b.r * 8));
    L.t1.push_back(take(qr_batch_t_bytes(b.r)));
    L.wp1.push_back(take(qr_batch_wp_bytes(rl, b.r)));
    L.z.push_back(take((size_t)b.r * b.r * 8));
    L.t2.push_back(take(qr_batch_t_bytes(b.r)));
    L.wp2.push_back(take(qr_batch_wp_bytes(b.r, b.r)));
  }
  L.total = off;
  return L;
}

}  // namespace
}  // namespace gn

using namespace gn;

extern "C" {

gn_status gn_batch_workspace_size(const gn_batch_problem* probs, int32_t count, size_t* bytes) {
  if (!bytes) return GN_ERR_ARG;
  GN_TRY(validate(probs, count));
  *bytes = layout(probs, count).total;
  return GN_OK;
}

gn_status gn_batch_prepare(const gn_batch_problem* probs, int32_t count, const int32_t* tile_policy,
                           gn_batch_plan* plan, void* ws, size_t ws_bytes, gn_stream_t stream_) {
  if (!plan || !ws) return GN_ERR_ARG;
  GN_TRY(validate(probs, count));
  if (!aligned16(ws)) return GN_ERR_ALIGN;
  int32_t pol[4];
  for (int i = 0; i < 4; ++i) {
    pol[i] = tile_policy ? tile_policy[i] : default_cfg(i);
    if (pol[i] < 0 || pol[i] >= kNumCfg) return GN_ERR_ARG;
  }
  for (int i = 1; i < 4; ++i)  // one launch, one workgroup size
    if (kCfgThreads[pol[i]] != kCfgThreads[pol[0]]) return GN_ERR_ARG;
  std::vector<PassItem> items;
  int64_t n_pass, n_core;
  build_items(probs, count, pol, items, n_pass, n_core);
  const Layout L = layout(probs, count);
  if (ws_bytes < L.total) return GN_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream_;
  char* base = (char*)ws;

  std::vector<BatchDesc> desc(count);
  std::vector<QrJob> qr1(count), qr2(count);
  std::vector<TruncJob> tj(count);
  std::vector<GaussJob> gj(2 * count);
  gn_batch_plan P{};
  P.count = count;
  P.n_pass_items = (int32_t)n_pass;
  P.n_core_items = (int32_t)n_core;
  for (int32_t p = 0; p < count; ++p) {
    const gn_batch_problem& b = probs[p];
    const int64_t l = b.l < 0 ? (b.r + 1) / 2 : b.l, rl = b.r + l;
    const int64_t ldx = round4(b.r), ldy = round4(rl);
    float* X = (float*)(base + L.x[p]);
    float* Y = (float*)(base + L.y[p]);
    float* Cf = (float*)(base + L.cf[p]);
    double* C = (double*)(base + L.c[p]);
    double* Z = (double*)(base + L.z[p]);
    desc[p] = BatchDesc{b.m, b.n, b.r, rl, (const float*)b.A, b.lda, X, ldx, Y, ldy,
                        (float*)b.AX, b.ldax, (float*)b.YtA, b.ldya, Cf, C};
    qr1[p] = QrJob{rl, b.r, C, b.r, b.core.Q1, b.r, b.core.R, b.r,
                   (double*)(base + L.t1[p]), (double*)(base + L.wp1[p]), nullptr, 0};
    qr2[p] = QrJob{b.r, b.r, Z, b.r, b.core.Q2, b.r, b.core.R2, b.r,
                   (double*)(base + L.t2[p]), (double*)(base + L.wp2[p]), b.core.k, b.r};
    const double nux = std::sqrt((double)b.n) + std::sqrt((double)b.r);
    const double nuy = std::sqrt((double)b.m) + std::sqrt((double)rl);
    const double tau = (b.eps > 0.0) ? b.eps * nux * nuy : 0.0;
    tj[p] = TruncJob{b.r, b.core.R, b.r, tau, b.core.k, b.core.status, Z, b.r};
    gj[2 * p] = GaussJob{b.seed, 1, b.n, b.r, X, ldx};
    gj[2 * p + 1] = GaussJob{b.seed, 2, b.m, rl, Y, ldy};
    P.max_m = std::max(P.max_m, b.m);
    P.max_n = std::max(P.max_n, b.n);
    P.max_r = std::max(P.max_r, b.r);
    P.max_rl = std::max(P.max_rl, rl);
    P.pass_flops += 2.0 * b.m * b.n * (double)(rl + b.r);
    P.pass_bytes += 4.0 * ((double)b.m * b.n + (double)b.m * rl + (double)b.n * b.r +
                           (double)b.m * b.r + (double)rl * b.n);
  }
  P.pass_threads = kCfgThreads[pol[0]];
  P.grid = (int32_t)std::max<int64_t>(n_pass, 1);
  P.ws_bytes = L.total;
  P.off_desc = L.desc;
  P.off_items = L.items;
  P.off_qr = L.qr1;
  P.off_qr2 = L.qr2;
  P.off_trunc = L.trunc;
  P.off_widen = L.desc;
  for (int i = 0; i < 4; ++i) P.tile_policy[i] = pol[i];

  auto up = [&](size_t off, const void* src, size_t bytes) {
    return hipMemcpyAsync(base + off, src, bytes, hipMemcpyHostToDevice, s) == hipSuccess;
  };
  if (!up(L.desc, desc.data(), desc.size() * sizeof(BatchDesc)) ||
      !up(L.items, items.data(), items.size() * sizeof(PassItem)) ||
      !up(L.qr1, qr1.data(), qr1.size() * sizeof(QrJob)) ||
      !up(L.qr2, qr2.data(), qr2.size() * sizeof(QrJob)) ||
      !up(L.trunc, tj.data(), tj.size() * sizeof(TruncJob)) ||
      !up(L.gauss, gj.data(), gj.size() * sizeof(GaussJob)))
    return GN_ERR_HIP;
  GN_TRY(launch_gaussian_batched((const GaussJob*)(base + L.gauss), 2 * count, GN_DT_F32, s));
  if (hipStreamSynchronize(s) != hipSuccess) return GN_ERR_HIP;
  *plan = P;
  return GN_OK;
}

gn_status gn_batch_solve(const gn_batch_plan* plan, int32_t stages, void* ws, size_t ws_bytes,
                         gn_stream_t stream_) {
  if (!plan || !ws) return GN_ERR_ARG;
  if (stages < 1 || stages > GN_BATCH_ALL) return GN_ERR_ARG;
  if (plan->count < 1) return GN_ERR_ARG;
  if (ws_bytes < plan->ws_bytes) return GN_ERR_WORKSPACE;
  if (plan->max_rl > kMaxCoreRows) return GN_ERR_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream_;
  char* base = (char*)ws;
  const BatchDesc* desc = (const BatchDesc*)(base + plan->off_desc);
  const PassItem* items = (const PassItem*)(base + plan->off_items);
  const unsigned z = (unsigned)plan->count;
  // sketch passes, then the core products (which read AX)
  if (stages & GN_BATCH_PASS) {
    if (plan->pass_threads == 256)
      batch_pass<256, kSmem256><<<dim3((unsigned)plan->grid), dim3(256), 0, s>>>(
          desc, items, plan->n_pass_items);
    else if (plan->pass_threads == 512)
      batch_pass<512, kSmem512><<<dim3((unsigned)plan->grid), dim3(512), 0, s>>>(
          desc, items, plan->n_pass_items);
    else
      return GN_ERR_ARG;
    GN_LAUNCH_CHECK();
  }
  if (!(stages & GN_BATCH_CORE)) return GN_OK;
  const int64_t gcore = std::max<int64_t>(plan->n_core_items, 1);
  batch_pass<256, kSmem256><<<dim3((unsigned)gcore), dim3(256), 0, s>>>(desc, items + plan->n_pass_items,
                                                         plan->n_core_items);
  GN_LAUNCH_CHECK();
  batch_widen<<<dim3(16, 1, z), dim3(256), 0, s>>>(desc);
  GN_LAUNCH_CHECK();
  // FP64 core of every problem: QR, kept rank, second QR when truncated
  GN_TRY(launch_qr_batched((const QrJob*)(base + plan->off_qr), plan->count, plan->max_rl,
                           plan->max_r, s));
  GN_TRY(launch_truncate_batched((const TruncJob*)(base + plan->off_trunc), plan->count,
                                 plan->max_r, s));
  return launch_qr_batched((const QrJob*)(base + plan->off_qr2), plan->count, plan->max_r,
                           plan->max_r, s);
}

}  // extern "C"
