// gn_residual_noalloc: the tile-wise residual ||A - F G||_F^2 of gn_residual for
// callers that cannot allocate device memory (code under stream capture, serving
// loops): the per-tile partial sums go to a fixed device array compiled into the
// library instead of a caller-provided workspace.
//
// The array lives in the library's code object, one copy per GPU, from the
// moment the library is loaded on that GPU until the process ends.  Its device
// address is looked up once per device (with that device current) and kept; the
// kernels only ever receive that address.  Every residual tile writes its own
// partial before the reduction reads it, so nothing has to be cleared between
// calls.  Calls that overlap in time on one GPU share the array and race.
#include <mutex>

#include "gn_internal.h"

using namespace gn;

namespace {

// 2 MiB: one double per 64 x 64 tile, 262144 tiles (m n <= 2^30 elements, e.g.
// 32768 x 32768).
constexpr size_t kScratchBytes = size_t(2) << 20;
constexpr int64_t kScratchDoubles = (int64_t)(kScratchBytes / sizeof(double));
constexpr int kMaxScratchDevices = 64;

static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxScratchDevices] = {};

// The device address of `scratch` on the current device (looked up on the
// first call on that device, with the device current).
gn_status scratch_address(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return GN_ERR_HIP;
  if (dev < 0 || dev >= kMaxScratchDevices) return GN_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GN_ERR_HIP;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return GN_OK;
}

}  // namespace

extern "C" {

gn_status gn_residual_noalloc(int64_t m, int64_t n, int64_t k, const void* A, int64_t lda,
                              int32_t a_dtype, const float* A_scales, const double* F, int64_t ldf,
                              const double* G, int64_t ldg, double* out_sumsq,
                              gn_stream_t stream) {
  if (!A || !F || !G || !out_sumsq) return GN_ERR_ARG;
  if (a_dtype < GN_DT_F64 || a_dtype > GN_DT_F16) return GN_ERR_ARG;
  if ((a_dtype == GN_DT_BF16 || a_dtype == GN_DT_F16) && !A_scales) return GN_ERR_ARG;
  if (m < 1 || n < 1 || k < 0 || lda < n || ldf < k || ldg < n) return GN_ERR_SHAPE;
  if (residual_ws_bytes(m, n) > kScratchBytes) return GN_ERR_UNSUPPORTED;
  double* partial = nullptr;
  GN_TRY(scratch_address(&partial));
  return launch_residual(m, n, k, MatRef{A, a_dtype, lda, 1}, A_scales,
                         MatRef{F, GN_DT_F64, ldf, 1}, MatRef{G, GN_DT_F64, ldg, 1}, partial,
                         out_sumsq, (hipStream_t)stream);
}

}  // extern "C"
