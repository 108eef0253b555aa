// Allocation-free rounding: tt_round with its workspace taken from a
// library-owned static device array instead of the context's arena.
//
// The array is a file-scope __device__ object, so each GPU that loads the
// library holds its own copy until the process ends.  Its device address is
// looked up once per device (hipGetSymbolAddress, with that device current)
// when a context is created there; host code only ever passes that looked-up
// address to kernels, never the array's name.
#include <mutex>

#include "kernels.h"
#include "round.h"

namespace qt {

constexpr int QT_MAX_DEVICES = 64;

static __device__ __align__(256) char scratch[QT_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[QT_MAX_DEVICES] = {};

// Looks up this device's copy of the scratch array (the device must be
// current).  Called by qt_ctx_create; later calls for the same device return
// the stored address.
qt_status noalloc_attach(int device) {
  QT_CHECK(device >= 0 && device < QT_MAX_DEVICES, QT_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return QT_OK;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr) {
    set_error(hip_msg(e, "hipGetSymbolAddress(noalloc scratch)"));
    return QT_EHIP;
  }
  g_scratch_ptr[device] = p;
  return QT_OK;
}

static void* noalloc_ptr(int device) {
  if (device < 0 || device >= QT_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace qt

using namespace qt;

extern "C" qt_status tt_round_noalloc(qt_ctx ctx, qt_tt* x, const qt_round_opts* opts,
                                      double* err_out, double* norm_out) {
  QT_CHECK(ctx && x && opts, QT_EINVAL, "tt_round_noalloc: null argument");
  qt::enter(ctx);
  QT_TRY(qt::tt_validate(x, "x"));
  QT_CHECK(opts->eps >= 0.0, QT_EINVAL, "tt_round_noalloc: eps < 0");
  QT_CHECK(opts->mode == QT_ROUND_SVD, QT_EINVAL,
           "tt_round_noalloc: only QT_ROUND_SVD applies to a materialized train");
  QT_CHECK(opts->precision == QT_PREC_F64, QT_EINVAL,
           "tt_round_noalloc: QT_PREC_F32 applies to the product-aware roundings only");
  void* base = noalloc_ptr(ctx->device);
  QT_CHECK(base, QT_EINVAL, "tt_round_noalloc: no scratch attached for the context's device");
  const int lmax_cap = opts->max_rank > 0 ? opts->max_rank : (1 << 30);
  const qt::RoundWs w = qt::round_ws_layout(x, lmax_cap);
  QT_CHECK(w.max_nb <= 1024, QT_ECAPACITY, "tt_round_noalloc: SVD block above 1024 columns");
  if (w.bytes > (size_t)QT_NOALLOC_SCRATCH_BYTES) {
    char msg[160];
    snprintf(msg, sizeof(msg),
             "tt_round_noalloc: needs %zu bytes of scratch, above the fixed %zu (use tt_round)",
             w.bytes, (size_t)QT_NOALLOC_SCRATCH_BYTES);
    qt::set_error(msg);
    return QT_ECAPACITY;
  }
  // the rounding carves its buffers from the static array; nothing in it may
  // allocate: no tile-shape timing (it would allocate its output), no
  // profiling events
  char* ws = ctx->ws;
  const size_t ws_size = ctx->ws_size, ws_top = ctx->ws_top;
  ctx->ws = (char*)base;
  ctx->ws_size = (size_t)QT_NOALLOC_SCRATCH_BYTES;
  ctx->ws_top = 0;
  qt::g_prof = nullptr;
  qt::g_no_alloc = true;
  const qt_status st = qt::round_impl(ctx, x, opts, err_out, norm_out, false, nullptr, 0, 0);
  qt::g_no_alloc = false;
  ctx->ws = ws;
  ctx->ws_size = ws_size;
  ctx->ws_top = ws_top;
  return st;
}
