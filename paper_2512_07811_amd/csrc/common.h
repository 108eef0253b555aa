// Shared definitions of the qtthom HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <array>
#include <map>
#include <vector>

#include "../../include/qtthom.h"

#define QT_MAX_CORES 64

namespace qt {

typedef double2 cplx;

__host__ __device__ inline cplx cmul(cplx a, cplx b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__host__ __device__ inline cplx cmulc(cplx a, cplx b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline cplx cadd(cplx a, cplx b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline cplx csub(cplx a, cplx b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline cplx cscale(cplx a, double s) { return make_double2(a.x * s, a.y * s); }
__host__ __device__ inline cplx cconj(cplx a) { return make_double2(a.x, -a.y); }
__host__ __device__ inline double cabs2(cplx a) { return a.x * a.x + a.y * a.y; }
__device__ inline cplx czero() { return make_double2(0.0, 0.0); }
// c += a * b
__device__ inline void cfma(cplx& c, cplx a, cplx b) {
  c.x = fma(a.x, b.x, c.x);
  c.x = fma(-a.y, b.y, c.x);
  c.y = fma(a.x, b.y, c.y);
  c.y = fma(a.y, b.x, c.y);
}

// A size read from device memory: value = mul * p[b * stride] + cst
// (cst alone when p is null).  b is the instance index of a batch.
struct Dim {
  const int32_t* p;
  int32_t stride;
  int32_t mul;
  int32_t cst;
};
__device__ inline int dimv(const Dim& d, int b) {
  return (d.p ? d.mul * d.p[(int64_t)b * d.stride] : 0) + d.cst;
}
inline Dim dconst(int v) { return Dim{nullptr, 0, 0, v}; }
inline Dim dref(const int32_t* p, int stride, int mul = 1) { return Dim{p, stride, mul, 0}; }

// 64-bit strides that may depend on one device rank: value = mul * p[b*stride] + cst.
struct Str {
  const int32_t* p;
  int32_t stride;
  int64_t mul;
  int64_t cst;
};
__device__ inline int64_t strv(const Str& s, int b) {
  return (s.p ? s.mul * (int64_t)s.p[(int64_t)b * s.stride] : 0) + s.cst;
}
inline Str sconst(int64_t v) { return Str{nullptr, 0, 0, v}; }
inline Str sref(const int32_t* p, int stride, int64_t mul = 1, int64_t cst = 0) {
  return Str{p, stride, mul, cst};
}

// A strided matrix operand: element (r, c) of batch item (b1, b2) of instance b at
// base + b*inst + b1*s1 + b2*s2 + r*rs + c*cs.
// Instance b of a batch reads base + (b / grp) * inst (grp > 1: several fields
// share one operator instance).
struct Mat {
  cplx* base;
  int64_t inst;
  Str off, s1, s2, rs, cs;
  int32_t grp;
};
inline Mat mat(const cplx* base, int64_t inst, Str rs, Str cs, Str s1 = Str{nullptr, 0, 0, 0},
               Str s2 = Str{nullptr, 0, 0, 0}, Str off = Str{nullptr, 0, 0, 0}) {
  return Mat{const_cast<cplx*>(base), inst, off, s1, s2, rs, cs, 1};
}
// The same for data of a (possibly per-instance) operator.
inline Mat mat_op(const qt_mpo* A, const cplx* base, Str rs, Str cs,
                  Str s1 = Str{nullptr, 0, 0, 0}, Str s2 = Str{nullptr, 0, 0, 0},
                  Str off = Str{nullptr, 0, 0, 0}) {
  Mat m = mat(base, A->inst_stride, rs, cs, s1, s2, off);
  m.grp = A->inst_group > 0 ? A->inst_group : 1;
  return m;
}

// Wave-level reductions (wave64).
__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ inline cplx wave_sum(cplx v) {
  v.x = wave_sum(v.x);
  v.y = wave_sum(v.y);
  return v;
}

// Reciprocal and reciprocal square root for the small serial kernels (QR
// reflectors, Jacobi rotations), whose steps are latency-bound: the hardware
// approximations v_rcp_f64 / v_rsq_f64 refined by two Newton steps each
// (error a few ulp, x > 0 finite), instead of the IEEE-rounded division and
// square-root sequences, which are several times longer.  The approximations
// do not cover the whole exponent range (a denormal argument comes back as
// infinity), so arguments outside [2^-960, 2^960] are scaled by an exact power
// of two first; that branch is taken only for numerically vanishing blocks
// (for instance the rounding of a Green-operator output that is zero in exact
// arithmetic).
__device__ inline double fast_rcp(double x) {
  double sc = 1.0;
  if (x < 0x1p-960) { x *= 0x1p+960; sc = 0x1p+960; }
  else if (x > 0x1p+960) { x *= 0x1p-960; sc = 0x1p-960; }
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r * sc;
}
__device__ inline double fast_rsq(double x) {
  double sc = 1.0;
  if (x < 0x1p-960) { x *= 0x1p+960; sc = 0x1p+480; }
  else if (x > 0x1p+960) { x *= 0x1p-960; sc = 0x1p-480; }
  double r = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  r = r * fma(-h * r, r, 1.5);
  r = r * fma(-h * r, r, 1.5);
  return r * sc;
}

// Sum over the 16 lanes of a DPP row; every lane of the row receives the same
// bits.  quad_perm [1,0,3,2] and [2,3,0,1] add within quads (lane i adds lane
// i^1, then i^2), row_half_mirror pairs quad 0 with 1 and 2 with 3, row_mirror
// pairs quad 0 with 3 and 1 with 2.  Each step adds two values that the partner
// lane adds in the other order, so by commutativity all 16 lanes round alike.
// (A rotate-based tree would associate differently per quad; lanes would then
// disagree in the last bit, which lets the sign of a cancelling difference,
// such as beta - alpha of a Jacobi pair with equal norms, differ between lanes.)
__device__ inline double row16_sum(double v) {
#define QT_DPP_STEP(ctrl)                                                           \
  {                                                                                 \
    int lo = __double2loint(v), hi = __double2hiint(v);                             \
    int l2 = __builtin_amdgcn_update_dpp(0, lo, ctrl, 0xF, 0xF, false);             \
    int h2 = __builtin_amdgcn_update_dpp(0, hi, ctrl, 0xF, 0xF, false);             \
    v += __hiloint2double(h2, l2);                                                  \
  }
  QT_DPP_STEP(0xB1)
  QT_DPP_STEP(0x4E)
  QT_DPP_STEP(0x141)
  QT_DPP_STEP(0x140)
#undef QT_DPP_STEP
  return v;
}
__device__ inline cplx row16_sum(cplx v) {
  v.x = row16_sum(v.x);
  v.y = row16_sum(v.y);
  return v;
}

// Householder reflector of a column x (head al = x_j, tail sum of squares
// sig2): beta = -e^{i arg al} ||x||, iu0 = 1 / (al - beta), t = 1 + |al| / ||x||,
// so that u = x / (al - beta) (u_j = 1) and H = I - t u u^H maps x to beta e_j.
// When ||x||^2 < 2^-900 the caller passes al and sig2 of the column scaled by
// sc = 2^600 (an exact power of two): squares and reciprocals of the unscaled
// values would leave the double range; u and t do not depend on the scale,
// beta and iu0 are returned for the unscaled column.
constexpr double QR_TINY = 0x1p-900, QR_SCALE = 0x1p+600;
__device__ inline void house_coef(cplx al, double sig2, double sc, double& t, cplx& beta,
                                  cplx& iu0) {
  // sc is 1 or QR_SCALE: its reciprocal without a division on the critical path
  const double isc = sc == 1.0 ? 1.0 : 1.0 / QR_SCALE;
  const double a2 = cabs2(al), x2 = a2 + sig2;
  if (x2 == 0.0) {
    t = 0.0; beta = cscale(al, isc); iu0 = make_double2(0.0, 0.0);
    return;
  }
  const double ixn = fast_rsq(x2), xn = x2 * ixn;
  double aa = 0.0;
  cplx ph = make_double2(1.0, 0.0);
  if (a2 > 0.0) {
    const double ia = fast_rsq(a2);
    aa = a2 * ia;
    ph = make_double2(al.x * ia, al.y * ia);
  }
  const cplx bs = make_double2(-ph.x * xn, -ph.y * xn);
  const cplx u0 = csub(al, bs);
  const double id = fast_rcp(cabs2(u0)) * sc;
  iu0 = make_double2(u0.x * id, -u0.y * id);
  beta = cscale(bs, isc);
  t = 1.0 + aa * ixn;
}

// Error reporting ---------------------------------------------------------
void set_error(const std::string& msg);
std::string hip_msg(hipError_t e, const char* what);

#define QT_HIP(call)                                  \
  do {                                                \
    hipError_t _e = (call);                           \
    if (_e != hipSuccess) {                           \
      ::qt::set_error(::qt::hip_msg(_e, #call));      \
      return QT_EHIP;                                 \
    }                                                 \
  } while (0)

#define QT_CHECK(cond, code, msg)                     \
  do {                                                \
    if (!(cond)) {                                    \
      ::qt::set_error(msg);                           \
      return code;                                    \
    }                                                 \
  } while (0)

#define QT_TRY(call)                                  \
  do {                                                \
    qt_status _s = (call);                            \
    if (_s < 0) return _s;                            \
  } while (0)

// Device status word bits (written by kernels, read by the host on sync).
enum : int32_t { ST_JACOBI_CAP = 1, ST_NONFINITE = 2 };
// The status word is followed (at byte 16) by QT_DIAG_N doubles of diagnostics
// written by the first kernel that raises ST_JACOBI_CAP: matrix order, squared
// Frobenius norm, largest |b_p^H b_q| / (||b_p|| ||b_q|| tol) of the last sweep,
// smallest rotated column norm^2 / Frobenius^2 of the last sweep, sweeps.
constexpr int QT_DIAG_N = 10;   // [0, 5): sweep cap, [5, 10): non-finite values
constexpr size_t QT_STATUS_BYTES = 16 + 8 * QT_DIAG_N;
__host__ __device__ inline double* status_diag(int32_t* status) {
  return (double*)((char*)status + 16);
}

// Device event counters (int64, indices below), read with qt_ctx_counters.
enum : int32_t { CNT_SVD_CALLS = 0, CNT_SVD_SWEEPS = 1, CNT_SKETCH_FAIL = 2, CNT_FALLBACK = 3,
                 CNT_GEMM_FLOPS = 4, CNT_GEMM_BYTES = 5, CNT_LEARNED = 6, CNT_N = 8 };

// Kernel classes that can be timed with events (qt_ctx_profile).
enum : int32_t { PROF_GEMM = 1, PROF_QR = 2, PROF_SVD = 4 };

// Live timing of one kernel class: event pairs recorded around its launches.
struct ProfSink {
  int cls = 0;
  hipStream_t stream = nullptr;
  std::vector<hipEvent_t> ev;   // start/stop pairs
  size_t used = 0;
  int depth = 0;                // open regions (nested ones add to the outer one)
  void begin();                 // record a start event (grows the pool)
  void end();                   // record the matching stop event
};
extern thread_local ProfSink* g_prof;
inline bool prof_on(int cls) { return g_prof && (g_prof->cls & cls); }
extern thread_local unsigned long long* g_counters;
// Split-K partial tiles of the structured GEMM (owned by the context).
struct SplitKBuf {
  cplx* p = nullptr;
  int64_t elems = 0;
};
extern thread_local SplitKBuf g_splitk;
constexpr int64_t QT_SPLITK_ELEMS = int64_t(1) << 22;   // 64 MiB of complex doubles

// Tile shapes of the structured GEMM (64 or 32 rows by 64 or 32 columns),
// chosen per call signature by timing each shape once (owned by the context).
// mode 0: always 64 x 64; 1: autotune; 2..5: always shape mode - 2.
struct GemmTuner {
  int mode = 1;
  std::map<std::array<int64_t, 10>, int> choice;
  cplx* scratch = nullptr;      // output of the timing launches
  int64_t scratch_elems = 0;
  qt_ctx owner = nullptr;       // caller-memory contexts time into their free arena
  hipEvent_t ev[8] = {};          // one pair per tile shape
};
extern thread_local GemmTuner* g_tuner;
// Set while an allocation-free entry point runs: the GEMM launcher then never
// times tile shapes (the timing would allocate its output buffer).
extern thread_local bool g_no_alloc;
// Set while the sketch contractions of a QT_PREC_F32 rounding are launched:
// the GEMM launcher then runs its FP32-MFMA variant.
extern thread_local bool g_gemm_f32;
struct GemmF32Scope {
  bool prev;
  explicit GemmF32Scope(bool on) : prev(g_gemm_f32) { g_gemm_f32 = on; }
  ~GemmF32Scope() { g_gemm_f32 = prev; }
};
qt_status noalloc_attach(int device);

struct LearnCtx;
}  // namespace qt

// Context: device, stream and a growable workspace arena.
struct qt_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_size = 0;
  size_t ws_top = 0;
  int32_t* status = nullptr;  // device status word
  unsigned long long* counters = nullptr;  // device [CNT_N] event counters
  qt::SplitKBuf splitk;                    // GEMM split-K partials
  qt::GemmTuner tuner;                     // GEMM tile shapes per call signature
  qt::ProfSink prof;
  qt::LearnCtx* learn = nullptr;   // learned-rank state (created on demand)
  // caller-owned device memory (qt_ctx_create_with_memory): the context's
  // fixed state at its head, the arena after it, persistent buffers (learned
  // state, logs) taken from its end; the library then never allocates
  bool ext = false;
  char* ext_lo = nullptr;        // first byte of the arena
  size_t ext_size = 0;           // arena + persistent bytes
  size_t ext_persist = 0;        // bytes taken from the end
  std::vector<std::array<size_t, 3>> ext_blocks;   // (offset, bytes, freed)
  int jacobi_default = 30;
  uint64_t sketch_counter = 0;  // distinct Gaussian streams across iterations
  uint64_t* dev_iter = nullptr;  // device copy of the iteration number (graph replays)
  bool capturing = false;        // a graph of one iteration is being captured
  hipStream_t cap_stream = nullptr;  // private stream for captures (default priority)
};

namespace qt {

// Workspace arena: a bump allocator reset at the start of each entry point.
// Growing the arena synchronizes the stream and reallocates.
struct Arena {
  qt_ctx ctx;
  size_t need = 0;
  explicit Arena(qt_ctx c) : ctx(c) { ctx->ws_top = 0; }
};
qt_status ws_reserve(qt_ctx ctx, size_t bytes);
void* ws_take(qt_ctx ctx, size_t bytes);
// Persistent device buffers of a context (learned state, logs): hipMalloc, or,
// with caller-owned memory, blocks taken from its end (QT_ENOMEM when the
// arena in use would be overrun).
qt_status ctx_dev_alloc(qt_ctx ctx, void** p, size_t bytes);
void ctx_dev_free(qt_ctx ctx, void* p);

// Host-side helpers for qt_tt metadata.
int64_t tt_slot_elems(const qt_tt* t, int k);
qt_status tt_validate(const qt_tt* t, const char* name);

}  // namespace qt
