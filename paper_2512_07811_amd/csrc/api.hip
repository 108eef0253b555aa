// Context, workspace, validation and the Algorithm 2 entry points
// (ls_iterate, homogenize) of the qtthom C ABI.
#include <algorithm>
#include <cstring>

#include "kernels.h"
#include "round.h"
#include "sketch.h"
#include "learned.h"

namespace qt {

static thread_local std::string g_last_error;
thread_local ProfSink* g_prof = nullptr;
thread_local unsigned long long* g_counters = nullptr;
thread_local SplitKBuf g_splitk;
thread_local GemmTuner* g_tuner = nullptr;
thread_local bool g_no_alloc = false;
thread_local bool g_gemm_f32 = false;

// Regions do not nest: work launched inside an open region (the finishing
// products of a large SVD, the products of a blocked QR) counts to that region.
void ProfSink::begin() {
  if (depth++ > 0) return;
  if (used + 2 > ev.size()) {
    for (int i = 0; i < 64; ++i) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      ev.push_back(e);
    }
  }
  hipEventRecord(ev[used], stream);
}

void ProfSink::end() {
  if (--depth > 0) return;
  if (used + 2 > ev.size()) return;
  hipEventRecord(ev[used + 1], stream);
  used += 2;
}

// Every public entry point binds the context's profiling sink and counters
// for the kernels it launches on this thread.
void enter(qt_ctx ctx) {
  if (!ctx) return;
  ctx->prof.stream = ctx->stream;
  g_prof = ctx->prof.cls ? &ctx->prof : nullptr;
  g_counters = ctx->counters;
  g_splitk = ctx->splitk;
  g_tuner = &ctx->tuner;
}

void set_error(const std::string& msg) { g_last_error = msg; }

std::string hip_msg(hipError_t e, const char* what) {
  return std::string(what) + ": " + hipGetErrorString(e);
}

qt_status ws_reserve(qt_ctx ctx, size_t bytes) {
  bytes = (bytes + 255) & ~(size_t)255;
  if (ctx->ws_top + bytes <= ctx->ws_size) return QT_OK;
  if (ctx->ext) {
    char msg[200];
    snprintf(msg, sizeof(msg),
             "caller-owned memory: the call needs %zu bytes of workspace, %zu are free "
             "(size the memory with qt_workspace_query / qt_ls_workspace_query)",
             ctx->ws_top + bytes, ctx->ws_size);
    set_error(msg);
    return QT_ENOMEM;
  }
  size_t want = std::max(ctx->ws_top + bytes, ctx->ws_size + ctx->ws_size / 2);
  // earlier work on the stream may still read the old arena
  QT_HIP(hipStreamSynchronize(ctx->stream));
  if (ctx->ws_top != 0) {
    // live allocations inside the current call would move: refuse
    set_error("workspace grew inside a call (internal sizing error)");
    return QT_ENOMEM;
  }
  if (ctx->ws) QT_HIP(hipFree(ctx->ws));
  ctx->ws = nullptr;
  ctx->ws_size = 0;
  hipError_t e = hipMalloc((void**)&ctx->ws, want);
  if (e != hipSuccess) {
    set_error(hip_msg(e, "hipMalloc(workspace)"));
    return QT_ENOMEM;
  }
  ctx->ws_size = want;
  return QT_OK;
}

qt_status ctx_dev_alloc(qt_ctx ctx, void** p, size_t bytes) {
  *p = nullptr;
  if (!ctx->ext) {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
      set_error(hip_msg(e, "hipMalloc(context buffer)"));
      return QT_ENOMEM;
    }
    return QT_OK;
  }
  bytes = (bytes + 255) & ~(size_t)255;
  // a freed block that is large enough is taken again (re-enabled logs of the
  // same capacity, learned state of the same shape)
  for (auto& b : ctx->ext_blocks)
    if (b[2] && b[1] >= bytes) {
      b[2] = 0;
      *p = ctx->ext_lo + b[0];
      return QT_OK;
    }
  if (ctx->ext_persist + bytes + ctx->ws_top > ctx->ext_size) {
    char msg[200];
    snprintf(msg, sizeof(msg),
             "caller-owned memory: %zu more bytes for persistent buffers, %zu are free", bytes,
             ctx->ext_size - ctx->ext_persist - ctx->ws_top);
    set_error(msg);
    return QT_ENOMEM;
  }
  ctx->ext_persist += bytes;
  const size_t off = ctx->ext_size - ctx->ext_persist;
  ctx->ext_blocks.push_back({off, bytes, 0});
  ctx->ws_size = off;
  *p = ctx->ext_lo + off;
  return QT_OK;
}

void ctx_dev_free(qt_ctx ctx, void* p) {
  if (!p) return;
  if (!ctx->ext) {
    hipFree(p);
    return;
  }
  const size_t off = (size_t)((char*)p - ctx->ext_lo);
  for (auto& b : ctx->ext_blocks)
    if (b[0] == off) b[2] = 1;
  // give back the freed blocks at the low end of the persistent region
  while (!ctx->ext_blocks.empty() && ctx->ext_blocks.back()[2]) {
    ctx->ext_persist -= ctx->ext_blocks.back()[1];
    ctx->ext_blocks.pop_back();
  }
  ctx->ws_size = ctx->ext_size - ctx->ext_persist;
}

void* ws_take(qt_ctx ctx, size_t bytes) {
  bytes = (bytes + 255) & ~(size_t)255;
  if (ctx->ws_top + bytes > ctx->ws_size) return nullptr;
  void* p = ctx->ws + ctx->ws_top;
  ctx->ws_top += bytes;
  return p;
}

int64_t tt_slot_elems(const qt_tt* t, int k) {
  return (int64_t)t->cap[k] * t->modes[k] * t->cap[k + 1];
}

qt_status tt_validate(const qt_tt* t, const char* name) {
  std::string nm(name);
  QT_CHECK(t->n >= 1 && t->n <= QT_MAX_CORES, QT_EINVAL, nm + ": core count out of range");
  QT_CHECK(t->batch >= 1, QT_EINVAL, nm + ": batch < 1");
  QT_CHECK(t->modes && t->cap && t->offsets && t->ranks && t->data, QT_EINVAL,
           nm + ": null pointer in descriptor");
  QT_CHECK(t->cap[0] == 1 && t->cap[t->n] == 1, QT_EINVAL, nm + ": boundary capacities must be 1");
  int64_t end = 0;
  for (int k = 0; k < t->n; ++k) {
    QT_CHECK(t->modes[k] >= 1, QT_EINVAL, nm + ": mode < 1");
    QT_CHECK(t->cap[k + 1] >= 1, QT_EINVAL, nm + ": capacity < 1");
    QT_CHECK(t->offsets[k] >= 0, QT_EINVAL, nm + ": negative offset");
    end = std::max(end, t->offsets[k] + tt_slot_elems(t, k));
  }
  QT_CHECK(t->batch == 1 || t->inst_stride >= end, QT_EINVAL, nm + ": instance stride too small");
  return QT_OK;
}

TTLayout make_layout(const std::vector<int32_t>& modes, const std::vector<int32_t>& cap) {
  TTLayout L;
  L.modes = modes;
  L.cap = cap;
  int64_t off = 0;
  for (size_t k = 0; k < modes.size(); ++k) {
    L.off.push_back(off);
    int64_t s = (int64_t)cap[k] * modes[k] * cap[k + 1];
    off += (s + 31) & ~(int64_t)31;
  }
  L.stride = off;
  return L;
}

__global__ void k_copy_ranks(int n1, int batch, const int32_t* src, int ss, int32_t* dst) {
  int b = blockIdx.x;
  if (b >= batch) return;
  for (int k = threadIdx.x; k < n1; k += blockDim.x) dst[(int64_t)b * n1 + k] = src[(int64_t)b * ss + k];
}

// Copy every core (actual ranks) of src into dst's slots; src may broadcast (batch 1).
static qt_status tt_copy(qt_ctx ctx, const qt_tt* src, qt_tt* dst) {
  const int n = dst->n, B = dst->batch;
  const int64_t sS = src->batch == 1 ? 0 : src->inst_stride;
  const int srs = src->batch == 1 ? 0 : n + 1;
  for (int k = 0; k < n; ++k) {
    int64_t cap = (int64_t)std::min(src->cap[k], dst->cap[k]) * src->modes[k] *
                  std::min(src->cap[k + 1], dst->cap[k + 1]);
    copy(ctx->stream, B, dref(src->ranks + k, srs, src->modes[k]), dref(src->ranks + k + 1, srs),
         cap, (const cplx*)src->data + src->offsets[k], sS, (cplx*)dst->data + dst->offsets[k],
         dst->inst_stride);
  }
  k_copy_ranks<<<B, 64, 0, ctx->stream>>>(n + 1, B, src->ranks, srs, dst->ranks);
  QT_HIP(hipGetLastError());
  return QT_OK;
}

static std::vector<int32_t> natural_caps(const std::vector<int32_t>& modes) {
  const int n = (int)modes.size();
  std::vector<int32_t> nat(n + 1, 1);
  for (int k = 1; k < n; ++k) {
    double left = 1, right = 1;
    for (int j = 0; j < k; ++j) left *= modes[j];
    for (int j = k; j < n; ++j) right *= modes[j];
    nat[k] = (int32_t)std::min(std::min(left, right), 1e9);
  }
  return nat;
}

static qt_status validate_ops(const qt_operands* ops, const qt_tt* e) {
  // kp (the scalar material train) is optional: without it the material acts
  // through the operator Kp on every path (elasticity: a Voigt operator)
  if (ops->kp.n > 0) QT_TRY(tt_validate(&ops->kp, "operands.kp"));
  QT_TRY(tt_validate(&ops->E, "operands.E"));
  QT_TRY(tt_validate(e, "e"));
  const int n = e->n;
  QT_CHECK(n == 3 * ops->L + 1, QT_EINVAL, "operands: n != 3L+1");
  QT_CHECK((ops->kp.n == n || (ops->kp.n == 0 && ops->Kp.n == n)) && ops->E.n == n &&
               ops->S.n == n && ops->Sinv.n == n && ops->G.n == n,
           QT_EINVAL, "operands: core counts differ");
  QT_CHECK(ops->kp.n == 0 || ops->kp.batch == 1, QT_EINVAL, "operands: kp must be a single train");
  QT_CHECK(ops->G2.n == 0 || ops->G2.n == n, QT_EINVAL, "operands: G2 core count");
  QT_CHECK(ops->E.batch == e->batch, QT_EINVAL, "operands: E batch must equal e batch");
  QT_CHECK(ops->E_norm != nullptr, QT_EINVAL, "operands: E_norm missing");
  for (int b = 0; b < e->batch; ++b)
    QT_CHECK(ops->E_norm[b] > 0.0, QT_EINVAL, "operands: every load E must be nonzero");
  for (int k = 0; k < n; ++k)
    QT_CHECK(e->modes[k] == (k == 0 ? ops->E.modes[0] : 2) && ops->E.modes[k] == e->modes[k],
             QT_EINVAL, "e: modes must be [d,2,...] with d the mode of E's component core");
  return QT_OK;
}

// The field must hold every train a rounding can leave: min(natural rank, max_rank).
static qt_status validate_field_cap(const qt_tt* e, int rmax) {
  std::vector<int32_t> nat = natural_caps(std::vector<int32_t>(e->modes, e->modes + e->n));
  for (int k = 0; k <= e->n; ++k) {
    int need = rmax > 0 ? std::min(nat[k], rmax) : nat[k];
    QT_CHECK(e->cap[k] >= need, QT_ECAPACITY, "e: capacity below min(natural rank, max_rank)");
  }
  return QT_OK;
}

// Capacities of the intermediates of one iteration.
struct IterPlan {
  std::vector<int32_t> modes, rc, c1, c2, c3, c4, c5, c6;
  TTLayout l1, l2, l3, l4, l5, l6, lr;
  size_t bytesA = 0, bytesB = 0;
};

static int32_t clampi(int64_t v) { return (int32_t)std::min<int64_t>(v, 1 << 30); }

static IterPlan plan_iteration(const qt_operands* ops, const qt_tt* e, int rmax) {
  IterPlan P;
  const int n = e->n;
  P.modes.assign(e->modes, e->modes + n);
  std::vector<int32_t> nat = natural_caps(P.modes);
  P.rc.resize(n + 1);
  P.c1.resize(n + 1); P.c2.resize(n + 1); P.c3.resize(n + 1); P.c4.resize(n + 1);
  P.c5.resize(n + 1); P.c6.resize(n + 1);
  for (int k = 0; k <= n; ++k) {
    int ce = e->cap[k];
    P.rc[k] = std::min(std::min(nat[k], rmax > 0 ? rmax : ce), ce);
    P.c1[k] = clampi((int64_t)(ops->kp.n ? ops->kp.cap[k] : ops->Kp.ranks[k]) * ce);
    int r1 = std::min<int64_t>(P.c1[k], std::min<int64_t>(nat[k], rmax > 0 ? rmax : P.c1[k]));
    P.c2[k] = clampi((int64_t)ops->S.ranks[k] * r1);
    int r2 = std::min<int64_t>(P.c2[k], std::min<int64_t>(nat[k], rmax > 0 ? rmax : P.c2[k]));
    P.c3[k] = clampi((int64_t)ops->G.ranks[k] * r2);
    int r3 = std::min<int64_t>(P.c3[k], std::min<int64_t>(nat[k], rmax > 0 ? rmax : P.c3[k]));
    // S^H eps^ is not rounded on its own: E - S^H eps^ is rounded once
    P.c4[k] = clampi((int64_t)ops->Sinv.ranks[k] * r3);
    P.c5[k] = (k == 0 || k == n) ? 1 : clampi((int64_t)ops->E.cap[k] + P.c4[k]);
    int r5 = std::min<int64_t>(P.c5[k], std::min<int64_t>(nat[k], rmax > 0 ? rmax : P.c5[k]));
    P.c6[k] = (k == 0 || k == n) ? 1 : clampi((int64_t)r5 + ce);
  }
  P.l1 = make_layout(P.modes, P.c1);
  P.l2 = make_layout(P.modes, P.c2);
  P.l3 = make_layout(P.modes, P.c3);
  P.l4 = make_layout(P.modes, P.c4);
  P.l5 = make_layout(P.modes, P.c5);
  P.l6 = make_layout(P.modes, P.c6);
  const int B = e->batch;
  P.bytesA = sizeof(cplx) * B * std::max({P.l1.stride, P.l3.stride, P.l5.stride});
  P.bytesB = sizeof(cplx) * B * std::max({P.l2.stride, P.l4.stride, P.l6.stride});
  return P;
}

// View of a rounded train with capacities reduced to what rounding can leave.
static qt_tt shrink(const qt_tt& t, const std::vector<int32_t>& capv, int rmax,
                    std::vector<int32_t>& store) {
  const int n = t.n;
  std::vector<int32_t> nat = natural_caps(std::vector<int32_t>(t.modes, t.modes + n));
  store.resize(n + 1);
  for (int k = 0; k <= n; ++k)
    store[k] = std::min<int32_t>(capv[k], std::min<int32_t>(nat[k], rmax > 0 ? rmax : capv[k]));
  qt_tt v = t;
  v.cap = store.data();
  return v;
}

static size_t round_bytes(const TTLayout& L, int B, int rmax) {
  qt_tt t = L.view(nullptr, nullptr, B);
  return round_ws_layout(&t, rmax > 0 ? rmax : (1 << 30)).bytes;
}

// Workspace of residual_norm beyond the difference train itself.
static size_t residual_bytes(const TTLayout& ld, int B, int rmax) {
  const int n = (int)ld.modes.size();
  int64_t env = 1, tcap = 1;
  for (int k = 0; k <= n; ++k) env = std::max<int64_t>(env, (int64_t)ld.cap[k] * ld.cap[k]);
  for (int k = 0; k < n; ++k)
    tcap = std::max<int64_t>(tcap, (int64_t)ld.cap[k] * ld.modes[k] * ld.cap[k + 1]);
  const size_t dot = sizeof(cplx) * B * (2 * env + tcap) + 4096;
  qt_tt t = ld.view(nullptr, nullptr, B);
  const size_t sweep = round_ws_layout(&t, rmax > 0 ? rmax : (1 << 30)).bytes;
  return std::max(dot, sweep) + sizeof(double) * 8 * B + sizeof(int32_t) * B + 4 * 256;
}

static size_t iteration_bytes(const IterPlan& P, int B, int rmax) {
  size_t r = 0;
  for (const TTLayout* L : {&P.l1, &P.l2, &P.l3, &P.l4, &P.l5})
    r = std::max(r, round_bytes(*L, B, rmax));
  r = std::max(r, residual_bytes(P.l6, B, rmax));
  const int n = (int)P.modes.size();
  return P.bytesA + P.bytesB + r + sizeof(int32_t) * B * (n + 1) * 2 + sizeof(double) * B * 4 +
         4096;
}

__global__ void k_take_re(int batch, const double* pairs, double* out) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < batch) out[b] = pairs[2 * b];
}

__global__ void k_residual(int batch, const double* norm, const double* inv_scale, double* out) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < batch) out[b] = norm[b] * inv_scale[b];
}

// Residual ||e' - e|| of the stopping rule (Alg. 2) for d = e' - e.
// Environment contractions give ||d||^2, ||e'||^2 and ||e||^2; their rounding
// error is about n R u (||e'||^2 + ||e||^2) (n cores, R the summed rank, u the
// unit roundoff), so where ||d||^2 > RES_DOT_TOL (||e'||^2 + ||e||^2) the dot
// value is accurate to a relative 2 n R u / RES_DOT_TOL (< 1e-8 at n R <= 1e4)
// and the instance takes it.  Closer to convergence the difference cancels
// and the left-orthogonalizing sweep of d (relative error ~ u ||e|| / ||d||)
// decides; instances that took the dot value get rank-0 interior bonds, so
// every kernel of that sweep finds nothing to do for them.
constexpr double RES_DOT_TOL = 1e-4;

__global__ void k_res_choose(int batch, int n, const double* __restrict__ pd,
                             const double* __restrict__ pe1, const double* __restrict__ pe0,
                             int32_t* dranks, double* rdot, int32_t* use_dot) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const double d2 = pd[2 * b], s2 = pe1[2 * b] + pe0[2 * b];
  const bool dot = d2 > RES_DOT_TOL * s2;
  use_dot[b] = dot ? 1 : 0;
  rdot[b] = dot ? sqrt(d2) : 0.0;
  if (dot)
    for (int k = 1; k < n; ++k) dranks[(int64_t)b * (n + 1) + k] = 0;
}

__global__ void k_res_merge(int batch, const int32_t* __restrict__ use_dot,
                            const double* __restrict__ rdot, double* dnorm) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < batch && use_dot[b]) dnorm[b] = rdot[b];
}

static qt_status residual_norm(qt_ctx ctx, const qt_tt* enew, const qt_tt* e, qt_tt* d,
                               double* dnorm, const qt_round_opts& ro) {
  const int B = d->batch, n = d->n;
  hipStream_t st = ctx->stream;
  double* pairs = (double*)ws_take(ctx, sizeof(double) * 6 * B);
  double* rdot = (double*)ws_take(ctx, sizeof(double) * B);
  int32_t* use = (int32_t*)ws_take(ctx, sizeof(int32_t) * B);
  QT_CHECK(pairs && rdot && use, QT_ENOMEM, "residual workspace");
  const size_t mark = ctx->ws_top;
  QT_TRY(dot_impl(ctx, d, d, pairs, false));
  ctx->ws_top = mark;
  QT_TRY(dot_impl(ctx, enew, enew, pairs + 2 * B, false));
  ctx->ws_top = mark;
  QT_TRY(dot_impl(ctx, e, e, pairs + 4 * B, false));
  ctx->ws_top = mark;
  k_res_choose<<<(B + 127) / 128, 128, 0, st>>>(B, n, pairs, pairs + 2 * B, pairs + 4 * B,
                                                d->ranks, rdot, use);
  // outside a graph capture, skip the sweep's launches when every instance
  // took the dot value (one small read; its kernels would all exit at once)
  bool sweep = true;
  if (!ctx->capturing) {
    std::vector<int32_t> hu(B);
    QT_HIP(hipMemcpyAsync(hu.data(), use, sizeof(int32_t) * B, hipMemcpyDeviceToHost, st));
    QT_HIP(hipStreamSynchronize(st));
    sweep = std::any_of(hu.begin(), hu.end(), [](int32_t u) { return u == 0; });
  }
  if (sweep) {
    qt_round_opts po = ro;
    po.mode = QT_ROUND_SVD;
    QT_TRY(round_impl(ctx, d, &po, nullptr, dnorm, true, nullptr, 0, 0));
  }
  k_res_merge<<<(B + 127) / 128, 128, 0, st>>>(B, use, rdot, dnorm);
  QT_HIP(hipGetLastError());
  return QT_OK;
}

// One iteration of Algorithm 2 with materialized products and SVD rounding.
static qt_status iterate_once(qt_ctx ctx, const qt_operands* ops, qt_tt* e, const IterPlan& P,
                              const qt_round_opts& ro, char* bufA, char* bufB, int32_t* rA,
                              int32_t* rB, double* dnorm, const double* dinv, double* res_out) {
  const int B = e->batch;
  const int rmax = ro.max_rank;
  const size_t mark = ctx->ws_top;
  std::vector<int32_t> s1, s2, s3, s5;
  // tau = round(k' (.) e)
  qt_tt t1 = P.l1.view(bufA, rA, B);
  if (ops->kp.n) QT_TRY(hadamard_impl(ctx, &ops->kp, e, &t1));
  else QT_TRY(mpo_impl(ctx, &ops->Kp, e, &t1));
  QT_TRY(round_impl(ctx, &t1, &ro, nullptr, nullptr, false, nullptr, 0, 0));
  ctx->ws_top = mark;
  qt_tt t1r = shrink(t1, P.c1, rmax, s1);
  // tau^ = round(S tau)
  qt_tt t2 = P.l2.view(bufB, rB, B);
  QT_TRY(mpo_impl(ctx, &ops->S, &t1r, &t2));
  QT_TRY(round_impl(ctx, &t2, &ro, nullptr, nullptr, false, nullptr, 0, 0));
  ctx->ws_top = mark;
  qt_tt t2r = shrink(t2, P.c2, rmax, s2);
  // eps^ = round(G tau^)
  qt_tt t3 = P.l3.view(bufA, rA, B);
  QT_TRY(mpo_impl(ctx, &ops->G, &t2r, &t3));
  QT_TRY(round_impl(ctx, &t3, &ro, nullptr, nullptr, false, nullptr, 0, 0));
  ctx->ws_top = mark;
  qt_tt t3r = shrink(t3, P.c3, rmax, s3);
  // S^dagger eps^ (materialized, not rounded on its own)
  qt_tt t4 = P.l4.view(bufB, rB, B);
  QT_TRY(mpo_impl(ctx, &ops->Sinv, &t3r, &t4));
  // e' = round(E - S^dagger eps^): the fourth and last rounding of the iteration
  qt_tt t5 = P.l5.view(bufA, rA, B);
  QT_TRY(add_impl(ctx, 1.0, 0.0, &ops->E, -1.0, 0.0, &t4, &t5));
  QT_TRY(round_impl(ctx, &t5, &ro, nullptr, nullptr, false, nullptr, 0, 0));
  ctx->ws_top = mark;
  qt_tt t5r = shrink(t5, P.c5, rmax, s5);
  // residual ||e' - e||
  qt_tt t6 = P.l6.view(bufB, rB, B);
  QT_TRY(add_impl(ctx, 1.0, 0.0, &t5r, -1.0, 0.0, e, &t6));
  QT_TRY(residual_norm(ctx, &t5r, e, &t6, dnorm, ro));
  ctx->ws_top = mark;
  if (res_out) {
    k_residual<<<(B + 127) / 128, 128, 0, ctx->stream>>>(B, dnorm, dinv, res_out);
    QT_HIP(hipGetLastError());
  }
  // e <- e'
  QT_TRY(tt_copy(ctx, &t5r, e));
  return QT_OK;
}

static qt_status check_status(qt_ctx ctx) {
  int32_t st = 0;
  QT_HIP(hipMemcpyAsync(&st, ctx->status, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
  QT_HIP(hipStreamSynchronize(ctx->stream));
  if (st) {
    QT_HIP(hipMemsetAsync(ctx->status, 0, sizeof(int32_t), ctx->stream));
    if (st & ST_NONFINITE) {
      double d[QT_DIAG_N];
      QT_HIP(hipMemcpyAsync(d, status_diag(ctx->status), sizeof(d), hipMemcpyDeviceToHost,
                            ctx->stream));
      QT_HIP(hipStreamSynchronize(ctx->stream));
      char msg[256];
      static const char* where[] = {"", "LDS Jacobi", "global-memory Jacobi",
                                    "triangle given to the Jacobi", "",
                                    "", "core from the Jacobi (tall)", "",
                                    "left vectors from the Jacobi (wide)", ""};
      const int w = (int)d[8];
      snprintf(msg, sizeof(msg),
               "non-finite values in a rounding (%s, order %d, values %.3e %.3e, count %d)",
               (w >= 1 && w <= 9) ? where[w] : "?", (int)d[5], d[6], d[7], (int)d[9]);
      set_error(msg);
      return QT_ENUMERIC;
    }
    if (st & ST_JACOBI_CAP) {
      double d[QT_DIAG_N];
      QT_HIP(hipMemcpyAsync(d, status_diag(ctx->status), sizeof(d), hipMemcpyDeviceToHost,
                            ctx->stream));
      QT_HIP(hipStreamSynchronize(ctx->stream));
      char msg[256];
      snprintf(msg, sizeof(msg),
               "Jacobi SVD reached its sweep cap (order %d, ||R||_F^2 %.3e, worst off-diagonal "
               "%.3e x tol, smallest rotated column %.3e of ||R||_F^2, %d sweeps)",
               (int)d[0], d[1], d[2], d[3], (int)d[4]);
      set_error(msg);
      return QT_ENUMERIC;
    }
  }
  return QT_OK;
}

struct IterSetup {
  IterPlan P;
  char* bufA = nullptr;
  char* bufB = nullptr;
  int32_t* rA = nullptr;
  int32_t* rB = nullptr;
  double* dnorm = nullptr;
  double* dinv = nullptr;
};

static qt_status setup_iteration(qt_ctx ctx, const qt_operands* ops, qt_tt* e,
                                 const qt_solve_opts* opts, IterSetup& S, size_t extra) {
  const int B = e->batch, n = e->n;
  const int rmax = opts->round.max_rank;
  S.P = plan_iteration(ops, e, rmax);
  ctx->ws_top = 0;
  QT_TRY(ws_reserve(ctx, iteration_bytes(S.P, B, rmax) + extra));
  S.bufA = (char*)ws_take(ctx, S.P.bytesA);
  S.bufB = (char*)ws_take(ctx, S.P.bytesB);
  S.rA = (int32_t*)ws_take(ctx, sizeof(int32_t) * B * (n + 1));
  S.rB = (int32_t*)ws_take(ctx, sizeof(int32_t) * B * (n + 1));
  S.dnorm = (double*)ws_take(ctx, sizeof(double) * B);
  S.dinv = (double*)ws_take(ctx, sizeof(double) * B);
  QT_CHECK(S.bufA && S.bufB && S.rA && S.rB && S.dnorm && S.dinv, QT_ENOMEM, "iteration workspace");
  std::vector<double> inv(B);
  const double N3 = std::ldexp(1.0, 3 * ops->L);
  for (int b = 0; b < B; ++b) inv[b] = 1.0 / (ops->E_norm[b] * std::sqrt(N3));
  QT_HIP(hipMemcpy(S.dinv, inv.data(), sizeof(double) * B, hipMemcpyHostToDevice));
  return QT_OK;
}


// ----------------------------------------------------------- sketch mode
// tau = R(Kp y), tau^ = R(S tau), eps^ = R(G tau^), t4 = R(S^H eps^) with the
// product-aware rounding R; then e' = SVD-round(E - t4) and the residual.
struct SketchPlan {
  std::vector<int32_t> modes, ce;
  std::vector<int32_t> ell1, ell2, ell3, ell4;
  std::vector<int32_t> c1r, c2r, c3r, c4r, c5, c5r, c6;
  TTLayout l1, l2, l3, l4, l5, l6;
  size_t bytesA = 0, bytesB = 0, ws = 0;
};

static std::vector<int32_t> capmin(const std::vector<int32_t>& c, int rmax) {
  std::vector<int32_t> r(c);
  if (rmax > 0)
    for (size_t k = 1; k + 1 < r.size(); ++k) r[k] = std::min(r[k], rmax);
  return r;
}

static SketchPlan plan_sketch(const qt_operands* ops, const qt_tt* e, const qt_round_opts& ro) {
  SketchPlan P;
  const int n = e->n, B = e->batch, rmax = ro.max_rank, os = ro.oversample;
  P.modes.assign(e->modes, e->modes + n);
  P.ce.assign(e->cap, e->cap + n + 1);
  std::vector<int32_t> nat = natural_caps(P.modes);
  qt_tt y = *e;
  P.ell1 = sketch_ranks(&ops->Kp, &y, rmax, os);
  P.c1r = capmin(P.ell1, rmax);
  y.cap = P.c1r.data();
  P.ell2 = sketch_ranks(&ops->S, &y, rmax, os);
  P.c2r = capmin(P.ell2, rmax);
  y.cap = P.c2r.data();
  P.ell3 = sketch_ranks(&ops->G, &y, rmax, os);
  P.c3r = capmin(P.ell3, rmax);
  y.cap = P.c3r.data();
  // t = S E - eps^ (rank c3r + 1), then e' = R(S^H t)
  P.c5.resize(n + 1);
  P.c6.resize(n + 1);
  for (int k = 0; k <= n; ++k) P.c5[k] = (k == 0 || k == n) ? 1 : P.c3r[k] + ops->SE.cap[k];
  y.cap = P.c5.data();
  P.ell4 = sketch_ranks(&ops->Sinv, &y, rmax, os);
  P.c4r = capmin(P.ell4, rmax);
  for (int k = 0; k <= n; ++k) P.c6[k] = (k == 0 || k == n) ? 1 : P.c4r[k] + P.ce[k];
  (void)nat;
  P.l1 = make_layout(P.modes, P.ell1);
  P.l2 = make_layout(P.modes, P.ell2);
  P.l3 = make_layout(P.modes, P.ell3);
  P.l4 = make_layout(P.modes, P.ell4);
  P.l5 = make_layout(P.modes, P.c5);
  P.l6 = make_layout(P.modes, P.c6);
  P.bytesA = sizeof(cplx) * B * std::max({P.l1.stride, P.l3.stride, P.l4.stride});
  P.bytesB = sizeof(cplx) * B * std::max({P.l2.stride, P.l5.stride, P.l6.stride});
  const int lmax = rmax > 0 ? rmax : (1 << 30);
  size_t ws = 0;
  qt_tt yv = *e, ov;
  ov = P.l1.view(nullptr, nullptr, B);
  ws = std::max(ws, sround_ws_layout(&ops->Kp, &yv, &ov, P.ell1, lmax).bytes);
  yv.cap = P.c1r.data();
  ov = P.l2.view(nullptr, nullptr, B);
  ws = std::max(ws, sround_ws_layout(&ops->S, &yv, &ov, P.ell2, lmax).bytes);
  yv.cap = P.c2r.data();
  ov = P.l3.view(nullptr, nullptr, B);
  ws = std::max(ws, sround_ws_layout(&ops->G, &yv, &ov, P.ell3, lmax).bytes);
  ws = std::max(ws, sandwich_ws_layout(ops->G2.n ? &ops->G2 : &ops->G, &yv).bytes);
  yv.cap = P.c5.data();
  ov = P.l4.view(nullptr, nullptr, B);
  ws = std::max(ws, sround_ws_layout(&ops->Sinv, &yv, &ov, P.ell4, lmax).bytes);
  {
    // <t, t> by environments (dot_impl)
    int64_t env = 1, tcap = 1;
    for (int k = 0; k <= n; ++k) env = std::max<int64_t>(env, (int64_t)P.c5[k] * P.c5[k]);
    for (int k = 0; k < n; ++k)
      tcap = std::max<int64_t>(tcap, (int64_t)P.c5[k] * P.modes[k] * P.c5[k + 1]);
    ws = std::max(ws, sizeof(cplx) * B * (2 * env + tcap) + sizeof(double) * 2 * B + 8192);
  }
  yv = *e;
  ws = std::max(ws, sandwich_ws_layout(&ops->K2, &yv).bytes);
  ws = std::max(ws, residual_bytes(P.l6, B, rmax));
  P.ws = ws;
  return P;
}

static qt_tt view_caps(const qt_tt& t, const std::vector<int32_t>& caps) {
  qt_tt v = t;
  v.cap = caps.data();
  return v;
}

// One product-aware rounding step s of the iteration.  Learned path: fixed
// widths predicted by the MLP from the previous iteration's features (the
// largest prediction over the batch, per bond); instance b keeps its learned
// rounding when its exact a-posteriori error sqrt(||x||^2 - ||x~||^2)/||x|| is
// at most eps, or, where the last SVD-truncated rounding of this step and
// instance could not meet eps (its error estimate e_s > eps: the rank cap
// binds), at most max(eps, accept * e_s).  The decision is taken on the
// device per instance; the host reads the number of instances that fell back
// and, when there are any, runs the SVD-truncated rounding of the whole batch
// into the spare buffer and copies it over the instances that fell back.  The
// factor never relaxes eps.
// lo_flags (device [B]): 1 where the output is left-orthogonal (a kept
// fixed-rank rounding, weight in the last core), 0 where it is right-
// orthogonal (SVD-truncated, weight in core 0).
__global__ void k_fill_i32(int64_t count, int32_t v, int32_t* p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

// out <- spare for the instances b with keep[b] == 0 (cores of every slot,
// ranks, error and estimate)
__global__ void k_take_fallback(int64_t per, int n1, int B, const int32_t* __restrict__ keep,
                                const cplx* __restrict__ spare, const int32_t* __restrict__ rk2,
                                const double* __restrict__ err2, cplx* out, int32_t* rk,
                                double* err) {
  const int b = blockIdx.y;
  if (keep[b]) return;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < per;
       e += (int64_t)gridDim.x * blockDim.x)
    out[(int64_t)b * per + e] = spare[(int64_t)b * per + e];
  if (blockIdx.x == 0) {
    for (int k = threadIdx.x; k < n1; k += blockDim.x) rk[(int64_t)b * n1 + k] = rk2[(int64_t)b * n1 + k];
    if (threadIdx.x == 0) {
      err[b] = err2[b];
      err[B + b] = err2[B + b];
    }
  }
}

__global__ void k_keep_to_flags(int B, const int32_t* __restrict__ keep, int32_t* lo) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) lo[b] = keep[b];
}

// Buffers of the learned path: spare outputs for the fallback (layout of each
// step's output), its ranks and errors, per-instance orientation flags and
// norm scratch; for batches, the compacted redo of the instances that fell
// back: their inputs (yc, ranks rc), per-instance operators (ac), norms (xc),
// sketch R diagonals (rdc) and indices (idx).
struct LearnBufs {
  char* spare = nullptr;
  int32_t* rS = nullptr;
  double* err2 = nullptr;
  int32_t* lo = nullptr;
  double* ntmp = nullptr;
  cplx* yc = nullptr;
  int32_t* rc = nullptr;
  cplx* ac = nullptr;
  double* xc = nullptr;
  double* rdc = nullptr;
  int32_t* idx = nullptr;
};

// idx[0..nf) = the instances b with keep[b] == 0, in order (one block)
__global__ void k_fail_index(int B, const int32_t* __restrict__ keep, int32_t* __restrict__ idx) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int j = 0;
  for (int b = 0; b < B; ++b)
    if (!keep[b]) idx[j++] = b;
}

// dst instance j <- src instance idx[j] / grp: `per` elements, optionally the
// ranks (n1 per instance) and one double (xn2)
__global__ void k_gather_inst(int64_t per, const int32_t* __restrict__ idx, int grp,
                              const cplx* __restrict__ src, int64_t sS, cplx* __restrict__ dst,
                              int64_t sD, int n1, const int32_t* __restrict__ rsrc,
                              int32_t* __restrict__ rdst, const double* __restrict__ xsrc,
                              double* __restrict__ xdst) {
  const int j = blockIdx.y;
  const int64_t b = idx[j] / grp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < per;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[j * sD + e] = src[b * sS + e];
  if (blockIdx.x == 0) {
    if (rdst)
      for (int k = threadIdx.x; k < n1; k += blockDim.x) rdst[(int64_t)j * n1 + k] = rsrc[b * n1 + k];
    if (xdst && threadIdx.x == 0) xdst[j] = xsrc[b];
  }
}

// out instance idx[j] <- spare instance j (cores, ranks, error bound and
// estimate, sketch R diagonals)
__global__ void k_scatter_fallback(int64_t per, int n1, int B, int nf, const int32_t* __restrict__ idx,
                                   const cplx* __restrict__ spare, const int32_t* __restrict__ rk2,
                                   const double* __restrict__ err2, cplx* out, int32_t* rk,
                                   double* err, const double* __restrict__ rdc, double* rd,
                                   int64_t rd_per) {
  const int j = blockIdx.y;
  const int64_t b = idx[j];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < per;
       e += (int64_t)gridDim.x * blockDim.x)
    out[b * per + e] = spare[(int64_t)j * per + e];
  if (rd)
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < rd_per;
         e += (int64_t)gridDim.x * blockDim.x)
      rd[b * rd_per + e] = rdc[(int64_t)j * rd_per + e];
  if (blockIdx.x == 0) {
    for (int k = threadIdx.x; k < n1; k += blockDim.x) rk[b * n1 + k] = rk2[(int64_t)j * n1 + k];
    if (threadIdx.x == 0) {
      err[b] = err2[j];
      err[B + b] = err2[nf + j];
    }
  }
}

static qt_status round_step(qt_ctx ctx, int step, const qt_mpo* A, const qt_tt* y,
                            const std::vector<int32_t>& ell_plan, const qt_round_opts& base,
                            const double* xn2, qt_tt* out, double* err_dev, uint64_t iter_id,
                            bool learned, bool logging, int32_t* lo_flags, qt_tt* spare,
                            double* err2, const LearnBufs& lb) {
  const int n = y->n, B = y->batch;
  LearnCtx* L = ctx->learn;
  const bool track = L && (learned || logging);
  double* rd = track ? L->rdiag_at(step) : nullptr;
  const size_t mark = ctx->ws_top;
  qt_round_opts so = base;
  so.mode = QT_ROUND_SKETCH;
  std::vector<int32_t> ell = ell_plan;
  const bool use_learned = learned && L->have_prev && L->params && !L->pred_ell[step].empty();
  // the SVD-truncated rounding's error as the learned path's reference: the
  // quadrature estimate (the reported bound adds the two parts linearly)
  double* est_dev = err_dev + B;
  if (use_learned) {
    const int rcap = base.max_rank > 0 ? base.max_rank : (1 << 30);
    for (size_t k = 1; k + 1 < ell.size(); ++k)
      ell[k] = std::min({ell[k], L->pred_ell[step][k], rcap});
    so.mode = QT_ROUND_LEARNED;
  }
  QT_TRY(sround_impl(ctx, A, y, nullptr, nullptr, ell, &so, xn2, out, err_dev, nullptr,
                     iter_id * 4 + step, nullptr, 0, 0, rd, est_dev));
  ctx->ws_top = mark;
  int32_t nfail = B;
  if (use_learned) {
    learn_decide(ctx, step, err_dev, base.eps);
    QT_HIP(hipMemcpyAsync(&nfail, L->nfail, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    QT_HIP(hipStreamSynchronize(ctx->stream));
    // kept instances: left-orthogonal fixed-rank output
    k_fill_i32<<<(B + 255) / 256, 256, 0, ctx->stream>>>(B, 1, lo_flags);
    qt_round_opts fo = base;
    fo.mode = QT_ROUND_SKETCH;
    const int64_t per = out->inst_stride;
    const int64_t rd_per = (int64_t)(n + 1) * RD_MAX;
    if (nfail > 0 && nfail < B && lb.yc) {
      // redo only the instances that fell back, as a compacted batch: gather
      // their inputs (and per-instance operators and norms), round them
      // SVD-truncated into the spare train, scatter the results back
      const int nf = nfail;
      k_fail_index<<<1, 64, 0, ctx->stream>>>(B, L->keep, lb.idx);
      dim3 gy((unsigned)std::min<int64_t>((y->inst_stride + 255) / 256, 64), nf);
      k_gather_inst<<<gy, 256, 0, ctx->stream>>>(y->inst_stride, lb.idx, 1, (const cplx*)y->data,
                                                 y->inst_stride, lb.yc, y->inst_stride, n + 1,
                                                 y->ranks, lb.rc, xn2, lb.xc);
      qt_tt yc = *y;
      yc.batch = nf;
      yc.data = lb.yc;
      yc.ranks = lb.rc;
      qt_mpo Ac = *A;
      if (A->inst_stride > 0) {
        dim3 ga((unsigned)std::min<int64_t>((A->inst_stride + 255) / 256, 64), nf);
        k_gather_inst<<<ga, 256, 0, ctx->stream>>>(
            A->inst_stride, lb.idx, A->inst_group > 0 ? A->inst_group : 1, (const cplx*)A->data,
            A->inst_stride, lb.ac, A->inst_stride, 0, nullptr, nullptr, nullptr, nullptr);
        Ac.data = lb.ac;
        Ac.inst_group = 1;
      }
      qt_tt sc = *spare;
      sc.batch = nf;
      QT_TRY(sround_impl(ctx, &Ac, &yc, nullptr, nullptr, ell_plan, &fo, lb.xc, &sc, err2, nullptr,
                         iter_id * 4 + step + (1ull << 40), nullptr, 0, 0, rd ? lb.rdc : nullptr,
                         err2 + nf));
      ctx->ws_top = mark;
      dim3 gs((unsigned)std::min<int64_t>((per + 255) / 256, 64), nf);
      k_scatter_fallback<<<gs, 256, 0, ctx->stream>>>(per, n + 1, B, nf, lb.idx,
                                                      (const cplx*)spare->data, spare->ranks, err2,
                                                      (cplx*)out->data, out->ranks, err_dev,
                                                      lb.rdc, rd, rd_per);
      k_keep_to_flags<<<(B + 255) / 256, 256, 0, ctx->stream>>>(B, L->keep, lo_flags);
      learn_set_ref(ctx, step, est_dev, L->keep);
    } else if (nfail > 0) {
      QT_TRY(sround_impl(ctx, A, y, nullptr, nullptr, ell_plan, &fo, xn2, spare, err2, nullptr,
                         iter_id * 4 + step + (1ull << 40), nullptr, 0, 0, rd, err2 + B));
      ctx->ws_top = mark;
      dim3 grid((unsigned)std::min<int64_t>((per + 255) / 256, 64), B);
      k_take_fallback<<<grid, 256, 0, ctx->stream>>>(per, n + 1, B, L->keep, (const cplx*)spare->data,
                                                     spare->ranks, err2, (cplx*)out->data,
                                                     out->ranks, err_dev);
      // fallen-back instances are right-orthogonal
      k_keep_to_flags<<<(B + 255) / 256, 256, 0, ctx->stream>>>(B, L->keep, lo_flags);
      learn_set_ref(ctx, step, est_dev, L->keep);
    }
  }
  if (!use_learned) {
    k_fill_i32<<<(B + 255) / 256, 256, 0, ctx->stream>>>(B, 0, lo_flags);
    if (learned && L) learn_set_ref(ctx, step, est_dev, nullptr);
  }
  // the stored sketch R diagonals are the fallback's where one ran (every
  // instance's after a whole-batch redo, the failed ones' after a compacted one)
  if (track) {
    const bool compacted = use_learned && nfail > 0 && nfail < B && lb.yc;
    if (compacted)
      learn_features(ctx, step, ell, xn2, base.eps, base.max_rank, &ell_plan, L->keep);
    else
      learn_features(ctx, step, (use_learned && nfail == 0) ? ell : ell_plan, xn2, base.eps,
                     base.max_rank);
  }
  if (!use_learned && logging) learn_log(ctx, step, out->ranks);
  QT_HIP(hipGetLastError());
  return QT_OK;
}

// After an iteration: the features just written become "previous"; the
// learned path predicts the next iteration's widths with the MLP.
static qt_status learn_advance(qt_ctx ctx, bool learned, const std::vector<int32_t>* ells[4]) {
  LearnCtx* L = ctx->learn;
  if (!L) return QT_OK;
  L->cur = 1 - L->cur;
  L->have_prev = true;
  ++L->iter;
  if (!learned || !L->params) return QT_OK;
  return learn_predict(ctx, ells);
}

// ||t||^2 of an orthogonalized train per instance: the squared norm of core
// n-1 where lo[b] (left-orthogonal), of core 0 otherwise.
__global__ void k_pick_norm(int B, const int32_t* lo, const double* last, const double* first,
                            double* out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) out[b] = lo[b] ? last[b] : first[b];
}

static void weight_norm2(hipStream_t st, const qt_tt& t, const int32_t* lo, double* tmp,
                         double* out) {
  const int n = t.n, rs = n + 1, B = t.batch;
  sumsq(st, B, dref(t.ranks + n - 1, rs, t.modes[n - 1]), dconst(1),
        (const cplx*)t.data + t.offsets[n - 1], t.inst_stride, tmp, 1.0);
  sumsq(st, B, dconst(1), dref(t.ranks + 1, rs, t.modes[0]), (const cplx*)t.data,
        t.inst_stride, tmp + B, 1.0);
  k_pick_norm<<<(B + 127) / 128, 128, 0, st>>>(B, lo, tmp, tmp + B, out);
}


static qt_status iterate_once_sketch(qt_ctx ctx, const qt_operands* ops, qt_tt* e,
                                     const SketchPlan& P, const qt_round_opts& ro, char* bufA,
                                     char* bufB, int32_t* rA, int32_t* rB, double* dnorm,
                                     const double* dinv, double* xn2, double* err_dev,
                                     double* res_out, uint64_t iter_id, bool learned,
                                     bool logging, const LearnBufs& lb) {
  const int B = e->batch, n = e->n;
  hipStream_t st = ctx->stream;
  const size_t mark = ctx->ws_top;
  if (learned || logging) QT_TRY(learn_ensure(ctx, n, B));
  int32_t* lo = lb.lo;
  qt_tt sp1 = P.l1.view(lb.spare, lb.rS, B), sp2 = P.l2.view(lb.spare, lb.rS, B);
  qt_tt sp3 = P.l3.view(lb.spare, lb.rS, B), sp4 = P.l4.view(lb.spare, lb.rS, B);
  // tau = R(k' e)
  QT_TRY(sandwich_impl(ctx, &ops->K2, e, 1.0, xn2));
  ctx->ws_top = mark;
  qt_tt t1 = P.l1.view(bufA, rA, B);
  QT_TRY(round_step(ctx, 0, &ops->Kp, e, P.ell1, ro, xn2, &t1, err_dev, iter_id, learned, logging,
                    lo, &sp1, lb.err2, lb));
  qt_tt t1r = view_caps(t1, P.c1r);
  // tau^ = R(S tau);  ||S tau|| = ||tau|| (S unitary)
  weight_norm2(st, t1r, lo, lb.ntmp, xn2);
  qt_tt t2 = P.l2.view(bufB, rB, B);
  QT_TRY(round_step(ctx, 1, &ops->S, &t1r, P.ell2, ro, xn2, &t2, err_dev, iter_id, learned, logging,
                    lo, &sp2, lb.err2, lb));
  qt_tt t2r = view_caps(t2, P.c2r);
  // eps^ = R(G tau^);  ||G t||^2 = <t, G t>/k0 (scalar conductivity: k0 G is a
  // projector), or <t, G2 t> with G2 = G^H G given as an operand (elasticity)
  if (ops->G2.n) QT_TRY(sandwich_impl(ctx, &ops->G2, &t2r, 1.0, xn2));
  else QT_TRY(sandwich_impl(ctx, &ops->G, &t2r, 1.0 / ops->k0, xn2));
  ctx->ws_top = mark;
  qt_tt t3 = P.l3.view(bufA, rA, B);
  QT_TRY(round_step(ctx, 2, &ops->G, &t2r, P.ell3, ro, xn2, &t3, err_dev, iter_id, learned, logging,
                    lo, &sp3, lb.err2, lb));
  qt_tt t3r = view_caps(t3, P.c3r);
  // t = S E - eps^;  ||t||^2 by environments (no cancellation: Gamma(0) = 0
  // makes eps^ vanish at the zero frequency, where S E lives)
  qt_tt tt = P.l5.view(bufB, rB, B);
  QT_TRY(add_impl(ctx, 1.0, 0.0, &ops->SE, -1.0, 0.0, &t3r, &tt));
  qt_tt ttr = view_caps(tt, P.c5);
  {
    double* pairs = (double*)ws_take(ctx, sizeof(double) * 2 * B);
    QT_CHECK(pairs, QT_ENOMEM, "iteration workspace (norm)");
    QT_TRY(dot_impl(ctx, &ttr, &ttr, pairs, false));
    k_take_re<<<(B + 127) / 128, 128, 0, st>>>(B, pairs, xn2);
    ctx->ws_top = mark;
  }
  // e' = R(S^H t) = E - S^H eps^
  qt_tt t4 = P.l4.view(bufA, rA, B);
  QT_TRY(round_step(ctx, 3, &ops->Sinv, &ttr, P.ell4, ro, xn2, &t4, err_dev, iter_id, learned,
                    logging, lo, &sp4, lb.err2, lb));
  qt_tt t4r = view_caps(t4, P.c4r);
  if (learned || logging) {
    const std::vector<int32_t>* ells[4] = {&P.ell1, &P.ell2, &P.ell3, &P.ell4};
    QT_TRY(learn_advance(ctx, learned, ells));
  }
  // residual ||e' - e||
  qt_tt t6 = P.l6.view(bufB, rB, B);
  QT_TRY(add_impl(ctx, 1.0, 0.0, &t4r, -1.0, 0.0, e, &t6));
  QT_TRY(residual_norm(ctx, &t4r, e, &t6, dnorm, ro));
  ctx->ws_top = mark;
  if (res_out) {
    k_residual<<<(B + 127) / 128, 128, 0, st>>>(B, dnorm, dinv, res_out);
    QT_HIP(hipGetLastError());
  }
  QT_TRY(tt_copy(ctx, &t4r, e));
  return QT_OK;
}

// One solver set-up shared by ls_iterate and homogenize (both modes).
struct Solver {
  bool sketch = false;
  IterPlan P;
  SketchPlan SP;
  char* bufA = nullptr;
  char* bufB = nullptr;
  int32_t* rA = nullptr;
  int32_t* rB = nullptr;
  double* dnorm = nullptr;
  double* dinv = nullptr;
  double* xn2 = nullptr;
  double* err = nullptr;
  LearnBufs lb;
  bool learned = false;
  bool logging = false;
};

// Arena bytes homogenize needs beyond the iteration: its residuals and the
// three A_eff dot products (environments of k_sel[c] against the field).
static size_t homogenize_extra(const qt_tt* k_sel, const qt_tt* e) {
  const int B = e->batch, d = e->modes[0];
  size_t need = 4096 + sizeof(double) * 4 * B;
  int64_t env = 1, tcap = 1;
  for (int c = 0; c < d; ++c) {
    for (int k = 0; k <= e->n; ++k)
      env = std::max<int64_t>(env, (int64_t)k_sel[c].cap[k] * e->cap[k]);
    for (int k = 0; k < e->n; ++k)
      tcap = std::max<int64_t>(tcap, (int64_t)k_sel[c].cap[k] * e->modes[k] * e->cap[k + 1]);
  }
  return need + sizeof(cplx) * B * (2 * env + tcap) + 1024;
}

// Arena bytes of ls_iterate beyond the iteration: its residual scratch.
static size_t ls_extra(const qt_tt* e) { return sizeof(double) * e->batch + 256; }

static size_t solver_arena_bytes(size_t bytesA, size_t bytesB, size_t ws, size_t extra,
                                 size_t spare, int B, int n) {
  return bytesA + bytesB + ws + extra + spare + sizeof(int32_t) * B * (n + 1) * 3 +
         sizeof(double) * B * 9 + sizeof(int32_t) * B + 14 * 256;
}

static size_t learn_spare_train_bytes(const SketchPlan& P, int B) {
  return (sizeof(cplx) * B * std::max({P.l1.stride, P.l2.stride, P.l3.stride, P.l4.stride}) + 255) &
         ~(size_t)255;
}
// inputs of the four roundings: the field, t1, t2 and S E - eps^ (layouts l1, l2, l5)
static int64_t learn_input_stride(const qt_tt* e, const SketchPlan& P) {
  return std::max({e->inst_stride, P.l1.stride, P.l2.stride, P.l5.stride});
}
static int64_t learn_op_stride(const qt_operands* ops) {
  return std::max({ops->Kp.inst_stride, ops->S.inst_stride, ops->G.inst_stride,
                   ops->Sinv.inst_stride});
}
static size_t learn_compact_bytes(const qt_operands* ops, const qt_tt* e, const SketchPlan& P) {
  const int64_t B = e->batch, n = e->n;
  return sizeof(cplx) * B * (learn_input_stride(e, P) + learn_op_stride(ops)) +
         sizeof(double) * B * ((n + 1) * RD_MAX + 1) + sizeof(int32_t) * B * (n + 2) + 8 * 256;
}

// Plan and arena sizes of a solve (no context needed: also the workspace query).
static qt_status solver_plan(const qt_operands* ops, const qt_tt* e, const qt_solve_opts* opts,
                             Solver& S, size_t& bytesA, size_t& bytesB, size_t& ws,
                             size_t& spare) {
  const int B = e->batch, n = e->n;
  const int rmax = opts->round.max_rank;
  S.sketch = opts->round.mode != QT_ROUND_SVD;
  QT_CHECK(opts->round.precision == QT_PREC_F64 ||
               (opts->round.precision == QT_PREC_F32 && S.sketch),
           QT_EINVAL, "solver: QT_PREC_F32 applies to the sketch and learned modes only");
  S.learned = opts->round.mode == QT_ROUND_LEARNED;
  if (S.learned)
    QT_CHECK(e->batch <= 1024, QT_EINVAL, "solver: learned rounding takes at most 1024 fields");
  if (S.sketch) {
    QT_CHECK(ops->Kp.n == n && ops->K2.n == n && ops->k0 > 0.0, QT_EINVAL,
             "solver: sketch mode needs Kp, K2 and k0 operands");
    QT_TRY(tt_validate(&ops->SE, "operands.SE"));
    QT_CHECK(ops->SE.n == n && ops->SE.batch == B, QT_EINVAL,
             "solver: operands.SE must match the field batch");
    for (int k = 0; k < n; ++k)
      QT_CHECK(ops->SE.modes[k] == e->modes[k], QT_EINVAL, "solver: operands.SE modes");
    S.SP = plan_sketch(ops, e, opts->round);
    bytesA = S.SP.bytesA; bytesB = S.SP.bytesB; ws = S.SP.ws;
  } else {
    QT_CHECK(ops->Kp.inst_stride == 0 && ops->K2.inst_stride == 0, QT_EINVAL,
             "solver: the plain (materializing) iteration needs shared operators");
    S.P = plan_iteration(ops, e, rmax);
    bytesA = S.P.bytesA; bytesB = S.P.bytesB; ws = iteration_bytes(S.P, B, rmax) - S.P.bytesA - S.P.bytesB;
  }
  // the learned path's fallback writes into a spare train of the largest step
  // layout; batches also hold the buffers of the compacted redo (after it)
  spare = 0;
  if (S.learned) {
    spare = learn_spare_train_bytes(S.SP, B);
    if (B > 1) spare += learn_compact_bytes(ops, e, S.SP);
  }
  return QT_OK;
}

static qt_status solver_setup(qt_ctx ctx, const qt_operands* ops, qt_tt* e,
                              const qt_solve_opts* opts, Solver& S, size_t extra) {
  const int B = e->batch, n = e->n;
  size_t bytesA = 0, bytesB = 0, ws = 0, spare = 0;
  QT_TRY(solver_plan(ops, e, opts, S, bytesA, bytesB, ws, spare));
  S.logging = ctx->learn && ctx->learn->log_count && S.sketch;
  if (S.learned)
    QT_CHECK(ctx->learn && ctx->learn->params, QT_EINVAL,
             "solver: learned rounding needs a predictor (qt_set_predictor)");
  ctx->ws_top = 0;
  // persistent learned state first (caller-owned memory takes it from the
  // end, outside the arena reserved next)
  if (S.learned || S.logging) QT_TRY(learn_ensure(ctx, n, B));
  QT_TRY(ws_reserve(ctx, solver_arena_bytes(bytesA, bytesB, ws, extra, spare, B, n)));
  S.bufA = (char*)ws_take(ctx, bytesA);
  S.bufB = (char*)ws_take(ctx, bytesB);
  S.rA = (int32_t*)ws_take(ctx, sizeof(int32_t) * B * (n + 1));
  S.rB = (int32_t*)ws_take(ctx, sizeof(int32_t) * B * (n + 1));
  S.dnorm = (double*)ws_take(ctx, sizeof(double) * B);
  S.dinv = (double*)ws_take(ctx, sizeof(double) * B);
  S.xn2 = (double*)ws_take(ctx, sizeof(double) * B);
  S.err = (double*)ws_take(ctx, sizeof(double) * 2 * B);   // bound, then estimate
  QT_CHECK(S.bufA && S.bufB && S.rA && S.rB && S.dnorm && S.dinv && S.xn2 && S.err, QT_ENOMEM,
           "iteration workspace");
  S.lb.rS = (int32_t*)ws_take(ctx, sizeof(int32_t) * B * (n + 1));
  S.lb.err2 = (double*)ws_take(ctx, sizeof(double) * 2 * B);
  S.lb.lo = (int32_t*)ws_take(ctx, sizeof(int32_t) * B);
  S.lb.ntmp = (double*)ws_take(ctx, sizeof(double) * 2 * B);
  if (spare) {
    const size_t train = learn_spare_train_bytes(S.SP, B);
    S.lb.spare = (char*)ws_take(ctx, train);
    QT_CHECK(S.lb.spare, QT_ENOMEM, "iteration workspace (learned path)");
    if (spare > train) {
      S.lb.yc = (cplx*)ws_take(ctx, sizeof(cplx) * B * learn_input_stride(e, S.SP));
      const int64_t as = learn_op_stride(ops);
      S.lb.ac = as > 0 ? (cplx*)ws_take(ctx, sizeof(cplx) * B * as) : nullptr;
      S.lb.rdc = (double*)ws_take(ctx, sizeof(double) * B * (n + 1) * RD_MAX);
      S.lb.xc = (double*)ws_take(ctx, sizeof(double) * B);
      S.lb.rc = (int32_t*)ws_take(ctx, sizeof(int32_t) * B * (n + 1));
      S.lb.idx = (int32_t*)ws_take(ctx, sizeof(int32_t) * B);
      QT_CHECK(S.lb.yc && (as == 0 || S.lb.ac) && S.lb.rdc && S.lb.xc && S.lb.rc && S.lb.idx,
               QT_ENOMEM, "iteration workspace (compacted fallback)");
    }
  }
  QT_CHECK(S.lb.rS && S.lb.err2 && S.lb.lo && S.lb.ntmp && (!spare || S.lb.spare), QT_ENOMEM,
           "iteration workspace (learned path)");
  std::vector<double> inv(B);
  const double N3 = std::ldexp(1.0, 3 * ops->L);
  for (int b = 0; b < B; ++b) inv[b] = 1.0 / (ops->E_norm[b] * std::sqrt(N3));
  QT_HIP(hipMemcpy(S.dinv, inv.data(), sizeof(double) * B, hipMemcpyHostToDevice));
  return QT_OK;
}

static qt_status solver_step(qt_ctx ctx, const qt_operands* ops, qt_tt* e, const Solver& S,
                             const qt_round_opts& ro, double* res_out) {
  if (S.sketch) {
    uint64_t id = ctx->sketch_counter++;
    return iterate_once_sketch(ctx, ops, e, S.SP, ro, S.bufA, S.bufB, S.rA, S.rB, S.dnorm, S.dinv,
                               S.xn2, S.err, res_out, id, S.learned, S.logging, S.lb);
  }
  return iterate_once(ctx, ops, e, S.P, ro, S.bufA, S.bufB, S.rA, S.rB, S.dnorm, S.dinv, res_out);
}

__global__ void k_inc_u64(uint64_t* p) { p[0] += 1; }

// Iterations 2..n of a sketch-mode ls_iterate as replays of one captured
// iteration: the capture runs on the context's private stream with the
// context stream swapped out (nothing executes while capturing), the replays
// run on the context stream.  The Gaussian stream of each replay comes from a
// device counter (incremented inside the graph), the residual goes to a
// scratch slot copied out after each replay.
static qt_status iterate_graph(qt_ctx ctx, const qt_operands* ops, qt_tt* e, const Solver& S,
                               const qt_round_opts& ro, int32_t n_iter, double* residual_out,
                               double* res_tmp) {
  const int B = e->batch;
  if (!ctx->cap_stream) QT_HIP(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  hipStream_t run = ctx->stream;
  const size_t mark = ctx->ws_top;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ctx->stream = ctx->cap_stream;
  ctx->capturing = true;
  qt_status st = QT_OK;
  hipError_t he = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
  if (he == hipSuccess) {
    st = iterate_once_sketch(ctx, ops, e, S.SP, ro, S.bufA, S.bufB, S.rA, S.rB, S.dnorm, S.dinv,
                             S.xn2, S.err, residual_out ? res_tmp : nullptr, 0, false, false, S.lb);
    k_inc_u64<<<1, 1, 0, ctx->cap_stream>>>(ctx->dev_iter);
    hipError_t he2 = hipStreamEndCapture(ctx->cap_stream, &graph);
    if (he == hipSuccess) he = he2;
  }
  ctx->stream = run;
  ctx->capturing = false;
  ctx->ws_top = mark;
  if (st != QT_OK || he != hipSuccess) {
    if (graph) hipGraphDestroy(graph);
    if (st != QT_OK) return st;
    set_error(hip_msg(he, "ls_iterate: graph capture"));
    return QT_EHIP;
  }
  he = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (he != hipSuccess) {
    hipGraphDestroy(graph);
    set_error(hip_msg(he, "ls_iterate: graph instantiation"));
    return QT_EHIP;
  }
  const uint64_t first = ctx->sketch_counter;
  he = hipMemcpyAsync(ctx->dev_iter, &first, sizeof(uint64_t), hipMemcpyHostToDevice, run);
  for (int it = 0; it < n_iter && he == hipSuccess; ++it) {
    he = hipGraphLaunch(exec, run);
    if (he == hipSuccess && residual_out)
      he = hipMemcpyAsync(residual_out + (int64_t)it * B, res_tmp, sizeof(double) * B,
                          hipMemcpyDeviceToDevice, run);
  }
  // the host copy of the counter must stay alive until the copy above ran
  hipError_t hs = hipStreamSynchronize(run);
  hipGraphExecDestroy(exec);
  hipGraphDestroy(graph);
  if (he == hipSuccess) he = hs;
  if (he != hipSuccess) {
    set_error(hip_msg(he, "ls_iterate: graph replay"));
    return QT_EHIP;
  }
  ctx->sketch_counter += n_iter;
  return QT_OK;
}

// Fixed device state of a context: status word, counters, graph iteration
// counter and the GEMM split-K buffer (256-byte aligned pieces).
static size_t fixed_piece(size_t b) { return (b + 255) & ~(size_t)255; }
static size_t ctx_fixed_bytes() {
  return fixed_piece(QT_STATUS_BYTES) + fixed_piece(sizeof(unsigned long long) * CNT_N) +
         fixed_piece(sizeof(uint64_t)) + fixed_piece(sizeof(cplx) * QT_SPLITK_ELEMS);
}

static void ctx_release(qt_ctx c) {
  if (!c->ext) {
    if (c->ws) hipFree(c->ws);
    if (c->status) hipFree(c->status);
    if (c->counters) hipFree(c->counters);
    if (c->splitk.p) hipFree(c->splitk.p);
    if (c->dev_iter) hipFree(c->dev_iter);
  }
  if (c->tuner.scratch) hipFree(c->tuner.scratch);
  for (hipEvent_t e : c->tuner.ev)
    if (e) hipEventDestroy(e);
  if (qt::g_tuner == &c->tuner) qt::g_tuner = nullptr;
  if (c->cap_stream) hipStreamDestroy(c->cap_stream);
  for (hipEvent_t e : c->prof.ev) hipEventDestroy(e);
  qt_learn_free(c);
  delete c;
}

static qt_status ctx_init(int device, void* stream, char* mem, size_t mem_bytes, qt_ctx* out) {
  QT_CHECK(out, QT_EINVAL, "qt_ctx_create: null out");
  *out = nullptr;
  QT_HIP(hipSetDevice(device));
  qt_ctx c = new qt_ctx_s();
  c->device = device;
  c->stream = (hipStream_t)stream;
  c->tuner.owner = c;
  hipError_t e = hipSuccess;
  if (mem) {
    // caller-owned memory: fixed state at its head, the arena after it
    c->ext = true;
    char* p = mem;
    c->status = (int32_t*)p;
    p += fixed_piece(QT_STATUS_BYTES);
    c->counters = (unsigned long long*)p;
    p += fixed_piece(sizeof(unsigned long long) * CNT_N);
    c->dev_iter = (uint64_t*)p;
    p += fixed_piece(sizeof(uint64_t));
    c->splitk.p = (cplx*)p;
    c->splitk.elems = QT_SPLITK_ELEMS;
    p += fixed_piece(sizeof(cplx) * QT_SPLITK_ELEMS);
    c->ext_lo = p;
    c->ext_size = mem_bytes - ctx_fixed_bytes();
    c->ws = p;
    c->ws_size = c->ext_size;
  } else {
    e = hipMalloc((void**)&c->status, QT_STATUS_BYTES);
    if (e == hipSuccess) e = hipMalloc((void**)&c->counters, sizeof(unsigned long long) * CNT_N);
    if (e == hipSuccess) {
      e = hipMalloc((void**)&c->splitk.p, sizeof(cplx) * QT_SPLITK_ELEMS);
      if (e == hipSuccess) c->splitk.elems = QT_SPLITK_ELEMS;
    }
    if (e == hipSuccess) e = hipMalloc((void**)&c->dev_iter, sizeof(uint64_t));
  }
  if (e == hipSuccess) e = hipMemset(c->status, 0, QT_STATUS_BYTES);
  if (e == hipSuccess) e = hipMemset(c->counters, 0, sizeof(unsigned long long) * CNT_N);
  if (e == hipSuccess) e = hipMemset(c->dev_iter, 0, sizeof(uint64_t));
  if (e != hipSuccess) {
    ctx_release(c);
    set_error(hip_msg(e, "qt_ctx_create: device state"));
    return QT_EHIP;
  }
  // the allocation-free entry points' scratch on this device
  qt_status s = noalloc_attach(device);
  if (s != QT_OK) {
    ctx_release(c);
    return s;
  }
  *out = c;
  return QT_OK;
}

}  // namespace qt

using namespace qt;

extern "C" {

const char* qt_last_error(void) { return g_last_error.c_str(); }

qt_status qt_ctx_create(int device, void* stream, size_t ws_bytes, qt_ctx* out) {
  QT_TRY(ctx_init(device, stream, nullptr, 0, out));
  if (ws_bytes) {
    qt_status s = ws_reserve(*out, ws_bytes);
    if (s != QT_OK) {
      ctx_release(*out);
      *out = nullptr;
      return s;
    }
  }
  return QT_OK;
}

size_t qt_ctx_fixed_bytes(void) { return ctx_fixed_bytes(); }

qt_status qt_workspace_query(const qt_tt* x, const qt_round_opts* opts, size_t* bytes) {
  QT_CHECK(x && opts && bytes, QT_EINVAL, "qt_workspace_query: null argument");
  QT_TRY(tt_validate(x, "x"));
  const int lmax_cap = opts->max_rank > 0 ? opts->max_rank : (1 << 30);
  *bytes = (round_ws_layout(x, lmax_cap, opts->mode == QT_ROUND_POLAR).bytes + 255) &
           ~(size_t)255;
  return QT_OK;
}

qt_status qt_ls_workspace_query(const qt_operands* ops, const qt_tt* k_sel, const qt_tt* e,
                                const qt_solve_opts* opts, size_t* bytes) {
  QT_CHECK(ops && e && opts && bytes, QT_EINVAL, "qt_ls_workspace_query: null argument");
  QT_TRY(validate_ops(ops, e));
  QT_TRY(validate_field_cap(e, opts->round.max_rank));
  if (k_sel)
    for (int c = 0; c < e->modes[0]; ++c) {
      QT_TRY(tt_validate(&k_sel[c], "k_sel"));
      QT_CHECK(k_sel[c].n == e->n, QT_EINVAL, "qt_ls_workspace_query: k_sel cores");
    }
  Solver S;
  size_t bytesA = 0, bytesB = 0, ws = 0, spare = 0;
  QT_TRY(solver_plan(ops, e, opts, S, bytesA, bytesB, ws, spare));
  const size_t extra = k_sel ? homogenize_extra(k_sel, e) : ls_extra(e);
  size_t b = (solver_arena_bytes(bytesA, bytesB, ws, extra, spare, e->batch, e->n) + 255) &
             ~(size_t)255;
  if (S.sketch) b += learn_state_bytes(e->n, e->batch);
  *bytes = b;
  return QT_OK;
}

qt_status qt_ctx_create_with_memory(int device, void* stream, void* mem, size_t mem_bytes,
                                    qt_ctx* out) {
  QT_CHECK(mem && ((uintptr_t)mem & 255) == 0, QT_EINVAL,
           "qt_ctx_create_with_memory: memory must be non-null and 256-byte aligned");
  QT_CHECK(mem_bytes >= ctx_fixed_bytes(), QT_ENOMEM,
           "qt_ctx_create_with_memory: memory below qt_ctx_fixed_bytes()");
  return ctx_init(device, stream, (char*)mem, mem_bytes, out);
}

void qt_ctx_destroy(qt_ctx ctx) {
  if (!ctx) return;
  hipStreamSynchronize(ctx->stream);
  ctx_release(ctx);
}

qt_status qt_ctx_profile(qt_ctx ctx, int32_t classes) {
  QT_CHECK(ctx, QT_EINVAL, "qt_ctx_profile: null ctx");
  QT_HIP(hipStreamSynchronize(ctx->stream));
  ctx->prof.cls = classes;
  ctx->prof.used = 0;
  return QT_OK;
}

qt_status qt_ctx_autotune(qt_ctx ctx, int32_t mode, int32_t* entries) {
  QT_CHECK(ctx && mode >= 0 && mode <= 5, QT_EINVAL, "qt_ctx_autotune: bad argument");
  ctx->tuner.mode = mode;
  if (entries) *entries = (int32_t)ctx->tuner.choice.size();
  return QT_OK;
}

qt_status qt_ctx_profile_read(qt_ctx ctx, double* total_ms, int64_t* launches) {
  QT_CHECK(ctx && total_ms && launches, QT_EINVAL, "qt_ctx_profile_read: bad argument");
  QT_HIP(hipStreamSynchronize(ctx->stream));
  double t = 0.0;
  for (size_t i = 0; i + 1 < ctx->prof.used; i += 2) {
    float ms = 0.f;
    QT_HIP(hipEventElapsedTime(&ms, ctx->prof.ev[i], ctx->prof.ev[i + 1]));
    t += ms;
  }
  *total_ms = t;
  *launches = (int64_t)(ctx->prof.used / 2);
  ctx->prof.used = 0;
  return QT_OK;
}

qt_status qt_ctx_counters(qt_ctx ctx, int64_t* out, int32_t n, int32_t reset) {
  QT_CHECK(ctx && out && n >= 0, QT_EINVAL, "qt_ctx_counters: bad argument");
  unsigned long long h[CNT_N] = {0};
  QT_HIP(hipMemcpyAsync(h, ctx->counters, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
  QT_HIP(hipStreamSynchronize(ctx->stream));
  for (int i = 0; i < n && i < CNT_N; ++i) out[i] = (int64_t)h[i];
  if (reset) QT_HIP(hipMemsetAsync(ctx->counters, 0, sizeof(h), ctx->stream));
  return QT_OK;
}

qt_status qt_ctx_sync(qt_ctx ctx) {
  QT_CHECK(ctx, QT_EINVAL, "qt_ctx_sync: null ctx");
  return check_status(ctx);
}

qt_status ls_iterate(qt_ctx ctx, const qt_operands* ops, qt_tt* e, const qt_solve_opts* opts,
                     int32_t n_iter, double* residual_out) {
  QT_CHECK(ctx && ops && e && opts, QT_EINVAL, "ls_iterate: null argument");
  enter(ctx);
  QT_TRY(validate_ops(ops, e));
  QT_CHECK(n_iter >= 0, QT_EINVAL, "ls_iterate: n_iter < 0");
  QT_TRY(validate_field_cap(e, opts->round.max_rank));
  Solver S;
  QT_TRY(solver_setup(ctx, ops, e, opts, S, ls_extra(e)));
  double* res_tmp = (double*)ws_take(ctx, sizeof(double) * e->batch);
  QT_CHECK(res_tmp, QT_ENOMEM, "ls_iterate: workspace");
  const bool graph = opts->graph && S.sketch && !S.learned && !S.logging && !ctx->prof.cls;
  // the first iteration runs eagerly (it also performs any one-time set-up)
  const int eager = graph ? std::min(n_iter, 1) : n_iter;
  for (int it = 0; it < eager; ++it) {
    QT_TRY(solver_step(ctx, ops, e, S, opts->round,
                       residual_out ? residual_out + (int64_t)it * e->batch : nullptr));
  }
  if (graph && n_iter > eager)
    QT_TRY(iterate_graph(ctx, ops, e, S, opts->round, n_iter - eager,
                         residual_out ? residual_out + (int64_t)eager * e->batch : nullptr,
                         res_tmp));
  return QT_OK;
}

qt_status homogenize(qt_ctx ctx, const qt_operands* ops, const qt_tt* k_sel, qt_tt* e,
                     const qt_solve_opts* opts, double* A_eff, int32_t* iters,
                     double* residuals) {
  QT_CHECK(ctx && ops && k_sel && e && opts && A_eff && iters, QT_EINVAL, "homogenize: null argument");
  enter(ctx);
  QT_TRY(validate_ops(ops, e));
  const int d = e->modes[0];   // components of the field (3 conductivity, 6 elasticity)
  for (int c = 0; c < d; ++c) {
    QT_TRY(tt_validate(&k_sel[c], "k_sel"));
    QT_CHECK((k_sel[c].batch == 1 || k_sel[c].batch == e->batch) && k_sel[c].n == e->n,
             QT_EINVAL, "homogenize: k_sel must hold 1 or batch trains");
  }
  QT_CHECK(opts->max_iter >= 1, QT_EINVAL, "homogenize: max_iter < 1");
  QT_TRY(validate_field_cap(e, opts->round.max_rank));
  const int B = e->batch;
  Solver S;
  QT_TRY(solver_setup(ctx, ops, e, opts, S, homogenize_extra(k_sel, e)));
  double* dres = (double*)ws_take(ctx, sizeof(double) * B);
  QT_CHECK(dres, QT_ENOMEM, "homogenize: workspace");
  QT_TRY(tt_copy(ctx, &ops->E, e));
  QT_TRY(qt_learn_reset(ctx));   // a new field: no previous-iteration features
  std::vector<double> hres(B);
  std::vector<int> done(B, 0), taken(B, 0);
  for (int b = 0; b < B; ++b) iters[b] = opts->max_iter;
  // A_eff[b][c] = Re <k_sel[c], e_b> / N^3 for the instances with take[b]
  // (the iterate of each field when it converges: fields of a batch that
  // converge early go on iterating with the others, so their A_eff is taken
  // at that iteration, as a separate solve of the field would take it)
  std::vector<double> hd(2 * B);
  const double N3 = std::ldexp(1.0, 3 * ops->L);
  auto take_aeff = [&](const std::vector<int>& take) -> qt_status {
    const size_t mark = ctx->ws_top;
    double* dd = (double*)ws_take(ctx, sizeof(double) * 2 * B);
    QT_CHECK(dd, QT_ENOMEM, "homogenize: workspace");
    const size_t top = ctx->ws_top;
    for (int c = 0; c < d; ++c) {
      ctx->ws_top = top;
      // dot workspace must fit in what setup reserved: environments are small
      qt_status s = dot_impl(ctx, &k_sel[c], e, dd, false);
      if (s == QT_ENOMEM || ctx->ws_top > ctx->ws_size) {
        ctx->ws_top = mark;
        set_error("homogenize: dot workspace");
        return QT_ENOMEM;
      }
      if (s != QT_OK) { ctx->ws_top = mark; return s; }
      QT_HIP(hipMemcpyAsync(hd.data(), dd, sizeof(double) * 2 * B, hipMemcpyDeviceToHost, ctx->stream));
      QT_HIP(hipStreamSynchronize(ctx->stream));
      for (int b = 0; b < B; ++b)
        if (take[b]) A_eff[(int64_t)b * d + c] = hd[2 * b] / N3;
    }
    ctx->ws_top = mark;
    for (int b = 0; b < B; ++b) taken[b] |= take[b];
    return QT_OK;
  };
  int it = 0;
  bool all = false;
  for (it = 1; it <= opts->max_iter && !all; ++it) {
    QT_TRY(solver_step(ctx, ops, e, S, opts->round, dres));
    QT_HIP(hipMemcpyAsync(hres.data(), dres, sizeof(double) * B, hipMemcpyDeviceToHost, ctx->stream));
    QT_TRY(check_status(ctx));
    all = true;
    std::vector<int> now(B, 0);
    bool any = false;
    for (int b = 0; b < B; ++b) {
      if (residuals) residuals[(int64_t)(it - 1) * B + b] = hres[b];
      if (!done[b] && hres[b] < opts->tol) { done[b] = 1; iters[b] = it; now[b] = 1; any = true; }
      all = all && done[b];
    }
    if (any) QT_TRY(take_aeff(now));
  }
  // fields that did not converge: the last iterate
  std::vector<int> rest(B, 0);
  bool any_rest = false;
  for (int b = 0; b < B; ++b) { rest[b] = !taken[b]; any_rest = any_rest || rest[b]; }
  if (any_rest) QT_TRY(take_aeff(rest));
  QT_TRY(check_status(ctx));
  return all ? QT_OK : QT_NOT_CONVERGED;
}

}  // extern "C"
