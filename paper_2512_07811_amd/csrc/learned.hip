// Learned-rank state: rank logs for training, per-bond features for the MLP
// predictor, and the device-side acceptance of learned roundings, for a batch
// of fields (every array below has a slice per instance).
//
// Features of bond k at rounding step s (24 floats): the sorted magnitudes of
// the R-diagonal of the sketch QR at bond k (a randomized estimate of the bond
// spectrum; ||Y|| ~ sqrt(l) ||x|| for a unit Gaussian sketch) sampled at the
// 16 fixed positions j = (i+1) h - 1, h = ceil(r_max / 16) (clamped to the last
// column l - 1 of a narrower sketch) as log10(|R_jj| / (sqrt(l) ||x||)) / 16
// clipped to [-1, 0]; the per-bond threshold log10(eps / sqrt(n-1)) / 16; the sketch width
// l / r_max; the bond position k / (n-1); a one-hot of the step (Hadamard,
// SFFT, Green, inverse SFFT); log10(eps) / 16.  Label: the rank kept by the
// SVD truncation at that bond in the NEXT iteration (features lag by one
// iteration so that the learned path can predict before it sketches).
#include "learned.h"

namespace qt {

struct EllArr {
  int32_t v[QT_MAX_CORES + 1];
};

// grid (ceil((n-1)/64), B): bond k of instance b
// alt / alt_of (may be null): instances b with alt_of[b] == 0 had their
// sketch at the widths alt instead of ell (the instances whose learned
// rounding fell back and was redone at the plan widths).
__global__ void k_features(const double* __restrict__ rd, EllArr ell, EllArr alt,
                           const int32_t* __restrict__ alt_of, const double* xn2, int n,
                           double eps, int rmax, int step, float* __restrict__ feat) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x + 1;   // bond 1..n-1
  const int b = blockIdx.y;
  if (k >= n) return;
  const int l = max((alt_of && alt_of[b] == 0) ? alt.v[k] : ell.v[k], 1);
  const double xn = sqrt(fmax(xn2[b], 1e-300));
  float* f = feat + ((int64_t)b * QT_MAX_CORES + (k - 1)) * QT_RANK_FEATURES;
  const double* r = rd + ((int64_t)b * (n + 1) + k) * RD_MAX;
  const int h = max((rmax + 15) / 16, 1);
  for (int i = 0; i < 16; ++i) {
    const int q = min((i + 1) * h - 1, l - 1);
    const double d = r[min(q, RD_MAX - 1)] / (sqrt((double)l) * xn);
    double lg = log10(fmax(d, 1e-16));
    lg = fmin(fmax(lg, -16.0), 0.0);
    f[i] = (float)(lg / 16.0);
  }
  f[16] = (float)(log10(fmax(eps, 1e-16) / sqrt((double)(n - 1))) / 16.0);
  f[17] = (float)((double)l / (double)max(rmax, 1));
  f[18] = (float)((double)k / (double)(n - 1));
  for (int s = 0; s < 4; ++s) f[19 + s] = (s == step) ? 1.f : 0.f;
  f[23] = (float)(log10(fmax(eps, 1e-16)) / 16.0);
}

// Appends (previous-iteration features, this rounding's kept rank) for every
// bond of every instance.  grid (ceil((n-1)/64), B).
__global__ void k_log_append(const float* __restrict__ prev, const int32_t* __restrict__ ranks,
                             int n, int n_cls, float* __restrict__ log_feat,
                             int32_t* __restrict__ log_label, int32_t* count, int capacity) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x + 1;
  const int b = blockIdx.y;
  if (k >= n) return;
  const int idx = atomicAdd(count, 1);
  if (idx >= capacity) return;
  const float* src = prev + ((int64_t)b * QT_MAX_CORES + (k - 1)) * QT_RANK_FEATURES;
  for (int i = 0; i < QT_RANK_FEATURES; ++i)
    log_feat[(int64_t)idx * QT_RANK_FEATURES + i] = src[i];
  const int r = ranks[(int64_t)b * (n + 1) + k];
  log_label[idx] = min(max((r + 7) / 8, 1), n_cls) - 1;
}

// keep[b] = err[b] <= (ref > eps ? max(eps, accept ref) : eps); fallbacks and
// attempts counted; one row per instance appended to the rounding log.
__global__ void k_learn_decide(int B, const double* __restrict__ err, const double* __restrict__ ref,
                               double eps, double accept, int32_t* keep, int32_t* nfail,
                               unsigned long long* counters, double* rlog, int32_t* rlog_count,
                               int rlog_cap, double iter, int step) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b == 0) *nfail = 0;
  __syncthreads();
  if (b >= B) return;
  const double es = ref[b];
  const double lim = es > eps ? fmax(eps, accept * es) : eps;
  const int k = err[b] <= lim ? 1 : 0;
  keep[b] = k;
  if (!k) atomicAdd(nfail, 1);
  if (counters) {
    atomicAdd(counters + CNT_LEARNED, 1ull);
    if (!k) atomicAdd(counters + CNT_FALLBACK, 1ull);
  }
  if (rlog && rlog_count) {
    const int idx = atomicAdd(rlog_count, 1);
    if (idx < rlog_cap) {
      double* row = rlog + (int64_t)idx * QT_LEARN_LOG_COLS;
      row[0] = iter;
      row[1] = step;
      row[2] = b;
      row[3] = err[b];
      row[4] = es;
      row[5] = k;
    }
  }
}

__global__ void k_learn_set_ref(int B, const double* __restrict__ est,
                                const int32_t* __restrict__ keep, double* ref) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B && (!keep || !keep[b])) ref[b] = est[b];
}

// pmax[s][k] = max over instances of pred[s][b][k]
__global__ void k_pred_max(int B, const int32_t* __restrict__ pred, int32_t* pmax) {
  const int s = blockIdx.x, k = threadIdx.x;
  if (k >= QT_MAX_CORES) return;
  int v = 1;
  for (int b = 0; b < B; ++b)
    v = max(v, pred[((int64_t)s * B + b) * QT_MAX_CORES + k]);
  pmax[s * QT_MAX_CORES + k] = v;
}

// freed in the reverse order of allocation (caller-owned memory gives its
// blocks back from the low end of the persistent region)
static void learn_free_state(qt_ctx ctx, LearnCtx* L) {
  ctx_dev_free(ctx, L->nfail);
  ctx_dev_free(ctx, L->keep);
  ctx_dev_free(ctx, L->ref);
  ctx_dev_free(ctx, L->pmax);
  ctx_dev_free(ctx, L->pcap);
  ctx_dev_free(ctx, L->pred);
  ctx_dev_free(ctx, L->feat);
  ctx_dev_free(ctx, L->rdiag);
  L->rdiag = nullptr; L->feat = nullptr; L->pred = nullptr; L->pcap = nullptr;
  L->pmax = nullptr; L->ref = nullptr; L->keep = nullptr; L->nfail = nullptr;
}

size_t learn_state_bytes(int n, int B) {
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t nf = (size_t)2 * 4 * B * QT_MAX_CORES * QT_RANK_FEATURES;
  const size_t np = (size_t)4 * B * QT_MAX_CORES;
  return al(sizeof(double) * 4 * B * (n + 1) * RD_MAX) + al(sizeof(float) * nf) +
         2 * al(sizeof(int32_t) * np) + al(sizeof(int32_t) * 4 * QT_MAX_CORES) +
         al(sizeof(double) * 4 * B) + al(sizeof(int32_t) * B) + al(sizeof(int32_t));
}

qt_status learn_ensure(qt_ctx ctx, int n, int B) {
  QT_CHECK(n <= QT_MAX_CORES && B >= 1, QT_EINVAL, "learned state: too many cores");
  if (!ctx->learn) ctx->learn = new LearnCtx();
  LearnCtx* L = ctx->learn;
  if (L->n == n && L->B == B && L->rdiag) return QT_OK;
  QT_HIP(hipStreamSynchronize(ctx->stream));
  learn_free_state(ctx, L);
  L->n = 0;
  L->B = 0;
  const size_t nf = (size_t)2 * 4 * B * QT_MAX_CORES * QT_RANK_FEATURES;
  const size_t np = (size_t)4 * B * QT_MAX_CORES;
  QT_TRY(ctx_dev_alloc(ctx, (void**)&L->rdiag, sizeof(double) * 4 * B * (n + 1) * RD_MAX));
  QT_TRY(ctx_dev_alloc(ctx, (void**)&L->feat, sizeof(float) * nf));
  QT_TRY(ctx_dev_alloc(ctx, (void**)&L->pred, sizeof(int32_t) * np));
  QT_TRY(ctx_dev_alloc(ctx, (void**)&L->pcap, sizeof(int32_t) * np));
  QT_TRY(ctx_dev_alloc(ctx, (void**)&L->pmax, sizeof(int32_t) * 4 * QT_MAX_CORES));
  QT_TRY(ctx_dev_alloc(ctx, (void**)&L->ref, sizeof(double) * 4 * B));
  QT_TRY(ctx_dev_alloc(ctx, (void**)&L->keep, sizeof(int32_t) * B));
  QT_TRY(ctx_dev_alloc(ctx, (void**)&L->nfail, sizeof(int32_t)));
  QT_HIP(hipMemsetAsync(L->rdiag, 0, sizeof(double) * 4 * B * (n + 1) * RD_MAX, ctx->stream));
  QT_HIP(hipMemsetAsync(L->ref, 0, sizeof(double) * 4 * B, ctx->stream));
  L->n = n;
  L->B = B;
  L->have_prev = false;
  L->cur = 0;
  for (int s = 0; s < 4; ++s) L->pred_ell[s].clear();
  return QT_OK;
}

void learn_features(qt_ctx ctx, int step, const std::vector<int32_t>& ell, const double* xn2,
                    double eps, int rmax, const std::vector<int32_t>* alt, const int32_t* alt_of) {
  LearnCtx* L = ctx->learn;
  EllArr e{}, a{};
  for (size_t k = 0; k < ell.size() && k <= QT_MAX_CORES; ++k) e.v[k] = ell[k];
  if (alt)
    for (size_t k = 0; k < alt->size() && k <= QT_MAX_CORES; ++k) a.v[k] = (*alt)[k];
  dim3 grid((L->n + 62) / 64, L->B);
  k_features<<<grid, 64, 0, ctx->stream>>>(L->rdiag_at(step), e, a, alt ? alt_of : nullptr, xn2,
                                           L->n, eps, rmax, step, L->feat_at(L->cur, step));
}

void learn_log(qt_ctx ctx, int step, const int32_t* ranks) {
  LearnCtx* L = ctx->learn;
  if (!L->log_count || !L->have_prev) return;
  dim3 grid((L->n + 62) / 64, L->B);
  k_log_append<<<grid, 64, 0, ctx->stream>>>(L->feat_at(1 - L->cur, step), ranks, L->n,
                                             L->log_cls, L->log_feat, L->log_label, L->log_count,
                                             L->log_cap);
}

void learn_decide(qt_ctx ctx, int step, const double* err, double eps) {
  LearnCtx* L = ctx->learn;
  const int B = L->B;
  // one block: the fail count is reset and accumulated in the same launch
  k_learn_decide<<<1, 1024, 0, ctx->stream>>>(B, err, L->ref + (int64_t)step * B, eps,
                                              (double)L->accept, L->keep, L->nfail,
                                              ctx->counters, L->rlog, L->rlog_count, L->rlog_cap,
                                              (double)L->iter, step);
}

void learn_set_ref(qt_ctx ctx, int step, const double* est, const int32_t* keep) {
  LearnCtx* L = ctx->learn;
  k_learn_set_ref<<<(L->B + 127) / 128, 128, 0, ctx->stream>>>(L->B, est, keep,
                                                               L->ref + (int64_t)step * L->B);
}

qt_status learn_predict(qt_ctx ctx, const std::vector<int32_t>* ells[4]) {
  LearnCtx* L = ctx->learn;
  const int n = L->n, B = L->B;
  // caps = plan widths per (step, instance, bond); features of bond k at row k-1
  std::vector<int32_t> caps((size_t)4 * B * QT_MAX_CORES, 1);
  for (int s = 0; s < 4; ++s)
    for (int b = 0; b < B; ++b)
      for (int k = 1; k < n; ++k)
        caps[((size_t)s * B + b) * QT_MAX_CORES + k - 1] = (*ells[s])[k];
  QT_HIP(hipMemcpyAsync(L->pcap, caps.data(), sizeof(int32_t) * caps.size(),
                        hipMemcpyHostToDevice, ctx->stream));
  QT_TRY(qt_mlp_infer(ctx, L->params, L->feat_at(L->cur, 0), 4 * B * QT_MAX_CORES,
                      QT_RANK_FEATURES, L->pred_cls, L->quantile, nullptr, L->pred, L->pcap));
  k_pred_max<<<4, QT_MAX_CORES, 0, ctx->stream>>>(B, L->pred, L->pmax);
  std::vector<int32_t> pr(4 * QT_MAX_CORES);
  QT_HIP(hipMemcpyAsync(pr.data(), L->pmax, sizeof(int32_t) * pr.size(), hipMemcpyDeviceToHost,
                        ctx->stream));
  QT_HIP(hipStreamSynchronize(ctx->stream));
  for (int s = 0; s < 4; ++s) {
    L->pred_ell[s].assign(n + 1, 1);
    for (int k = 1; k < n; ++k) L->pred_ell[s][k] = pr[s * QT_MAX_CORES + k - 1];
  }
  return QT_OK;
}

}  // namespace qt

using namespace qt;

extern "C" qt_status qt_ranklog_enable(qt_ctx ctx, int32_t capacity, int32_t n_cls) {
  QT_CHECK(ctx && capacity >= 0 && n_cls >= 2, QT_EINVAL, "qt_ranklog_enable: bad argument");
  if (!ctx->learn) ctx->learn = new LearnCtx();
  LearnCtx* L = ctx->learn;
  QT_HIP(hipStreamSynchronize(ctx->stream));
  ctx->ws_top = 0;   // between calls: nothing lives in the arena
  ctx_dev_free(ctx, L->log_count);
  ctx_dev_free(ctx, L->log_label);
  ctx_dev_free(ctx, L->log_feat);
  L->log_feat = nullptr; L->log_label = nullptr; L->log_count = nullptr; L->log_cap = 0;
  if (capacity == 0) return QT_OK;
  QT_TRY(ctx_dev_alloc(ctx, (void**)&L->log_feat,
                       sizeof(float) * (size_t)capacity * QT_RANK_FEATURES));
  QT_TRY(ctx_dev_alloc(ctx, (void**)&L->log_label, sizeof(int32_t) * (size_t)capacity));
  QT_TRY(ctx_dev_alloc(ctx, (void**)&L->log_count, sizeof(int32_t)));
  QT_HIP(hipMemset(L->log_count, 0, sizeof(int32_t)));
  L->log_cap = capacity;
  L->log_cls = n_cls;
  return QT_OK;
}

extern "C" qt_status qt_ranklog_get(qt_ctx ctx, float* features, int32_t* labels,
                                    int32_t max_count, int32_t* count) {
  QT_CHECK(ctx && count && max_count >= 0, QT_EINVAL, "qt_ranklog_get: bad argument");
  QT_CHECK(ctx->learn && ctx->learn->log_count, QT_EINVAL, "qt_ranklog_get: log not enabled");
  LearnCtx* L = ctx->learn;
  int32_t c = 0;
  QT_HIP(hipMemcpyAsync(&c, L->log_count, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
  QT_HIP(hipStreamSynchronize(ctx->stream));
  c = std::min(c, L->log_cap);
  *count = c;
  const int32_t m = std::min(c, max_count);
  if (m > 0) {
    QT_CHECK(features && labels, QT_EINVAL, "qt_ranklog_get: null output buffer");
    QT_HIP(hipMemcpyAsync(features, L->log_feat, sizeof(float) * (size_t)m * QT_RANK_FEATURES,
                          hipMemcpyDeviceToDevice, ctx->stream));
    QT_HIP(hipMemcpyAsync(labels, L->log_label, sizeof(int32_t) * (size_t)m,
                          hipMemcpyDeviceToDevice, ctx->stream));
  }
  return QT_OK;
}

extern "C" qt_status qt_learn_log_enable(qt_ctx ctx, int32_t capacity) {
  QT_CHECK(ctx && capacity >= 0, QT_EINVAL, "qt_learn_log_enable: bad argument");
  if (!ctx->learn) ctx->learn = new LearnCtx();
  LearnCtx* L = ctx->learn;
  QT_HIP(hipStreamSynchronize(ctx->stream));
  ctx->ws_top = 0;
  ctx_dev_free(ctx, L->rlog_count);
  ctx_dev_free(ctx, L->rlog);
  L->rlog = nullptr; L->rlog_count = nullptr; L->rlog_cap = 0;
  if (capacity == 0) return QT_OK;
  QT_TRY(ctx_dev_alloc(ctx, (void**)&L->rlog,
                       sizeof(double) * (size_t)capacity * QT_LEARN_LOG_COLS));
  QT_TRY(ctx_dev_alloc(ctx, (void**)&L->rlog_count, sizeof(int32_t)));
  QT_HIP(hipMemset(L->rlog_count, 0, sizeof(int32_t)));
  L->rlog_cap = capacity;
  return QT_OK;
}

extern "C" qt_status qt_learn_log_get(qt_ctx ctx, double* rows, int32_t max_rows,
                                      int32_t* count) {
  QT_CHECK(ctx && count && max_rows >= 0, QT_EINVAL, "qt_learn_log_get: bad argument");
  QT_CHECK(ctx->learn && ctx->learn->rlog_count, QT_EINVAL, "qt_learn_log_get: log not enabled");
  LearnCtx* L = ctx->learn;
  int32_t c = 0;
  QT_HIP(hipMemcpyAsync(&c, L->rlog_count, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
  QT_HIP(hipStreamSynchronize(ctx->stream));
  c = std::min(c, L->rlog_cap);
  *count = c;
  const int32_t m = std::min(c, max_rows);
  if (m > 0) {
    QT_CHECK(rows, QT_EINVAL, "qt_learn_log_get: null output buffer");
    QT_HIP(hipMemcpyAsync(rows, L->rlog, sizeof(double) * (size_t)m * QT_LEARN_LOG_COLS,
                          hipMemcpyDeviceToHost, ctx->stream));
    QT_HIP(hipStreamSynchronize(ctx->stream));
  }
  return QT_OK;
}

extern "C" qt_status qt_set_predictor(qt_ctx ctx, const float* params, int32_t n_cls,
                                      float quantile, float accept_factor) {
  QT_CHECK(ctx && n_cls >= 2 && n_cls <= 32 && quantile > 0.f && quantile <= 1.f &&
               accept_factor <= 2.f, QT_EINVAL, "qt_set_predictor: bad argument");
  if (!ctx->learn) ctx->learn = new LearnCtx();
  LearnCtx* L = ctx->learn;
  L->params = params;
  L->pred_cls = n_cls;
  L->quantile = quantile;
  L->accept = accept_factor > 0.f ? accept_factor : 1.0f;
  return QT_OK;
}

extern "C" qt_status qt_learn_reset(qt_ctx ctx) {
  QT_CHECK(ctx, QT_EINVAL, "qt_learn_reset: null ctx");
  if (ctx->learn) {
    LearnCtx* L = ctx->learn;
    L->have_prev = false;
    for (int s = 0; s < 4; ++s) L->pred_ell[s].clear();
    if (L->ref) QT_HIP(hipMemsetAsync(L->ref, 0, sizeof(double) * 4 * L->B, ctx->stream));
  }
  return QT_OK;
}

void qt_learn_free(qt_ctx ctx) {
  if (!ctx || !ctx->learn) return;
  LearnCtx* L = ctx->learn;
  learn_free_state(ctx, L);
  ctx_dev_free(ctx, L->log_count);
  ctx_dev_free(ctx, L->log_label);
  ctx_dev_free(ctx, L->log_feat);
  ctx_dev_free(ctx, L->rlog_count);
  ctx_dev_free(ctx, L->rlog);
  delete L;
  ctx->learn = nullptr;
}
