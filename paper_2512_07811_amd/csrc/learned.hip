// Learned-rank state: rank logs for training, per-bond features for the MLP
// predictor, and the a-posteriori acceptance bookkeeping of the learned path.
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

__global__ void k_features(const double* __restrict__ rd, EllArr ell, const double* xn2, int n,
                           double eps, int rmax, int step, float* __restrict__ feat) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x + 1;   // bond 1..n-1
  if (k >= n) return;
  const int l = max(ell.v[k], 1);
  const double xn = sqrt(fmax(xn2[0], 1e-300));
  float* f = feat + (int64_t)(k - 1) * QT_RANK_FEATURES;
  const double* r = rd + (int64_t)k * RD_MAX;
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

// Appends (previous-iteration features, this rounding's kept rank) for every bond.
__global__ void k_log_append(const float* __restrict__ prev, const int32_t* __restrict__ ranks,
                             int n, int n_cls, float* __restrict__ log_feat,
                             int32_t* __restrict__ log_label, int32_t* count, int capacity) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x + 1;
  if (k >= n) return;
  const int idx = atomicAdd(count, 1);
  if (idx >= capacity) return;
  for (int i = 0; i < QT_RANK_FEATURES; ++i)
    log_feat[(int64_t)idx * QT_RANK_FEATURES + i] = prev[(int64_t)(k - 1) * QT_RANK_FEATURES + i];
  const int r = ranks[k];
  log_label[idx] = min(max((r + 7) / 8, 1), n_cls) - 1;
}

qt_status learn_ensure(qt_ctx ctx, int n) {
  QT_CHECK(n <= QT_MAX_CORES, QT_EINVAL, "learned state: too many cores");
  if (!ctx->learn) ctx->learn = new LearnCtx();
  LearnCtx* L = ctx->learn;
  if (L->n == n && L->rdiag) return QT_OK;
  if (L->rdiag) {
    QT_HIP(hipStreamSynchronize(ctx->stream));
    hipFree(L->rdiag);
    hipFree(L->feat);
    hipFree(L->pred);
  }
  L->n = n;
  QT_HIP(hipMalloc((void**)&L->rdiag, sizeof(double) * 4 * (n + 1) * RD_MAX));
  QT_HIP(hipMemset(L->rdiag, 0, sizeof(double) * 4 * (n + 1) * RD_MAX));
  QT_HIP(hipMalloc((void**)&L->feat, sizeof(float) * 2 * 4 * QT_MAX_CORES * QT_RANK_FEATURES));
  QT_HIP(hipMalloc((void**)&L->pred, sizeof(int32_t) * 2 * 4 * QT_MAX_CORES));
  L->have_prev = false;
  L->cur = 0;
  return QT_OK;
}

void learn_features(qt_ctx ctx, int step, const std::vector<int32_t>& ell, const double* xn2,
                    double eps, int rmax) {
  LearnCtx* L = ctx->learn;
  EllArr e{};
  for (size_t k = 0; k < ell.size() && k <= QT_MAX_CORES; ++k) e.v[k] = ell[k];
  k_features<<<1, 64, 0, ctx->stream>>>(L->rdiag + (int64_t)step * (L->n + 1) * RD_MAX, e, xn2,
                                        L->n, eps, rmax, step, L->feat_at(L->cur, step));
}

void learn_log(qt_ctx ctx, int step, const int32_t* ranks) {
  LearnCtx* L = ctx->learn;
  if (!L->log_count || !L->have_prev) return;
  k_log_append<<<1, 64, 0, ctx->stream>>>(L->feat_at(1 - L->cur, step), ranks, L->n, L->log_cls,
                                          L->log_feat, L->log_label, L->log_count, L->log_cap);
}

}  // namespace qt

using namespace qt;

extern "C" qt_status qt_ranklog_enable(qt_ctx ctx, int32_t capacity, int32_t n_cls) {
  QT_CHECK(ctx && capacity >= 0 && n_cls >= 2, QT_EINVAL, "qt_ranklog_enable: bad argument");
  if (!ctx->learn) ctx->learn = new LearnCtx();
  LearnCtx* L = ctx->learn;
  QT_HIP(hipStreamSynchronize(ctx->stream));
  if (L->log_feat) { hipFree(L->log_feat); hipFree(L->log_label); hipFree(L->log_count); }
  L->log_feat = nullptr; L->log_label = nullptr; L->log_count = nullptr; L->log_cap = 0;
  if (capacity == 0) return QT_OK;
  QT_HIP(hipMalloc((void**)&L->log_feat, sizeof(float) * (size_t)capacity * QT_RANK_FEATURES));
  QT_HIP(hipMalloc((void**)&L->log_label, sizeof(int32_t) * (size_t)capacity));
  QT_HIP(hipMalloc((void**)&L->log_count, sizeof(int32_t)));
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
    ctx->learn->have_prev = false;
    for (int s = 0; s < 4; ++s) {
      ctx->learn->pred_ell[s].clear();
      ctx->learn->ref_err[s] = 0.0;
    }
  }
  return QT_OK;
}

void qt_learn_free(qt_ctx ctx) {
  if (!ctx || !ctx->learn) return;
  LearnCtx* L = ctx->learn;
  if (L->rdiag) { hipFree(L->rdiag); hipFree(L->feat); hipFree(L->pred); }
  if (L->log_feat) { hipFree(L->log_feat); hipFree(L->log_label); hipFree(L->log_count); }
  delete L;
  ctx->learn = nullptr;
}
