// Learned-rank state of a context (rank logs, features, predictions).
#pragma once

#include "kernels.h"
#include "sketch.h"

#define QT_RANK_FEATURES 24

namespace qt {

struct LearnCtx {
  int n = 0;
  double* rdiag = nullptr;      // [4][n+1][RD_MAX] sorted sketch-QR diagonals
  float* feat = nullptr;        // [2][4][QT_MAX_CORES][F] features (double-buffered)
  int32_t* pred = nullptr;      // [2][4][QT_MAX_CORES] predicted ranks / caps
  int cur = 0;                  // feature buffer written this iteration
  bool have_prev = false;       // features of a previous iteration exist
  std::vector<int32_t> pred_ell[4];              // host copy of the predicted ranks
  double ref_err[4] = {0.0, 0.0, 0.0, 0.0};     // last SVD-truncated error per step
  // predictor
  const float* params = nullptr;
  int pred_cls = 0;
  float quantile = 0.9f;
  // a learned rounding is kept iff error <= eps, or, where ref_err[step] > eps
  // (rank cap), iff error <= max(eps, accept * ref_err[step])
  float accept = 1.0f;
  long long fallbacks = 0;
  long long learned_roundings = 0;
  // rank log (training data)
  float* log_feat = nullptr;
  int32_t* log_label = nullptr;
  int32_t* log_count = nullptr;
  int log_cap = 0;
  int log_cls = 8;
  float* feat_at(int buf, int step) {
    return feat + ((int64_t)buf * 4 + step) * QT_MAX_CORES * QT_RANK_FEATURES;
  }
  int32_t* pred_at(int buf, int step) { return pred + ((int64_t)buf * 4 + step) * QT_MAX_CORES; }
};

qt_status learn_ensure(qt_ctx ctx, int n);
void learn_features(qt_ctx ctx, int step, const std::vector<int32_t>& ell, const double* xn2,
                    double eps, int rmax);
void learn_log(qt_ctx ctx, int step, const int32_t* ranks);

}  // namespace qt

void qt_learn_free(qt_ctx ctx);
extern "C" qt_status qt_mlp_infer(qt_ctx ctx, const float* params, const float* X, int32_t n,
                                  int32_t n_in, int32_t n_cls, float quantile, float* logits,
                                  int32_t* ranks, const int32_t* rank_cap);
