// Learned-rank state of a context (rank logs, features, predictions and the
// device-side acceptance of learned roundings), for a batch of B fields.
#pragma once

#include "kernels.h"
#include "sketch.h"

#define QT_RANK_FEATURES 24
// one row of the learned-rounding log: iteration, step, instance, learned
// error, reference error e_s of the step, kept (1) or fell back (0)
#define QT_LEARN_LOG_COLS 6

namespace qt {

struct LearnCtx {
  int n = 0, B = 0;
  double* rdiag = nullptr;      // [4][B][n+1][RD_MAX] sorted sketch-QR diagonals
  float* feat = nullptr;        // [2][4][B][QT_MAX_CORES][F] features (double-buffered)
  int32_t* pred = nullptr;      // [4][B][QT_MAX_CORES] predicted ranks
  int32_t* pcap = nullptr;      // [4][B][QT_MAX_CORES] plan widths (the predictions' caps)
  int32_t* pmax = nullptr;      // [4][QT_MAX_CORES] largest prediction over the batch
  double* ref = nullptr;        // [4][B] error estimate of the step's last SVD-truncated rounding
  int32_t* keep = nullptr;      // [B] the current learned rounding is kept
  int32_t* nfail = nullptr;     // [1] instances of the current rounding that fell back
  int cur = 0;                  // feature buffer written this iteration
  bool have_prev = false;       // features of a previous iteration exist
  std::vector<int32_t> pred_ell[4];              // host copy of the batch's predicted widths
  // predictor
  const float* params = nullptr;
  int pred_cls = 0;
  float quantile = 0.9f;
  // a learned rounding of instance b is kept iff error <= eps, or, where
  // ref[step][b] > eps (rank cap), iff error <= max(eps, accept * ref[step][b])
  float accept = 1.0f;
  // rank log (training data)
  float* log_feat = nullptr;
  int32_t* log_label = nullptr;
  int32_t* log_count = nullptr;
  int log_cap = 0;
  int log_cls = 8;
  // learned-rounding log (diagnostics): rows of QT_LEARN_LOG_COLS doubles
  double* rlog = nullptr;
  int32_t* rlog_count = nullptr;
  int rlog_cap = 0;
  uint64_t iter = 0;            // iteration number written to the rounding log
  float* feat_at(int buf, int step) {
    return feat + (((int64_t)buf * 4 + step) * B) * QT_MAX_CORES * QT_RANK_FEATURES;
  }
  int32_t* pred_at(int step) { return pred + (int64_t)step * B * QT_MAX_CORES; }
  int32_t* pcap_at(int step) { return pcap + (int64_t)step * B * QT_MAX_CORES; }
  double* rdiag_at(int step) { return rdiag + (int64_t)step * B * (n + 1) * RD_MAX; }
};

qt_status learn_ensure(qt_ctx ctx, int n, int B);
// device bytes of the learned state of n cores and B instances
size_t learn_state_bytes(int n, int B);
// features of this step's roundings from their sketch R diagonals; alt /
// alt_of (optional): widths of the instances b with alt_of[b] == 0
void learn_features(qt_ctx ctx, int step, const std::vector<int32_t>& ell, const double* xn2,
                    double eps, int rmax, const std::vector<int32_t>* alt = nullptr,
                    const int32_t* alt_of = nullptr);
void learn_log(qt_ctx ctx, int step, const int32_t* ranks);
// keep[b] = (err[b] <= reference of step s for instance b); counts the learned
// roundings and the fallbacks on the device; appends to the rounding log.
void learn_decide(qt_ctx ctx, int step, const double* err, double eps);
// ref[step][b] = est[b] for the instances that were rounded SVD-truncated
// (all when keep is null).
void learn_set_ref(qt_ctx ctx, int step, const double* est, const int32_t* keep);
// Widths of the next iteration: MLP inference on every instance's features,
// capped per (step, bond) by the plan widths, the largest over the batch to
// the host (pred_ell).
qt_status learn_predict(qt_ctx ctx, const std::vector<int32_t>* ells[4]);

}  // namespace qt

void qt_learn_free(qt_ctx ctx);
extern "C" qt_status qt_mlp_infer(qt_ctx ctx, const float* params, const float* X, int32_t n,
                                  int32_t n_in, int32_t n_cls, float quantile, float* logits,
                                  int32_t* ranks, const int32_t* rank_cap);
