// Drivers of the product-aware rounding: the sketch followed either by the
// right-to-left truncated-SVD sweep with the remaining error budget
// (QT_ROUND_SKETCH) or by nothing (QT_ROUND_LEARNED: fixed, predicted ranks),
// with the exact a-posteriori error ||x - x~||^2 = ||x||^2 - ||x~||^2 of the
// orthogonal projection.
#include <algorithm>

#include "kernels.h"
#include "round.h"
#include "sketch.h"

namespace qt {

// e_s^2 = max(||x||^2 - ||x~||^2, 0) (exact for the orthogonal projection of the
// sketch).  The truncation of interior bonds moves the result's left
// interfaces out of the sketch's span, so its error is not orthogonal to the
// projection error: the budget is split linearly (triangle inequality),
// delta[b] = max(eps ||x|| - e_s, 0)/sqrt(n-1), so that
// ||x - z|| <= e_s + sqrt(sum of discarded tails^2) <= eps ||x||.
// Relative floor of the truncation threshold for eps > 0: singular values of
// rounding noise (about 1e-16 of the norm each) never survive a truncation.
constexpr double QT_NOISE_FLOOR = 1e-14;

__global__ void k_budget(int batch, int nbonds, double eps, const double* xn2, const double* yn2,
                         double* delta, double* disc2, double* es2, int32_t* fail,
                         unsigned long long* counters) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  double e2 = fmax(xn2[b] - yn2[b], 0.0);
  double bud = eps * sqrt(fmax(xn2[b], 0.0)) - sqrt(e2);
  double dl = nbonds > 0 ? fmax(bud, 0.0) / sqrt((double)nbonds) : 0.0;
  // eps > 0: no bond keeps directions below the rounding-noise floor, also
  // when the projection alone exhausts the budget (the rank cap binds)
  if (eps > 0.0 && nbonds > 0) dl = fmax(dl, QT_NOISE_FLOOR * sqrt(xn2[b]));
  delta[b] = dl;
  disc2[b] = 0.0;
  es2[b] = e2;
  if (fail) fail[b] = bud < 0.0 ? 1 : 0;
  if (bud < 0.0 && counters) atomicAdd(counters + CNT_SKETCH_FAIL, 1ull);
}

// Reported error: (e_s + sqrt(discarded tails^2)) / ||x||, a rigorous upper
// bound of ||x - z|| / ||x|| (exact when nothing is truncated after the sketch);
// est (optional): sqrt(e_s^2 + tails^2) / ||x||, the estimate that treats the
// two errors as orthogonal (within a few per cent of the true error in the
// capped tests), used where two roundings' errors are compared.
__global__ void k_sketch_err(int batch, const double* xn2, const double* es2, const double* disc2,
                             double* err, double* est) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  double x = xn2[b];
  const double d2 = disc2 ? disc2[b] : 0.0;
  if (err) err[b] = x > 0.0 ? (sqrt(es2[b]) + sqrt(d2)) / sqrt(x) : 0.0;
  if (est) est[b] = x > 0.0 ? sqrt((es2[b] + d2) / x) : 0.0;
}

std::vector<int32_t> sketch_ranks(const qt_mpo* A, const qt_tt* y, int rmax, int oversample) {
  const int n = y->n;
  std::vector<int32_t> ell(n + 1, 1);
  for (int k = 1; k < n; ++k) {
    double left = 1, right = 1;
    for (int j = 0; j < k; ++j) left *= y->modes[j];
    for (int j = k; j < n; ++j) right *= y->modes[j];
    int64_t nat = (int64_t)std::min(std::min(left, right), 1e9);
    int64_t prod = (int64_t)A->ranks[k] * y->cap[k];
    int64_t want = rmax > 0 ? (int64_t)rmax + std::max(oversample, 0) : prod;
    ell[k] = (int32_t)std::max<int64_t>(1, std::min({nat, prod, want}));
  }
  return ell;
}

SRoundWs sround_ws_layout(const qt_mpo* A, const qt_tt* y, const qt_tt* out,
                          const std::vector<int32_t>& ell, int lmax_cap) {
  SRoundWs w;
  SketchWs sk = sketch_ws_layout(A, y, ell);
  RoundWs rw = round_ws_layout(out, lmax_cap);
  w.om_off.assign(y->n, 0);
  int64_t o = 0;
  for (int k = 0; k < y->n; ++k) {
    w.om_off[k] = o;
    o += ((int64_t)ell[k] * y->modes[k] * ell[k + 1] + 31) & ~(int64_t)31;
  }
  w.om_tot = std::max<int64_t>(o, 1);
  const int B = y->batch;
  w.sweep = rw;
  w.bytes = sk.bytes + rw.sweep_bytes +
            sizeof(cplx) * (w.om_tot + (int64_t)B * (2 * rw.slot + rw.vv + rw.carry)) +
            sizeof(double) * B * 6 + sizeof(int32_t) * B * (y->n + 2) * 2 + 16 * 256;
  return w;
}

qt_status sround_impl(qt_ctx ctx, const qt_mpo* A, const qt_tt* y, const cplx* omega_in,
                      const std::vector<int64_t>* om_off_in, const std::vector<int32_t>& ell,
                      const qt_round_opts* o, const double* xn2, qt_tt* out, double* err_out,
                      int32_t* fail, uint64_t stream_id, double* svlog, int64_t svb,
                      int64_t svi, double* rdiag, double* err_est) {
  const int n = y->n, B = y->batch;
  hipStream_t st = ctx->stream;
  const int lmax_cap = o->max_rank > 0 ? o->max_rank : (1 << 30);
  SRoundWs w = sround_ws_layout(A, y, out, ell, lmax_cap);
  const cplx* omega = omega_in;
  const std::vector<int64_t>* om_off = om_off_in;
  if (!omega) {
    cplx* om = (cplx*)ws_take(ctx, sizeof(cplx) * w.om_tot);
    QT_CHECK(om, QT_ENOMEM, "sketch rounding: workspace too small");
    gauss_fill(st, w.om_tot, o->seed, stream_id, om, ctx->capturing ? ctx->dev_iter : nullptr);
    omega = om;
    om_off = &w.om_off;
  }
  double* yn2 = (double*)ws_take(ctx, sizeof(double) * B);
  double* delta = (double*)ws_take(ctx, sizeof(double) * B);
  double* disc2 = (double*)ws_take(ctx, sizeof(double) * B);
  double* es2 = (double*)ws_take(ctx, sizeof(double) * B);
  int32_t* rkl = (int32_t*)ws_take(ctx, sizeof(int32_t) * B * (n + 1));
  QT_CHECK(yn2 && delta && disc2 && es2 && rkl, QT_ENOMEM, "sketch rounding: workspace too small");
  QT_TRY(sketch_impl(ctx, A, y, omega, *om_off, ell, out, yn2, rdiag,
                     o->precision == QT_PREC_F32));
  k_budget<<<(B + 127) / 128, 128, 0, st>>>(B, n - 1, o->eps, xn2, yn2, delta, disc2, es2, fail,
                                            ctx->counters);
  if (o->mode == QT_ROUND_SKETCH && n > 1) {
    cplx* scratch = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.sweep.slot);
    cplx* Bsv = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.sweep.slot);
    cplx* V = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.sweep.vv);
    cplx* Cb = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.sweep.carry);
    QT_CHECK(scratch && Bsv && V && Cb, QT_ENOMEM, "sketch rounding: workspace too small");
    copy_i32(st, (int64_t)B * (n + 1), out->ranks, rkl);
    SweepBufs buf{scratch, Bsv, V, Cb, w.sweep.slot, w.sweep.vv, w.sweep.carry};
    QT_TRY(take_sweep_extra(ctx, B, w.sweep, buf));
    const int sweeps = o->jacobi_max_sweeps > 0 ? o->jacobi_max_sweeps : ctx->jacobi_default;
    QT_TRY(right_sweep_impl(ctx, out, rkl, (const cplx*)out->data + out->offsets[n - 1],
                            out->inst_stride, buf, delta, disc2, lmax_cap, sweeps, svlog, svb, svi));
    if (err_out || err_est)
      k_sketch_err<<<(B + 127) / 128, 128, 0, st>>>(B, xn2, es2, disc2, err_out, err_est);
  } else {
    if (err_out || err_est)
      k_sketch_err<<<(B + 127) / 128, 128, 0, st>>>(B, xn2, es2, nullptr, err_out, err_est);
  }
  QT_HIP(hipGetLastError());
  return QT_OK;
}

static qt_status validate_mpo(const qt_mpo* A, const qt_tt* y) {
  QT_CHECK(A->n == y->n, QT_EINVAL, "operator and train core counts differ");
  QT_CHECK(A->ranks[0] == 1 && A->ranks[A->n] == 1, QT_EINVAL, "operator boundary ranks");
  QT_CHECK(A->inst_stride >= 0 && A->inst_group >= 1, QT_EINVAL,
           "operator instance stride/group");
  for (int k = 0; k < y->n; ++k) {
    QT_CHECK(A->modes_in[k] == y->modes[k] && A->modes_out[k] == y->modes[k], QT_EINVAL,
             "operator modes must equal train modes (square operator)");
  }
  return QT_OK;
}

}  // namespace qt

using namespace qt;

extern "C" qt_status tt_sketch_round(qt_ctx ctx, const qt_mpo* A, const qt_tt* y,
                                     const qt_tt* omega, const qt_round_opts* opts,
                                     const double* xnorm2, qt_tt* out, double* err_out,
                                     int32_t* fail_out) {
  qt::enter(ctx);
  QT_CHECK(ctx && A && y && opts && xnorm2 && out, QT_EINVAL, "tt_sketch_round: null argument");
  QT_TRY(tt_validate(y, "y"));
  QT_TRY(tt_validate(out, "out"));
  QT_TRY(validate_mpo(A, y));
  QT_CHECK(out->n == y->n && out->batch == y->batch, QT_EINVAL, "tt_sketch_round: out shape");
  QT_CHECK(out->data != y->data, QT_EINVAL, "tt_sketch_round: out aliases y");
  QT_CHECK(opts->mode == QT_ROUND_SKETCH || opts->mode == QT_ROUND_LEARNED, QT_EINVAL,
           "tt_sketch_round: mode must be QT_ROUND_SKETCH or QT_ROUND_LEARNED");
  QT_CHECK(opts->precision == QT_PREC_F64 || opts->precision == QT_PREC_F32, QT_EINVAL,
           "tt_sketch_round: precision must be QT_PREC_F64 or QT_PREC_F32");
  const int n = y->n;
  std::vector<int32_t> ell;
  std::vector<int64_t> off;
  if (omega) {
    QT_TRY(tt_validate(omega, "omega"));
    QT_CHECK(omega->n == n && omega->batch == 1, QT_EINVAL, "tt_sketch_round: omega shape");
    ell.assign(omega->cap, omega->cap + n + 1);
    off.assign(omega->offsets, omega->offsets + n);
  } else {
    ell = sketch_ranks(A, y, opts->max_rank, opts->oversample);
  }
  for (int k = 0; k <= n; ++k)
    QT_CHECK(out->cap[k] >= ell[k], QT_ECAPACITY, "tt_sketch_round: out capacity below sketch ranks");
  ctx->ws_top = 0;
  const int lmax_cap = opts->max_rank > 0 ? opts->max_rank : (1 << 30);
  QT_TRY(ws_reserve(ctx, sround_ws_layout(A, y, out, ell, lmax_cap).bytes));
  return sround_impl(ctx, A, y, omega ? (const cplx*)omega->data : nullptr, omega ? &off : nullptr,
                     ell, opts, xnorm2, out, err_out, fail_out, 0, nullptr, 0, 0);
}

extern "C" qt_status tt_sandwich(qt_ctx ctx, const qt_mpo* Q, const qt_tt* y, double scale,
                                 double* out) {
  qt::enter(ctx);
  QT_CHECK(ctx && Q && y && out, QT_EINVAL, "tt_sandwich: null argument");
  QT_TRY(tt_validate(y, "y"));
  QT_TRY(validate_mpo(Q, y));
  ctx->ws_top = 0;
  QT_TRY(ws_reserve(ctx, sandwich_ws_layout(Q, y).bytes));
  return sandwich_impl(ctx, Q, y, scale, out);
}
