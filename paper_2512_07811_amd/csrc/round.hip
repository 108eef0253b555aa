// TT rounding on device (Sec. 2.2 of arXiv 2512.07811):
//   left sweep:  [Q_k, R_k] = qr(core_k as (r'_k p_k x r_{k+1})); core_{k+1} <- R_k core_{k+1}
//   ||x|| = ||core_{n-1}||;  delta = eps ||x|| / sqrt(n-1)
//   right sweep: SVD of core_k as (r'_k x p_k l_{k+1}); keep the smallest l whose
//                discarded tail <= delta (cap max_rank); core_k <- V^H[:l];
//                core_{k-1} <- core_{k-1} U[:, :l] Sigma[:l]
// Every size is read by the kernels from device rank arrays, so the sweep is a
// fixed launch sequence with no host synchronisation.
#include "kernels.h"
#include "round.h"
#include "sketch.h"

namespace qt {

__global__ void k_init_left(int n, int batch, const int32_t* ranks, int32_t* rk_left) {
  int b = blockIdx.x;
  if (b >= batch) return;
  for (int k = threadIdx.x; k <= n; k += blockDim.x)
    rk_left[(int64_t)b * (n + 1) + k] = (k == 0 || k == n) ? 1 : ranks[(int64_t)b * (n + 1) + k];
}

RoundWs round_ws_layout(const qt_tt* x, int lmax_cap, bool polar) {
  RoundWs w;
  const int n = x->n;
  int64_t slot = 1, rr = 1, vv = 1, carry = 1, tau = 1;
  for (int k = 0; k < n; ++k) {
    int64_t s = (int64_t)x->cap[k] * x->modes[k] * x->cap[k + 1];
    slot = std::max(slot, s);
    rr = std::max<int64_t>(rr, (int64_t)x->cap[k + 1] * x->cap[k + 1]);
    int lnext = std::min(x->cap[k + 1], lmax_cap);
    int64_t nb = std::min<int64_t>(x->cap[k], (int64_t)x->modes[k] * lnext);
    vv = std::max(vv, nb * nb);
    carry = std::max<int64_t>(carry, (int64_t)x->cap[k] * std::min(x->cap[k], lmax_cap));
    tau = std::max<int64_t>(tau, x->cap[k + 1]);
    w.max_nb = std::max<int64_t>(w.max_nb, nb);
    const int64_t mbk = std::max<int64_t>(x->cap[k], (int64_t)x->modes[k] * lnext);
    if (k >= 1 && nb <= 1024 && qr_blocked_wanted((int)mbk, (int)nb)) {
      // the SVD's first QR (mbk x nb) and second QR (nb x nb): the panel
      // width depends on the rows, so either may need more
      for (const int64_t rows : {mbk, nb}) {
        if (rows == nb && !qr_blocked_wanted((int)nb, (int)nb)) continue;
        int64_t v, t, wq;
        qr_blocked_ws_elems((int)rows, (int)nb, &v, &t, &wq);
        w.sb_v = std::max(w.sb_v, v);
        w.sb_t = std::max(w.sb_t, t);
        w.sb_w = std::max(w.sb_w, wq);
        w.sb_tau = std::max(w.sb_tau, qr_blocked_tau_elems((int)rows, (int)nb));
      }
    }
    if (k < n - 1 && qr_blocked_wanted(x->cap[k] * x->modes[k], x->cap[k + 1])) {
      int64_t v, t, wq;
      qr_blocked_ws_elems(x->cap[k] * x->modes[k], x->cap[k + 1], &v, &t, &wq);
      w.qb_v = std::max(w.qb_v, v);
      w.qb_t = std::max(w.qb_t, t);
      w.qb_w = std::max(w.qb_w, wq);
      w.qb_tau = std::max(w.qb_tau, qr_blocked_tau_elems(x->cap[k] * x->modes[k], x->cap[k + 1]));
    }
  }
  w.slot = slot; w.rr = rr; w.vv = vv; w.carry = carry; w.tau = tau;
  const int B = x->batch;
  w.max_nb = std::max<int64_t>(w.max_nb, 1);
  // tau: nb reflector scalars, then 8 sizes of the SVD's second QR and
  // finishing products (4 doubles)
  w.sweep_bytes = sizeof(cplx) * B * (slot + vv) + sizeof(double) * B * (w.max_nb + 4) + 3 * 256;
  if (w.sb_v > 0)
    w.sweep_bytes += sizeof(cplx) * B * (w.sb_v + w.sb_t + 2 * w.sb_w) +
                     sizeof(double) * B * w.sb_tau + sizeof(int32_t) * B * 4 + 7 * 256;
  w.bytes = sizeof(cplx) * B * (3 * slot + rr + vv + carry) + sizeof(double) * B * (tau + 4) +
            sizeof(int32_t) * B * (n + 1) + 16 * 256 + w.sweep_bytes;
  if (w.qb_v > 0)
    w.bytes += sizeof(cplx) * B * (w.qb_v + w.qb_t + 2 * w.qb_w) + sizeof(double) * B * w.qb_tau +
               sizeof(int32_t) * B + 8 * 256;
  if (polar && n > 1) {
    int nc = 1, mc = 1;
    for (int k = 1; k < n; ++k) {
      nc = std::max(nc, x->cap[k]);
      mc = std::max(mc, x->modes[k] * std::min(x->cap[k + 1], lmax_cap));
    }
    w.polar = true;
    w.pol = polar_sizes(nc, mc, std::min(nc, lmax_cap));
    w.bytes += polar_ws_bytes(B, w.pol);
  }
  return w;
}

qt_status round_impl(qt_ctx ctx, qt_tt* x, const qt_round_opts* o, double* err_out,
                     double* norm_out, bool left_only, double* svlog, int64_t svstride_bond,
                     int64_t svstride_inst, bool orth_only, bool left_orth) {
  const int n = x->n, B = x->batch;
  hipStream_t st = ctx->stream;
  const int lmax_cap = o->max_rank > 0 ? o->max_rank : (1 << 30);
  const bool polar = o->mode == QT_ROUND_POLAR;
  RoundWs w = round_ws_layout(x, lmax_cap, polar);
  QT_CHECK(w.max_nb <= 1024, QT_ECAPACITY, "tt_round: SVD block above 1024 columns");
  const int sweeps = o->jacobi_max_sweeps > 0 ? o->jacobi_max_sweeps : ctx->jacobi_default;
  cplx* scratch = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.slot);
  cplx* Wq = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.slot);
  cplx* Bsv = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.slot);
  cplx* Rb = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.rr);
  cplx* Vb = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.vv);
  cplx* Cb = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.carry);
  double* tau = (double*)ws_take(ctx, sizeof(double) * B * w.tau);
  double* norm = (double*)ws_take(ctx, sizeof(double) * B);
  double* delta = (double*)ws_take(ctx, sizeof(double) * B);
  double* disc2 = (double*)ws_take(ctx, sizeof(double) * B);
  int32_t* rkl = (int32_t*)ws_take(ctx, sizeof(int32_t) * B * (n + 1));
  QT_CHECK(scratch && Wq && Bsv && Rb && Vb && Cb && tau && norm && delta && disc2 && rkl,
           QT_ENOMEM, "tt_round: workspace too small");
  QrBlkWs qb{};
  if (w.qb_v > 0) {
    qb.V = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.qb_v);
    qb.v_stride = w.qb_v;
    qb.T = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.qb_t);
    qb.t_stride = w.qb_t;
    qb.W1 = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.qb_w);
    qb.W2 = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.qb_w);
    qb.w_stride = w.qb_w;
    qb.tau = (double*)ws_take(ctx, sizeof(double) * B * w.qb_tau);
    qb.tau_stride = w.qb_tau;
    qb.s_dev = (int32_t*)ws_take(ctx, sizeof(int32_t) * B);
    QT_CHECK(qb.V && qb.T && qb.W1 && qb.W2 && qb.tau && qb.s_dev, QT_ENOMEM,
             "tt_round: blocked QR workspace too small");
  }
  cplx* X = (cplx*)x->data;
  const int64_t sX = x->inst_stride;
  const int rs = n + 1;
  int32_t* rk = x->ranks;
  const cplx one = make_double2(1.0, 0.0);

  if (n == 1) {
    norm_delta(st, B, dconst(1), dconst(x->modes[0]), X + x->offsets[0], sX, norm, delta, disc2,
               0.0, 0);
    finalize_err(st, B, disc2, norm, err_out, norm_out);
    QT_HIP(hipGetLastError());
    return QT_OK;
  }
  k_init_left<<<B, 64, 0, st>>>(n, B, rk, rkl);
  if (orth_only) {
    // exact right orthogonalization: the right sweep's QRs from x's own last
    // core, no left sweep, nothing truncated, no error or norm
    QT_CHECK(!polar && !err_out && !norm_out && !svlog, QT_EINVAL,
             "right orthogonalization: SVD mode without error outputs");
    SweepBufs buf{scratch, Bsv, Vb, Cb, w.slot, w.vv, w.carry};
    QT_TRY(take_sweep_extra(ctx, B, w, buf));
    buf.exact = true;
    QT_TRY(right_sweep_impl(ctx, x, rkl, X + x->offsets[n - 1], sX, buf, delta, disc2, lmax_cap,
                            sweeps, nullptr, 0, 0));
    QT_HIP(hipGetLastError());
    return QT_OK;
  }
  if (left_orth) {
    // cores 0..n-2 already have orthonormal (or zero) columns: ||x|| is the
    // last core's norm, and the truncation sweep starts from that core
    QT_CHECK(!left_only, QT_EINVAL, "rounding: left_orth with left_only");
    norm_delta(st, B, dref(rkl + n - 1, rs), dconst(x->modes[n - 1]), X + x->offsets[n - 1], sX,
               norm, delta, disc2, o->eps, n - 1);
    SweepBufs buf{scratch, Bsv, Vb, Cb, w.slot, w.vv, w.carry};
    QT_TRY(take_sweep_extra(ctx, B, w, buf));
    PolarWs pw{};
    if (polar) {
      QT_TRY(polar_ws_take(ctx, B, w.pol, pw));
      buf.polar = &pw;
      buf.polar_nq = polar_quintic_steps(o->eps, n - 1, std::min(w.pol.ncap, w.pol.mcap));
      buf.polar_seed = o->seed;
    }
    QT_TRY(right_sweep_impl(ctx, x, rkl, X + x->offsets[n - 1], sX, buf, delta, disc2, lmax_cap,
                            sweeps, svlog, svstride_bond, svstride_inst));
    finalize_err(st, B, disc2, norm, err_out, norm_out);
    QT_HIP(hipGetLastError());
    return QT_OK;
  }
  // ---- left orthogonalization sweep
  for (int k = 0; k < n - 1; ++k) {
    const int p = x->modes[k];
    const cplx* in = (k == 0) ? X + x->offsets[0] : scratch;
    const int64_t sin = (k == 0) ? sX : w.slot;
    // left_only (norm of the train): R is all that is carried, Q is not formed
    if (qr_blocked_wanted(x->cap[k] * p, x->cap[k + 1]))
      qr_blocked(st, B, x->cap[k] * p, x->cap[k + 1], dref(rkl + k, rs, p), dref(rk + k + 1, rs),
                 in, sin, Wq, w.slot, qb, left_only ? nullptr : X + x->offsets[k], sX, Rb, w.rr,
                 rkl + k + 1, rs);
    else
      qr_auto(st, B, x->cap[k] * p, x->cap[k + 1], dref(rkl + k, rs, p), dref(rk + k + 1, rs),
              in, sin, Wq, w.slot, tau, w.tau, left_only ? nullptr : X + x->offsets[k], sX, Rb,
              w.rr, rkl + k + 1, rs);
    const int p1 = x->modes[k + 1];
    // scratch (s x p1 r_{k+2}) = R (s x r_{k+1}) * core_{k+1} (r_{k+1} x p1 r_{k+2})
    gemm(st, B, dref(rkl + k + 1, rs), dref(rk + k + 2, rs, p1), dref(rk + k + 1, rs),
         x->cap[k + 1], p1 * x->cap[k + 2], false, Rb, w.rr, false, X + x->offsets[k + 1], sX,
         scratch, w.slot, one, false);
  }
  // the last core (r'_{n-1} x p_{n-1}) is in scratch: ||x|| and delta
  norm_delta(st, B, dref(rkl + n - 1, rs), dconst(x->modes[n - 1]), scratch, w.slot, norm, delta,
             disc2, o->eps, n - 1);
  if (left_only) {
    // norm only: x is left as scratch (its cores were consumed, not rewritten)
    finalize_err(st, B, disc2, norm, err_out, norm_out);
    QT_HIP(hipGetLastError());
    return QT_OK;
  }
  // ---- right truncation sweep
  SweepBufs buf{scratch, Bsv, Vb, Cb, w.slot, w.vv, w.carry};
  QT_TRY(take_sweep_extra(ctx, B, w, buf));
  PolarWs pw{};
  if (polar) {
    QT_TRY(polar_ws_take(ctx, B, w.pol, pw));
    buf.polar = &pw;
    buf.polar_nq = polar_quintic_steps(o->eps, n - 1, std::min(w.pol.ncap, w.pol.mcap));
    buf.polar_seed = o->seed;
  }
  QT_TRY(right_sweep_impl(ctx, x, rkl, scratch, w.slot, buf, delta, disc2, lmax_cap, sweeps, svlog,
                          svstride_bond, svstride_inst));
  finalize_err(st, B, disc2, norm, err_out, norm_out);
  QT_HIP(hipGetLastError());
  return QT_OK;
}

// Sweep cap of the Jacobi at orders above 100 (R^H and W in global memory):
// twice the context default unless the caller set a cap of its own; graded
// spectra with long tails of negligible singular values need more sweeps
// there (33 at order 160 on the columns of R's unpreconditioned B).
static int sweeps_global(qt_ctx ctx, int sweeps) {
  return sweeps == ctx->jacobi_default ? 2 * sweeps : sweeps;
}

qt_status take_sweep_extra(qt_ctx ctx, int B, const RoundWs& w, SweepBufs& buf) {
  buf.U = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.slot);
  buf.RV = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.vv);
  buf.nbmax = w.max_nb + 4;
  buf.tau = (double*)ws_take(ctx, sizeof(double) * B * buf.nbmax);
  QT_CHECK(buf.U && buf.RV && buf.tau, QT_ENOMEM, "rounding: sweep workspace too small");
  buf.qb = QrBlkWs{};
  if (w.sb_v > 0) {
    QrBlkWs& q = buf.qb;
    q.V = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.sb_v);
    q.v_stride = w.sb_v;
    q.T = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.sb_t);
    q.t_stride = w.sb_t;
    q.W1 = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.sb_w);
    q.W2 = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.sb_w);
    q.w_stride = w.sb_w;
    q.tau = (double*)ws_take(ctx, sizeof(double) * B * w.sb_tau);
    q.tau_stride = w.sb_tau;
    q.s_dev = (int32_t*)ws_take(ctx, sizeof(int32_t) * B);
    q.dims = (int32_t*)ws_take(ctx, sizeof(int32_t) * B * 3);
    QT_CHECK(q.V && q.T && q.W1 && q.W2 && q.tau && q.s_dev && q.dims, QT_ENOMEM,
             "rounding: blocked QR workspace of the SVD too small");
  }
  return QT_OK;
}

qt_status right_sweep_impl(qt_ctx ctx, qt_tt* x, const int32_t* rkl, const cplx* center,
                           int64_t cstride, const SweepBufs& buf, const double* delta,
                           double* disc2, int lmax_cap, int sweeps, double* svlog, int64_t svb,
                           int64_t svi) {
  const int sweeps_glb = sweeps_global(ctx, sweeps);
  const int n = x->n, B = x->batch, rs = n + 1;
  hipStream_t st = ctx->stream;
  cplx* X = (cplx*)x->data;
  const int64_t sX = x->inst_stride;
  int32_t* rk = x->ranks;
  const cplx one = make_double2(1.0, 0.0);
  for (int k = n - 1; k >= 1; --k) {
    const int nbk = std::min(x->cap[k], x->modes[k] * std::min(x->cap[k + 1], lmax_cap));
    QT_CHECK(nbk <= 1024, QT_ECAPACITY,
             "rounding: SVD block above 1024 columns (cap the rank or the sketch width)");
  }
  // the SVD reads its input again after writing the core (carry = A core^H):
  // a centre stored in x's own last core is staged into the scratch first
  if (center == X + x->offsets[n - 1]) {
    copy(st, B, dref(rkl + n - 1, rs), dref(rk + n, rs, x->modes[n - 1]),
         (int64_t)x->cap[n - 1] * x->modes[n - 1] * x->cap[n], center, cstride, buf.scratch,
         buf.slot);
    center = buf.scratch;
    cstride = buf.slot;
  }
  for (int k = n - 1; k >= 1; --k) {
    const int p = x->modes[k];
    const int lmax = std::min(lmax_cap, x->cap[k]);
    const cplx* in = (k == n - 1) ? center : buf.scratch;
    const int64_t sin = (k == n - 1) ? cstride : buf.slot;
    const int mcap = x->cap[k], ccap = p * std::min(x->cap[k + 1], lmax_cap);
    double* svk = svlog ? svlog + k * svb : nullptr;
    const bool prof = prof_on(PROF_SVD);
    if (prof) g_prof->begin();
    const int nsw = std::min(mcap, ccap) > 100 ? sweeps_glb : sweeps;
    const bool ok = buf.polar ?
        (polar_trunc(st, B, mcap, ccap, dref(rkl + k, rs), dref(rk + k + 1, rs, p), in, sin,
                     *buf.polar, X + x->offsets[k], sX, buf.C, buf.carry, rk + k, rs, delta,
                     disc2, lmax, buf.polar_nq, buf.polar_seed, (uint64_t)k), true) :
        svd_trunc_fast(st, B, mcap, ccap, dref(rkl + k, rs), dref(rk + k + 1, rs, p),
                                   in, sin, buf.Bsv, buf.U, buf.slot, buf.V, buf.RV, buf.vv,
                                   buf.tau, buf.nbmax, buf.qb.V ? &buf.qb : nullptr,
                                   X + x->offsets[k], sX, buf.C,
                                   buf.carry, rk + k, rs, delta, disc2, lmax, nsw, ctx->status,
                                   svk, svi, ctx->counters, buf.exact);
    QT_CHECK(ok, QT_ECAPACITY, "rounding: SVD block above 1024 columns");
    if (prof) g_prof->end();
    const int pp = x->modes[k - 1];
    // scratch (r'_{k-1} p x l_k) = core_{k-1} (r'_{k-1} p x r'_k) * carry (r'_k x l_k)
    gemm(st, B, dref(rkl + k - 1, rs, pp), dref(rk + k, rs), dref(rkl + k, rs),
         x->cap[k - 1] * pp, x->cap[k], false, X + x->offsets[k - 1], sX, false, buf.C, buf.carry,
         buf.scratch, buf.slot, one, false);
  }
  copy(st, B, dconst(x->modes[0]), dref(rk + 1, rs), (int64_t)x->modes[0] * x->cap[1],
       buf.scratch, buf.slot, X + x->offsets[0], sX);
  QT_HIP(hipGetLastError());
  return QT_OK;
}

}  // namespace qt

extern "C" qt_status tt_round(qt_ctx ctx, qt_tt* x, const qt_round_opts* opts, double* err_out,
                              double* norm_out) {
  qt::enter(ctx);
  QT_CHECK(ctx && x && opts, QT_EINVAL, "tt_round: null argument");
  QT_TRY(qt::tt_validate(x, "x"));
  QT_CHECK(opts->eps >= 0.0, QT_EINVAL, "tt_round: eps < 0");
  QT_CHECK(opts->mode == QT_ROUND_SVD || opts->mode == QT_ROUND_POLAR, QT_EINVAL,
           "tt_round: QT_ROUND_SVD or QT_ROUND_POLAR apply to a materialized train");
  QT_CHECK(opts->precision == QT_PREC_F64, QT_EINVAL,
           "tt_round: QT_PREC_F32 applies to the product-aware roundings only");
  ctx->ws_top = 0;
  const int lmax_cap = opts->max_rank > 0 ? opts->max_rank : (1 << 30);
  QT_TRY(qt::ws_reserve(ctx, qt::round_ws_layout(x, lmax_cap,
                                                 opts->mode == QT_ROUND_POLAR).bytes));
  return qt::round_impl(ctx, x, opts, err_out, norm_out, false, nullptr, 0, 0);
}
