// Internal interfaces of the product-aware (sketch) rounding.
#pragma once

#include "kernels.h"
#include "polar.h"
#include "round.h"

namespace qt {

struct SketchWs {
  std::vector<int64_t> Woff;
  int64_t Wtot = 1, T1 = 1, T2 = 1, M = 1, T3 = 1, Z = 1, Y = 1, R = 1, tau = 1;
  // blocked QRs of the sketches Y_k beyond registers and LDS (0: none)
  int64_t qb_v = 0, qb_t = 0, qb_w = 0, qb_tau = 0;
  size_t bytes = 0;
};
SketchWs sketch_ws_layout(const qt_mpo* A, const qt_tt* y, const std::vector<int32_t>& ell);

// Randomize-then-orthogonalize of x = A (*) y with sketch cores omega (slot k at
// om_off[k], shape (ell[k], p_k, ell[k+1]), shared by all instances).  out gets
// left-orthogonal cores 0..n-2 and the centre in core n-1; ynorm2[b] = ||x~||^2.
// rdiag (optional): [B][n+1][RD_MAX] sorted |R_jj| of the QR of Y_k written at
// bond k+1 of each instance, the input of the rank-predictor features.
// f32: the contractions that only choose the bases (right sketches W_k and
// Y_k = Z_k W_{k+1}) run on the FP32-MFMA GEMM; the projection (T3, Z, M) and
// everything after it stay FP64, so the output is still the exact orthogonal
// projection of x onto the chosen subspace and ||x~||^2 is exact.
constexpr int RD_MAX = 128;
qt_status sketch_impl(qt_ctx ctx, const qt_mpo* A, const qt_tt* y, const cplx* omega,
                      const std::vector<int64_t>& om_off, const std::vector<int32_t>& ell,
                      qt_tt* out, double* ynorm2, double* rdiag = nullptr, bool f32 = false);

struct SandwichWs {
  int64_t E = 1, F = 1, G = 1;
  size_t bytes = 0;
};
SandwichWs sandwich_ws_layout(const qt_mpo* Q, const qt_tt* y);
// out[b] = scale * Re <y_b, Q y_b>
qt_status sandwich_impl(qt_ctx ctx, const qt_mpo* Q, const qt_tt* y, double scale, double* out);

void gauss_fill(hipStream_t st, int64_t count, uint64_t seed, uint64_t stream, cplx* out,
                const uint64_t* base = nullptr);
void sumsq(hipStream_t st, int batch, Dim rows, Dim cols, const cplx* X, int64_t sX, double* out,
           double scale);

// Right-to-left truncated-SVD sweep on a train whose cores 0..n-2 are
// left-orthogonal with left ranks rkl (device, separate from x->ranks); the
// centre (core n-1) is read from `center`.  Writes x->ranks and the cores.
struct SweepBufs {
  cplx* scratch;
  cplx* Bsv;
  cplx* V;
  cplx* C;
  int64_t slot, vv, carry;
  cplx* U;     // reflectors, then the kept left Jacobi vectors (slot)
  cplx* RV;    // Jacobi matrix of orders above 100 (vv)
  double* tau; // nbmax entries: reflector scalars, then 4 for the SVD's sizes
  int64_t nbmax;
  QrBlkWs qb;  // blocked QRs of large SVD blocks (V null when none)
  // polar-decomposition truncation instead of the SVD (null: SVD)
  const PolarWs* polar = nullptr;
  int polar_nq = 0;
  uint64_t polar_seed = 0;
  // exact right orthogonalization: the SVD blocks' QR only, nothing truncated
  bool exact = false;
};
qt_status take_sweep_extra(qt_ctx ctx, int B, const RoundWs& w, SweepBufs& buf);
qt_status right_sweep_impl(qt_ctx ctx, qt_tt* x, const int32_t* rkl, const cplx* center,
                           int64_t cstride, const SweepBufs& buf, const double* delta,
                           double* disc2, int lmax_cap, int sweeps, double* svlog, int64_t svb,
                           int64_t svi);

struct SRoundWs {
  std::vector<int64_t> om_off;
  int64_t om_tot = 1;
  RoundWs sweep;
  size_t bytes = 0;
};
std::vector<int32_t> sketch_ranks(const qt_mpo* A, const qt_tt* y, int rmax, int oversample);
SRoundWs sround_ws_layout(const qt_mpo* A, const qt_tt* y, const qt_tt* out,
                          const std::vector<int32_t>& ell, int lmax_cap);
// Product-aware rounding of A (*) y into out (mode QT_ROUND_SKETCH or
// QT_ROUND_LEARNED).  xn2: device ||A y||^2 per instance.  omega_in null ->
// Gaussian cores drawn from (o->seed, stream_id).  fail[b] = 1 when the
// sketch alone already exceeds eps*||x||.  err_out: the rigorous error bound;
// err_est (optional): the quadrature estimate (see k_sketch_err).
qt_status sround_impl(qt_ctx ctx, const qt_mpo* A, const qt_tt* y, const cplx* omega_in,
                      const std::vector<int64_t>* om_off_in, const std::vector<int32_t>& ell,
                      const qt_round_opts* o, const double* xn2, qt_tt* out, double* err_out,
                      int32_t* fail, uint64_t stream_id, double* svlog, int64_t svb,
                      int64_t svi, double* rdiag = nullptr, double* err_est = nullptr);

}  // namespace qt
