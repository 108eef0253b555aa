// Internal interfaces shared by the entry points.
#pragma once

#include "kernels.h"
#include "polar.h"

namespace qt {

struct RoundWs {
  int64_t slot = 1, rr = 1, vv = 1, carry = 1, tau = 1, max_nb = 0;
  // blocked left-sweep QR (elements per instance; 0 when no core needs it)
  int64_t qb_v = 0, qb_t = 0, qb_w = 0, qb_tau = 0;
  int64_t sb_v = 0, sb_t = 0, sb_w = 0, sb_tau = 0;   // blocked QRs of the SVD blocks
  size_t bytes = 0;
  size_t sweep_bytes = 0;   // extra for the fast SVD (reflectors, R V, tau, sigma)
  bool polar = false;       // polar-decomposition truncation (QT_ROUND_POLAR)
  PolarSizes pol;
};
RoundWs round_ws_layout(const qt_tt* x, int lmax_cap, bool polar = false);

// left_only: QR sweep that carries only the R factors and reports the norm
// (no truncation; Q is never formed, x's cores are consumed as scratch).
// svlog: optional [bond][instance][nb] log of sorted singular values.
// orth_only: no rounding, an exact right orthogonalization of x (cores 1..n-1
// with orthonormal rows, ranks min(r_k, p_k r_{k+1})) by the right sweep's QRs
// (SVD mode, no error, norm or log outputs).
// left_orth: the caller guarantees that cores 0..n-2 have orthonormal or zero
// columns; the left QR sweep is skipped (the truncation sweep and its delta
// rule start from the last core, whose norm is ||x||).
qt_status round_impl(qt_ctx ctx, qt_tt* x, const qt_round_opts* o, double* err_out,
                     double* norm_out, bool left_only, double* svlog, int64_t svstride_bond,
                     int64_t svstride_inst, bool orth_only = false, bool left_orth = false);
qt_status hadamard_impl(qt_ctx ctx, const qt_tt* a, const qt_tt* b, qt_tt* out);
qt_status mpo_impl(qt_ctx ctx, const qt_mpo* A, const qt_tt* x, qt_tt* out);
qt_status add_impl(qt_ctx ctx, double are, double aim, const qt_tt* x, double bre, double bim,
                   const qt_tt* y, qt_tt* out);
qt_status dot_impl(qt_ctx ctx, const qt_tt* a, const qt_tt* b, double* out, bool reserve);

// Host-side description of a train laid out in a caller buffer.
struct TTLayout {
  std::vector<int32_t> modes, cap;
  std::vector<int64_t> off;
  int64_t stride = 0;
  qt_tt view(void* data, int32_t* ranks, int batch) const {
    qt_tt t;
    t.n = (int32_t)modes.size();
    t.batch = batch;
    t.modes = modes.data();
    t.cap = cap.data();
    t.offsets = off.data();
    t.inst_stride = stride;
    t.ranks = ranks;
    t.data = data;
    return t;
  }
};
TTLayout make_layout(const std::vector<int32_t>& modes, const std::vector<int32_t>& cap);

}  // namespace qt
