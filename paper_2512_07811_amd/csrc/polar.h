// Polar-decomposition truncation of a bond (GEMM-based, see polar.hip).
#pragma once

#include "kernels.h"

namespace qt {

struct PolarSizes {
  int ncap = 1, mcap = 1, lcap = 1;
  int64_t y = 1, g = 1, c = 1, r = 1, tau = 1;   // elements per instance
  // blocked-QR workspace of the subspace iteration's ncap x lcap QRs (zero
  // when one workgroup's registers or LDS hold them)
  int64_t qb_v = 0, qb_t = 0, qb_w = 0, qb_tau = 0;
};
PolarSizes polar_sizes(int ncap, int mcap, int lcap);
size_t polar_ws_bytes(int B, const PolarSizes& s);

struct PolarWs {
  PolarSizes s;
  cplx *Y0, *Y1, *G, *P, *H, *Z0, *Z1, *Om, *V, *W, *C, *Wq, *R;
  double* tau;
  double* nrm;     // [3][B]
  int32_t* sq;     // [B]
  QrBlkWs qb;      // V null: the QRs run in one workgroup
};
qt_status polar_ws_take(qt_ctx ctx, int B, const PolarSizes& s, PolarWs& w);
// Quintic steps that bring relative singular values down to a twentieth of
// the cutoff eps / (sqrt(nbonds) qcap) within [0.7, 1.21].
int polar_quintic_steps(double eps, int nbonds, int qcap);

// Truncates the centre A (n x m packed, n <= ncap, m <= mcap) of every
// instance: keeps the directions of singular values above delta[b] / min(n, m)
// (at least one, at most lmax), writes the core (l x m packed) and the carry
// (n x l packed), l to l_out and adds the discarded weight to disc2.  The
// Gaussian start block of the subspace iteration is Philox(seed, stream).
void polar_trunc(hipStream_t st, int B, int ncap, int mcap, Dim n, Dim m, const cplx* A,
                 int64_t sA, const PolarWs& w, cplx* core, int64_t sCore, cplx* carry,
                 int64_t sCarry, int32_t* l_out, int l_stride, const double* delta,
                 double* disc2, int lmax, int nq, uint64_t seed, uint64_t stream);

}  // namespace qt
