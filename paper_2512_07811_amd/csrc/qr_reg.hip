// Register-resident Householder QR for the small, latency-bound factorizations
// of the rounding sweeps.
//
// One 1024-thread workgroup (16 wave64s = 64 row groups of 16 lanes) per
// matrix.  Column c lives in group c % 64 (wave (c % 64) / 4, DPP row c % 4),
// register slot c / 64; row i lives in lane i % 16 of that group, register row
// i / 16.  Step j: the group owning column j forms the reflector
// H = I - tau u u^H (u_j = 1, H x = beta e_1, beta = -e^{i arg x_j} ||x||,
// tau = 1 + |x_j|/||x||) and publishes u in LDS;
// every group updates its own trailing columns in registers, reducing over its
// 16 lanes with DPP.  One barrier per column.  The reflectors stay in LDS
// (column-major, at most 144 x 64 or 96 x 96 complex = 144 KiB), so that
// Q = H_0..H_{s-1} [I; 0] is then accumulated backwards in the same registers
// with no barrier at all: every group owns its columns and the reflectors are
// read-only by then.  (U is unused scratch kept for the common QR signature.)
#include "kernels.h"

namespace qt {

constexpr int QG = 64;  // row groups per workgroup

template <int RPL, int CPS, bool ORIENT>
__global__ __launch_bounds__(1024) void k_qr_reg(Dim Md, Dim Nd, const cplx* __restrict__ A,
                                                 int64_t sA, cplx* __restrict__ U, int64_t sU,
                                                 double* __restrict__ tau, int64_t sTau,
                                                 cplx* __restrict__ Q, int64_t sQ,
                                                 cplx* __restrict__ R, int64_t sR, int32_t* s_out,
                                                 int s_stride) {
  constexpr int MAXM = 16 * RPL;
  constexpr int SMAX = MAXM < QG * CPS ? MAXM : QG * CPS;
  const int b = blockIdx.x;
  const int m0 = dimv(Md, b), n0 = dimv(Nd, b);
  // ORIENT: factor B = A when m0 >= n0, else B = A^H (so B is never wide)
  const bool trans = ORIENT && (m0 < n0);
  const int m = trans ? n0 : m0, n = trans ? m0 : n0;
  const int s = min(m, n);
  const bool want_q = Q != nullptr;   // decided before Q is offset
  A += b * sA; U += b * sU; tau += b * sTau; R += b * sR;
  if (want_q) Q += b * sQ;
  const int g = threadIdx.x & 15;          // lane in the row group
  const int grp = threadIdx.x >> 4;        // row group 0..63 (= column residue)
  __shared__ cplx ul[SMAX * MAXM];     // reflector j in ul[j * MAXM ...]
  __shared__ double tl[SMAX];
  cplx a[CPS][RPL];
#pragma unroll
  for (int cs = 0; cs < CPS; ++cs) {
    const int c = grp + QG * cs;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = g + 16 * r;
      cplx v = make_double2(0.0, 0.0);
      if (i < m && c < n) v = trans ? cconj(A[(int64_t)c * n0 + i]) : A[(int64_t)i * n + c];
      a[cs][r] = v;
    }
  }
  for (int j = 0; j < s; ++j) {
    if (grp == (j % QG)) {
      const int csj = j / QG;
      cplx col[RPL];
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        col[r] = make_double2(0.0, 0.0);
#pragma unroll
        for (int cs = 0; cs < CPS; ++cs)
          if (cs == csj) col[r] = a[cs][r];
      }
      double sig2 = 0.0;
      cplx al = make_double2(0.0, 0.0);
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int i = g + 16 * r;
        if (i > j && i < m) sig2 += cabs2(col[r]);
        if (i == j) al = col[r];
      }
      sig2 = row16_sum(sig2);
      al = row16_sum(al);  // one lane contributes
      double t;
      cplx beta, iu0;
      {
        double sc = 1.0, s2 = sig2;
        const double x2 = cabs2(al) + sig2;
        if (x2 > 0.0 && x2 < QR_TINY) {   // uniform over the row group
          sc = QR_SCALE;
          s2 = 0.0;
#pragma unroll
          for (int r = 0; r < RPL; ++r) {
            const int i = g + 16 * r;
            if (i > j && i < m) s2 += cabs2(cscale(col[r], sc));
          }
          s2 = row16_sum(s2);
        }
        house_coef(cscale(al, sc), s2, sc, t, beta, iu0);
      }
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int i = g + 16 * r;
        cplx u;
        if (i < j || i >= m) u = make_double2(0.0, 0.0);
        else if (i == j) u = make_double2(1.0, 0.0);
        else u = cmul(col[r], iu0);
        ul[j * MAXM + i] = u;
        // the owner keeps R's column: beta on the diagonal, zeros below
        cplx keep = (i == j) ? beta : (i > j ? make_double2(0.0, 0.0) : col[r]);
#pragma unroll
        for (int cs = 0; cs < CPS; ++cs)
          if (cs == csj) a[cs][r] = keep;
      }
      if (g == 0) {
        tl[j] = t;
        tau[j] = t;
      }
    }
    __syncthreads();
    const double t = tl[j];
    if (t != 0.0) {
      const cplx* uj = ul + j * MAXM;
#pragma unroll
      for (int cs = 0; cs < CPS; ++cs) {
        const int c = grp + QG * cs;
        const bool act = (c > j) && (c < n);
        cplx w = make_double2(0.0, 0.0);
#pragma unroll
        for (int r = 0; r < RPL; ++r) cfma(w, cconj(uj[g + 16 * r]), a[cs][r]);
        w = row16_sum(w);
        const cplx f = act ? cscale(w, -t) : make_double2(0.0, 0.0);
#pragma unroll
        for (int r = 0; r < RPL; ++r) cfma(a[cs][r], uj[g + 16 * r], f);
      }
    }
  }
  // R (s x n): upper trapezoid of the factored matrix
#pragma unroll
  for (int cs = 0; cs < CPS; ++cs) {
    const int c = grp + QG * cs;
    if (c >= n) continue;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = g + 16 * r;
      if (i < s) R[(int64_t)i * n + c] = (c >= i) ? a[cs][r] : make_double2(0.0, 0.0);
    }
  }
  // Q (m x s) accumulated backwards: Q <- H_j Q for j = s-1 .. 0 (skipped
  // when only R is wanted)
  if (!want_q) {
    if (threadIdx.x == 0 && s_out) s_out[(int64_t)b * s_stride] = s;
    return;
  }
#pragma unroll
  for (int cs = 0; cs < CPS; ++cs) {
    const int c = grp + QG * cs;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = g + 16 * r;
      a[cs][r] = make_double2((i == c && c < s) ? 1.0 : 0.0, 0.0);
    }
  }
  // the last step's barrier made every reflector visible; no more barriers
  for (int j = s - 1; j >= 0; --j) {
    const double t = tl[j];
    if (t != 0.0) {
      const cplx* uj = ul + j * MAXM;
#pragma unroll
      for (int cs = 0; cs < CPS; ++cs) {
        const int c = grp + QG * cs;
        const bool act = (c >= j) && (c < s);
        cplx w = make_double2(0.0, 0.0);
#pragma unroll
        for (int r = 0; r < RPL; ++r) cfma(w, cconj(uj[g + 16 * r]), a[cs][r]);
        w = row16_sum(w);
        const cplx f = act ? cscale(w, -t) : make_double2(0.0, 0.0);
#pragma unroll
        for (int r = 0; r < RPL; ++r) cfma(a[cs][r], uj[g + 16 * r], f);
      }
    }
  }
#pragma unroll
  for (int cs = 0; cs < CPS; ++cs) {
    const int c = grp + QG * cs;
    if (c >= s) continue;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = g + 16 * r;
      if (i < m) Q[(int64_t)i * s + c] = a[cs][r];
    }
  }
  if (threadIdx.x == 0 && s_out) s_out[(int64_t)b * s_stride] = s;
}

template <int RPL, int CPS>
static void launch_qr_reg(hipStream_t st, int batch, bool orient, Dim m, Dim n, const cplx* A,
                          int64_t sA, cplx* U, int64_t sU, double* tau, int64_t sTau, cplx* Q,
                          int64_t sQ, cplx* R, int64_t sR, int32_t* s_out, int s_stride) {
  if (orient)
    k_qr_reg<RPL, CPS, true><<<batch, 1024, 0, st>>>(m, n, A, sA, U, sU, tau, sTau, Q, sQ, R, sR,
                                                     s_out, s_stride);
  else
    k_qr_reg<RPL, CPS, false><<<batch, 1024, 0, st>>>(m, n, A, sA, U, sU, tau, sTau, Q, sQ, R, sR,
                                                      s_out, s_stride);
}

// Capacities covered without register spills: m <= 144 with n <= 64, and
// m <= 96 with n <= 128.
bool qr_reg(hipStream_t st, int batch, int mcap, int ncap, Dim m, Dim n, const cplx* A, int64_t sA,
            cplx* U, int64_t sU, double* tau, int64_t sTau, cplx* Q, int64_t sQ, cplx* R,
            int64_t sR, int32_t* s_out, int s_stride, bool orient) {
  const int rpl = (mcap + 15) / 16, cps = (ncap + QG - 1) / QG;
  if (rpl < 1 || cps < 1 || cps > 2) return false;
#define QR_CASE(RR, CC)                                                                       \
  if (rpl <= RR && cps <= CC) {                                                               \
    launch_qr_reg<RR, CC>(st, batch, orient, m, n, A, sA, U, sU, tau, sTau, Q, sQ, R, sR,     \
                          s_out, s_stride);                                                   \
    return true;                                                                              \
  }
  QR_CASE(2, 1) QR_CASE(4, 1) QR_CASE(6, 1) QR_CASE(9, 1)
  QR_CASE(2, 2) QR_CASE(4, 2) QR_CASE(6, 2)
#undef QR_CASE
  return false;
}

// ---------------------------------------------------------------------------
// Memory-resident variant with the same work split (16-lane groups, DPP sums,
// one barrier per column) for matrices that do not fit in registers: the
// matrix lives in LDS when m*n*16 bytes fit (dynamic shared memory), else in
// the global scratch W (L2-resident for these sizes).
// Rows per lane handled per batch of loads: the loops below issue all loads of
// a chunk of QM_CH rows before using any of them (the memory latency, not the
// arithmetic, bounds these steps), and keep the chunk in registers when the
// column is short enough (m - j <= 16 QM_CH) to be updated in place.
constexpr int QM_CH = 9;

// H = I - t u u^H (u_j = 1, u below the diagonal of column j) applied to the
// column col over rows j..m-1 by one 16-lane group (lane g).
__device__ inline void qm_apply(const cplx* __restrict__ uj, cplx* __restrict__ col, int j, int m,
                                int g, double t) {
  if (m - j <= 16 * QM_CH) {
    cplx uu[QM_CH], cc[QM_CH];
#pragma unroll
    for (int r = 0; r < QM_CH; ++r) {
      const int i = j + g + 16 * r;
      uu[r] = make_double2(0.0, 0.0);
      cc[r] = make_double2(0.0, 0.0);
      if (i < m) {
        uu[r] = (i == j) ? make_double2(1.0, 0.0) : uj[i];
        cc[r] = col[i];
      }
    }
    cplx w = make_double2(0.0, 0.0);
#pragma unroll
    for (int r = 0; r < QM_CH; ++r) cfma(w, cconj(uu[r]), cc[r]);
    w = row16_sum(w);
    const cplx f = cscale(w, -t);
#pragma unroll
    for (int r = 0; r < QM_CH; ++r) {
      const int i = j + g + 16 * r;
      if (i < m) {
        cfma(cc[r], uu[r], f);
        col[i] = cc[r];
      }
    }
    return;
  }
  cplx w = make_double2(0.0, 0.0);
  for (int i0 = j; i0 < m; i0 += 16 * QM_CH) {
    cplx uu[QM_CH], cc[QM_CH];
#pragma unroll
    for (int r = 0; r < QM_CH; ++r) {
      const int i = i0 + g + 16 * r;
      uu[r] = make_double2(0.0, 0.0);
      cc[r] = make_double2(0.0, 0.0);
      if (i < m) {
        uu[r] = (i == j) ? make_double2(1.0, 0.0) : uj[i];
        cc[r] = col[i];
      }
    }
#pragma unroll
    for (int r = 0; r < QM_CH; ++r) cfma(w, cconj(uu[r]), cc[r]);
  }
  w = row16_sum(w);
  const cplx f = cscale(w, -t);
  for (int i0 = j; i0 < m; i0 += 16 * QM_CH) {
    cplx uu[QM_CH], cc[QM_CH];
#pragma unroll
    for (int r = 0; r < QM_CH; ++r) {
      const int i = i0 + g + 16 * r;
      uu[r] = make_double2(0.0, 0.0);
      cc[r] = make_double2(0.0, 0.0);
      if (i < m) {
        uu[r] = (i == j) ? make_double2(1.0, 0.0) : uj[i];
        cc[r] = col[i];
      }
    }
#pragma unroll
    for (int r = 0; r < QM_CH; ++r) {
      const int i = i0 + g + 16 * r;
      if (i < m) {
        cfma(cc[r], uu[r], f);
        col[i] = cc[r];
      }
    }
  }
}

template <bool IN_LDS>
__global__ __launch_bounds__(1024) void k_qr_mem(Dim Md, Dim Nd, const cplx* __restrict__ A,
                                                 int64_t sA, cplx* __restrict__ W, int64_t sW,
                                                 double* __restrict__ tau, int64_t sTau,
                                                 cplx* __restrict__ Q, int64_t sQ,
                                                 cplx* __restrict__ R, int64_t sR, int32_t* s_out,
                                                 int s_stride, int orient) {
  extern __shared__ cplx dyn[];
  const int b = blockIdx.x;
  const int m0 = dimv(Md, b), n0 = dimv(Nd, b);
  const bool trans = orient && (m0 < n0);   // factor A^H when A is wide
  const int m = trans ? n0 : m0, n = trans ? m0 : n0;
  const int s = min(m, n);
  const bool want_q = Q != nullptr;   // decided before Q is offset
  A += b * sA; W += b * sW; tau += b * sTau; R += b * sR;
  if (want_q) Q += b * sQ;
  // column-major m x n work matrix; the reflector of step j (u_j = 1 implicit)
  // is kept below the diagonal of column j and read from there by all groups
  cplx* M = IN_LDS ? dyn : W;
  __shared__ double tsh[2];
  const int g = threadIdx.x & 15, grp = threadIdx.x >> 4;
  for (int64_t e = threadIdx.x; e < (int64_t)m * n; e += blockDim.x) {
    const int i = (int)(e / n), c = (int)(e % n);
    M[(int64_t)c * m + i] = trans ? cconj(A[(int64_t)c * n0 + i]) : A[e];
  }
  __syncthreads();
  for (int j = 0; j < s; ++j) {
    const int buf = j & 1;
    cplx* colj = M + (int64_t)j * m;
    if (grp == (j % QG)) {
      double sig2 = 0.0;
      for (int i0 = j + 1; i0 < m; i0 += 16 * QM_CH) {
        cplx xx[QM_CH];
#pragma unroll
        for (int r = 0; r < QM_CH; ++r) {
          const int i = i0 + g + 16 * r;
          xx[r] = i < m ? colj[i] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int r = 0; r < QM_CH; ++r) sig2 += cabs2(xx[r]);
      }
      sig2 = row16_sum(sig2);
      const cplx al = colj[j];
      double t;
      cplx beta, iu0;
      {
        double sc = 1.0, s2 = sig2;
        const double x2 = cabs2(al) + sig2;
        if (x2 > 0.0 && x2 < QR_TINY) {   // uniform over the row group
          sc = QR_SCALE;
          s2 = 0.0;
          for (int i = j + 1 + g; i < m; i += 16) s2 += cabs2(cscale(colj[i], sc));
          s2 = row16_sum(s2);
        }
        house_coef(cscale(al, sc), s2, sc, t, beta, iu0);
      }
      for (int i0 = j + 1; i0 < m; i0 += 16 * QM_CH) {
        cplx xx[QM_CH];
#pragma unroll
        for (int r = 0; r < QM_CH; ++r) {
          const int i = i0 + g + 16 * r;
          xx[r] = i < m ? colj[i] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int r = 0; r < QM_CH; ++r) {
          const int i = i0 + g + 16 * r;
          if (i < m) colj[i] = cmul(xx[r], iu0);
        }
      }
      if (g == 0) {
        colj[j] = beta;
        tsh[buf] = t;
        tau[j] = t;
      }
    }
    __syncthreads();
    const double t = tsh[buf];
    if (t != 0.0) {
      // column c always belongs to group c % 64, so the next owner reads its
      // own updates (no barrier needed between the update and the next step)
      for (int c = grp; c < n; c += QG) {
        if (c <= j) continue;
        qm_apply(colj, M + (int64_t)c * m, j, m, g, t);
      }
    }
  }
  __syncthreads();
  for (int64_t e = threadIdx.x; e < (int64_t)s * n; e += blockDim.x) {
    const int i = (int)(e / n), c = (int)(e % n);
    R[e] = (c >= i) ? M[(int64_t)c * m + i] : make_double2(0.0, 0.0);
  }
  if (!want_q) {   // only R is wanted
    if (threadIdx.x == 0 && s_out) s_out[(int64_t)b * s_stride] = s;
    return;
  }
  __syncthreads();   // R is read from M before M is overwritten below
  // Q (m x s) formed in place over the reflectors (backward accumulation):
  // at step j, H_j is applied to columns j+1..s-1, then column j, whose
  // reflector is no longer needed, becomes H_j e_j.  The R factor was copied
  // out above; Q is written out coalesced at the end.
  for (int j = s - 1; j >= 0; --j) {
    const double t = tau[j];
    const cplx* uj = M + (int64_t)j * m;
    if (t != 0.0) {
      for (int c = j + 1 + grp; c < s; c += QG) qm_apply(uj, M + (int64_t)c * m, j, m, g, t);
    }
    __syncthreads();
    cplx* colj = M + (int64_t)j * m;
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
      cplx v;
      if (i < j) v = make_double2(0.0, 0.0);
      else if (i == j) v = make_double2(1.0 - t, 0.0);
      else v = cscale(colj[i], -t);
      colj[i] = v;
    }
    __syncthreads();
  }
  for (int64_t e = threadIdx.x; e < (int64_t)m * s; e += blockDim.x) {
    const int i = (int)(e / s), c = (int)(e % s);
    Q[e] = M[(int64_t)c * m + i];
  }
  if (threadIdx.x == 0 && s_out) s_out[(int64_t)b * s_stride] = s;
}

constexpr size_t QR_LDS_BYTES = 160 * 1024 - 64;

bool qr_reg_fits(int mcap, int ncap) {
  const int rpl = (mcap + 15) / 16, cps = (ncap + QG - 1) / QG;
  if (rpl < 1 || cps < 1) return false;
  return (cps == 1 && rpl <= 9) || (cps == 2 && rpl <= 6);
}

bool qr_lds_fits(int mcap, int ncap) {
  return sizeof(cplx) * (size_t)mcap * ncap <= QR_LDS_BYTES;
}

void qr_mem(hipStream_t st, int batch, int mcap, int ncap, Dim m, Dim n, const cplx* A,
            int64_t sA, cplx* W, int64_t sW, double* tau, int64_t sTau, cplx* Q, int64_t sQ,
            cplx* R, int64_t sR, int32_t* s_out, int s_stride, bool orient) {
  static bool attr_set = false;
  if (!attr_set) {
    hipFuncSetAttribute((const void*)k_qr_mem<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)QR_LDS_BYTES);
    attr_set = true;
  }
  const size_t lds = sizeof(cplx) * (size_t)mcap * ncap;
  if (lds <= QR_LDS_BYTES) {
    k_qr_mem<true><<<batch, 1024, lds, st>>>(m, n, A, sA, W, sW, tau, sTau, Q, sQ, R, sR, s_out,
                                             s_stride, orient ? 1 : 0);
  } else {
    k_qr_mem<false><<<batch, 1024, 0, st>>>(m, n, A, sA, W, sW, tau, sTau, Q, sQ, R, sR, s_out,
                                            s_stride, orient ? 1 : 0);
  }
}

}  // namespace qt
