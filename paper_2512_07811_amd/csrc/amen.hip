// AMEn approximation of a TT x TTO product, y ~ A x (Sec. 2.1 of arXiv
// 2512.07811; Algorithm 2 applies it to the Green multiply): the cores of y
// are swept left to right, each taken from the local projection of A x onto
// the frames of y, and enriched with an approximation z of the residual
// A x - y (Dolgov and Savostyanov, SIAM J. Sci. Comput. 2014).
//
// One sweep, with y and z right-orthogonal on entry, all trains unpacked to
// capacity-padded cores (zeros beyond the actual ranks, so that every GEMM
// has host-known sizes):
//   right interfaces   PR[k] = [Phi^{yAx}_R ; Phi^{zAx}_R] (stacked rows: the
//                      z rows right after y's actual rank, zeros after them,
//                      so that a QR meets the padding's zero columns last),
//                      PZY[k] = Phi^{zy}_R
//   core k             T2 = (PL x_k) A_k              (PL = Phi^{yAx}_L)
//                      YE = T2 PR[k+1] = [local solution | enrichment]
//                      y_k <- Q of QR(YE)             (the span of AMEn's
//                      [y_k | e_k], e_k = YE_z - y_k PZY^T: the correction
//                      is a combination of the first block's columns; Q's
//                      columns of the padding's zero columns are zeroed)
//                      PL <- Q^H T2
//                      z_k <- Q of QR(Phi^{zAx}_L A_k x_k Phi^{zAx}_R
//                                     - Phi^{zy}_L y_k Phi^{zy}_R)
//   last core          the local solutions of y and z
// then one TT rounding of y at eps (the SVD rounding's delta rule and cap),
// which leaves y right-orthogonal, and a right orthogonalization of z (QR
// sweep from its last core; y and z get the same one before the first sweep).
#include "kernels.h"
#include "round.h"

namespace qt {

// padded core (R x p x R2, zeros outside) <- packed core (r x p x r2) of
// instance b (ranks read from the device)
__global__ void k_amen_unpack(int p, int R, int R2, const int32_t* __restrict__ ranks, int rs,
                              int k, const cplx* __restrict__ src, int64_t sS,
                              cplx* __restrict__ dst, int64_t sD) {
  const int b = blockIdx.y;
  const int64_t cnt = (int64_t)R * p * R2;
  const int r = ranks[(int64_t)b * rs + k], r2 = ranks[(int64_t)b * rs + k + 1];
  src += b * sS;
  dst += b * sD;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cnt;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % R2);
    const int i = (int)((e / R2) % p);
    const int a = (int)(e / ((int64_t)R2 * p));
    dst[e] = (a < r && c < r2) ? src[((int64_t)a * p + i) * r2 + c] : make_double2(0.0, 0.0);
  }
}

// dst[e] = src[e * stride] for e < count per instance (a column of a matrix)
__global__ void k_amen_column(int64_t count, const cplx* __restrict__ src, int64_t stride,
                              int64_t sS, cplx* __restrict__ dst, int64_t sD) {
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) dst[b * sD + e] = src[b * sS + e * stride];
}

__global__ void k_amen_fill_ranks(int batch, int n, const int32_t* __restrict__ caps,
                                  int32_t* __restrict__ ranks) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < batch * (n + 1)) ranks[t] = caps[t % (n + 1)];
}

__global__ void k_amen_zero(int64_t count, cplx* p, int64_t stride) {
  const int b = blockIdx.y;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    p[b * stride + e] = make_double2(0.0, 0.0);
}

// PR[n] = [1; 1], the other boundaries = 1
__global__ void k_amen_ones(int batch, cplx* p, int64_t stride, int count) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < batch * count) p[(t / count) * stride + t % count] = make_double2(1.0, 0.0);
}

// Columns of Q whose R diagonal is exactly zero come from columns of the
// factored matrix that are exactly zero (capacity padding: a zero column stays
// zero under the earlier reflectors, so its reflector is the identity and
// R_jj = 0); the Householder Q still holds a unit vector there.  Zeroing those
// columns leaves the frame of the nonzero columns, with zero-padded slots.
__global__ void k_amen_dead_columns(int m, int s, int n, cplx* __restrict__ Q, int64_t sQ,
                                    const cplx* __restrict__ R, int64_t sR) {
  const int b = blockIdx.y;
  Q += b * sQ;
  R += b * sR;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)m * s;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(e % s);
    const cplx d = R[(int64_t)j * n + j];
    if (d.x == 0.0 && d.y == 0.0) Q[e] = make_double2(0.0, 0.0);
  }
}

namespace {

struct Sizes {
  int n = 0, B = 0;
  std::vector<int32_t> p, ra, cx, cy, cz, ly, lz;
  std::vector<int64_t> offx, offy, offz, offly, offlz, offPR, offPZY;
  int64_t sx = 0, sy = 0, sz = 0, sly = 0, slz = 0, sPR = 0, sPZY = 0;
  int64_t PL = 1, PZL = 1, PZYL = 1, T1 = 1, T2 = 1, YE = 1, ZA = 1, G = 1, H = 1;
  int64_t qW = 1, qR = 1, qtau = 1;
  bool qb = false;
  int64_t qb_v = 0, qb_t = 0, qb_w = 0, qb_tau = 0;
};

int64_t al32(int64_t v) { return (v + 31) & ~(int64_t)31; }

Sizes amen_sizes(const qt_mpo* A, const qt_tt* x, const qt_tt* y, const qt_tt* z) {
  Sizes s;
  const int n = x->n;
  s.n = n;
  s.B = x->batch;
  s.p.assign(x->modes, x->modes + n);
  s.ra.assign(A->ranks, A->ranks + n + 1);
  s.cx.assign(x->cap, x->cap + n + 1);
  s.cy.assign(y->cap, y->cap + n + 1);
  s.cz.assign(z->cap, z->cap + n + 1);
  // new frames: QR of (ly_k p) x (cy_{k+1} + cz_{k+1}) and (lz_k p) x cz_{k+1}
  s.ly.assign(n + 1, 1);
  s.lz.assign(n + 1, 1);
  for (int k = 0; k + 1 < n; ++k) {
    s.ly[k + 1] = std::min<int32_t>(s.ly[k] * s.p[k], s.cy[k + 1] + s.cz[k + 1]);
    s.lz[k + 1] = std::min<int32_t>(s.lz[k] * s.p[k], s.cz[k + 1]);
  }
  auto slots = [&](const std::vector<int32_t>& c, std::vector<int64_t>& off, int64_t& tot) {
    off.assign(n, 0);
    tot = 0;
    for (int k = 0; k < n; ++k) {
      off[k] = tot;
      tot += al32((int64_t)c[k] * s.p[k] * c[k + 1]);
    }
    tot = std::max<int64_t>(tot, 32);
  };
  slots(s.cx, s.offx, s.sx);
  slots(s.cy, s.offy, s.sy);
  slots(s.cz, s.offz, s.sz);
  slots(s.ly, s.offly, s.sly);
  slots(s.lz, s.offlz, s.slz);
  s.offPR.assign(n + 1, 0);
  s.offPZY.assign(n + 1, 0);
  for (int k = 1; k <= n; ++k) {
    const int64_t rows = k < n ? s.cy[k] + s.cz[k] : 2;
    s.offPR[k] = s.sPR;
    s.sPR += al32(rows * s.ra[k] * s.cx[k]);
    s.offPZY[k] = s.sPZY;
    s.sPZY += al32((int64_t)s.cz[k] * s.cy[k]);
  }
  auto mx = [](int64_t& a, int64_t b) { a = std::max(a, b); };
  for (int k = 0; k < n; ++k) {
    const int64_t p = s.p[k], a = s.ra[k], a1 = s.ra[k + 1], x = s.cx[k], x1 = s.cx[k + 1];
    const int64_t Rc = k + 1 < n ? s.cy[k + 1] + s.cz[k + 1] : 2;
    mx(s.PL, (int64_t)s.ly[k] * a * x);
    mx(s.PZL, (int64_t)s.lz[k] * a * x);
    mx(s.PZYL, (int64_t)s.lz[k] * s.ly[k]);
    mx(s.T1, std::max<int64_t>(s.ly[k], s.lz[k]) * a * p * x1);
    mx(s.T2, std::max<int64_t>(s.ly[k], s.lz[k]) * p * a1 * x1);
    mx(s.YE, (int64_t)s.ly[k] * p * Rc);
    mx(s.ZA, (int64_t)s.lz[k] * p * s.cz[k + 1]);
    mx(s.G, (int64_t)s.lz[k] * p * s.cy[k + 1]);
    mx(s.H, (int64_t)s.lz[k] * p * s.ly[k + 1]);
    if (k >= 1) {   // right pass: R1 (x p x Rc a1), R2 (p Rc a x), G1 (cy p x cz)
      mx(s.T1, x * p * Rc * a1);
      mx(s.T2, p * Rc * a * x);
      mx(s.G, (int64_t)s.cy[k] * p * s.cz[k + 1]);
    }
    const int64_t mq = (int64_t)s.ly[k] * p, nq = Rc;
    mx(s.qW, mq * nq);
    mx(s.qR, nq * nq);
    mx(s.qtau, nq + 8);
    mx(s.qW, (int64_t)s.lz[k] * p * s.cz[k + 1]);
    if (k + 1 < n && qr_blocked_wanted((int)mq, (int)nq)) {
      int64_t v, t, w;
      qr_blocked_ws_elems((int)mq, (int)nq, &v, &t, &w);
      s.qb = true;
      mx(s.qb_v, v);
      mx(s.qb_t, t);
      mx(s.qb_w, w);
      mx(s.qb_tau, qr_blocked_tau_elems((int)mq, (int)nq));
    }
  }
  return s;
}

size_t amen_bytes(const Sizes& s) {
  const int64_t B = s.B;
  int64_t e = s.sx + s.sy + s.sz + s.sly + s.slz + s.sPR + s.sPZY + 2 * s.PL + 2 * s.PZL +
              2 * s.PZYL + s.T1 + s.T2 + s.YE + s.ZA + s.G + s.H + s.qW + s.qR;
  if (s.qb) e += s.qb_v + s.qb_t + 2 * s.qb_w;
  size_t bytes = sizeof(cplx) * B * e + sizeof(double) * B * (s.qtau + s.qb_tau) +
                 sizeof(int32_t) * (2 * B * (s.n + 1) + 2 * (s.n + 1) + 2 * B) + 40 * 256;
  return bytes;
}

}  // namespace

qt_status amen_impl(qt_ctx ctx, const qt_mpo* A, const qt_tt* x, qt_tt* y, qt_tt* z, double eps,
                    int max_rank, int sweeps, double* err_out) {
  // the sweep projects onto right-orthogonal frames: bring y and z there
  // (an exact right orthogonalization: a QR sweep from the last core)
  qt_round_opts r0{};
  r0.mode = QT_ROUND_SVD;
  {
    const size_t m0 = ctx->ws_top;
    QT_TRY(round_impl(ctx, y, &r0, nullptr, nullptr, false, nullptr, 0, 0, true));
    ctx->ws_top = m0;
    QT_TRY(round_impl(ctx, z, &r0, nullptr, nullptr, false, nullptr, 0, 0, true));
    ctx->ws_top = m0;
  }
  const Sizes s = amen_sizes(A, x, y, z);
  const int n = s.n, B = s.B, rs = n + 1;
  hipStream_t st = ctx->stream;
  auto take = [&](int64_t elems) { return (cplx*)ws_take(ctx, sizeof(cplx) * B * elems); };
  cplx* X = take(s.sx);
  cplx* Y = take(s.sy);
  cplx* Zo = take(s.sz);
  cplx* Yn = take(s.sly);
  cplx* Zn = take(s.slz);
  cplx* PR = take(s.sPR);
  cplx* PZY = take(s.sPZY);
  cplx* PL[2] = {take(s.PL), take(s.PL)};
  cplx* PZL[2] = {take(s.PZL), take(s.PZL)};
  cplx* PZYL[2] = {take(s.PZYL), take(s.PZYL)};
  cplx* T1 = take(s.T1);
  cplx* T2 = take(s.T2);
  cplx* YE = take(s.YE);
  cplx* ZA = take(s.ZA);
  cplx* G = take(s.G);
  cplx* H = take(s.H);
  cplx* qW = take(s.qW);
  cplx* qR = take(s.qR);
  double* qtau = (double*)ws_take(ctx, sizeof(double) * B * s.qtau);
  int32_t* rk_y = (int32_t*)ws_take(ctx, sizeof(int32_t) * B * (n + 1));
  int32_t* rk_z = (int32_t*)ws_take(ctx, sizeof(int32_t) * B * (n + 1));
  int32_t* caps = (int32_t*)ws_take(ctx, sizeof(int32_t) * 2 * (n + 1));
  int32_t* qs = (int32_t*)ws_take(ctx, sizeof(int32_t) * 2 * B);
  QT_CHECK(X && Y && Zo && Yn && Zn && PR && PZY && PL[1] && PZL[1] && PZYL[1] && T1 && T2 &&
               YE && ZA && G && H && qW && qR && qtau && rk_y && rk_z && caps && qs,
           QT_ENOMEM, "tt_amen_mv: workspace too small");
  QrBlkWs qb{};
  if (s.qb) {
    qb.V = take(s.qb_v);
    qb.v_stride = s.qb_v;
    qb.T = take(s.qb_t);
    qb.t_stride = s.qb_t;
    qb.W1 = take(s.qb_w);
    qb.W2 = take(s.qb_w);
    qb.w_stride = s.qb_w;
    qb.tau = (double*)ws_take(ctx, sizeof(double) * B * s.qb_tau);
    qb.tau_stride = s.qb_tau;
    qb.s_dev = (int32_t*)ws_take(ctx, sizeof(int32_t) * B);
    QT_CHECK(qb.V && qb.T && qb.W1 && qb.W2 && qb.tau && qb.s_dev, QT_ENOMEM,
             "tt_amen_mv: blocked QR workspace too small");
  }
  const size_t mark = ctx->ws_top;
  {
    std::vector<int32_t> hc(2 * (n + 1));
    for (int k = 0; k <= n; ++k) {
      hc[k] = s.ly[k];
      hc[n + 1 + k] = s.lz[k];
    }
    QT_HIP(hipMemcpyAsync(caps, hc.data(), sizeof(int32_t) * hc.size(), hipMemcpyHostToDevice, st));
  }
  const Str S0{nullptr, 0, 0, 0};
  auto sc = [](int64_t v) { return sconst(v); };
  auto dc = [](int v) { return dconst(v); };
  const cplx one = make_double2(1.0, 0.0), mone = make_double2(-1.0, 0.0);
  const cplx* Ad = (const cplx*)A->data;
  auto unpack = [&](const qt_tt* t, const std::vector<int32_t>& cap, const std::vector<int64_t>& off,
                    int64_t stride, cplx* dst) {
    for (int k = 0; k < n; ++k) {
      const int64_t cnt = (int64_t)cap[k] * s.p[k] * cap[k + 1];
      dim3 grid((unsigned)std::min<int64_t>((cnt + 255) / 256, 4096), B);
      k_amen_unpack<<<grid, 256, 0, st>>>(s.p[k], cap[k], cap[k + 1], t->ranks, rs, k,
                                          (const cplx*)t->data + t->offsets[k], t->inst_stride,
                                          dst + off[k], stride);
    }
  };
  // Q (mcap x min(mcap, ncap), row-major) of the row-major mcap x ncap matrix
  // Amat; sA and sQ are the instance strides of the two buffers
  auto qr_any = [&](int mcap, int ncap, cplx* Amat, int64_t sA, cplx* Q, int64_t sQ,
                    int32_t* sout) {
    if (s.qb && qr_blocked_wanted(mcap, ncap))
      qr_blocked(st, B, mcap, ncap, dc(mcap), dc(ncap), Amat, sA, qW, s.qW, qb, Q, sQ, qR, s.qR,
                 sout, 1);
    else
      qr_auto(st, B, mcap, ncap, dc(mcap), dc(ncap), Amat, sA, qW, s.qW, qtau, s.qtau, Q, sQ, qR,
              s.qR, sout, 1);
    const int sc_ = std::min(mcap, ncap);
    dim3 grid((unsigned)std::min<int64_t>(((int64_t)mcap * sc_ + 255) / 256, 2048), B);
    k_amen_dead_columns<<<grid, 256, 0, st>>>(mcap, sc_, ncap, Q, sQ, qR, s.qR);
  };
  // (A_k x_k) applied to the left interface IN (rows m): T2[m][i][a'][x']
  auto apply_local = [&](int k, int m, const cplx* IN, int64_t sIN) {
    const int p = s.p[k], a = s.ra[k], a1 = s.ra[k + 1], xx = s.cx[k], x1 = s.cx[k + 1];
    const cplx* Xk = X + s.offx[k];
    // T1[(m, a), (j, x')] = IN[(m, a), x] x_k[x, (j, x')]
    gemm_ex(st, B, 1, 1, dc(m * a), dc(p * x1), dc(xx), m * a, p * x1,
            mat(IN, sIN, sc(xx), sc(1)), false,
            mat(Xk, s.sx, sc((int64_t)p * x1), sc(1)), false, mat(T1, s.T1, sc((int64_t)p * x1), sc(1)),
            one, false);
    const cplx* Ak = Ad + A->offsets[k];
    if (A->diag[k]) {
      // item (m, i): T2 (a' x x') = A_k[:, i, :]^T T1[(m, :), (i, :)]
      gemm_ex(st, B, m, p, dc(a1), dc(x1), dc(a), a1, x1,
              mat_op(A, Ak, sc(1), sc((int64_t)p * a1), S0, sc(a1)), false,
              mat(T1, s.T1, sc((int64_t)p * x1), sc(1), sc((int64_t)a * p * x1), sc(x1)), false,
              mat(T2, s.T2, sc(x1), sc(1), sc((int64_t)p * a1 * x1), sc((int64_t)a1 * x1)), one,
              false);
    } else {
      for (int j = 0; j < p; ++j)
        gemm_ex(st, B, m, p, dc(a1), dc(x1), dc(a), a1, x1,
                mat_op(A, Ak + (int64_t)j * a1, sc(1), sc((int64_t)p * p * a1), S0,
                       sc((int64_t)p * a1)),
                false, mat(T1 + (int64_t)j * x1, s.T1, sc((int64_t)p * x1), sc(1),
                           sc((int64_t)a * p * x1), S0),
                false,
                mat(T2, s.T2, sc(x1), sc(1), sc((int64_t)p * a1 * x1), sc((int64_t)a1 * x1)), one,
                j > 0);
    }
  };

  for (int sw = 0; sw < sweeps; ++sw) {
    unpack(x, s.cx, s.offx, s.sx, X);
    unpack(y, s.cy, s.offy, s.sy, Y);
    unpack(z, s.cz, s.offz, s.sz, Zo);
    k_amen_ones<<<(B * 2 + 127) / 128, 128, 0, st>>>(B, PR + s.offPR[n], s.sPR, 2);
    k_amen_ones<<<(B + 127) / 128, 128, 0, st>>>(B, PZY + s.offPZY[n], s.sPZY, 1);
    // ---- right interfaces from the old (right-orthogonal) frames
    for (int k = n - 1; k >= 1; --k) {
      const int p = s.p[k], a = s.ra[k], a1 = s.ra[k + 1], xx = s.cx[k], x1 = s.cx[k + 1];
      const int Y1 = s.cy[k + 1], Z1 = s.cz[k + 1];
      const int Rc = k + 1 < n ? Y1 + Z1 : 2;
      const cplx* Xk = X + s.offx[k];
      const cplx* Pn = PR + s.offPR[k + 1];
      // R1[(x, j), (r, a')] = x_k[(x, j), x'] PR[k+1][(r, a'), x']
      gemm_ex(st, B, 1, 1, dc(xx * p), dc(Rc * a1), dc(x1), xx * p, Rc * a1,
              mat(Xk, s.sx, sc(x1), sc(1)), false, mat(Pn, s.sPR, sc(1), sc(x1)), false,
              mat(T1, s.T1, sc((int64_t)Rc * a1), sc(1)), one, false);
      // R2[i][r][a][x] = sum_{j, a'} A_k[a, i, j, a'] R1[(x, j), (r, a')]
      const cplx* Ak = Ad + A->offsets[k];
      const Mat R2 = mat(T2, s.T2, sc((int64_t)a * xx), sc(xx), sc(1), sc((int64_t)Rc * a * xx));
      if (A->diag[k]) {
        gemm_ex(st, B, xx, p, dc(Rc), dc(a), dc(a1), Rc, a,
                mat(T1, s.T1, sc(a1), sc(1), sc((int64_t)p * Rc * a1), sc((int64_t)Rc * a1)), false,
                mat_op(A, Ak, sc(1), sc((int64_t)p * a1), S0, sc(a1)), false, R2, one, false);
      } else {
        for (int j = 0; j < p; ++j)
          gemm_ex(st, B, xx, p, dc(Rc), dc(a), dc(a1), Rc, a,
                  mat(T1 + (int64_t)j * Rc * a1, s.T1, sc(a1), sc(1), sc((int64_t)p * Rc * a1), S0),
                  false,
                  mat_op(A, Ak + (int64_t)j * a1, sc(1), sc((int64_t)p * p * a1), S0,
                         sc((int64_t)p * a1)),
                  false, R2, one, j > 0);
      }
      // PR[k] rows: the y frames' (ry_k of them), then the z frames' right
      // after them, zeros to the end (sum over i of conj(frame_k[., i, .]) R2[i])
      cplx* Pk = PR + s.offPR[k];
      const int64_t ax = (int64_t)a * xx;
      {
        const int64_t cnt = (int64_t)(s.cy[k] + s.cz[k]) * ax;
        k_amen_zero<<<dim3((unsigned)std::min<int64_t>((cnt + 255) / 256, 2048), B), 256, 0, st>>>(
            cnt, Pk, s.sPR);
      }
      for (int i = 0; i < p; ++i) {
        gemm_ex(st, B, 1, 1, dc(s.cy[k]), dc(a * xx), dc(Y1), s.cy[k], a * xx,
                mat(Y + s.offy[k] + (int64_t)i * Y1, s.sy, sc((int64_t)p * Y1), sc(1)), true,
                mat(T2 + (int64_t)i * Rc * ax, s.T2, sc(ax), sc(1)), false, mat(Pk, s.sPR, sc(ax), sc(1)),
                one, i > 0);
        gemm_ex(st, B, 1, 1, dc(s.cz[k]), dc(a * xx), dc(Z1), s.cz[k], a * xx,
                mat(Zo + s.offz[k] + (int64_t)i * Z1, s.sz, sc((int64_t)p * Z1), sc(1)), true,
                mat(T2 + (int64_t)i * Rc * ax, s.T2, sc(ax), sc(1), S0, S0,
                    sref(y->ranks + k + 1, rs, ax)),
                false,
                mat(Pk, s.sPR, sc(ax), sc(1), S0, S0, sref(y->ranks + k, rs, ax)), one, i > 0);
      }
      // PZY[k][z, y] = sum conj(z_k[z, (i, Z')]) (y_k PZY[k+1]^T)[(y, i), Z']
      gemm_ex(st, B, 1, 1, dc(s.cy[k] * p), dc(Z1), dc(Y1), s.cy[k] * p, Z1,
              mat(Y + s.offy[k], s.sy, sc(Y1), sc(1)), false,
              mat(PZY + s.offPZY[k + 1], s.sPZY, sc(1), sc(Y1)), false,
              mat(G, s.G, sc(Z1), sc(1)), one, false);
      gemm_ex(st, B, 1, 1, dc(s.cz[k]), dc(s.cy[k]), dc(p * Z1), s.cz[k], s.cy[k],
              mat(Zo + s.offz[k], s.sz, sc((int64_t)p * Z1), sc(1)), true,
              mat(G, s.G, sc(1), sc((int64_t)p * Z1)), false,
              mat(PZY + s.offPZY[k], s.sPZY, sc(s.cy[k]), sc(1)), one, false);
    }
    // ---- left sweep
    k_amen_ones<<<(B + 127) / 128, 128, 0, st>>>(B, PL[0], s.PL, 1);
    k_amen_ones<<<(B + 127) / 128, 128, 0, st>>>(B, PZL[0], s.PZL, 1);
    k_amen_ones<<<(B + 127) / 128, 128, 0, st>>>(B, PZYL[0], s.PZYL, 1);
    int cur = 0;
    for (int k = 0; k < n; ++k) {
      const int p = s.p[k], a1 = s.ra[k + 1], x1 = s.cx[k + 1];
      const int l = s.ly[k], lz = s.lz[k];
      const bool last = k == n - 1;
      const int Y1 = last ? 1 : s.cy[k + 1], Z1 = last ? 1 : s.cz[k + 1];
      const int Rc = last ? 2 : Y1 + Z1;
      const int64_t A1X1 = (int64_t)a1 * x1;
      const cplx* Pn = PR + s.offPR[k + 1];
      // y side: T2 = (PL x_k) A_k, YE = T2 PR[k+1]^T
      apply_local(k, l, PL[cur], s.PL);
      gemm_ex(st, B, 1, 1, dc(l * p), dc(Rc), dc((int)A1X1), l * p, Rc,
              mat(T2, s.T2, sc(A1X1), sc(1)), false, mat(Pn, s.sPR, sc(1), sc(A1X1)), false,
              mat(YE, s.YE, sc(Rc), sc(1)), one, false, Dim{nullptr, 0, 0, 1 << 30}, A1X1);
      if (last) {
        k_amen_column<<<dim3((unsigned)((l * p + 255) / 256), B), 256, 0, st>>>(
            (int64_t)l * p, YE, Rc, s.YE, Yn + s.offly[k], s.sly);
      } else {
        const int l1 = s.ly[k + 1];
        qr_any(l * p, Rc, YE, s.YE, Yn + s.offly[k], s.sly, qs);
        // PL <- Q^H T2
        gemm_ex(st, B, 1, 1, dc(l1), dc((int)A1X1), dc(l * p), l1, (int)A1X1,
                mat(Yn + s.offly[k], s.sly, sc(1), sc(l1)), true, mat(T2, s.T2, sc(A1X1), sc(1)),
                false, mat(PL[cur ^ 1], s.PL, sc(A1X1), sc(1)), one, false,
                Dim{nullptr, 0, 0, 1 << 30}, (int64_t)l * p);
      }
      // z side: ZA = (PZL x_k) A_k PR[k+1]_z^T - PZYL y_k PZY[k+1]^T
      apply_local(k, lz, PZL[cur], s.PZL);
      // the z rows of PR[k+1] follow its ry_{k+1} y rows
      gemm_ex(st, B, 1, 1, dc(lz * p), dc(Z1), dc((int)A1X1), lz * p, Z1,
              mat(T2, s.T2, sc(A1X1), sc(1)), false,
              mat(Pn, s.sPR, sc(1), sc(A1X1), S0, S0, sref(y->ranks + k + 1, rs, A1X1)), false,
              mat(ZA, s.ZA, sc(Z1), sc(1)), one, false, Dim{nullptr, 0, 0, 1 << 30}, A1X1);
      // G[z][i][y'] = PZYL[z, s] YE[(s, i), y'] (the local solution's columns)
      gemm_ex(st, B, p, 1, dc(lz), dref(y->ranks + k + 1, rs), dc(l), lz, Y1,
              mat(PZYL[cur], s.PZYL, sc(l), sc(1)), false,
              mat(YE, s.YE, sc((int64_t)p * Rc), sc(1), sc(Rc)), false,
              mat(G, s.G, sc((int64_t)p * Y1), sc(1), sc(Y1)), one, false);
      // ZA -= G PZY[k+1]^T
      gemm_ex(st, B, 1, 1, dc(lz * p), dc(Z1), dref(y->ranks + k + 1, rs), lz * p, Z1,
              mat(G, s.G, sc(Y1), sc(1)), false,
              mat(PZY + s.offPZY[k + 1], s.sPZY, sc(1), sc(Y1)), false, mat(ZA, s.ZA, sc(Z1), sc(1)),
              mone, true);
      if (last) {
        copy(st, B, dc(lz * p), dc(1), (int64_t)lz * p, ZA, s.ZA, Zn + s.offlz[k], s.slz);
        break;
      }
      const int lz1 = s.lz[k + 1], l1 = s.ly[k + 1];
      qr_any(lz * p, Z1, ZA, s.ZA, Zn + s.offlz[k], s.slz, qs + B);
      // PZL <- Qz^H T2
      gemm_ex(st, B, 1, 1, dc(lz1), dc((int)A1X1), dc(lz * p), lz1, (int)A1X1,
              mat(Zn + s.offlz[k], s.slz, sc(1), sc(lz1)), true, mat(T2, s.T2, sc(A1X1), sc(1)),
              false, mat(PZL[cur ^ 1], s.PZL, sc(A1X1), sc(1)), one, false);
      // PZYL <- Qz^H (PZYL (x) I_p) Q
      gemm_ex(st, B, p, 1, dc(lz), dc(l1), dc(l), lz, l1, mat(PZYL[cur], s.PZYL, sc(l), sc(1)), false,
              mat(Yn + s.offly[k], s.sly, sc((int64_t)p * l1), sc(1), sc(l1)), false,
              mat(H, s.H, sc((int64_t)p * l1), sc(1), sc(l1)), one, false);
      gemm_ex(st, B, 1, 1, dc(lz1), dc(l1), dc(lz * p), lz1, l1,
              mat(Zn + s.offlz[k], s.slz, sc(1), sc(lz1)), true, mat(H, s.H, sc(l1), sc(1)), false,
              mat(PZYL[cur ^ 1], s.PZYL, sc(l1), sc(1)), one, false);
      cur ^= 1;
    }
    // ---- truncation of y, right-orthogonalization of z, back into y and z
    k_amen_fill_ranks<<<(B * (n + 1) + 127) / 128, 128, 0, st>>>(B, n, caps, rk_y);
    k_amen_fill_ranks<<<(B * (n + 1) + 127) / 128, 128, 0, st>>>(B, n, caps + n + 1, rk_z);
    TTLayout ly;
    ly.modes = s.p;
    ly.cap = s.ly;
    ly.off = s.offly;
    ly.stride = s.sly;
    qt_tt ty = ly.view(Yn, rk_y, B);
    TTLayout lz;
    lz.modes = s.p;
    lz.cap = s.lz;
    lz.off = s.offlz;
    lz.stride = s.slz;
    qt_tt tz = lz.view(Zn, rk_z, B);
    qt_round_opts ro{};
    ro.eps = eps;
    ro.max_rank = max_rank;
    ro.mode = QT_ROUND_SVD;
    ctx->ws_top = mark;
    // the sweep left y's cores 0..n-2 as Q factors (orthonormal columns, the
    // padding's zeroed): the rounding needs no left QR sweep
    QT_TRY(round_impl(ctx, &ty, &ro, sw + 1 == sweeps ? err_out : nullptr, nullptr, false, nullptr,
                      0, 0, false, true));
    ctx->ws_top = mark;
    QT_TRY(round_impl(ctx, &tz, &r0, nullptr, nullptr, false, nullptr, 0, 0, true));
    ctx->ws_top = mark;
    for (int k = 0; k < n; ++k) {
      copy(st, B, dref(rk_y + k, rs, s.p[k]), dref(rk_y + k + 1, rs),
           (int64_t)s.cy[k] * s.p[k] * s.cy[k + 1], Yn + s.offly[k], s.sly,
           (cplx*)y->data + y->offsets[k], y->inst_stride);
      copy(st, B, dref(rk_z + k, rs, s.p[k]), dref(rk_z + k + 1, rs),
           (int64_t)s.cz[k] * s.p[k] * s.cz[k + 1], Zn + s.offlz[k], s.slz,
           (cplx*)z->data + z->offsets[k], z->inst_stride);
    }
    copy_i32(st, (int64_t)B * (n + 1), rk_y, y->ranks);
    copy_i32(st, (int64_t)B * (n + 1), rk_z, z->ranks);
  }
  QT_HIP(hipGetLastError());
  return QT_OK;
}

size_t amen_ws_bytes(const qt_mpo* A, const qt_tt* x, const qt_tt* y, const qt_tt* z, int max_rank) {
  const Sizes s = amen_sizes(A, x, y, z);
  TTLayout ly;
  ly.modes = s.p;
  ly.cap = s.ly;
  ly.off = s.offly;
  ly.stride = s.sly;
  std::vector<int32_t> dummy(1);
  qt_tt ty = ly.view(nullptr, dummy.data(), s.B);
  TTLayout lz;
  lz.modes = s.p;
  lz.cap = s.lz;
  lz.off = s.offlz;
  lz.stride = s.slz;
  qt_tt tz = lz.view(nullptr, dummy.data(), s.B);
  const int lmax = max_rank > 0 ? max_rank : (1 << 30);
  return std::max({amen_bytes(s) + std::max(round_ws_layout(&ty, lmax).bytes,
                                            round_ws_layout(&tz, 1 << 30).bytes),
                   round_ws_layout(y, 1 << 30).bytes, round_ws_layout(z, 1 << 30).bytes});
}

}  // namespace qt

using namespace qt;

extern "C" qt_status tt_amen_mv(qt_ctx ctx, const qt_mpo* A, const qt_tt* x, qt_tt* y, qt_tt* z,
                                double eps, int32_t max_rank, int32_t sweeps, double* err_out) {
  qt::enter(ctx);
  QT_CHECK(ctx && A && x && y && z, QT_EINVAL, "tt_amen_mv: null argument");
  QT_TRY(qt::tt_validate(x, "x"));
  QT_TRY(qt::tt_validate(y, "y"));
  QT_TRY(qt::tt_validate(z, "z"));
  QT_CHECK(eps >= 0.0 && max_rank >= 0 && sweeps >= 1, QT_EINVAL,
           "tt_amen_mv: eps < 0, max_rank < 0 or sweeps < 1");
  const int n = x->n;
  QT_CHECK(A->n == n && y->n == n && z->n == n, QT_EINVAL, "tt_amen_mv: core counts differ");
  QT_CHECK(y->batch == x->batch && z->batch == x->batch, QT_EINVAL, "tt_amen_mv: batches differ");
  QT_CHECK(A->inst_stride == 0 || A->inst_group >= 1, QT_EINVAL, "tt_amen_mv: bad operator group");
  int64_t left = 1;
  std::vector<int64_t> right(n + 1, 1);
  for (int k = n - 1; k >= 0; --k) right[k] = std::min<int64_t>(right[k + 1] * x->modes[k], 1 << 30);
  for (int k = 0; k < n; ++k) {
    QT_CHECK(A->modes_out[k] == x->modes[k] && A->modes_in[k] == x->modes[k] &&
                 y->modes[k] == x->modes[k] && z->modes[k] == x->modes[k],
             QT_EINVAL, "tt_amen_mv: modes differ (A must be square on x's modes)");
    left = std::min<int64_t>(left * x->modes[k], 1 << 30);
    // y must hold the rounded result: min(max_rank, natural bound) at every bond
    const int64_t need = std::min<int64_t>({left, right[k + 1], max_rank > 0 ? max_rank : (1 << 30)});
    QT_CHECK(k + 1 == n || y->cap[k + 1] >= need, QT_EINVAL,
             "tt_amen_mv: y's capacity is below min(max_rank, natural rank) at a bond");
  }
  ctx->ws_top = 0;
  QT_TRY(qt::ws_reserve(ctx, qt::amen_ws_bytes(A, x, y, z, max_rank)));
  return qt::amen_impl(ctx, A, x, y, z, eps, max_rank, sweeps, err_out);
}
