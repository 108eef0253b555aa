// Product-aware randomized rounding of x = Op (*) y (x never materialized).
//
// x has cores X_k(i) = sum_j D_k(i, j) (Kronecker) Y_k(j) (TT x TTO contraction,
// Sec. 2.1 of arXiv 2512.07811; a Hadamard product is the diagonal case, eq.
// tt_to_tto).  Its rank R_k = r_D r_y is never formed.  Randomize-then-
// orthogonalize (Al Daas et al., SIAM J. Sci. Comput. 2023) with a Gaussian
// train Omega of ranks l_k:
//   right pass  W_k = sum_i X_k(i) W_{k+1} Omega_k(i)^T        (R_k x l_k)
//   left pass   Y_k = Z_k W_{k+1};  Q_k = qr(Y_k);  M_k = Q_k^H Z_k;
//               Z_{k+1} = M_k X_{k+1}
// Every contraction with X_k is split into GEMMs with D_k and Y_k separately,
// so the work is O(p l R (r_D + r_y)) per core instead of O(p R^3).
//
// Also here: <y, Q y> for a diagonal/component operator Q (exact squared norm
// of a product through Op^H Op), and the Philox4x32-10 Gaussian generator.
#include "kernels.h"
#include "round.h"
#include "sketch.h"

namespace qt {

// ------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of
//   (hi0, lo0) = mulhilo(0xD2511F53, c0), (hi1, lo1) = mulhilo(0xCD9E8D57, c2)
//   c = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0);  k += (0x9E3779B9, 0xBB67AE85)
// Gaussian t of stream s: counter (t_lo, t_hi, s_lo, s_hi), key = seed; the
// first two outputs u0, u1 map to (x + 1) 2^-32 in (0, 1]; Box-Muller
// z = sqrt(-2 ln u0) cos(2 pi u1).
__host__ __device__ inline void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__device__ inline double gauss(uint64_t seed, uint64_t stream, uint64_t t) {
  uint32_t c[4] = {(uint32_t)t, (uint32_t)(t >> 32), (uint32_t)stream, (uint32_t)(stream >> 32)};
  philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  double u0 = ((double)c[0] + 1.0) * 2.3283064365386963e-10;
  double u1 = ((double)c[1] + 1.0) * 2.3283064365386963e-10;
  return sqrt(-2.0 * log(u0)) * cos(6.283185307179586 * u1);
}

// stream = (base ? 4 * base[0] : 0) + add: a captured graph reads the iteration
// number from device memory, so that every replay draws new Gaussians.
__global__ void k_gauss_fill(int64_t count, uint64_t seed, const uint64_t* base, uint64_t add,
                             cplx* out) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stream = (base ? 4 * base[0] : 0) + add;
  if (t < count) out[t] = make_double2(gauss(seed, stream, (uint64_t)t), 0.0);
}

void gauss_fill(hipStream_t st, int64_t count, uint64_t seed, uint64_t stream, cplx* out,
                const uint64_t* base) {
  if (count <= 0) return;
  k_gauss_fill<<<(unsigned)((count + 255) / 256), 256, 0, st>>>(count, seed, base, stream, out);
}

// ----------------------------------------------------------- helpers
__global__ void k_fill_one(int batch, cplx* p, int64_t stride) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < batch) p[b * stride] = make_double2(1.0, 0.0);
}

__global__ void k_init_ranks_one(int n, int batch, int32_t* r) {
  int b = blockIdx.x;
  if (b >= batch) return;
  if (threadIdx.x == 0) {
    r[(int64_t)b * (n + 1)] = 1;
    r[(int64_t)b * (n + 1) + n] = 1;
  }
}

__global__ void k_sumsq(Dim Rd, Dim Cd, const cplx* X, int64_t sX, double* out, double scale) {
  __shared__ double red[16];
  const int b = blockIdx.x;
  const int64_t cnt = (int64_t)dimv(Rd, b) * dimv(Cd, b);
  X += b * sX;
  double a = 0.0;
  for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) a += cabs2(X[e]);
  a = wave_sum(a);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
    out[b] = scale * t;
  }
}

void sumsq(hipStream_t st, int batch, Dim rows, Dim cols, const cplx* X, int64_t sX, double* out,
           double scale) {
  k_sumsq<<<batch, 256, 0, st>>>(rows, cols, X, sX, out, scale);
}

static const Str S0{nullptr, 0, 0, 0};
static inline Str sc(int64_t v) { return sconst(v); }

SketchWs sketch_ws_layout(const qt_mpo* A, const qt_tt* y, const std::vector<int32_t>& ell) {
  SketchWs w;
  const int n = y->n;
  w.Woff.assign(n + 1, 0);
  int64_t acc = 0;
  for (int k = 1; k <= n; ++k) {
    w.Woff[k] = acc;
    int64_t s = (int64_t)A->ranks[k] * y->cap[k] * ell[k];
    acc += (s + 31) & ~(int64_t)31;
  }
  w.Wtot = std::max<int64_t>(acc, 1);
  auto mx = [](int64_t& a, int64_t b) { a = std::max(a, b); };
  for (int k = 0; k < n; ++k) {
    const int64_t p = y->modes[k];
    const int64_t kd = (A->diag[k] ? p : p * p) * A->ranks[k + 1];
    mx(w.T1, (int64_t)A->ranks[k + 1] * y->cap[k + 1] * ell[k] * p);
    mx(w.T2, (A->diag[k] ? p : p * p) * A->ranks[k + 1] * y->cap[k] * ell[k]);
    mx(w.M, (int64_t)ell[k] * A->ranks[k] * y->cap[k]);
    mx(w.M, (int64_t)ell[k + 1] * A->ranks[k + 1] * y->cap[k + 1]);
    mx(w.T3, (int64_t)ell[k] * y->cap[k] * kd);
    mx(w.Z, (int64_t)ell[k] * p * A->ranks[k + 1] * y->cap[k + 1]);
    mx(w.Y, (int64_t)ell[k] * p * ell[k + 1]);
    mx(w.R, (int64_t)ell[k + 1] * ell[k + 1]);
    mx(w.tau, ell[k + 1]);
    if (k < n - 1 && qr_blocked_wanted((int)(ell[k] * p), ell[k + 1])) {
      int64_t v, t, wq;
      qr_blocked_ws_elems((int)(ell[k] * p), ell[k + 1], &v, &t, &wq);
      mx(w.qb_v, v);
      mx(w.qb_t, t);
      mx(w.qb_w, wq);
      mx(w.qb_tau, qr_blocked_tau_elems((int)(ell[k] * p), ell[k + 1]));
    }
  }
  const int B = y->batch;
  w.bytes = sizeof(cplx) * B * (w.Wtot + w.T1 + w.T2 + w.M + w.T3 + w.Z + 2 * w.Y + w.R) +
            sizeof(double) * B * (w.tau + 2) + 16 * 256;
  if (w.qb_v > 0)
    w.bytes += sizeof(cplx) * B * (w.qb_v + w.qb_t + 2 * w.qb_w) +
               sizeof(double) * B * w.qb_tau + sizeof(int32_t) * B + 8 * 256;
  return w;
}

// |R_jj| of the sketch QR at bond k+1, sorted descending; block b handles
// instance b (R slice sR, rank s_rank[b * rs], output slice so)
__global__ void k_rdiag(const cplx* R, int64_t sR, int ldr, const int32_t* s_rank, int rs,
                        double* out, int64_t so) {
  __shared__ double v[RD_MAX];
  const int b = blockIdx.x;
  R += b * sR;
  out += b * so;
  const int s = min(s_rank[(int64_t)b * rs], RD_MAX);
  for (int j = threadIdx.x; j < RD_MAX; j += blockDim.x)
    v[j] = j < s ? sqrt(cabs2(R[(int64_t)j * ldr + j])) : 0.0;
  __syncthreads();
  for (int j = threadIdx.x; j < RD_MAX; j += blockDim.x) {
    const double x = v[j];
    int pos = 0;
    for (int i = 0; i < RD_MAX; ++i) pos += (v[i] > x) || (v[i] == x && i < j);
    out[pos] = x;
  }
}

qt_status sketch_impl(qt_ctx ctx, const qt_mpo* A, const qt_tt* y, const cplx* omega,
                      const std::vector<int64_t>& om_off, const std::vector<int32_t>& ell,
                      qt_tt* out, double* ynorm2, double* rdiag, bool f32) {
  const int n = y->n, B = y->batch;
  hipStream_t st = ctx->stream;
  SketchWs w = sketch_ws_layout(A, y, ell);
  cplx* Wall = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.Wtot);
  cplx* T1 = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.T1);
  cplx* T2 = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.T2);
  cplx* Mb = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.M);
  cplx* T3 = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.T3);
  cplx* Zb = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.Z);
  cplx* Yb = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.Y);
  cplx* Wq = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.Y);
  cplx* Rb = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.R);
  double* tau = (double*)ws_take(ctx, sizeof(double) * B * w.tau);
  QT_CHECK(Wall && T1 && T2 && Mb && T3 && Zb && Yb && Wq && Rb && tau, QT_ENOMEM,
           "sketch: workspace too small");
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
             "sketch: blocked QR workspace too small");
  }
  const int rs = n + 1;
  int32_t* ry = y->ranks;
  int32_t* ro = out->ranks;
  const cplx* Yd = (const cplx*)y->data;
  const cplx* Dd = (const cplx*)A->data;
  cplx* Od = (cplx*)out->data;
  const int64_t iW = w.Wtot, iT1 = w.T1, iT2 = w.T2, iM = w.M, iT3 = w.T3, iZ = w.Z, iY = w.Y;
  const cplx one = make_double2(1.0, 0.0);

  // ---- right pass: W_n = 1
  k_fill_one<<<(B + 127) / 128, 128, 0, st>>>(B, Wall + w.Woff[n], iW);
  for (int k = n - 1; k >= 1; --k) {
    GemmF32Scope prec(f32);
    const int p = y->modes[k];
    const int lk = ell[k], lk1 = ell[k + 1];
    const int rd = A->ranks[k], rd1 = A->ranks[k + 1];
    const bool diag = A->diag[k] != 0;
    const int kd = (diag ? p : p * p) * rd1;
    const cplx* Om = omega + om_off[k];
    const cplx* Yk = Yd + y->offsets[k];
    // T1[(a', b'), (g, i)] = sum_g' W_{k+1}[(a', b'), g'] Omega_k[(g, i), g']
    gemm_ex(st, B, 1, 1, dref(ry + k + 1, rs, rd1), dconst(lk * p), dconst(lk1), rd1 * y->cap[k + 1],
            lk * p, mat(Wall + w.Woff[k + 1], iW, sc(lk1), sc(1)), false,
            mat(Om, 0, sc(1), sc(lk1)), false, mat(T1, iT1, sc(lk * p), sc(1)), one, false);
    // T2[(i [j] a')][b][g] = sum_b' Y_k[b, j, b'] T1[(a', b'), (g, i)]
    const int64_t t2_ia = (int64_t)rd1 * y->cap[k] * lk;      // one (i) or (i, j) block
    const int64_t t2_a = (int64_t)y->cap[k] * lk;
    if (diag) {
      gemm_ex(st, B, p, rd1, dref(ry + k, rs), dconst(lk), dref(ry + k + 1, rs), y->cap[k], lk,
              mat(Yk, y->inst_stride, sref(ry + k + 1, rs, p), sc(1), sref(ry + k + 1, rs, 1)), false,
              mat(T1, iT1, sc(lk * p), sc(p), sc(1), sref(ry + k + 1, rs, (int64_t)lk * p)), false,
              mat(T2, iT2, sc(lk), sc(1), sc(t2_ia), sc(t2_a)), one, false);
    } else {
      for (int i = 0; i < p; ++i)
        gemm_ex(st, B, p, rd1, dref(ry + k, rs), dconst(lk), dref(ry + k + 1, rs), y->cap[k], lk,
                mat(Yk, y->inst_stride, sref(ry + k + 1, rs, p), sc(1), sref(ry + k + 1, rs, 1)),
                false,
                mat(T1 + i, iT1, sc(lk * p), sc(p), S0, sref(ry + k + 1, rs, (int64_t)lk * p)), false,
                mat(T2 + (int64_t)i * p * t2_ia, iT2, sc(lk), sc(1), sc(t2_ia), sc(t2_a)), one,
                false);
    }
    // W_k[(a, b)][g] = sum_K D_k[a][K] T2[K][b][g]
    gemm_ex(st, B, 1, 1, dconst(rd), dref(ry + k, rs, lk), dconst(kd), rd, y->cap[k] * lk,
            mat_op(A, Dd + A->offsets[k], sc(kd), sc(1)), false, mat(T2, iT2, sc(t2_a), sc(1)), false,
            mat(Wall + w.Woff[k], iW, sref(ry + k, rs, lk), sc(1)), one, false,
            dconst(1 << 30), kd);
  }
  // ---- left pass: M_{-1} = 1, out ranks r_0 = r_n = 1
  k_fill_one<<<(B + 127) / 128, 128, 0, st>>>(B, Mb, iM);
  k_init_ranks_one<<<B, 64, 0, st>>>(n, B, ro);
  for (int k = 0; k < n; ++k) {
    const int p = y->modes[k];
    const int lk = ell[k];
    const int rd = A->ranks[k], rd1 = A->ranks[k + 1];
    const bool diag = A->diag[k] != 0;
    const int kd = (diag ? p : p * p) * rd1;
    const cplx* Yk = Yd + y->offsets[k];
    const int64_t t3_s = (int64_t)y->cap[k] * kd;
    // T3[s][b][K] = sum_a M[s][(a, b)] D_k[a][K]
    gemm_ex(st, B, lk, 1, dref(ry + k, rs), dconst(kd), dconst(rd), y->cap[k], kd,
            mat(Mb, iM, sc(1), sref(ry + k, rs, 1), sref(ry + k, rs, rd)), false,
            mat_op(A, Dd + A->offsets[k], sc(kd), sc(1)), false, mat(T3, iT3, sc(kd), sc(1), sc(t3_s)),
            one, false, dref(ro + k, rs), rd);
    // Z[(s, i)][(a', b')] = sum_j sum_b T3[s][b][(i [j] a')] Y_k[b, j, b']
    Mat Zc = mat(Zb, iZ, sref(ry + k + 1, rs, 1), sc(1), sref(ry + k + 1, rs, (int64_t)p * rd1),
                 sref(ry + k + 1, rs, rd1));
    if (diag) {
      gemm_ex(st, B, lk, p, dconst(rd1), dref(ry + k + 1, rs), dref(ry + k, rs), rd1,
              y->cap[k + 1], mat(T3, iT3, sc(1), sc(kd), sc(t3_s), sc(rd1)), false,
              mat(Yk, y->inst_stride, sref(ry + k + 1, rs, p), sc(1), S0, sref(ry + k + 1, rs, 1)),
              false, Zc, one, false, dref(ro + k, rs));
    } else {
      for (int j = 0; j < p; ++j)
        gemm_ex(st, B, lk, p, dconst(rd1), dref(ry + k + 1, rs), dref(ry + k, rs), rd1,
                y->cap[k + 1],
                mat(T3 + (int64_t)j * rd1, iT3, sc(1), sc(kd), sc(t3_s), sc((int64_t)p * rd1)),
                false,
                mat(Yk, y->inst_stride, sref(ry + k + 1, rs, p), sc(1), S0, S0,
                    sref(ry + k + 1, rs, j)),
                false, Zc, one, j > 0, dref(ro + k, rs));
    }
    if (k == n - 1) {
      // last core (s, p, 1) = Z; ||x~||^2
      copy(st, B, dref(ro + k, rs, p), dconst(1), (int64_t)lk * p, Zb, iZ, Od + out->offsets[k],
           out->inst_stride);
      if (ynorm2) sumsq(st, B, dref(ro + k, rs, p), dconst(1), Zb, iZ, ynorm2, 1.0);
      break;
    }
    const int lk1 = ell[k + 1];
    // Y_k = Z W_{k+1}   ((s p) x l_{k+1})
    GemmF32Scope prec(f32);
    gemm_ex(st, B, 1, 1, dref(ro + k, rs, p), dconst(lk1), dref(ry + k + 1, rs, rd1), lk * p, lk1,
            mat(Zb, iZ, sref(ry + k + 1, rs, rd1), sc(1)), false,
            mat(Wall + w.Woff[k + 1], iW, sc(lk1), sc(1)), false, mat(Yb, iY, sc(lk1), sc(1)),
            one, false, dconst(1 << 30), (int64_t)rd1 * y->cap[k + 1]);
    g_gemm_f32 = false;
    // Q_k = qr(Y_k) -> out core k, new rank s' -> ro[k+1]
    if (qb.V && qr_blocked_wanted(lk * p, lk1))
      qr_blocked(st, B, lk * p, lk1, dref(ro + k, rs, p), dconst(lk1), Yb, iY, Wq, iY, qb,
                 Od + out->offsets[k], out->inst_stride, Rb, w.R, ro + k + 1, rs);
    else
      qr_auto(st, B, lk * p, lk1, dref(ro + k, rs, p), dconst(lk1), Yb, iY, Wq, iY, tau, w.tau,
              Od + out->offsets[k], out->inst_stride, Rb, w.R, ro + k + 1, rs);
    if (rdiag)
      k_rdiag<<<B, 128, 0, st>>>(Rb, w.R, lk1, ro + k + 1, rs, rdiag + (int64_t)(k + 1) * RD_MAX,
                                 (int64_t)(n + 1) * RD_MAX);
    // M_k = Q_k^H Z   (s' x R_{k+1})
    gemm_ex(st, B, 1, 1, dref(ro + k + 1, rs), dref(ry + k + 1, rs, rd1), dref(ro + k, rs, p), lk1,
            rd1 * y->cap[k + 1],
            mat(Od + out->offsets[k], out->inst_stride, sc(1), sref(ro + k + 1, rs, 1)), true,
            mat(Zb, iZ, sref(ry + k + 1, rs, rd1), sc(1)), false,
            mat(Mb, iM, sref(ry + k + 1, rs, rd1), sc(1)), one, false);
  }
  QT_HIP(hipGetLastError());
  return QT_OK;
}

// ----------------------------------------------------- <y, Q y>
SandwichWs sandwich_ws_layout(const qt_mpo* Q, const qt_tt* y) {
  SandwichWs w;
  for (int k = 0; k <= y->n; ++k)
    w.E = std::max<int64_t>(w.E, (int64_t)y->cap[k] * Q->ranks[k] * y->cap[k]);
  for (int k = 0; k < y->n; ++k) {
    const int64_t p = y->modes[k];
    w.F = std::max<int64_t>(w.F, (int64_t)y->cap[k] * Q->ranks[k] * p * y->cap[k + 1]);
    w.G = std::max<int64_t>(w.G, (int64_t)y->cap[k] * p * Q->ranks[k + 1] * y->cap[k + 1]);
  }
  w.bytes = sizeof(cplx) * y->batch * (2 * w.E + w.F + w.G) + 8 * 256;
  return w;
}

__global__ void k_store_re(int batch, const cplx* E, int64_t sE, double scale, double* out) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < batch) out[b] = scale * E[b * sE].x;
}

qt_status sandwich_impl(qt_ctx ctx, const qt_mpo* Q, const qt_tt* y, double scale, double* out) {
  const int n = y->n, B = y->batch, rs = n + 1;
  hipStream_t st = ctx->stream;
  SandwichWs w = sandwich_ws_layout(Q, y);
  cplx* E0 = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.E);
  cplx* E1 = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.E);
  cplx* F = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.F);
  cplx* G = (cplx*)ws_take(ctx, sizeof(cplx) * B * w.G);
  QT_CHECK(E0 && E1 && F && G, QT_ENOMEM, "sandwich: workspace too small");
  int32_t* ry = y->ranks;
  const cplx* Yd = (const cplx*)y->data;
  const cplx* Qd = (const cplx*)Q->data;
  const cplx one = make_double2(1.0, 0.0);
  k_fill_one<<<(B + 127) / 128, 128, 0, st>>>(B, E0, w.E);
  for (int k = 0; k < n; ++k) {
    const int p = y->modes[k];
    const int rq = Q->ranks[k], rq1 = Q->ranks[k + 1];
    const int cy = y->cap[k], cy1 = y->cap[k + 1];
    const cplx* Yk = Yd + y->offsets[k];
    const cplx* Qk = Qd + Q->offsets[k];
    // E layout [b][q][b2] with row stride cy over (b, q); F[(b, q)][(j, b'')] row stride p*cy1
    gemm_ex(st, B, 1, 1, dref(ry + k, rs, rq), dref(ry + k + 1, rs, p), dref(ry + k, rs), cy * rq,
            p * cy1, mat(E0, w.E, sc(cy), sc(1)), false,
            mat(Yk, y->inst_stride, sref(ry + k + 1, rs, p), sc(1)), false,
            mat(F, w.F, sc((int64_t)p * cy1), sc(1)), one, false);
    // G2[b][i][q'][b''] = sum_q sum_j Q[q, i, j, q'] F[b][q][j][b'']
    const int64_t g_b = (int64_t)p * rq1 * cy1, g_i = (int64_t)rq1 * cy1;
    if (Q->diag[k]) {
      gemm_ex(st, B, cy, p, dconst(rq1), dref(ry + k + 1, rs), dconst(rq), rq1, cy1,
              mat_op(Q, Qk, sc(1), sc((int64_t)p * rq1), S0, sc(rq1)), false,
              mat(F, w.F, sc((int64_t)p * cy1), sc(1), sc((int64_t)rq * p * cy1),
                  sref(ry + k + 1, rs, 1)),
              false, mat(G, w.G, sc(cy1), sc(1), sc(g_b), sc(g_i)), one, false, dref(ry + k, rs));
    } else {
      for (int j = 0; j < p; ++j)
        gemm_ex(st, B, cy, p, dconst(rq1), dref(ry + k + 1, rs), dconst(rq), rq1, cy1,
                mat_op(Q, Qk + (int64_t)j * rq1, sc(1), sc((int64_t)p * p * rq1), S0,
                    sc((int64_t)p * rq1)),
                false,
                mat(F, w.F, sc((int64_t)p * cy1), sc(1), sc((int64_t)rq * p * cy1), S0,
                    sref(ry + k + 1, rs, j)),
                false, mat(G, w.G, sc(cy1), sc(1), sc(g_b), sc(g_i)), one, j > 0,
                dref(ry + k, rs));
    }
    // E'[b'][q'][b''] = sum_{(b, i)} conj(Y[b, i, b']) G2[(b, i)][q'][b'']
    gemm_ex(st, B, rq1, 1, dref(ry + k + 1, rs), dref(ry + k + 1, rs), dref(ry + k, rs, p), cy1,
            cy1, mat(Yk, y->inst_stride, sc(1), sref(ry + k + 1, rs, 1)), true,
            mat(G, w.G, sc(g_i), sc(1), sc(cy1)), false,
            mat(E1, w.E, sc((int64_t)rq1 * cy1), sc(1), sc(cy1)), one, false);
    std::swap(E0, E1);
  }
  k_store_re<<<(B + 127) / 128, 128, 0, st>>>(B, E0, w.E, scale, out);
  QT_HIP(hipGetLastError());
  return QT_OK;
}

}  // namespace qt
