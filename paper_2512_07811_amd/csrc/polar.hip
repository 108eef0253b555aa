// Truncation of one bond by polar decomposition (Sec. 2.2, "Compression via
// Polar Decomposition" of arXiv 2512.07811), on the MFMA GEMM.
//
// For the centre A (n x m, n = r'_k rows, m = p_k r_{k+1} columns) of the
// right-to-left sweep, with T = A^H:
//   T = U H            polar factor U^H = lim Y_j of Y_0 = A / ||A||_F under
//                      Y <- p(Y Y^H) Y with odd polynomials (Newton-Schulz
//                      type): the singular values s of Y map s -> f(s) and
//                      converge to 1, the singular vectors stay; H = A U
//   H - d~ I = U' H'   U' = the sign of the Hermitian matrix Z_0 =
//                      (H - d~ I) / ||H - d~ I||_F under the same iteration
//   P+ = (I + U') / 2, l = round(trace P+) (>= 1, <= lmax)
//   C+ = orthonormal basis of range(P+): subspace iteration from a Gaussian
//        block, C <- qr(P+ H^2 C) (H also ranks the directions when the cap
//        binds)
//   core = C+^H U^H (l x m, orthonormal rows), carry = H C+ (n x l)
// The kept part carry * core = A (U C+)(U C+)^H is an orthogonal projection of
// A (to the accuracy of U on the kept directions), and the discarded weight is
// ||A - carry core||_F, formed explicitly.
//
// Iteration: quintic steps f(s) = a s + b s^3 + c s^5 (a, b, c = 3.4445,
// -4.7750, 2.0315) multiply small singular values by 3.44 and keep [0, 1]
// inside [0, 1.21], then cubic steps g(s) = (3 s - s^3) / 2 converge
// quadratically to 1.  The quintic count is chosen from the smallest value
// that must converge (a twentieth of the cutoff relative to ||A||): singular
// values within about 5 % of the cutoff may land on either side of it.
#include <cmath>

#include "kernels.h"
#include "polar.h"
#include "sketch.h"

namespace qt {

constexpr double PQ_A = 3.4445, PQ_B = -4.7750, PQ_C = 2.0315;
constexpr int PSUB_STEPS = 4;   // subspace-iteration steps with H^2

static inline Str str_of(Dim d) { return Str{d.p, d.stride, d.mul, d.cst}; }

PolarSizes polar_sizes(int ncap, int mcap, int lcap) {
  PolarSizes s;
  s.ncap = ncap; s.mcap = mcap; s.lcap = lcap;
  s.y = (int64_t)ncap * mcap;
  s.g = (int64_t)ncap * ncap;
  s.c = (int64_t)ncap * lcap;
  s.r = (int64_t)lcap * lcap;
  s.tau = lcap + 4;
  // every bond's QR is (rows x min(rows, lcap)) with rows <= ncap, and the
  // blocked QR's panel width depends on the rows: the largest need over them
  for (int m = 1; m <= ncap; ++m) {
    const int c = std::min(m, lcap);
    if (!qr_blocked_wanted(m, c)) continue;
    int64_t v, t, w;
    qr_blocked_ws_elems(m, c, &v, &t, &w);
    s.qb_v = std::max(s.qb_v, v);
    s.qb_t = std::max(s.qb_t, t);
    s.qb_w = std::max(s.qb_w, w);
    s.qb_tau = std::max(s.qb_tau, qr_blocked_tau_elems(m, c));
  }
  return s;
}

// The blocked-QR workspace of w covers an ncap x lcap factorization.
static bool polar_qb_fits(const PolarWs& w, int ncap, int lcap) {
  if (!w.qb.V || !qr_blocked_wanted(ncap, lcap)) return false;
  int64_t v, t, q;
  qr_blocked_ws_elems(ncap, lcap, &v, &t, &q);
  return v <= w.s.qb_v && t <= w.s.qb_t && q <= w.s.qb_w &&
         qr_blocked_tau_elems(ncap, lcap) <= w.s.qb_tau;
}

size_t polar_ws_bytes(int B, const PolarSizes& s) {
  size_t b = sizeof(cplx) * B * (2 * s.y + 5 * s.g + 5 * s.c + s.r) +
             sizeof(double) * B * (s.tau + 4) + sizeof(int32_t) * B + 16 * 256;
  if (s.qb_v > 0)
    b += sizeof(cplx) * B * (s.qb_v + s.qb_t + 2 * s.qb_w) + sizeof(double) * B * s.qb_tau +
         sizeof(int32_t) * B + 6 * 256;
  return b;
}

qt_status polar_ws_take(qt_ctx ctx, int B, const PolarSizes& s, PolarWs& w) {
  w.s = s;
  w.Y0 = (cplx*)ws_take(ctx, sizeof(cplx) * B * s.y);
  w.Y1 = (cplx*)ws_take(ctx, sizeof(cplx) * B * s.y);
  w.G = (cplx*)ws_take(ctx, sizeof(cplx) * B * s.g);
  w.P = (cplx*)ws_take(ctx, sizeof(cplx) * B * s.g);
  w.H = (cplx*)ws_take(ctx, sizeof(cplx) * B * s.g);
  w.Z0 = (cplx*)ws_take(ctx, sizeof(cplx) * B * s.g);
  w.Z1 = (cplx*)ws_take(ctx, sizeof(cplx) * B * s.g);
  w.Om = (cplx*)ws_take(ctx, sizeof(cplx) * B * s.c);
  w.V = (cplx*)ws_take(ctx, sizeof(cplx) * B * s.c);
  w.W = (cplx*)ws_take(ctx, sizeof(cplx) * B * s.c);
  w.C = (cplx*)ws_take(ctx, sizeof(cplx) * B * s.c);
  w.Wq = (cplx*)ws_take(ctx, sizeof(cplx) * B * s.c);
  w.R = (cplx*)ws_take(ctx, sizeof(cplx) * B * s.r);
  w.tau = (double*)ws_take(ctx, sizeof(double) * B * s.tau);
  w.nrm = (double*)ws_take(ctx, sizeof(double) * B * 4);
  w.sq = (int32_t*)ws_take(ctx, sizeof(int32_t) * B);
  QT_CHECK(w.Y0 && w.Y1 && w.G && w.P && w.H && w.Z0 && w.Z1 && w.Om && w.V && w.W && w.C &&
               w.Wq && w.R && w.tau && w.nrm && w.sq,
           QT_ENOMEM, "polar rounding: workspace too small");
  w.qb = QrBlkWs{};
  if (s.qb_v > 0) {
    QrBlkWs& q = w.qb;
    q.V = (cplx*)ws_take(ctx, sizeof(cplx) * B * s.qb_v);
    q.v_stride = s.qb_v;
    q.T = (cplx*)ws_take(ctx, sizeof(cplx) * B * s.qb_t);
    q.t_stride = s.qb_t;
    q.W1 = (cplx*)ws_take(ctx, sizeof(cplx) * B * s.qb_w);
    q.W2 = (cplx*)ws_take(ctx, sizeof(cplx) * B * s.qb_w);
    q.w_stride = s.qb_w;
    q.tau = (double*)ws_take(ctx, sizeof(double) * B * s.qb_tau);
    q.tau_stride = s.qb_tau;
    q.s_dev = (int32_t*)ws_take(ctx, sizeof(int32_t) * B);
    QT_CHECK(q.V && q.T && q.W1 && q.W2 && q.tau && q.s_dev, QT_ENOMEM,
             "polar rounding: blocked QR workspace too small");
  }
  return QT_OK;
}

int polar_quintic_steps(double eps, int nbonds, int qcap) {
  // smallest relative singular value (of ||A||) that must converge: a
  // twentieth of the cutoff delta / q = eps ||x|| / (sqrt(n - 1) q), ||A|| = ||x||
  const double e = std::max(eps, 1e-15);
  const double smin = e / (std::sqrt((double)std::max(nbonds, 1)) * std::max(qcap, 1) * 20.0);
  const int k = (int)std::ceil(std::log(0.7 / smin) / std::log(3.4445));
  return std::min(std::max(k, 3), 40);
}

// Frobenius norm squared of the n x m matrix X (row pitch ld) of each instance.
__global__ void k_pol_sumsq(Dim Nd, Dim Md, const cplx* X, int64_t ld, int64_t sX, double* out) {
  __shared__ double red[16];
  const int b = blockIdx.x;
  const int n = dimv(Nd, b), m = dimv(Md, b);
  X += b * sX;
  double a = 0.0;
  for (int64_t e = threadIdx.x; e < (int64_t)n * m; e += blockDim.x)
    a += cabs2(X[(e / m) * ld + e % m]);
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
    out[b] = t;
  }
}

// Y = A / ||A||_F (A packed with row pitch m, Y with row pitch ldY).
__global__ void k_pol_load(Dim Nd, Dim Md, const cplx* A, int64_t sA, const double* nA2,
                           cplx* Y, int64_t ldY, int64_t sY) {
  const int b = blockIdx.y;
  const int n = dimv(Nd, b), m = dimv(Md, b);
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * m) return;
  const double s = nA2[b] > 0.0 ? 1.0 / sqrt(nA2[b]) : 0.0;
  const int64_t i = e / m, j = e % m;
  Y[b * sY + i * ldY + j] = cscale(A[b * sA + e], s);
}

// Y = A (A packed with row pitch m, Y with row pitch ldY)
__global__ void k_pol_copy(Dim Nd, Dim Md, const cplx* A, int64_t sA, cplx* Y, int64_t ldY,
                           int64_t sY) {
  const int b = blockIdx.y;
  const int n = dimv(Nd, b), m = dimv(Md, b);
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * m) return;
  Y[b * sY + (e / m) * ldY + e % m] = A[b * sA + e];
}

// P = a I + b G (n x n, pitch ld)
__global__ void k_pol_poly(Dim Nd, const cplx* G, cplx* P, int64_t ld, int64_t sG, double a,
                           double bb) {
  const int b = blockIdx.y;
  const int n = dimv(Nd, b);
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int64_t i = e / n, j = e % n;
  cplx v = cscale(G[b * sG + i * ld + j], bb);
  if (i == j) v.x += a;
  P[b * sG + i * ld + j] = v;
}

// H <- (H + H^H) / 2 and Z = H - d~ I with d~ = delta / min(n, m): one thread
// per pair (i <= j).
__global__ void k_pol_shift(Dim Nd, Dim Md, cplx* H, cplx* Z, int64_t ld, int64_t sG,
                            const double* delta) {
  const int b = blockIdx.y;
  const int n = dimv(Nd, b), m = dimv(Md, b);
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int64_t i = e / n, j = e % n;
  if (i > j) return;
  cplx* Hb = H + b * sG;
  cplx* Zb = Z + b * sG;
  const cplx hij = Hb[i * ld + j], hji = Hb[j * ld + i];
  const cplx h = make_double2(0.5 * (hij.x + hji.x), 0.5 * (hij.y - hji.y));
  const double dt = delta[b] / (double)max(min(n, m), 1);
  Hb[i * ld + j] = h;
  Hb[j * ld + i] = cconj(h);
  cplx z = h;
  if (i == j) z.x -= dt;
  Zb[i * ld + j] = z;
  Zb[j * ld + i] = cconj(z);
}

// Z *= 1 / sqrt(nZ2)
__global__ void k_pol_scale(Dim Nd, cplx* Z, int64_t ld, int64_t sG, const double* nZ2) {
  const int b = blockIdx.y;
  const int n = dimv(Nd, b);
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const double s = nZ2[b] > 0.0 ? 1.0 / sqrt(nZ2[b]) : 0.0;
  const int64_t i = e / n, j = e % n;
  Z[b * sG + i * ld + j] = cscale(Z[b * sG + i * ld + j], s);
}

// P+ = (I + Z) / 2 in place, l = round(trace P+) clamped to [1, min(lmax, n)];
// with no direction above the cutoff, P+ = I (the subspace iteration with H
// then finds the dominant direction).  One block per instance.
__global__ void k_pol_pplus(Dim Nd, cplx* Z, int64_t ld, int64_t sG, int lmax, int32_t* l_out,
                            int l_stride) {
  __shared__ double red[16];
  __shared__ int none;
  const int b = blockIdx.x;
  const int n = dimv(Nd, b);
  cplx* Zb = Z + b * sG;
  double t = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) t += 0.5 * (1.0 + Zb[(int64_t)i * ld + i].x);
  t = wave_sum(t);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    const long l0 = lround(s);
    none = l0 < 1 ? 1 : 0;
    const int l = (int)min<long>(max<long>(l0, 1), (long)min(lmax, n));
    l_out[(int64_t)b * l_stride] = l;
  }
  __syncthreads();
  const int ident = none;
  for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += blockDim.x) {
    const int64_t i = e / n, j = e % n;
    cplx v = ident ? make_double2(0.0, 0.0) : cscale(Zb[i * ld + j], 0.5);
    if (i == j) v.x += ident ? 1.0 : 0.5;
    Zb[i * ld + j] = v;
  }
}

__global__ void k_pol_disc(int batch, const double* r2, double* disc2) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < batch) disc2[b] += r2[b];
}

// Y <- p(Y Y^H) Y with p(G) = a I + b G + c G^2 (c = 0: cubic step); Y is n x m
// with pitch ldY; ping-pong between Y and Yn.  Returns the buffer holding the
// result.
static cplx* poly_step(hipStream_t st, int B, Dim n, Dim m, int ncap, int mcap, cplx* Y,
                       cplx* Yn, int64_t ldY, int64_t sY, const PolarWs& w, double a, double bb,
                       double c) {
  const int64_t ldG = w.s.ncap, sG = w.s.g;
  const cplx one = make_double2(1.0, 0.0);
  const Str s1 = sconst(1);
  // G = Y Y^H
  gemm_ex(st, B, 1, 1, n, n, m, ncap, ncap, mat(Y, sY, sconst(ldY), s1), false,
          mat(Y, sY, s1, sconst(ldY)), true, mat(w.G, sG, sconst(ldG), s1), one, false,
          Dim{nullptr, 0, 0, 1 << 30}, mcap);
  // P = a I + b G (+ c G G)
  const int64_t ng = (int64_t)ncap * ncap;
  dim3 grid((unsigned)((ng + 255) / 256), B);
  k_pol_poly<<<grid, 256, 0, st>>>(n, w.G, w.P, ldG, sG, a, bb);
  if (c != 0.0)
    gemm_ex(st, B, 1, 1, n, n, n, ncap, ncap, mat(w.G, sG, sconst(ldG), s1), false,
            mat(w.G, sG, sconst(ldG), s1), false, mat(w.P, sG, sconst(ldG), s1),
            make_double2(c, 0.0), true, Dim{nullptr, 0, 0, 1 << 30}, ncap);
  // Yn = P Y
  gemm_ex(st, B, 1, 1, n, m, n, ncap, mcap, mat(w.P, sG, sconst(ldG), s1), false,
          mat(Y, sY, sconst(ldY), s1), false, mat(Yn, sY, sconst(ldY), s1), one, false,
          Dim{nullptr, 0, 0, 1 << 30}, ncap);
  return Yn;
}

static cplx* sign_iterate(hipStream_t st, int B, Dim n, Dim m, int ncap, int mcap, cplx* Y,
                          cplx* Yn, int64_t ldY, int64_t sY, const PolarWs& w, int nq, int nc) {
  for (int i = 0; i < nq; ++i) {
    cplx* r = poly_step(st, B, n, m, ncap, mcap, Y, Yn, ldY, sY, w, PQ_A, PQ_B, PQ_C);
    Yn = Y;
    Y = r;
  }
  for (int i = 0; i < nc; ++i) {
    cplx* r = poly_step(st, B, n, m, ncap, mcap, Y, Yn, ldY, sY, w, 1.5, -0.5, 0.0);
    Yn = Y;
    Y = r;
  }
  return Y;
}

void polar_trunc(hipStream_t st, int B, int ncap, int mcap, Dim n, Dim m, const cplx* A,
                 int64_t sA, const PolarWs& w, cplx* core, int64_t sCore, cplx* carry,
                 int64_t sCarry, int32_t* l_out, int l_stride, const double* delta,
                 double* disc2, int lmax, int nq, uint64_t seed, uint64_t stream) {
  const PolarSizes& s = w.s;
  const int lcap = std::min(ncap, lmax);
  const int64_t ldY = s.mcap, sY = s.y, ldG = s.ncap, sG = s.g, sC = s.c;
  const cplx one = make_double2(1.0, 0.0);
  const Str s1 = sconst(1);
  const Dim l = dref(l_out, l_stride);
  const Str sl = str_of(l), sm = str_of(m);
  double* nA2 = w.nrm;
  double* nZ2 = w.nrm + B;
  double* nC2 = w.nrm + 2 * B;
  constexpr int NC = 7;
  // ---- polar factor: Y -> U^H
  sumsq(st, B, n, m, A, sA, nA2, 1.0);
  {
    const int64_t cnt = (int64_t)ncap * mcap;
    dim3 grid((unsigned)((cnt + 255) / 256), B);
    k_pol_load<<<grid, 256, 0, st>>>(n, m, A, sA, nA2, w.Y0, ldY, sY);
  }
  cplx* U = sign_iterate(st, B, n, m, ncap, mcap, w.Y0, w.Y1, ldY, sY, w, nq, NC);
  // H = A U = A (U^H)^H   (n x n)
  gemm_ex(st, B, 1, 1, n, n, m, ncap, ncap, mat(A, sA, sm, s1), false,
          mat(U, sY, s1, sconst(ldY)), true, mat(w.H, sG, sconst(ldG), s1), one, false,
          Dim{nullptr, 0, 0, 1 << 30}, mcap);
  // ---- sign of H - d~ I
  const int64_t ng = (int64_t)ncap * ncap;
  dim3 gg((unsigned)((ng + 255) / 256), B);
  k_pol_shift<<<gg, 256, 0, st>>>(n, m, w.H, w.Z0, ldG, sG, delta);
  k_pol_sumsq<<<B, 256, 0, st>>>(n, n, w.Z0, ldG, sG, nZ2);
  k_pol_scale<<<gg, 256, 0, st>>>(n, w.Z0, ldG, sG, nZ2);
  cplx* Z = sign_iterate(st, B, n, n, ncap, ncap, w.Z0, w.Z1, ldG, sG, w, nq, NC);
  k_pol_pplus<<<B, 256, 0, st>>>(n, Z, ldG, sG, lmax, l_out, l_stride);
  // ---- C+ by subspace iteration: C = qr(P+ Om), then C <- qr(P+ H C) twice
  gauss_fill(st, (int64_t)B * sC, seed, stream, w.Om);
  gemm_ex(st, B, 1, 1, n, l, n, ncap, lcap, mat(Z, sG, sconst(ldG), s1), false,
          mat(w.Om, sC, sconst(lcap), s1), false, mat(w.V, sC, sl, s1), one, false,
          Dim{nullptr, 0, 0, 1 << 30}, ncap);
  // C = Q of the n x l block M (panels + MFMA GEMMs when one workgroup cannot
  // hold it: the work matrix is Wq either way)
  const bool blocked = polar_qb_fits(w, ncap, lcap);
  auto qr_c = [&](const cplx* M) {
    if (blocked)
      qr_blocked(st, B, ncap, lcap, n, l, M, sC, w.Wq, sC, w.qb, w.C, sC, w.R, s.r, w.sq, 1);
    else
      qr_auto(st, B, ncap, lcap, n, l, M, sC, w.Wq, sC, w.tau, s.tau, w.C, sC, w.R, s.r, w.sq, 1);
  };
  qr_c(w.V);
  // C <- qr(P+ H^2 C): inside range(P+) the directions converge at the rate
  // (sigma_{l+1} / sigma_l)^2 per step towards the l largest (the rank cap)
  for (int it = 0; it < PSUB_STEPS; ++it) {
    gemm_ex(st, B, 1, 1, n, l, n, ncap, lcap, mat(w.H, sG, sconst(ldG), s1), false,
            mat(w.C, sC, sl, s1), false, mat(w.W, sC, sl, s1), one, false,
            Dim{nullptr, 0, 0, 1 << 30}, ncap);
    gemm_ex(st, B, 1, 1, n, l, n, ncap, lcap, mat(w.H, sG, sconst(ldG), s1), false,
            mat(w.W, sC, sl, s1), false, mat(w.V, sC, sl, s1), one, false,
            Dim{nullptr, 0, 0, 1 << 30}, ncap);
    gemm_ex(st, B, 1, 1, n, l, n, ncap, lcap, mat(Z, sG, sconst(ldG), s1), false,
            mat(w.V, sC, sl, s1), false, mat(w.W, sC, sl, s1), one, false,
            Dim{nullptr, 0, 0, 1 << 30}, ncap);
    qr_c(w.W);
  }
  // ---- core = C^H U^H (l x m, packed), carry = H C (n x l, packed)
  gemm_ex(st, B, 1, 1, l, m, n, lcap, mcap, mat(w.C, sC, s1, sl), true,
          mat(U, sY, sconst(ldY), s1), false, mat(core, sCore, sm, s1), one, false,
          Dim{nullptr, 0, 0, 1 << 30}, ncap);
  gemm_ex(st, B, 1, 1, n, l, n, ncap, lcap, mat(w.H, sG, sconst(ldG), s1), false,
          mat(w.C, sC, sl, s1), false, mat(carry, sCarry, sl, s1), one, false,
          Dim{nullptr, 0, 0, 1 << 30}, ncap);
  // discarded weight ||A - carry core||^2, formed explicitly (the difference
  // of squared norms would lose everything below sqrt(u) ||A||)
  cplx* Rd = (U == w.Y0) ? w.Y1 : w.Y0;
  {
    const int64_t cnt = (int64_t)ncap * mcap;
    dim3 grid((unsigned)((cnt + 255) / 256), B);
    k_pol_copy<<<grid, 256, 0, st>>>(n, m, A, sA, Rd, ldY, sY);
  }
  gemm_ex(st, B, 1, 1, n, m, l, ncap, mcap, mat(carry, sCarry, sl, s1), false,
          mat(core, sCore, sm, s1), false, mat(Rd, sY, sconst(ldY), s1),
          make_double2(-1.0, 0.0), true, Dim{nullptr, 0, 0, 1 << 30}, lcap);
  k_pol_sumsq<<<B, 256, 0, st>>>(n, m, Rd, ldY, sY, nC2);
  k_pol_disc<<<(B + 127) / 128, 128, 0, st>>>(B, nC2, disc2);
}

}  // namespace qt
