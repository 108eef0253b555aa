// Dense complex-double building blocks of TT rounding on gfx950:
// tiled GEMM, single-workgroup Householder QR, one-sided Jacobi SVD with
// truncation, norms and copies.  Matrix sizes are read from device memory so
// that a whole rounding sweep is issued without host synchronisation.
#include "kernels.h"

namespace qt {

// ------------------------------------------------------------------ GEMM
// 64 x 64 output tile per 256-thread workgroup, K chunks of 16 staged in LDS;
// each thread owns a 4 x 4 block of outputs (rows ty+16i, cols tx+16j).
constexpr int GT_M = 64, GT_N = 64, GT_K = 16;

template <bool CA, bool CB>
__global__ __launch_bounds__(256) void k_gemm(Dim Md, Dim Nd, Dim Kd, const cplx* __restrict__ A,
                                              int64_t sA, const cplx* __restrict__ B, int64_t sB,
                                              cplx* __restrict__ C, int64_t sC, cplx alpha,
                                              int accumulate) {
  const int b = blockIdx.z;
  const int M = dimv(Md, b), N = dimv(Nd, b), K = dimv(Kd, b);
  const int m0 = blockIdx.y * GT_M, n0 = blockIdx.x * GT_N;
  if (m0 >= M || n0 >= N) return;
  A += b * sA;
  B += b * sB;
  C += b * sC;
  __shared__ cplx As[GT_K][GT_M + 1];
  __shared__ cplx Bs[GT_K][GT_N + 1];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  cplx acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = make_double2(0.0, 0.0);

  for (int k0 = 0; k0 < K; k0 += GT_K) {
    // A tile: op(A)[m0 + mm, k0 + kk]
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int idx = tid + 256 * e;
      int mm, kk;
      cplx v = make_double2(0.0, 0.0);
      if (!CA) {
        mm = idx >> 4; kk = idx & 15;
        int gm = m0 + mm, gk = k0 + kk;
        if (gm < M && gk < K) v = A[(int64_t)gm * K + gk];
      } else {
        kk = idx >> 6; mm = idx & 63;
        int gm = m0 + mm, gk = k0 + kk;
        if (gm < M && gk < K) v = cconj(A[(int64_t)gk * M + gm]);
      }
      As[kk][mm] = v;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int idx = tid + 256 * e;
      int kk, nn;
      cplx v = make_double2(0.0, 0.0);
      if (!CB) {
        kk = idx >> 6; nn = idx & 63;
        int gk = k0 + kk, gn = n0 + nn;
        if (gk < K && gn < N) v = B[(int64_t)gk * N + gn];
      } else {
        nn = idx >> 4; kk = idx & 15;
        int gk = k0 + kk, gn = n0 + nn;
        if (gk < K && gn < N) v = cconj(B[(int64_t)gn * K + gk]);
      }
      Bs[kk][nn] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < GT_K; ++kk) {
      cplx a[4], bb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) cfma(acc[i][j], a[i], bb[j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int gm = m0 + ty + 16 * i;
    if (gm >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int gn = n0 + tx + 16 * j;
      if (gn >= N) continue;
      cplx v = cmul(alpha, acc[i][j]);
      int64_t o = (int64_t)gm * N + gn;
      if (accumulate) v = cadd(v, C[o]);
      C[o] = v;
    }
  }
}

void gemm(hipStream_t st, int batch, Dim M, Dim N, Dim K, int Mcap, int Ncap, bool conjA,
          const cplx* A, int64_t sA, bool conjB, const cplx* B, int64_t sB, cplx* C, int64_t sC,
          cplx alpha, bool accumulate) {
  if (Mcap <= 0 || Ncap <= 0 || batch <= 0) return;
  dim3 grid((Ncap + GT_N - 1) / GT_N, (Mcap + GT_M - 1) / GT_M, batch);
  int acc = accumulate ? 1 : 0;
  if (!conjA && !conjB)
    k_gemm<false, false><<<grid, 256, 0, st>>>(M, N, K, A, sA, B, sB, C, sC, alpha, acc);
  else if (conjA && !conjB)
    k_gemm<true, false><<<grid, 256, 0, st>>>(M, N, K, A, sA, B, sB, C, sC, alpha, acc);
  else if (!conjA && conjB)
    k_gemm<false, true><<<grid, 256, 0, st>>>(M, N, K, A, sA, B, sB, C, sC, alpha, acc);
  else
    k_gemm<true, true><<<grid, 256, 0, st>>>(M, N, K, A, sA, B, sB, C, sC, alpha, acc);
}

// ------------------------------------------------------- block reductions
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += red[i];
  __syncthreads();
  return t;
}

// -------------------------------------------------------------------- QR
// Householder reflector H = I - tau u u^H with u_0 = 1, H x = beta e_1,
// beta = -e^{i arg x_0} ||x||, tau = 1 + |x_0|/||x|| (tau = 0 for x = 0).
__global__ __launch_bounds__(1024) void k_qr(Dim Md, Dim Nd, const cplx* __restrict__ A, int64_t sA,
                                            cplx* __restrict__ W, int64_t sW,
                                            double* __restrict__ tau, int64_t sTau,
                                            cplx* __restrict__ Q, int64_t sQ, cplx* __restrict__ R,
                                            int64_t sR, int32_t* s_out, int s_stride) {
  const int b = blockIdx.x;
  const int m = dimv(Md, b), n = dimv(Nd, b);
  const int s = min(m, n);
  A += b * sA; W += b * sW; tau += b * sTau; Q += b * sQ; R += b * sR;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
  __shared__ double red[16];
  __shared__ cplx sh_inv_u0, sh_beta;
  __shared__ double sh_tau;
  for (int64_t e = tid; e < (int64_t)m * n; e += blockDim.x) W[e] = A[e];
  __syncthreads();
  for (int j = 0; j < s; ++j) {
    double part = 0.0;
    for (int i = j + 1 + tid; i < m; i += blockDim.x) part += cabs2(W[(int64_t)i * n + j]);
    double sig2 = block_sum(part, red);
    if (tid == 0) {
      cplx al = W[(int64_t)j * n + j];
      double aa = sqrt(cabs2(al));
      double xn = sqrt(aa * aa + sig2);
      if (xn == 0.0) {
        sh_tau = 0.0; sh_beta = al; sh_inv_u0 = make_double2(0.0, 0.0);
      } else {
        cplx ph = aa > 0.0 ? make_double2(al.x / aa, al.y / aa) : make_double2(1.0, 0.0);
        cplx beta = make_double2(-ph.x * xn, -ph.y * xn);
        cplx u0 = csub(al, beta);               // = ph * (aa + xn)
        double d = cabs2(u0);
        sh_inv_u0 = make_double2(u0.x / d, -u0.y / d);
        sh_beta = beta;
        sh_tau = 1.0 + aa / xn;
      }
      tau[j] = sh_tau;
    }
    __syncthreads();
    const cplx iu0 = sh_inv_u0;
    const double tj = sh_tau;
    for (int i = j + 1 + tid; i < m; i += blockDim.x) {
      int64_t o = (int64_t)i * n + j;
      W[o] = cmul(W[o], iu0);
    }
    if (tid == 0) W[(int64_t)j * n + j] = sh_beta;
    __syncthreads();
    if (tj != 0.0) {
      for (int c = j + 1 + wv; c < n; c += nw) {
        cplx acc = (lane == 0) ? W[(int64_t)j * n + c] : make_double2(0.0, 0.0);
        for (int i = j + 1 + lane; i < m; i += 64) cfma(acc, cconj(W[(int64_t)i * n + j]), W[(int64_t)i * n + c]);
        acc = wave_sum(acc);
        cplx f = cscale(acc, -tj);
        if (lane == 0) W[(int64_t)j * n + c] = cadd(W[(int64_t)j * n + c], f);
        for (int i = j + 1 + lane; i < m; i += 64) {
          int64_t o = (int64_t)i * n + c;
          W[o] = cadd(W[o], cmul(W[(int64_t)i * n + j], f));
        }
      }
    }
    __syncthreads();
  }
  // R (s x n), upper trapezoid
  for (int64_t e = tid; e < (int64_t)s * n; e += blockDim.x) {
    int i = (int)(e / n), c = (int)(e % n);
    R[e] = (c >= i) ? W[(int64_t)i * n + c] : make_double2(0.0, 0.0);
  }
  // Q (m x s) = H_0 ... H_{s-1} [I; 0], accumulated backwards
  for (int64_t e = tid; e < (int64_t)m * s; e += blockDim.x) {
    int i = (int)(e / s), c = (int)(e % s);
    Q[e] = make_double2(i == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int j = s - 1; j >= 0; --j) {
    const double tj = tau[j];
    if (tj == 0.0) continue;
    for (int c = j + wv; c < s; c += nw) {
      cplx acc = (lane == 0) ? Q[(int64_t)j * s + c] : make_double2(0.0, 0.0);
      for (int i = j + 1 + lane; i < m; i += 64) cfma(acc, cconj(W[(int64_t)i * n + j]), Q[(int64_t)i * s + c]);
      acc = wave_sum(acc);
      cplx f = cscale(acc, -tj);
      if (lane == 0) Q[(int64_t)j * s + c] = cadd(Q[(int64_t)j * s + c], f);
      for (int i = j + 1 + lane; i < m; i += 64) {
        int64_t o = (int64_t)i * s + c;
        Q[o] = cadd(Q[o], cmul(W[(int64_t)i * n + j], f));
      }
    }
    __syncthreads();
  }
  if (tid == 0 && s_out) s_out[(int64_t)b * s_stride] = s;
}

void qr(hipStream_t st, int batch, Dim m, Dim n, const cplx* A, int64_t sA, cplx* W, int64_t sW,
        double* tau, int64_t sTau, cplx* Q, int64_t sQ, cplx* R, int64_t sR, int32_t* s_out,
        int s_stride) {
  k_qr<<<batch, 1024, 0, st>>>(m, n, A, sA, W, sW, tau, sTau, Q, sQ, R, sR, s_out, s_stride);
}

void qr_auto(hipStream_t st, int batch, int mcap, int ncap, Dim m, Dim n, const cplx* A,
             int64_t sA, cplx* W, int64_t sW, double* tau, int64_t sTau, cplx* Q, int64_t sQ,
             cplx* R, int64_t sR, int32_t* s_out, int s_stride) {
  const bool prof = prof_on(PROF_QR);
  if (prof) g_prof->begin();
  if (!qr_reg(st, batch, mcap, ncap, m, n, A, sA, W, sW, tau, sTau, Q, sQ, R, sR, s_out, s_stride))
    qr_mem(st, batch, mcap, ncap, m, n, A, sA, W, sW, tau, sTau, Q, sQ, R, sR, s_out, s_stride);
  if (prof) g_prof->end();
}

// ------------------------------------------------------------ Jacobi SVD
// Columns of B (mb x nb, stored column-major: column c at B + c*mb) are made
// mutually orthogonal by plane rotations [b_p, b_q] <- [b_p, b_q] J with
//   J = [[c, s e^{i phi}], [-s e^{-i phi}, c]],  gamma = b_p^H b_q = |gamma| e^{i phi},
//   zeta = (beta - alpha)/(2|gamma|), t = sign(zeta)/(|zeta| + sqrt(1 + zeta^2)),
//   c = 1/sqrt(1 + t^2), s = c t;  the same J accumulates into V.
// Pairs follow a round-robin (circle) schedule: every round is a set of
// disjoint pairs, one per wave at a time.
// Convergence: rotate only while |gamma| > 2 mb eps sqrt(alpha beta) (the
// rounding bound of a length-mb dot product), and never between columns whose
// norms are below 1e-17 ||B||_F (they carry no significant digits; rotating
// them can cycle on underflowed values).
constexpr double JAC_EPS = 2.0 * 2.220446049250313e-16;
constexpr double JAC_NEGL = 1e-34;
constexpr int SVD_MAXNB = 1024;

__global__ __launch_bounds__(256) void k_svd_trunc(
    Dim Md, Dim Cd, const cplx* __restrict__ A, int64_t sA, cplx* __restrict__ Bw, int64_t sB,
    cplx* __restrict__ Vw, int64_t sV, cplx* __restrict__ core, int64_t sCore,
    cplx* __restrict__ carry, int64_t sCarry, int32_t* l_out, int l_stride,
    const double* __restrict__ delta, double* __restrict__ disc2, int lmax, int max_sweeps,
    int32_t* status, double* svlog, int64_t svstride) {
  const int b = blockIdx.x;
  const int m = dimv(Md, b), nc = dimv(Cd, b);
  const bool tall = m >= nc;
  const int mb = tall ? m : nc, nb = tall ? nc : m;
  A += b * sA; Bw += b * sB; Vw += b * sV; core += b * sCore; carry += b * sCarry;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
  __shared__ double sig[SVD_MAXNB];
  __shared__ int perm[SVD_MAXNB];
  __shared__ int sh_rot;
  __shared__ int sh_l;
  // B = A (tall) or A^H (wide), column-major
  for (int64_t e = tid; e < (int64_t)mb * nb; e += blockDim.x) {
    int c = (int)(e / mb), i = (int)(e % mb);
    Bw[e] = tall ? A[(int64_t)i * nc + c] : cconj(A[(int64_t)c * nc + i]);
  }
  for (int64_t e = tid; e < (int64_t)nb * nb; e += blockDim.x) {
    int c = (int)(e / nb), i = (int)(e % nb);
    Vw[e] = make_double2(i == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  const int nbp = (nb + 1) & ~1;
  const double jtol = JAC_EPS * (double)mb;
  __shared__ double red_f[16];
  double fro = 0.0;
  for (int64_t e = tid; e < (int64_t)mb * nb; e += blockDim.x) fro += cabs2(Bw[e]);
  fro = wave_sum(fro);
  if (lane == 0) red_f[wv] = fro;
  __syncthreads();
  fro = 0.0;
  for (int i = 0; i < nw; ++i) fro += red_f[i];
  const double negl = JAC_NEGL * fro;
  int sweep = 0;
  bool converged = (nb < 2);
  for (; sweep < max_sweeps && !converged; ++sweep) {
    if (tid == 0) sh_rot = 0;
    __syncthreads();
    for (int r = 0; r < nbp - 1; ++r) {
      for (int pi = wv; pi < nbp / 2; pi += nw) {
        int p, q;
        if (pi == 0) { p = nbp - 1; q = r; }
        else { p = (r + pi) % (nbp - 1); q = (r - pi + nbp - 1) % (nbp - 1); }
        if (p >= nb || q >= nb) continue;
        if (p > q) { int t = p; p = q; q = t; }
        cplx* bp = Bw + (int64_t)p * mb;
        cplx* bq = Bw + (int64_t)q * mb;
        double al = 0.0, be = 0.0;
        cplx ga = make_double2(0.0, 0.0);
        for (int i = lane; i < mb; i += 64) {
          cplx x = bp[i], y = bq[i];
          al += cabs2(x);
          be += cabs2(y);
          cfma(ga, cconj(x), y);
        }
        al = wave_sum(al); be = wave_sum(be); ga = wave_sum(ga);
        double g = sqrt(cabs2(ga));
        if (al <= negl || be <= negl) continue;
        if (g == 0.0 || !(g > jtol * sqrt(al * be))) continue;
        double zeta = (be - al) / (2.0 * g);
        double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        cplx e = make_double2(ga.x / g, ga.y / g);            // e^{i phi}
        cplx se = cscale(e, s), sec = cscale(cconj(e), s);
        for (int i = lane; i < mb; i += 64) {
          cplx x = bp[i], y = bq[i];
          bp[i] = csub(cscale(x, c), cmul(sec, y));
          bq[i] = cadd(cmul(se, x), cscale(y, c));
        }
        cplx* vp = Vw + (int64_t)p * nb;
        cplx* vq = Vw + (int64_t)q * nb;
        for (int i = lane; i < nb; i += 64) {
          cplx x = vp[i], y = vq[i];
          vp[i] = csub(cscale(x, c), cmul(sec, y));
          vq[i] = cadd(cmul(se, x), cscale(y, c));
        }
        if (lane == 0) sh_rot = 1;
      }
      __syncthreads();
    }
    converged = (sh_rot == 0);
    __syncthreads();
  }
  if (!converged && tid == 0) {
    const int32_t old = atomicOr(status, (int32_t)ST_JACOBI_CAP);
    if (!(old & ST_JACOBI_CAP)) {
      double* d = status_diag(status);
      d[0] = nb;
      d[1] = d[2] = d[3] = -1.0;   // not tracked by this variant
      d[4] = max_sweeps;
    }
  }
  // singular values
  for (int c = wv; c < nb; c += nw) {
    double a = 0.0;
    for (int i = lane; i < mb; i += 64) a += cabs2(Bw[(int64_t)c * mb + i]);
    a = wave_sum(a);
    if (lane == 0) sig[c] = sqrt(a);
  }
  __syncthreads();
  for (int c = tid; c < nb; c += blockDim.x) {
    double v = sig[c];
    int pos = 0;
    for (int d = 0; d < nb; ++d) pos += (sig[d] > v) || (sig[d] == v && d < c);
    perm[pos] = c;
  }
  __syncthreads();
  if (tid == 0) {
    double dl = delta[b];
    // tail[l] = sqrt(sum_{j >= l} s_j^2): smallest l >= 1 with tail[l] <= dl
    double tail2 = 0.0;
    int l = nb;
    for (int j = nb - 1; j >= 0; --j) {
      double sj = sig[perm[j]];
      if (sqrt(tail2 + sj * sj) <= dl) { tail2 += sj * sj; l = j; }
      else break;
    }
    if (l < 1) l = 1;
    if (l > lmax) l = lmax;
    if (l > nb) l = nb;
    double d2 = 0.0;
    bool finite = true;
    for (int j = 0; j < nb; ++j) {
      double sj = sig[perm[j]];
      if (!isfinite(sj)) finite = false;
      if (j >= l) d2 += sj * sj;
    }
    if (!finite) {
      const int32_t old = atomicOr(status, (int32_t)ST_NONFINITE);
      if (!(old & ST_NONFINITE)) {
        double* d = status_diag(status) + 5;
        d[0] = nb;
        d[1] = fro;
        d[2] = -1.0;
        d[3] = 2.0;   // global-memory Jacobi
        d[4] = sweep;
      }
    }
    disc2[b] += d2;
    sh_l = l;
    if (l_out) l_out[(int64_t)b * l_stride] = l;
  }
  __syncthreads();
  const int l = sh_l;
  if (svlog)
    for (int j = tid; j < nb; j += blockDim.x) svlog[b * svstride + j] = sig[perm[j]];
  if (tall) {
    // A V = U Sigma = B:  core = V^H[:l] (l x nc),  carry = B[:, perm[:l]] (m x l)
    for (int64_t e = tid; e < (int64_t)l * nc; e += blockDim.x) {
      int r = (int)(e / nc), c = (int)(e % nc);
      core[e] = cconj(Vw[(int64_t)perm[r] * nb + c]);
    }
    for (int64_t e = tid; e < (int64_t)m * l; e += blockDim.x) {
      int i = (int)(e / l), r = (int)(e % l);
      carry[e] = Bw[(int64_t)perm[r] * mb + i];
    }
  } else {
    // A^H W = U' Sigma = B:  A = W Sigma U'^H;  core = (B[:, perm[r]]/sigma)^H,
    // carry = W[:, perm[:l]] Sigma
    for (int64_t e = tid; e < (int64_t)l * nc; e += blockDim.x) {
      int r = (int)(e / nc), c = (int)(e % nc);
      double sv = sig[perm[r]];
      cplx v;
      if (sv > 0.0) v = cscale(cconj(Bw[(int64_t)perm[r] * mb + c]), 1.0 / sv);
      else v = make_double2(c == r ? 1.0 : 0.0, 0.0);
      core[e] = v;
    }
    for (int64_t e = tid; e < (int64_t)m * l; e += blockDim.x) {
      int i = (int)(e / l), r = (int)(e % l);
      carry[e] = cscale(Vw[(int64_t)perm[r] * nb + i], sig[perm[r]]);
    }
  }
}

void svd_trunc(hipStream_t st, int batch, Dim m, Dim c, const cplx* A, int64_t sA, cplx* Bw,
               int64_t sB, cplx* Vw, int64_t sV, cplx* core, int64_t sCore, cplx* carry,
               int64_t sCarry, int32_t* l_out, int l_stride, const double* delta, double* disc2,
               int lmax, int max_sweeps, int32_t* status, double* svlog, int64_t svstride,
               int nbcap) {
  (void)nbcap;
  k_svd_trunc<<<batch, 256, 0, st>>>(m, c, A, sA, Bw, sB, Vw, sV, core, sCore, carry, sCarry,
                                     l_out, l_stride, delta, disc2, lmax, max_sweeps, status,
                                     svlog, svstride);
}

// ------------------------------------------------------------ small kernels
__global__ __launch_bounds__(256) void k_norm_delta(Dim Rd, Dim Cd, const cplx* X, int64_t sX,
                                                    double* norm, double* delta, double* disc2,
                                                    double eps, int nb_bonds) {
  __shared__ double red[16];
  const int b = blockIdx.x;
  const int64_t cnt = (int64_t)dimv(Rd, b) * dimv(Cd, b);
  X += b * sX;
  double a = 0.0;
  for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) a += cabs2(X[e]);
  a = block_sum(a, red);
  if (threadIdx.x == 0) {
    double nr = sqrt(a);
    if (norm) norm[b] = nr;
    if (delta) delta[b] = nb_bonds > 0 ? eps * nr / sqrt((double)nb_bonds) : 0.0;
    if (disc2) disc2[b] = 0.0;
  }
}

void norm_delta(hipStream_t st, int batch, Dim rows, Dim cols, const cplx* X, int64_t sX,
                double* norm, double* delta, double* disc2, double eps, int nb_bonds) {
  k_norm_delta<<<batch, 256, 0, st>>>(rows, cols, X, sX, norm, delta, disc2, eps, nb_bonds);
}

__global__ void k_copy(Dim Rd, Dim Cd, const cplx* src, int64_t sS, cplx* dst, int64_t sD) {
  const int b = blockIdx.y;
  const int64_t cnt = (int64_t)dimv(Rd, b) * dimv(Cd, b);
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < cnt) dst[b * sD + e] = src[b * sS + e];
}

void copy(hipStream_t st, int batch, Dim rows, Dim cols, int64_t cap_elems, const cplx* src,
          int64_t sS, cplx* dst, int64_t sD) {
  if (cap_elems <= 0) return;
  dim3 grid((unsigned)((cap_elems + 255) / 256), batch);
  k_copy<<<grid, 256, 0, st>>>(rows, cols, src, sS, dst, sD);
}

__global__ void k_finalize_err(int batch, const double* disc2, const double* norm, double* err,
                               double* norm_out) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  double nr = norm[b];
  if (err) err[b] = nr > 0.0 ? sqrt(disc2[b]) / nr : 0.0;
  if (norm_out) norm_out[b] = nr;
}

void finalize_err(hipStream_t st, int batch, const double* disc2, const double* norm, double* err,
                  double* norm_out) {
  k_finalize_err<<<(batch + 127) / 128, 128, 0, st>>>(batch, disc2, norm, err, norm_out);
}

__global__ void k_scale_vec(int batch, const double* in, const double* scale, double* out) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < batch) out[b] = in[b] * scale[b];
}

void scale_vec(hipStream_t st, int batch, const double* in, const double* scale, double* out) {
  k_scale_vec<<<(batch + 127) / 128, 128, 0, st>>>(batch, in, scale, out);
}

__global__ void k_copy_i32(int64_t count, const int32_t* __restrict__ src, int32_t* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) dst[t] = src[t];
}

void copy_i32(hipStream_t st, int64_t count, const int32_t* src, int32_t* dst) {
  if (count <= 0) return;
  k_copy_i32<<<(unsigned)((count + 255) / 256), 256, 0, st>>>(count, src, dst);
}

}  // namespace qt
