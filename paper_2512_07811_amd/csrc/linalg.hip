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
