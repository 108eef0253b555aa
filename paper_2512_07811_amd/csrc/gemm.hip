// General strided, batched complex-double GEMM used by the structured
// (product-aware) contractions.  Every size and stride may depend on device
// ranks, so the launch grid covers capacities and idle tiles exit at once.
#include "kernels.h"

namespace qt {

constexpr int XT_M = 64, XT_N = 64, XT_K = 16;

template <bool CA, bool CB>
__global__ __launch_bounds__(256) void k_gemm_ex(int nb1, int nb2, int ntn, Dim Md, Dim Nd,
                                                 Dim Kd, Mat A, Mat B, Mat C, cplx alpha,
                                                 int accumulate, Dim lim1,
                                                 unsigned long long* counters) {
  const int nbt = nb1 * nb2;
  const int tn = blockIdx.x % ntn;
  const int z = blockIdx.x / ntn;
  const int b = z / nbt;
  const int rem = z % nbt;
  const int b1 = rem / nb2, b2 = rem % nb2;
  const int M = dimv(Md, b), N = dimv(Nd, b), K = dimv(Kd, b);
  const int m0 = blockIdx.y * XT_M, n0 = tn * XT_N;
  if (m0 >= M || n0 >= N || b1 >= dimv(lim1, b)) return;
  if (counters && m0 == 0 && n0 == 0 && threadIdx.x == 0 && K > 0) {
    // algorithmic work of this product: 8 real flops per complex MAC and the
    // compulsory traffic of reading A, B and writing C once
    atomicAdd(counters + CNT_GEMM_FLOPS, 8ull * M * N * K);
    atomicAdd(counters + CNT_GEMM_BYTES, 16ull * ((unsigned long long)M * K + (unsigned long long)K * N +
                                                  (unsigned long long)M * N));
  }
  const cplx* Ab = A.base + b * A.inst + strv(A.off, b) + b1 * strv(A.s1, b) + b2 * strv(A.s2, b);
  const cplx* Bb = B.base + b * B.inst + strv(B.off, b) + b1 * strv(B.s1, b) + b2 * strv(B.s2, b);
  cplx* Cb = C.base + b * C.inst + strv(C.off, b) + b1 * strv(C.s1, b) + b2 * strv(C.s2, b);
  const int64_t ars = strv(A.rs, b), acs = strv(A.cs, b);
  const int64_t brs = strv(B.rs, b), bcs = strv(B.cs, b);
  const int64_t crs = strv(C.rs, b), ccs = strv(C.cs, b);
  const bool a_kfast = (acs == 1);
  const bool b_nfast = (bcs == 1);
  __shared__ cplx As[XT_K][XT_M + 1];
  __shared__ cplx Bs[XT_K][XT_N + 1];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  cplx acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = make_double2(0.0, 0.0);

  for (int k0 = 0; k0 < K; k0 += XT_K) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int idx = tid + 256 * e;
      int mm, kk;
      if (a_kfast) { mm = idx >> 4; kk = idx & 15; }
      else { kk = idx >> 6; mm = idx & 63; }
      int gm = m0 + mm, gk = k0 + kk;
      cplx v = make_double2(0.0, 0.0);
      if (gm < M && gk < K) {
        v = Ab[gm * ars + gk * acs];
        if (CA) v = cconj(v);
      }
      As[kk][mm] = v;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int idx = tid + 256 * e;
      int kk, nn;
      if (b_nfast) { kk = idx >> 6; nn = idx & 63; }
      else { nn = idx >> 4; kk = idx & 15; }
      int gk = k0 + kk, gn = n0 + nn;
      cplx v = make_double2(0.0, 0.0);
      if (gk < K && gn < N) {
        v = Bb[gk * brs + gn * bcs];
        if (CB) v = cconj(v);
      }
      Bs[kk][nn] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < XT_K; ++kk) {
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
      cplx* o = Cb + gm * crs + gn * ccs;
      if (accumulate) v = cadd(v, *o);
      *o = v;
    }
  }
}

void gemm_ex(hipStream_t st, int batch, int nb1, int nb2, Dim M, Dim N, Dim K, int Mcap, int Ncap,
             Mat A, bool conjA, Mat B, bool conjB, Mat C, cplx alpha, bool accumulate, Dim lim1) {
  if (Mcap <= 0 || Ncap <= 0 || batch <= 0 || nb1 <= 0 || nb2 <= 0) return;
  const int ntn = (Ncap + XT_N - 1) / XT_N;
  const int64_t gx = (int64_t)ntn * batch * nb1 * nb2;
  dim3 grid((unsigned)gx, (Mcap + XT_M - 1) / XT_M, 1);
  const int acc = accumulate ? 1 : 0;
  unsigned long long* cnt = g_counters;
  const bool prof = prof_on(PROF_GEMM);
  if (prof) g_prof->begin();
  if (!conjA && !conjB)
    k_gemm_ex<false, false><<<grid, 256, 0, st>>>(nb1, nb2, ntn, M, N, K, A, B, C, alpha, acc, lim1, cnt);
  else if (conjA && !conjB)
    k_gemm_ex<true, false><<<grid, 256, 0, st>>>(nb1, nb2, ntn, M, N, K, A, B, C, alpha, acc, lim1, cnt);
  else if (!conjA && conjB)
    k_gemm_ex<false, true><<<grid, 256, 0, st>>>(nb1, nb2, ntn, M, N, K, A, B, C, alpha, acc, lim1, cnt);
  else
    k_gemm_ex<true, true><<<grid, 256, 0, st>>>(nb1, nb2, ntn, M, N, K, A, B, C, alpha, acc, lim1, cnt);
  if (prof) g_prof->end();
}

}  // namespace qt
