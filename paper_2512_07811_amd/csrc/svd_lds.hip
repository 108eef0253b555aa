// Truncated SVD for the right-to-left sweep, A (m x c) packed row-major:
//   1. B = A (m >= c) or A^H (m < c); B = Q R by Householder QR;
//   2. one-sided (Hestenes) Jacobi on the columns of X = T^H for an upper
//      triangle T, until X W = U Sigma has orthogonal columns (W is not
//      formed); the rows of a triangular factor are better separated than
//      its columns, so this converges in fewer sweeps than Jacobi on T
//      (Drmac and Veselic, SIAM J. Matrix Anal. Appl. 29, 2008):
//        tall (A = Q R):   T = R; R = W Sigma U^H, A = (Q W) Sigma U^H, and
//                          the right singular vectors of A are U;
//        wide (A^H = Q R): a second QR without Q, R^H = Q2 R2, and T = R2:
//                          R = R2^H Q2^H has the left singular vectors U of
//                          R2^H, A = R^H Q^H = W' Sigma (Q U)^H, and the right
//                          singular vectors of A are Q U;
//   3. truncation (smallest l whose discarded tail <= delta, l <= lmax);
//   4. core = the first l right singular vectors as rows (U^H[:l] from the
//      converged columns, or (Q U[:, :l])^H by one GEMM), and
//      carry = A core^H, which equals U_A Sigma[:, :l] (A V_l = U_A Sigma_l),
//      by one GEMM on the original A: carry core = A V_l V_l^H is the
//      orthogonal projection of A, whatever the accuracy of W.
// Rotation: gamma = b_p^H b_q = |gamma| e^{i phi}, zeta = (beta - alpha)/(2|gamma|),
// t = sign(zeta)/(|zeta| + sqrt(1 + zeta^2)), c = 1/sqrt(1 + t^2), s = c t,
// [b_p, b_q] <- [b_p, b_q] [[c, s e^{i phi}], [-s e^{-i phi}, c]].
#include "kernels.h"

namespace qt {

constexpr int SL_NB = 68;            // orders up to 68: five rows per lane
constexpr int SL_NB_BIG = 100;       // up to 100: X fills 160000 bytes of LDS
constexpr double SL_EPS = 2.0 * 2.220446049250313e-16;
constexpr double SL_NEGL = 1e-34;

// Flags a non-finite output of the Jacobi (stage 6: the core of a tall
// instance, 8: the left vectors of a wide one) with the order, kept rank and
// extreme kept sigmas.
__device__ inline void flag_out(int32_t* status, int stage, int nb, int l, double smax,
                                double smin) {
  const int32_t old = atomicOr(status, (int32_t)ST_NONFINITE);
  if (!(old & ST_NONFINITE)) {
    double* d = status_diag(status) + 5;
    d[0] = nb;
    d[1] = smax;
    d[2] = smin;
    d[3] = stage;
    d[4] = l;
  }
}

// Truncation after convergence (thread 0): sorted order perm of the column
// norms sig, the smallest l >= 1 whose tail does not exceed delta, l <= lmax;
// returns l, adds the discarded tail to disc2, flags non-finite sigmas.
__device__ inline int jacobi_truncate(const double* sig, const int* perm, int nb, double dl,
                                      int lmax, double* disc2_b, int32_t* status, double fro,
                                      int sweeps_done, double variant) {
  double tail2 = 0.0;
  int l = nb;
  for (int j = nb - 1; j >= 0; --j) {
    const double sj = sig[perm[j]];
    if (sqrt(tail2 + sj * sj) <= dl) { tail2 += sj * sj; l = j; }
    else break;
  }
  if (l < 1) l = 1;
  if (l > lmax) l = lmax;
  if (l > nb) l = nb;
  double d2 = 0.0;
  bool finite = true;
  for (int j = 0; j < nb; ++j) {
    const double sj = sig[perm[j]];
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
      d[3] = variant;
      d[4] = sweeps_done;
    }
  }
  *disc2_b += d2;
  return l;
}

// Sum over the block (every thread gets the result); red holds 16 doubles.
__device__ inline double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

// Maximum / minimum over the block (every thread gets the result).
__device__ inline double block_max(double v, double* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double s = red[0];
  for (int i = 1; i < nw; ++i) s = fmax(s, red[i]);
  return s;
}
__device__ inline double block_min(double v, double* red) {
  return -block_max(-v, red);
}

// Sweep-cap diagnostics (thread 0): order, Frobenius norm^2, largest
// |gamma| / sqrt(alpha beta) / tol and smallest rotated column norm^2 /
// Frobenius^2 of the last sweep, sweeps done.
__device__ inline void flag_sweep_cap(int32_t* status, int nb, double fro, double worst2,
                                      double small2, double jtol, int sweeps_done) {
  const int32_t old = atomicOr(status, (int32_t)ST_JACOBI_CAP);
  if (!(old & ST_JACOBI_CAP)) {
    double* d = status_diag(status);
    d[0] = nb;
    d[1] = fro;
    d[2] = sqrt(worst2) / jtol;
    d[3] = small2 / fro;
    d[4] = sweeps_done;
  }
}

// Kept columns whose squared norm is at or below the rotation floor were
// never rotated, so they are not orthogonal to the others.  Their weight in
// the matrix is below 1e-17 of its norm, so any orthonormal completion
// serves: the sorted kept columns perm[t0..l) become, one by one, the unit
// vector e_j with the largest weight w_j = 1 - sum_q |U[j, q]|^2 outside the
// current span (at least (nb - r) / nb), with the previous columns projected
// out twice (classical Gram-Schmidt with reorthogonalization), normalized.
// Columns perm[0..t0) must have unit norm.  Whole block; h holds l complex
// values, w (nb doubles) is scratch.
__device__ void complete_columns(cplx* X, const int* perm, int nb, int t0, int l, cplx* h,
                                 double* red, double* w) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
  for (int j = tid; j < nb; j += blockDim.x) {
    double a = 1.0;
    for (int q = 0; q < t0; ++q) a -= cabs2(X[(int64_t)perm[q] * nb + j]);
    w[j] = a;
  }
  __syncthreads();
  for (int r = t0; r < l; ++r) {
    double best = -1.0;
    for (int j = tid; j < nb; j += blockDim.x) best = fmax(best, w[j]);
    best = block_max(best, red);
    double jb = (double)nb;
    for (int j = tid; j < nb; j += blockDim.x)
      if (w[j] == best) jb = fmin(jb, (double)j);
    const int js = (int)block_min(jb, red);
    cplx* v = X + (int64_t)perm[r] * nb;
    for (int i = tid; i < nb; i += blockDim.x) v[i] = make_double2(i == js ? 1.0 : 0.0, 0.0);
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
      for (int q = wv; q < r; q += nw) {
        const cplx* u = X + (int64_t)perm[q] * nb;
        cplx a = make_double2(0.0, 0.0);
        for (int i = lane; i < nb; i += 64) cfma(a, cconj(u[i]), v[i]);
        a = wave_sum(a);
        if (lane == 0) h[q] = a;
      }
      __syncthreads();
      for (int i = tid; i < nb; i += blockDim.x) {
        cplx acc = v[i];
        for (int q = 0; q < r; ++q) acc = csub(acc, cmul(h[q], X[(int64_t)perm[q] * nb + i]));
        v[i] = acc;
      }
      __syncthreads();
    }
    double n2 = 0.0;
    for (int i = tid; i < nb; i += blockDim.x) n2 += cabs2(v[i]);
    const double inv = 1.0 / sqrt(block_sum(n2, red));
    for (int i = tid; i < nb; i += blockDim.x) {
      const cplx u = cscale(v[i], inv);
      v[i] = u;
      w[i] -= cabs2(u);
    }
    __syncthreads();
  }
}

// Kept columns to unit norm in place (perm[0..t0), above the floor), the
// completion of the rest, then the outputs: core = U^H[:l] (tall) or
// Ul = U[:, :l] (wide).  sig is scratch after the normalization.
__device__ void jacobi_outputs(cplx* X, double* sig, const int* perm, int nb, int l, double negl,
                               bool tall, cplx* core, cplx* Ul, cplx* h, double* red,
                               int32_t* status) {
  const int tid = threadIdx.x;
  int t0 = l;
  for (int r = 0; r < l; ++r) {
    const double sv = sig[perm[r]];
    if (!(sv * sv > negl)) { t0 = r; break; }
  }
  const double s_first = sig[perm[0]], s_last = sig[perm[l - 1]];
  for (int64_t e = tid; e < (int64_t)t0 * nb; e += blockDim.x) {
    const int r = (int)(e / nb), i = (int)(e % nb);
    const int c = perm[r];
    X[(int64_t)c * nb + i] = cscale(X[(int64_t)c * nb + i], 1.0 / sig[c]);
  }
  __syncthreads();
  if (t0 < l) complete_columns(X, perm, nb, t0, l, h, red, sig);
  bool fin = true;
  for (int64_t e = tid; e < (int64_t)l * nb; e += blockDim.x) {
    const int r = (int)(e / nb), i = (int)(e % nb);
    const cplx u = X[(int64_t)perm[r] * nb + i];
    fin = fin && isfinite(u.x) && isfinite(u.y);
    if (tall) core[e] = cconj(u);     // row r of U^H
    else Ul[e] = u;
  }
  if (!fin) flag_out(status, tall ? 6 : 8, nb, l, s_first, s_last);
}

// One workgroup per instance; T (nb x nb, row-major) in Rin, X = T^H in LDS
// (NBMAX <= 100).  Outputs: tall: core =
// U^H[:l] (l x nb, row-major); wide: Ul = U[:, :l] (column r at Ul + r * nb),
// from which the caller forms core = (Q U[:, :l])^H.
template <int NBMAX>
__global__ __launch_bounds__(1024) void k_jacobi_lds(
    Dim Md, Dim Cd, const cplx* __restrict__ Rin, int64_t sR, cplx* __restrict__ Ul, int64_t sU,
    cplx* __restrict__ core, int64_t sCore, int32_t* l_out, int l_stride,
    const double* __restrict__ delta, double* __restrict__ disc2, int lmax, int max_sweeps,
    int32_t* status, double* svlog, int64_t svstride, unsigned long long* counters) {
  __shared__ cplx Rs[NBMAX * NBMAX];
  __shared__ cplx hb[NBMAX];          // projections of the column completion
  __shared__ double sig[NBMAX];
  __shared__ int perm[NBMAX];
  __shared__ double red[16];
  __shared__ int sh_l;
  const int b = blockIdx.x;
  const int m = dimv(Md, b), nc = dimv(Cd, b);
  const bool tall = m >= nc;
  const int nb = tall ? nc : m;
  Rin += b * sR; Ul += b * sU; core += b * sCore;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
  double fro = 0.0;
  for (int e = tid; e < nb * nb; e += blockDim.x) {
    const cplx v = cconj(Rin[e]);         // column c of T^H = conj(row c of T)
    Rs[e] = v;
    fro += cabs2(v);
  }
  fro = wave_sum(fro);
  if (lane == 0) red[wv] = fro;
  __syncthreads();
  fro = 0.0;
  for (int i = 0; i < nw; ++i) fro += red[i];
  if (tid == 0 && !isfinite(fro)) {
    const int32_t old = atomicOr(status, (int32_t)ST_NONFINITE);
    if (!(old & ST_NONFINITE)) {
      double* d = status_diag(status) + 5;
      d[0] = nb;
      d[1] = fro;
      d[2] = -1.0;
      d[3] = 3.0;   // the triangle handed to the Jacobi
      d[4] = 0.0;
    }
  }
  const double negl = SL_NEGL * fro;
  const double jtol = SL_EPS * (double)nb, jtol2 = jtol * jtol;
  const int nbp = (nb + 1) & ~1;
  const int g = tid & 15, grp = tid >> 4, ngrp = blockDim.x >> 4;
  bool converged = nb < 2;
  int sweeps_done = 0;
  // each 16-lane row group owns one pair per round; sums reduce over the group by DPP
  // per lane: any rotation in the current sweep; in the last allowed sweep
  // also the largest gamma^2 / (alpha beta) and the smallest rotated column
  // norm^2 (diagnostics of the sweep cap); convergence is one block-wide OR
  // per sweep
  double worst2 = 0.0, small2 = 0.0;
  for (int sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
    ++sweeps_done;
    int any_rot = 0;
    worst2 = 0.0;
    small2 = fro;
    for (int r = 0; r < nbp - 1; ++r) {
      for (int pi0 = 0; pi0 < nbp / 2; pi0 += ngrp) {
        // waves whose four groups all lie beyond the last pair of this round
        // have nothing to do (wave-uniform skip)
        if (pi0 + 4 * wv >= nbp / 2) continue;
        const int pi = pi0 + grp;
        int p = 0, q = 0;
        bool valid = pi < nbp / 2;
        if (valid) {
          const int mod = nbp - 1;
          if (pi == 0) { p = mod; q = r; }
          else {
            p = r + pi;
            if (p >= mod) p -= mod;
            q = r - pi;
            if (q < 0) q += mod;
          }
          if (p >= nb || q >= nb) valid = false;
          if (p > q) { int t = p; p = q; q = t; }
        }
        cplx* bp = Rs + p * nb;
        cplx* bq = Rs + q * nb;
        // the pair's columns stay in registers between the dot products and
        // the rotation up to order 68 (at most five rows per lane); above,
        // the rotation reads them again from LDS (register budget of 1024
        // threads)
        constexpr int RPL = (NBMAX + 15) / 16;
        constexpr bool KEEP = RPL <= 5;
        cplx xs[KEEP ? RPL : 1], ys[KEEP ? RPL : 1];
        double al = 0.0, be = 0.0;
        cplx ga = make_double2(0.0, 0.0);
#pragma unroll
        for (int it = 0; it < RPL; ++it) {
          const int i = g + 16 * it;
          cplx x = make_double2(0.0, 0.0), y = make_double2(0.0, 0.0);
          if (valid && i < nb) {
            x = bp[i];
            y = bq[i];
          }
          if (KEEP) {
            xs[it] = x;
            ys[it] = y;
          }
          al += cabs2(x);
          be += cabs2(y);
          cfma(ga, cconj(x), y);
        }
        al = row16_sum(al); be = row16_sum(be); ga = row16_sum(ga);
        const double g2 = cabs2(ga);
        const bool rot = valid && al > negl && be > negl && g2 > 0.0 && g2 > jtol2 * al * be;
        if (rot) {
          const double ig = fast_rsq(g2);                       // 1 / |gamma|
          const double zeta = 0.5 * (be - al) * ig;
          const double z2 = fma(zeta, zeta, 1.0);
          const double w = z2 * fast_rsq(z2);                   // sqrt(1 + zeta^2)
          const double t = copysign(fast_rcp(fabs(zeta) + w), zeta);
          const double c = fast_rsq(fma(t, t, 1.0)), s = c * t;
          const cplx e = make_double2(ga.x * ig, ga.y * ig);
          const cplx se = cscale(e, s), sec = cscale(cconj(e), s);
#pragma unroll
          for (int it = 0; it < RPL; ++it) {
            const int i = g + 16 * it;
            if (i < nb) {
              const cplx x = KEEP ? xs[it] : bp[i], y = KEEP ? ys[it] : bq[i];
              bp[i] = csub(cscale(x, c), cmul(sec, y));
              bq[i] = cadd(cmul(se, x), cscale(y, c));
            }
          }
          any_rot = 1;
          if (sweep + 1 == max_sweeps) {   // read only when the cap is reached
            worst2 = fmax(worst2, g2 * fast_rcp(al * be));
            small2 = fmin(small2, fmin(al, be));
          }
        }
      }
      __syncthreads();
    }
    converged = !__syncthreads_or(any_rot);
  }
  if (!converged) {   // block-uniform
    const double w2 = block_max(worst2, red), s2 = block_min(small2, red);
    if (tid == 0) flag_sweep_cap(status, nb, fro, w2, s2, jtol, sweeps_done);
  }
  if (tid == 0 && counters) {
    atomicAdd(counters + CNT_SVD_CALLS, 1ull);
    atomicAdd(counters + CNT_SVD_SWEEPS, (unsigned long long)sweeps_done);
  }
  for (int c = wv; c < nb; c += nw) {
    double a = 0.0;
    for (int i = lane; i < nb; i += 64) a += cabs2(Rs[c * nb + i]);
    a = wave_sum(a);
    if (lane == 0) sig[c] = sqrt(a);
  }
  __syncthreads();
  for (int c = tid; c < nb; c += blockDim.x) {
    const double v = sig[c];
    int pos = 0;
    for (int d = 0; d < nb; ++d) pos += (sig[d] > v) || (sig[d] == v && d < c);
    perm[pos] = c;
  }
  __syncthreads();
  if (tid == 0) {
    const int l = jacobi_truncate(sig, perm, nb, delta[b], lmax, disc2 + b, status, fro,
                                  sweeps_done, 1.0);
    sh_l = l;
    if (l_out) l_out[(int64_t)b * l_stride] = l;
  }
  __syncthreads();
  const int l = sh_l;
  if (svlog)
    for (int j = tid; j < nb; j += blockDim.x) svlog[b * svstride + j] = sig[perm[j]];
  // U[:, r] = (X W)[:, perm[r]] / sigma
  jacobi_outputs(Rs, sig, perm, nb, l, negl, tall, core, Ul, hb, red, status);
}


// Global-memory variant for orders 100 < nb <= 1024 (same algorithm, schedule
// and thresholds): X in the work matrix Xw (column-major, nb x nb per
// instance); each 16-lane group streams its pair's columns in chunks of SG_CH
// rows per lane (all loads of a chunk issued before use).  Outputs as the LDS
// variant.
constexpr int SG_NB = 1024;
constexpr int SG_CH = 6;
constexpr int SG_RPL = 8;            // register variant: orders up to 32 * SG_RPL = 256

// Sum over a group of GL = 16 or 32 lanes (every lane of the group gets it).
template <int GL>
__device__ inline double group_sum(double v) {
  v = row16_sum(v);
  if (GL == 32) v += __shfl_xor(v, 16, 64);
  return v;
}
template <int GL>
__device__ inline cplx group_sum(cplx v) {
  return make_double2(group_sum<GL>(v.x), group_sum<GL>(v.y));
}

// RPL = 0: 16-lane groups stream their pair's columns from X in chunks, once
// for the dot products and once for the rotation.  RPL > 0 (orders up to
// GL RPL): GL-lane groups keep the pair's columns in registers between the
// dot products and the rotation, one load and one store per element.  The
// 64 groups of 16 lanes take the 64 pairs of a step of order <= 128 in one
// pass and those of orders <= 144 in two; 32-lane groups orders up to 256.
template <int RPL, int GL>
__global__ __launch_bounds__(1024) void k_jacobi_glb(
    Dim Md, Dim Cd, const cplx* __restrict__ Rin, int64_t sR, cplx* __restrict__ Xw, int64_t sX,
    cplx* __restrict__ Ul, int64_t sU, cplx* __restrict__ core, int64_t sCore, int32_t* l_out,
    int l_stride, const double* __restrict__ delta, double* __restrict__ disc2, int lmax,
    int max_sweeps, int32_t* status, double* svlog, int64_t svstride,
    unsigned long long* counters) {
  __shared__ double sig[SG_NB];
  __shared__ int perm[SG_NB];
  __shared__ cplx hb[SG_NB];
  __shared__ double red[16];
  __shared__ int sh_l;
  const int b = blockIdx.x;
  const int m = dimv(Md, b), nc = dimv(Cd, b);
  const bool tall = m >= nc;
  const int nb = tall ? nc : m;
  Rin += b * sR; Xw += b * sX; Ul += b * sU; core += b * sCore;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
  const int64_t nn = (int64_t)nb * nb;
  double fro = 0.0;
  for (int64_t e = tid; e < nn; e += blockDim.x) {
    const cplx v = cconj(Rin[e]);         // column c of T^H = conj(row c of T)
    fro += cabs2(v);
    Xw[e] = v;
  }
  fro = wave_sum(fro);
  if (lane == 0) red[wv] = fro;
  __syncthreads();
  fro = 0.0;
  for (int i = 0; i < nw; ++i) fro += red[i];
  if (tid == 0 && !isfinite(fro)) {
    const int32_t old = atomicOr(status, (int32_t)ST_NONFINITE);
    if (!(old & ST_NONFINITE)) {
      double* d = status_diag(status) + 5;
      d[0] = nb; d[1] = fro; d[2] = -1.0; d[3] = 3.0; d[4] = 0.0;
    }
  }
  const double negl = SL_NEGL * fro;
  const double jtol = SL_EPS * (double)nb, jtol2 = jtol * jtol;
  const int nbp = (nb + 1) & ~1;
  static_assert(GL == 16 || GL == 32, "pair groups of 16 or 32 lanes");
  static_assert(RPL > 0 || GL == 16, "the streaming variant uses 16-lane groups");
  const int g = tid % GL, grp = tid / GL, ngrp = blockDim.x / GL;
  bool converged = nb < 2;
  int sweeps_done = 0;
  // per lane: any rotation in the current sweep; in the last allowed sweep
  // also the largest gamma^2 / (alpha beta) and the smallest rotated column
  // norm^2 (diagnostics of the sweep cap); convergence is one block-wide OR
  // per sweep
  double worst2 = 0.0, small2 = 0.0;
  for (int sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
    ++sweeps_done;
    int any_rot = 0;
    worst2 = 0.0;
    small2 = fro;
    for (int r = 0; r < nbp - 1; ++r) {
      for (int pi0 = 0; pi0 < nbp / 2; pi0 += ngrp) {
        // wave-uniform: no pair for this wave
        if (pi0 + (64 / GL) * wv >= nbp / 2) continue;
        const int pi = pi0 + grp;
        int p = 0, q = 0;
        bool valid = pi < nbp / 2;
        if (valid) {
          const int mod = nbp - 1;
          if (pi == 0) { p = mod; q = r; }
          else {
            p = r + pi;
            if (p >= mod) p -= mod;
            q = r - pi;
            if (q < 0) q += mod;
          }
          if (p >= nb || q >= nb) valid = false;
          if (p > q) { int t = p; p = q; q = t; }
        }
        cplx* bp = Xw + (int64_t)p * nb;
        cplx* bq = Xw + (int64_t)q * nb;
        double al = 0.0, be = 0.0;
        cplx ga = make_double2(0.0, 0.0);
        cplx xr[RPL > 0 ? RPL : 1], yr[RPL > 0 ? RPL : 1];
        if constexpr (RPL > 0) {
#pragma unroll
          for (int it = 0; it < RPL; ++it) {
            const int i = g + GL * it;
            xr[it] = (valid && i < nb) ? bp[i] : make_double2(0.0, 0.0);
            yr[it] = (valid && i < nb) ? bq[i] : make_double2(0.0, 0.0);
          }
#pragma unroll
          for (int it = 0; it < RPL; ++it) {
            al += cabs2(xr[it]);
            be += cabs2(yr[it]);
            cfma(ga, cconj(xr[it]), yr[it]);
          }
        } else if (valid) {
          for (int i0 = g; i0 < nb; i0 += 16 * SG_CH) {
            cplx xs[SG_CH], ys[SG_CH];
#pragma unroll
            for (int u = 0; u < SG_CH; ++u) {
              const int i = i0 + 16 * u;
              xs[u] = i < nb ? bp[i] : make_double2(0.0, 0.0);
              ys[u] = i < nb ? bq[i] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < SG_CH; ++u) {
              al += cabs2(xs[u]);
              be += cabs2(ys[u]);
              cfma(ga, cconj(xs[u]), ys[u]);
            }
          }
        }
        al = group_sum<GL>(al); be = group_sum<GL>(be); ga = group_sum<GL>(ga);
        const double g2 = cabs2(ga);
        const bool rot = valid && al > negl && be > negl && g2 > 0.0 && g2 > jtol2 * al * be;
        if (rot) {
          const double ig = fast_rsq(g2);
          const double zeta = 0.5 * (be - al) * ig;
          const double z2 = fma(zeta, zeta, 1.0);
          const double w = z2 * fast_rsq(z2);
          const double t = copysign(fast_rcp(fabs(zeta) + w), zeta);
          const double c = fast_rsq(fma(t, t, 1.0)), s = c * t;
          const cplx e = make_double2(ga.x * ig, ga.y * ig);
          const cplx se = cscale(e, s), sec = cscale(cconj(e), s);
          if constexpr (RPL > 0) {
#pragma unroll
            for (int it = 0; it < RPL; ++it) {
              const int i = g + GL * it;
              if (i < nb) {
                bp[i] = csub(cscale(xr[it], c), cmul(sec, yr[it]));
                bq[i] = cadd(cmul(se, xr[it]), cscale(yr[it], c));
              }
            }
          } else
          for (int i0 = g; i0 < nb; i0 += 16 * SG_CH) {
            cplx xs[SG_CH], ys[SG_CH];
#pragma unroll
            for (int u = 0; u < SG_CH; ++u) {
              const int i = i0 + 16 * u;
              xs[u] = i < nb ? bp[i] : make_double2(0.0, 0.0);
              ys[u] = i < nb ? bq[i] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < SG_CH; ++u) {
              const int i = i0 + 16 * u;
              if (i < nb) {
                bp[i] = csub(cscale(xs[u], c), cmul(sec, ys[u]));
                bq[i] = cadd(cmul(se, xs[u]), cscale(ys[u], c));
              }
            }
          }
          any_rot = 1;
          if (sweep + 1 == max_sweeps) {   // read only when the cap is reached
            worst2 = fmax(worst2, g2 * fast_rcp(al * be));
            small2 = fmin(small2, fmin(al, be));
          }
        }
      }
      __syncthreads();
    }
    converged = !__syncthreads_or(any_rot);
  }
  if (!converged) {   // block-uniform
    const double w2 = block_max(worst2, red), s2 = block_min(small2, red);
    if (tid == 0) flag_sweep_cap(status, nb, fro, w2, s2, jtol, sweeps_done);
  }
  if (tid == 0 && counters) {
    atomicAdd(counters + CNT_SVD_CALLS, 1ull);
    atomicAdd(counters + CNT_SVD_SWEEPS, (unsigned long long)sweeps_done);
  }
  for (int c = wv; c < nb; c += nw) {
    double a = 0.0;
    for (int i = lane; i < nb; i += 64) a += cabs2(Xw[(int64_t)c * nb + i]);
    a = wave_sum(a);
    if (lane == 0) sig[c] = sqrt(a);
  }
  __syncthreads();
  for (int c = tid; c < nb; c += blockDim.x) {
    const double v = sig[c];
    int pos = 0;
    for (int d = 0; d < nb; ++d) pos += (sig[d] > v) || (sig[d] == v && d < c);
    perm[pos] = c;
  }
  __syncthreads();
  if (tid == 0) {
    const int l = jacobi_truncate(sig, perm, nb, delta[b], lmax, disc2 + b, status, fro,
                                  sweeps_done, 2.0);
    sh_l = l;
    if (l_out) l_out[(int64_t)b * l_stride] = l;
  }
  __syncthreads();
  const int l = sh_l;
  if (svlog)
    for (int j = tid; j < nb; j += blockDim.x) svlog[b * svstride + j] = sig[perm[j]];
  jacobi_outputs(Xw, sig, perm, nb, l, negl, tall, core, Ul, hb, red, status);
}

// Sizes of the two finishing products per instance (ds ints each):
// [0..2] = (l, nc, nb) of core = U[:, :l]^H Q^H for A^H = Q R (zeros when
// tall); [3..5] = (m, l, nc) of carry = A core^H.
__global__ void k_fin_dims(int batch, Dim Md, Dim Cd, const int32_t* l_in, int l_stride,
                           int32_t* fd, int ds) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const int m = dimv(Md, b), nc = dimv(Cd, b), l = l_in[(int64_t)b * l_stride];
  const bool tall = m >= nc;
  int32_t* d = fd + (int64_t)b * ds;
  d[0] = tall ? 0 : l; d[1] = tall ? 0 : nc; d[2] = tall ? 0 : m;
  d[3] = m; d[4] = l; d[5] = nc;
}

// Wide instances (A^H = Q R): R^H (packed nb x nb) into X for the second QR,
// and its order in fd[6] (0 for tall instances, whose R is kept).
__global__ void k_qr2_prep(Dim Md, Dim Cd, const cplx* __restrict__ R, int64_t sR,
                           cplx* __restrict__ X, int64_t sX, int32_t* fd, int ds) {
  const int b = blockIdx.x;
  const int m = dimv(Md, b), nc = dimv(Cd, b);
  const bool wide = m < nc;
  if (threadIdx.x == 0) fd[(int64_t)b * ds + 6] = wide ? m : 0;
  if (!wide) return;
  R += b * sR; X += b * sX;
  for (int64_t e = threadIdx.x; e < (int64_t)m * m; e += blockDim.x) {
    const int64_t i = e / m, j = e % m;
    X[e] = cconj(R[j * m + i]);
  }
}

// Identity factors of an exact (untruncated) block: rank l = min(m, c); a
// wide instance gets U = I (l x l, row r = column r of U) in Uw, a tall one
// the core I (c x c, rows of V^H).
__global__ void k_orth_identity(Dim Md, Dim Cd, cplx* __restrict__ Uw, int64_t sU,
                                cplx* __restrict__ core, int64_t sCore, int32_t* l_out,
                                int l_stride) {
  const int b = blockIdx.x;
  const int m = dimv(Md, b), c = dimv(Cd, b);
  const bool tall = m >= c;
  const int l = tall ? c : m;
  cplx* dst = tall ? core + b * sCore : Uw + b * sU;
  for (int64_t e = threadIdx.x; e < (int64_t)l * l; e += blockDim.x)
    dst[e] = make_double2(e / l == e % l ? 1.0 : 0.0, 0.0);
  if (threadIdx.x == 0) l_out[(int64_t)b * l_stride] = l;
}

bool svd_trunc_fast(hipStream_t st, int batch, int mcap, int ccap, Dim m, Dim c, const cplx* A,
                    int64_t sA, cplx* Qw, cplx* Uw, int64_t sQ, cplx* Rw, cplx* Xw, int64_t sR,
                    double* tau, int64_t sT, const QrBlkWs* qb, cplx* core, int64_t sCore,
                    cplx* carry, int64_t sCarry, int32_t* l_out, int l_stride,
                    const double* delta, double* disc2, int lmax, int max_sweeps,
                    int32_t* status, double* svlog, int64_t svstride,
                    unsigned long long* counters, bool exact) {
  const int mbcap = std::max(mcap, ccap), nbcap = std::min(mcap, ccap);
  if (nbcap > SG_NB) return false;
  // blocks beyond one workgroup's LDS with >= 256 columns: panel + GEMM QRs
  // (work matrix in the QR scratch Uw)
  const bool blocked = qb && qr_blocked_wanted(mbcap, nbcap);
  if (blocked)
    qr_blocked(st, batch, mbcap, nbcap, m, c, A, sA, Uw, sQ, *qb, Qw, sQ, Rw, sR, nullptr, 0,
               true);
  else if (!qr_reg(st, batch, mbcap, nbcap, m, c, A, sA, Uw, sQ, tau, sT, Qw, sQ, Rw, sR,
                   nullptr, 0, true))
    qr_mem(st, batch, mbcap, nbcap, m, c, A, sA, Uw, sQ, tau, sT, Qw, sQ, Rw, sR, nullptr, 0, true);
  // per-instance sizes in the last 4 doubles of each tau slice (the QRs use
  // the first nb <= sT - 4)
  int32_t* fd = reinterpret_cast<int32_t*>(tau + sT - 4);
  const int ds = (int)(2 * sT);
  if (exact) {
    // no truncation: U = I for wide instances (core = Q^H of A^H = Q R,
    // carry = A Q = R^H), core = I for tall ones (carry = A), rank min(m, c)
    k_orth_identity<<<batch, 256, 0, st>>>(m, c, Uw, sQ, core, sCore, l_out, l_stride);
  } else {
  // wide instances: R2 of the second QR (R^H = Q2 R2) over R, Q2 not formed
  k_qr2_prep<<<batch, 256, 0, st>>>(m, c, Rw, sR, Xw, sR, fd, ds);
  const Dim d2 = dref(fd + 6, ds);
  if (blocked && qr_blocked_wanted(nbcap, nbcap))
    qr_blocked(st, batch, nbcap, nbcap, d2, d2, Xw, sR, Uw, sQ, *qb, nullptr, 0, Rw, sR, nullptr,
               0, false);
  else if (!qr_reg(st, batch, nbcap, nbcap, d2, d2, Xw, sR, Uw, sQ, tau, sT, nullptr, 0, Rw, sR,
                   nullptr, 0, false))
    qr_mem(st, batch, nbcap, nbcap, d2, d2, Xw, sR, Uw, sQ, tau, sT, nullptr, 0, Rw, sR, nullptr,
           0, false);
  // U[:, :l] of wide instances into the QR scratch Uw (free after the QRs)
  if (nbcap <= SL_NB)
    k_jacobi_lds<SL_NB><<<batch, 1024, 0, st>>>(m, c, Rw, sR, Uw, sQ, core, sCore, l_out,
                                                 l_stride, delta, disc2, lmax, max_sweeps, status,
                                                 svlog, svstride, counters);
  else if (nbcap <= SL_NB_BIG)
    k_jacobi_lds<SL_NB_BIG><<<batch, 1024, 0, st>>>(m, c, Rw, sR, Uw, sQ, core, sCore, l_out,
                                                     l_stride, delta, disc2, lmax, max_sweeps,
                                                     status, svlog, svstride, counters);
#define QT_JGLB(RPL, GL)                                                                     \
  k_jacobi_glb<RPL, GL><<<batch, 1024, 0, st>>>(m, c, Rw, sR, Xw, sR, Uw, sQ, core, sCore, l_out, \
                                                l_stride, delta, disc2, lmax, max_sweeps,     \
                                                status, svlog, svstride, counters)
  else if (nbcap <= 16 * 8)
    QT_JGLB(8, 16);
  else if (nbcap <= 16 * 9)
    QT_JGLB(9, 16);
  else if (nbcap <= 32 * SG_RPL)
    QT_JGLB(SG_RPL, 32);
  else
    QT_JGLB(0, 16);
#undef QT_JGLB
  }
  // finishing products on the MFMA GEMM (each instance's sizes are zero in the
  // product of the orientation it does not have):
  //   core  = U[:, :l]^H Q^H  (l x nc)  for A^H = Q R;
  //   carry = A core^H        (m x l)   for every instance
  k_fin_dims<<<(batch + 127) / 128, 128, 0, st>>>(batch, m, c, l_out, l_stride, fd, ds);
  const Str one{nullptr, 0, 0, 1};
  const Str s_nc{fd + 1, ds, 1, 0}, s_nb{fd + 2, ds, 1, 0};
  const Str s_l{fd + 4, ds, 1, 0}, s_k{fd + 5, ds, 1, 0};
  const cplx c1 = make_double2(1.0, 0.0);
  gemm_ex(st, batch, 1, 1, dref(fd + 0, ds), dref(fd + 1, ds), dref(fd + 2, ds), nbcap, mbcap,
          mat(Uw, sQ, s_nb, one), true, mat(Qw, sQ, one, s_nb), true,
          mat(core, sCore, s_nc, one), c1, false, Dim{nullptr, 0, 0, 1 << 30}, nbcap);
  gemm_ex(st, batch, 1, 1, dref(fd + 3, ds), dref(fd + 4, ds), dref(fd + 5, ds), mcap, nbcap,
          mat(A, sA, s_k, one), false, mat(core, sCore, one, s_k), true,
          mat(carry, sCarry, s_l, one), c1, false, Dim{nullptr, 0, 0, 1 << 30}, ccap);
  return true;
}

}  // namespace qt
