// Truncated SVD for the right-to-left sweep, small sizes (min(m, c) <= 100;
// R and V in LDS up to 68, R in LDS and V in global memory up to 100):
//   1. B = A (m >= c) or A^H (m < c); B = Q R by the register-resident QR;
//   2. one-sided (Hestenes) Jacobi on the columns of R^H (lower triangular),
//      which converge in fewer sweeps than R's (the rows of a triangular
//      factor are better separated than its columns; Drmac and Veselic,
//      SIAM J. Matrix Anal. Appl. 29, 2008): R^H W = U Sigma, so R = W Sigma U^H
//      (R^H and W in LDS, 16 waves, round-robin pairs, one barrier per round);
//   3. truncation (smallest l whose discarded tail <= delta, l <= lmax);
//   4. outputs: for A = Q R:   core = U^H[:l] = ((R^H W)[:, r] / sigma_r)^H,
//                              carry = Q W[:, :l] Sigma[:l];
//               for A^H = Q R: core = (Q W[:, r])^H,  carry = (R^H W)[:, :l].
// Rotation: gamma = b_p^H b_q = |gamma| e^{i phi}, zeta = (beta - alpha)/(2|gamma|),
// t = sign(zeta)/(|zeta| + sqrt(1 + zeta^2)), c = 1/sqrt(1 + t^2), s = c t,
// [b_p, b_q] <- [b_p, b_q] [[c, s e^{i phi}], [-s e^{-i phi}, c]].
#include "kernels.h"

namespace qt {

constexpr int SL_NB = 68;            // LDS holds two SL_NB x SL_NB complex matrices
constexpr int SL_NB_BIG = 100;       // LDS holds R only (160000 bytes), V in global memory
constexpr double SL_EPS = 2.0 * 2.220446049250313e-16;
constexpr double SL_NEGL = 1e-34;

// Flags a non-finite output of the truncated SVD (stage 5 + 2 * out + tall:
// out 0 core, 1 carry) with the order, kept rank and extreme kept sigmas.
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

// NBMAX: largest order; VG: V kept in global memory (Vg + b * sV, nb x nb);
// the large variant re-reads R from LDS for the rotation to stay within the
// register budget of 1024 threads.
template <int NBMAX, bool VG>
__global__ __launch_bounds__(1024) void k_jacobi_lds(
    Dim Md, Dim Cd, const cplx* __restrict__ Rin, int64_t sR, cplx* __restrict__ RVp, int64_t sRV,
    double* __restrict__ sigp, int64_t sSig, cplx* __restrict__ core, int64_t sCore,
    cplx* __restrict__ carry, int64_t sCarry, int32_t* l_out, int l_stride,
    const double* __restrict__ delta, double* __restrict__ disc2, int lmax, int max_sweeps,
    int32_t* status, double* svlog, int64_t svstride, unsigned long long* counters,
    cplx* __restrict__ Vg, int64_t sV) {
  __shared__ cplx Rs[NBMAX * NBMAX];
  __shared__ cplx Vl[VG ? 1 : NBMAX * NBMAX];
  __shared__ double sig[NBMAX];
  __shared__ int perm[NBMAX];
  __shared__ double red[16];
  __shared__ int sh_rot, sh_l;
  __shared__ unsigned long long sh_worst, sh_small;   // bit patterns of positive doubles
  const int b = blockIdx.x;
  const int m = dimv(Md, b), nc = dimv(Cd, b);
  const bool tall = m >= nc;
  const int nb = tall ? nc : m;
  Rin += b * sR; RVp += b * sRV; sigp += b * sSig; core += b * sCore; carry += b * sCarry;
  cplx* Vs = VG ? Vg + b * sV : Vl;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
  for (int e = tid; e < nb * nb; e += blockDim.x) {
    const int i = e / nb, c = e % nb;       // R row-major (nb x nb)
    Rs[e] = cconj(Rin[e]);                  // column c of R^H = conj(row c of R)
    Vs[c * nb + i] = make_double2(i == c ? 1.0 : 0.0, 0.0);
  }
  double fro = 0.0;
  for (int e = tid; e < nb * nb; e += blockDim.x) fro += cabs2(Rin[e]);
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
  for (int sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
    ++sweeps_done;
    if (tid == 0) {
      sh_rot = 0;
      sh_worst = 0ull;
      sh_small = (unsigned long long)__double_as_longlong(1.0);
    }
    __syncthreads();
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
        // the rotation (at most NBMAX / 16 rounded up rows per lane)
        constexpr int RPL = (NBMAX + 15) / 16;
        cplx xs[RPL], ys[RPL];
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
          if (!VG) {
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
              // the large variant re-reads R from LDS (registers hold V)
              const cplx x = VG ? bp[i] : xs[it], y = VG ? bq[i] : ys[it];
              bp[i] = csub(cscale(x, c), cmul(sec, y));
              bq[i] = cadd(cmul(se, x), cscale(y, c));
            }
          }
          cplx* vp = Vs + p * nb;
          cplx* vq = Vs + q * nb;
#pragma unroll
          for (int it = 0; it < RPL; ++it) {     // all loads first, then the updates
            const int i = g + 16 * it;
            xs[it] = i < nb ? vp[i] : make_double2(0.0, 0.0);
            ys[it] = i < nb ? vq[i] : make_double2(0.0, 0.0);
          }
#pragma unroll
          for (int it = 0; it < RPL; ++it) {
            const int i = g + 16 * it;
            if (i < nb) {
              vp[i] = csub(cscale(xs[it], c), cmul(sec, ys[it]));
              vq[i] = cadd(cmul(se, xs[it]), cscale(ys[it], c));
            }
          }
          if (g == 0) {
            sh_rot = 1;
            atomicMax(&sh_worst, (unsigned long long)__double_as_longlong(
                                     sqrt(g2 / (al * be)) / jtol));
            atomicMin(&sh_small, (unsigned long long)__double_as_longlong(fmin(al, be) / fro));
          }
        }
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
      d[1] = fro;
      d[2] = __longlong_as_double((long long)sh_worst);
      d[3] = __longlong_as_double((long long)sh_small);
      d[4] = sweeps_done;
    }
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
    const double dl = delta[b];
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
        d[3] = 1.0;   // LDS Jacobi
        d[4] = sweeps_done;
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
  // W[:, perm[:l]] column-major and sorted sigma for the finalizer
  for (int e = tid; e < l * nb; e += blockDim.x) {
    const int r = e / nb, i = e % nb;
    RVp[e] = Vs[perm[r] * nb + i];
  }
  for (int r = tid; r < l; r += blockDim.x) sigp[r] = sig[perm[r]];
  bool fin = true;
  if (tall) {
    // core = U^H[:l]  (l x nc), nc = nb; U[:, r] = (R^H W)[:, r] / sigma_r
    for (int e = tid; e < l * nb; e += blockDim.x) {
      const int r = e / nb, c = e % nb;
      const double sv = sig[perm[r]];
      const cplx v = sv > 0.0 ? cscale(cconj(Rs[perm[r] * nb + c]), 1.0 / sv)
                              : make_double2(c == r ? 1.0 : 0.0, 0.0);
      fin = fin && isfinite(v.x) && isfinite(v.y);
      core[e] = v;
    }
  } else {
    // carry = (R^H W)[:, perm[:l]] = U Sigma  (m x l), m = nb
    for (int e = tid; e < nb * l; e += blockDim.x) {
      const int i = e / l, r = e % l;
      const cplx v = Rs[perm[r] * nb + i];
      fin = fin && isfinite(v.x) && isfinite(v.y);
      carry[e] = v;
    }
  }
  for (int e = tid; e < l * nb; e += blockDim.x) {
    const cplx v = RVp[e];
    fin = fin && isfinite(v.x) && isfinite(v.y);
  }
  if (!fin) flag_out(status, tall ? 6 : 8, nb, l, sig[perm[0]], sig[perm[l - 1]]);
}


// Global-memory variant for orders 100 < nb <= 1024 (same algorithm, schedule
// and thresholds): R^H in the work matrix Rt, W in Vw (both column-major,
// nb x nb per instance); each 16-lane group streams its pair's columns in
// chunks of SG_CH rows per lane (all loads of a chunk issued before use).
// Rio: R (row-major) on entry, W[:, perm[:l]] (column-major) on exit.
constexpr int SG_NB = 1024;
constexpr int SG_CH = 6;

__global__ __launch_bounds__(1024) void k_jacobi_glb(
    Dim Md, Dim Cd, cplx* Rio, int64_t sR, cplx* __restrict__ Rt, int64_t sRt,
    cplx* __restrict__ Vw, int64_t sV, double* __restrict__ sigp, int64_t sSig,
    cplx* __restrict__ core, int64_t sCore, cplx* __restrict__ carry, int64_t sCarry,
    int32_t* l_out, int l_stride, const double* __restrict__ delta, double* __restrict__ disc2,
    int lmax, int max_sweeps, int32_t* status, double* svlog, int64_t svstride,
    unsigned long long* counters) {
  __shared__ double sig[SG_NB];
  __shared__ int perm[SG_NB];
  __shared__ double red[16];
  __shared__ int sh_rot, sh_l;
  __shared__ unsigned long long sh_worst, sh_small;
  const int b = blockIdx.x;
  const int m = dimv(Md, b), nc = dimv(Cd, b);
  const bool tall = m >= nc;
  const int nb = tall ? nc : m;
  Rio += b * sR; Rt += b * sRt; Vw += b * sV; sigp += b * sSig; core += b * sCore;
  carry += b * sCarry;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
  const int64_t nn = (int64_t)nb * nb;
  double fro = 0.0;
  for (int64_t e = tid; e < nn; e += blockDim.x) {
    const cplx v = Rio[e];
    fro += cabs2(v);
    Rt[e] = cconj(v);                       // column c of R^H = conj(row c of R)
    Vw[e] = make_double2((e / nb) == (e % nb) ? 1.0 : 0.0, 0.0);
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
  const int g = tid & 15, grp = tid >> 4, ngrp = blockDim.x >> 4;
  bool converged = nb < 2;
  int sweeps_done = 0;
  for (int sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
    ++sweeps_done;
    if (tid == 0) {
      sh_rot = 0;
      sh_worst = 0ull;
      sh_small = (unsigned long long)__double_as_longlong(1.0);
    }
    __syncthreads();
    for (int r = 0; r < nbp - 1; ++r) {
      for (int pi0 = 0; pi0 < nbp / 2; pi0 += ngrp) {
        if (pi0 + 4 * wv >= nbp / 2) continue;   // wave-uniform: no pair for this wave
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
        cplx* bp = Rt + (int64_t)p * nb;
        cplx* bq = Rt + (int64_t)q * nb;
        double al = 0.0, be = 0.0;
        cplx ga = make_double2(0.0, 0.0);
        if (valid) {
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
        al = row16_sum(al); be = row16_sum(be); ga = row16_sum(ga);
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
#pragma unroll 1
          for (int half = 0; half < 2; ++half) {   // R^H columns, then W columns
            cplx* cp = half == 0 ? bp : Vw + (int64_t)p * nb;
            cplx* cq = half == 0 ? bq : Vw + (int64_t)q * nb;
            for (int i0 = g; i0 < nb; i0 += 16 * SG_CH) {
              cplx xs[SG_CH], ys[SG_CH];
#pragma unroll
              for (int u = 0; u < SG_CH; ++u) {
                const int i = i0 + 16 * u;
                xs[u] = i < nb ? cp[i] : make_double2(0.0, 0.0);
                ys[u] = i < nb ? cq[i] : make_double2(0.0, 0.0);
              }
#pragma unroll
              for (int u = 0; u < SG_CH; ++u) {
                const int i = i0 + 16 * u;
                if (i < nb) {
                  cp[i] = csub(cscale(xs[u], c), cmul(sec, ys[u]));
                  cq[i] = cadd(cmul(se, xs[u]), cscale(ys[u], c));
                }
              }
            }
          }
          if (g == 0) {
            sh_rot = 1;
            atomicMax(&sh_worst, (unsigned long long)__double_as_longlong(
                                     sqrt(g2 / (al * be)) / jtol));
            atomicMin(&sh_small, (unsigned long long)__double_as_longlong(fmin(al, be) / fro));
          }
        }
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
      d[1] = fro;
      d[2] = __longlong_as_double((long long)sh_worst);
      d[3] = __longlong_as_double((long long)sh_small);
      d[4] = sweeps_done;
    }
  }
  if (tid == 0 && counters) {
    atomicAdd(counters + CNT_SVD_CALLS, 1ull);
    atomicAdd(counters + CNT_SVD_SWEEPS, (unsigned long long)sweeps_done);
  }
  for (int c = wv; c < nb; c += nw) {
    double a = 0.0;
    for (int i = lane; i < nb; i += 64) a += cabs2(Rt[(int64_t)c * nb + i]);
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
    const double dl = delta[b];
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
    if (!finite) flag_out(status, 2, nb, l, fro, -1.0);
    disc2[b] += d2;
    sh_l = l;
    if (l_out) l_out[(int64_t)b * l_stride] = l;
  }
  __syncthreads();
  const int l = sh_l;
  if (svlog)
    for (int j = tid; j < nb; j += blockDim.x) svlog[b * svstride + j] = sig[perm[j]];
  for (int r = tid; r < l; r += blockDim.x) sigp[r] = sig[perm[r]];
  bool fin = true;
  if (tall) {
    for (int64_t e = tid; e < (int64_t)l * nb; e += blockDim.x) {
      const int r = (int)(e / nb), c = (int)(e % nb);
      const double sv = sig[perm[r]];
      const cplx v = sv > 0.0 ? cscale(cconj(Rt[(int64_t)perm[r] * nb + c]), 1.0 / sv)
                              : make_double2(c == r ? 1.0 : 0.0, 0.0);
      fin = fin && isfinite(v.x) && isfinite(v.y);
      core[e] = v;
    }
  } else {
    for (int64_t e = tid; e < (int64_t)nb * l; e += blockDim.x) {
      const int i = (int)(e / l), r = (int)(e % l);
      const cplx v = Rt[(int64_t)perm[r] * nb + i];
      fin = fin && isfinite(v.x) && isfinite(v.y);
      carry[e] = v;
    }
  }
  // W[:, perm[:l]] over R (consumed at entry) for the finishing products,
  // scaled by sigma for the carry Q W Sigma (A = Q R)
  for (int64_t e = tid; e < (int64_t)l * nb; e += blockDim.x) {
    const int r = (int)(e / nb), i = (int)(e % nb);
    const cplx w = Vw[(int64_t)perm[r] * nb + i];
    const cplx v = tall ? cscale(w, sig[perm[r]]) : w;
    fin = fin && isfinite(v.x) && isfinite(v.y);
    Rio[e] = v;
  }
  if (!fin) flag_out(status, tall ? 6 : 8, nb, l, sig[perm[0]], sig[perm[l - 1]]);
}

// Sizes of the two finishing products of the global-memory variant:
// [0..2] = (m, l, nb) for A = Q R (tall), [3..5] = (l, nc, nb) for A^H = Q R;
// zeros for the orientation an instance does not have.
__global__ void k_fin_dims(int batch, Dim Md, Dim Cd, const int32_t* l_in, int l_stride,
                           int32_t* fd, int ds) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const int m = dimv(Md, b), nc = dimv(Cd, b), l = l_in[(int64_t)b * l_stride];
  const bool tall = m >= nc;
  int32_t* d = fd + (int64_t)b * ds;
  d[0] = tall ? m : 0; d[1] = tall ? l : 0; d[2] = tall ? nc : 0;
  d[3] = tall ? 0 : l; d[4] = tall ? 0 : nc; d[5] = tall ? 0 : m;
}

// Applies Q (mb x nb, row-major) to the kept columns of W: the carry
// Q W Sigma (A = Q R) or the core rows (Q W)^H (A^H = Q R).
__global__ __launch_bounds__(1024) void k_svd_finalize(Dim Md, Dim Cd, const cplx* __restrict__ Q,
                                                       int64_t sQ, const cplx* __restrict__ RVp,
                                                       int64_t sRV, const double* __restrict__ sigp,
                                                       int64_t sSig, const int32_t* l_in,
                                                       int l_stride, cplx* __restrict__ core,
                                                       int64_t sCore, cplx* __restrict__ carry,
                                                       int64_t sCarry, int32_t* status) {
  const int b = blockIdx.x;
  const int m = dimv(Md, b), nc = dimv(Cd, b);
  const bool tall = m >= nc;
  const int mb = tall ? m : nc, nb = tall ? nc : m;
  const int l = l_in[(int64_t)b * l_stride];
  Q += b * sQ; RVp += b * sRV; sigp += b * sSig; core += b * sCore; carry += b * sCarry;
  for (int e = threadIdx.x; e < mb * l; e += blockDim.x) {
    const int i = e / l, r = e % l;
    cplx acc = make_double2(0.0, 0.0);
    const cplx* qi = Q + (int64_t)i * nb;
    const cplx* rv = RVp + (int64_t)r * nb;
    for (int c = 0; c < nb; ++c) cfma(acc, qi[c], rv[c]);
    if (tall) {
      const cplx v = cscale(acc, sigp[r]);
      if (!(isfinite(v.x) && isfinite(v.y))) flag_out(status, 9, nb, l, sigp[0], sigp[l - 1]);
      carry[(int64_t)i * l + r] = v;                       // carry (m x l)
    } else {
      const cplx v = cconj(acc);
      if (!(isfinite(v.x) && isfinite(v.y))) flag_out(status, 7, nb, l, sigp[0], sigp[l - 1]);
      core[(int64_t)r * nc + i] = v;                       // core (l x nc), row r
    }
  }
}

bool svd_trunc_fast(hipStream_t st, int batch, int mcap, int ccap, Dim m, Dim c, const cplx* A,
                    int64_t sA, cplx* Qw, cplx* Uw, int64_t sQ, cplx* Rw, cplx* RVw, int64_t sR,
                    double* tau, double* sig, int64_t sT, cplx* core, int64_t sCore, cplx* carry,
                    int64_t sCarry, int32_t* l_out, int l_stride, const double* delta,
                    double* disc2, int lmax, int max_sweeps, int32_t* status, double* svlog,
                    int64_t svstride, unsigned long long* counters) {
  const int mbcap = std::max(mcap, ccap), nbcap = std::min(mcap, ccap);
  if (nbcap > SG_NB) return false;
  if (!qr_reg(st, batch, mbcap, nbcap, m, c, A, sA, Uw, sQ, tau, sT, Qw, sQ, Rw, sR, nullptr, 0,
              true))
    qr_mem(st, batch, mbcap, nbcap, m, c, A, sA, Uw, sQ, tau, sT, Qw, sQ, Rw, sR, nullptr, 0, true);
  if (nbcap > SL_NB_BIG) {
    // R^H in RVw, W in the QR scratch Uw (free after the QR), W[:, perm] back over R
    k_jacobi_glb<<<batch, 1024, 0, st>>>(m, c, Rw, sR, RVw, sR, Uw, sQ, sig, sT, core, sCore,
                                         carry, sCarry, l_out, l_stride, delta, disc2, lmax,
                                         max_sweeps, status, svlog, svstride, counters);
    // finishing products on the MFMA GEMM: carry = Q (W Sigma) for A = Q R,
    // core = W^H Q^H for A^H = Q R; each instance's sizes are zero in the
    // product of the other orientation
    int32_t* fd = reinterpret_cast<int32_t*>(tau);
    const int ds = (int)(2 * sT);
    k_fin_dims<<<(batch + 127) / 128, 128, 0, st>>>(batch, m, c, l_out, l_stride, fd, ds);
    const Dim tM = dref(fd + 0, ds), tN = dref(fd + 1, ds), tK = dref(fd + 2, ds);
    const Dim wM = dref(fd + 3, ds), wN = dref(fd + 4, ds), wK = dref(fd + 5, ds);
    const Str snb{fd + 2, ds, 1, 0}, sl{fd + 1, ds, 1, 0};
    const Str wnb{fd + 5, ds, 1, 0}, wnc{fd + 4, ds, 1, 0};
    const Str one{nullptr, 0, 0, 1};
    const cplx c1 = make_double2(1.0, 0.0);
    gemm_ex(st, batch, 1, 1, tM, tN, tK, mbcap, nbcap, mat(Qw, sQ, snb, one), false,
            mat(Rw, sR, one, snb), false, mat(carry, sCarry, sl, one), c1, false,
            Dim{nullptr, 0, 0, 1 << 30}, nbcap);
    gemm_ex(st, batch, 1, 1, wM, wN, wK, nbcap, mbcap, mat(Rw, sR, wnb, one), true,
            mat(Qw, sQ, one, wnb), true, mat(core, sCore, wnc, one), c1, false,
            Dim{nullptr, 0, 0, 1 << 30}, nbcap);
    return true;
  }
  if (nbcap <= SL_NB)
    k_jacobi_lds<SL_NB, false><<<batch, 1024, 0, st>>>(
        m, c, Rw, sR, RVw, sR, sig, sT, core, sCore, carry, sCarry, l_out, l_stride, delta, disc2,
        lmax, max_sweeps, status, svlog, svstride, counters, nullptr, 0);
  else   // V in the QR scratch Uw (mbcap x nbcap >= nb x nb per instance), free after the QR
    k_jacobi_lds<SL_NB_BIG, true><<<batch, 1024, 0, st>>>(
        m, c, Rw, sR, RVw, sR, sig, sT, core, sCore, carry, sCarry, l_out, l_stride, delta, disc2,
        lmax, max_sweeps, status, svlog, svstride, counters, Uw, sQ);
  k_svd_finalize<<<batch, 1024, 0, st>>>(m, c, Qw, sQ, RVw, sR, sig, sT, l_out, l_stride, core,
                                         sCore, carry, sCarry, status);
  return true;
}

}  // namespace qt
