// Blocked Householder QR (compact WY form) for unfoldings too large for one
// workgroup's LDS: the left orthogonalization sweep of the rounding (Sec. 2.2)
// at large ranks.
//
// A (m x n, row-major) is copied to a column-major work matrix M (leading
// dimension mcap).  For each panel of QB_NB columns starting at j0:
//   - one workgroup per instance factors the panel with Householder
//     reflectors H_j = I - t_j u_j u_j^H (u_j[j] = 1, t_j real), writes the
//     reflectors explicitly to V and builds the upper-triangular T with
//     H_j0 ... H_j0+NB-1 = I - V T V^H (T[:, i] = -t_i T V^H u_i, T[i][i] = t_i);
//   - the trailing columns are updated by three structured products on the
//     MFMA GEMM: W1 = V^H A, W2 = T^H W1, A -= V W2.
// Q (m x s) is then formed backward from [I; 0] with the same three products
// per panel (W1 = V^H Q, W2 = T W1, Q -= V W2), and R (s x n) is the upper
// triangle of M.  All sizes are device values (ranks); the launch sequence is
// fixed by the host capacities, and panels past s = min(m, n) exit at once.
#include "kernels.h"

namespace qt {

constexpr int QB_NB = 32;     // panel width
constexpr int QB_T = 512;     // threads of the panel workgroup (QB_T / 16 == QB_NB)
constexpr int QB_TILE = 32;   // transpose tile

// Sum over the workgroup; every thread returns the same value (the per-wave
// sums are added in a fixed order).
__device__ inline double qb_block_sum(double v, double* sh) {
  v = wave_sum(v);
  __syncthreads();   // sh may still be read from the previous call
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < QB_T / 64; ++i) s += sh[i];
  return s;
}

// M (column-major, ld) <- A (row-major m x n); s_dev[b] = min(m, n).
// trans (may be null; stride 3 per instance): factor B = A^H for that
// instance, whose column c is row c of A, conjugated.
__global__ __launch_bounds__(256) void k_qrb_load(int tiles_r, int tiles_c, Dim Md, Dim Nd,
                                                  const int32_t* trans,
                                                  const cplx* __restrict__ A, int64_t sA,
                                                  cplx* __restrict__ M, int64_t sM, int ld,
                                                  int32_t* s_dev) {
  const int per = tiles_r * tiles_c;
  const int b = blockIdx.x / per, t = blockIdx.x % per;
  const int m = dimv(Md, b), n = dimv(Nd, b);
  if (t == 0 && threadIdx.x == 0) s_dev[b] = min(m, n);
  const int r0 = (t / tiles_c) * QB_TILE, c0 = (t % tiles_c) * QB_TILE;
  A += b * sA;
  M += b * sM;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  if (trans && trans[(int64_t)b * 3 + 2]) {   // B (n x m) = A^H, no transpose through LDS
    if (r0 >= n || c0 >= m) return;
    for (int c = ty; c < QB_TILE; c += 8) {
      const int cc = c0 + c, i = r0 + tx;
      if (cc < m && i < n) M[(int64_t)cc * ld + i] = cconj(A[(int64_t)cc * n + i]);
    }
    return;
  }
  if (r0 >= m || c0 >= n) return;
  __shared__ cplx tile[QB_TILE][QB_TILE + 1];
  for (int r = ty; r < QB_TILE; r += 8) {
    const int i = r0 + r, c = c0 + tx;
    tile[r][tx] = (i < m && c < n) ? A[(int64_t)i * n + c] : czero();
  }
  __syncthreads();
  for (int c = ty; c < QB_TILE; c += 8) {
    const int i = r0 + tx, cc = c0 + c;
    if (i < m && cc < n) M[(int64_t)cc * ld + i] = tile[tx][c];
  }
}

// R (row-major s x n) <- upper triangle of M.
__global__ __launch_bounds__(256) void k_qrb_rout(int tiles_r, int tiles_c, Dim Md, Dim Nd,
                                                  const cplx* __restrict__ M, int64_t sM, int ld,
                                                  cplx* __restrict__ R, int64_t sR) {
  const int per = tiles_r * tiles_c;
  const int b = blockIdx.x / per, t = blockIdx.x % per;
  const int m = dimv(Md, b), n = dimv(Nd, b), s = min(m, n);
  const int r0 = (t / tiles_c) * QB_TILE, c0 = (t % tiles_c) * QB_TILE;
  if (r0 >= s || c0 >= n) return;
  __shared__ cplx tile[QB_TILE][QB_TILE + 1];
  M += b * sM;
  R += b * sR;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int c = ty; c < QB_TILE; c += 8) {
    const int i = r0 + tx, cc = c0 + c;
    tile[c][tx] = (i < s && cc < n && cc >= i) ? M[(int64_t)cc * ld + i] : czero();
  }
  __syncthreads();
  for (int r = ty; r < QB_TILE; r += 8) {
    const int i = r0 + r, c = c0 + tx;
    if (i < s && c < n) R[(int64_t)i * n + c] = tile[tx][r];
  }
}

// M <- [I_s; 0] (m x s, column-major).
__global__ __launch_bounds__(256) void k_qrb_qinit(int per, int64_t cap_elems, Dim Md, Dim Nd,
                                                   cplx* __restrict__ M, int64_t sM, int ld) {
  const int b = blockIdx.x / per;
  const int m = dimv(Md, b), n = dimv(Nd, b), s = min(m, n);
  M += b * sM;
  for (int64_t e = (int64_t)(blockIdx.x % per) * 256 + threadIdx.x; e < cap_elems;
       e += (int64_t)per * 256) {
    const int c = (int)(e / ld), i = (int)(e % ld);
    if (c < s && i < m) M[e] = make_double2(i == c ? 1.0 : 0.0, 0.0);
  }
}

// Q (row-major m x s) <- M (column-major); s_out[b] = s.
__global__ __launch_bounds__(256) void k_qrb_qout(int tiles_r, int tiles_c, Dim Md, Dim Nd,
                                                  const cplx* __restrict__ M, int64_t sM, int ld,
                                                  cplx* __restrict__ Q, int64_t sQ,
                                                  int32_t* s_out, int s_stride) {
  const int per = tiles_r * tiles_c;
  const int b = blockIdx.x / per, t = blockIdx.x % per;
  const int m = dimv(Md, b), n = dimv(Nd, b), s = min(m, n);
  if (t == 0 && threadIdx.x == 0 && s_out) s_out[(int64_t)b * s_stride] = s;
  const int r0 = (t / tiles_c) * QB_TILE, c0 = (t % tiles_c) * QB_TILE;
  if (r0 >= m || c0 >= s) return;
  __shared__ cplx tile[QB_TILE][QB_TILE + 1];
  M += b * sM;
  Q += b * sQ;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int c = ty; c < QB_TILE; c += 8) {
    const int i = r0 + tx, cc = c0 + c;
    tile[c][tx] = (i < m && cc < s) ? M[(int64_t)cc * ld + i] : czero();
  }
  __syncthreads();
  for (int r = ty; r < QB_TILE; r += 8) {
    const int i = r0 + r, c = c0 + tx;
    if (i < m && c < s) Q[(int64_t)i * s + c] = tile[tx][r];
  }
}

__global__ void k_qrb_sout(int batch, const int32_t* __restrict__ s_dev, int32_t* s_out,
                           int s_stride) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < batch) s_out[(int64_t)b * s_stride] = s_dev[b];
}

// Factor panel [j0, j0 + nbw) of M (rows j0..m-1), apply its reflectors to the
// other panel columns below n, write V's panel columns (zero above the
// diagonal, one on it; columns past nbw zero) and the panel's T (row-major
// QB_NB x QB_NB).  Thread t owns rows j0 + t + QB_T q for the whole panel, so
// its own updates need no barrier before it reads them again.
__global__ __launch_bounds__(QB_T) void k_qrb_panel(int j0, Dim Md, Dim Nd, cplx* __restrict__ M,
                                                    int64_t sM, int ld, cplx* __restrict__ V,
                                                    int64_t sV, double* __restrict__ tau,
                                                    int64_t sTau, cplx* __restrict__ T,
                                                    int64_t sT) {
  const int b = blockIdx.x;
  const int m = dimv(Md, b), n = dimv(Nd, b), s = min(m, n);
  if (j0 >= s) return;
  const int nbw = min(QB_NB, s - j0), pend = min(j0 + QB_NB, n);
  M += b * sM;
  V += b * sV;
  tau += b * sTau;
  T += b * sT + (int64_t)(j0 / QB_NB) * QB_NB * QB_NB;
  __shared__ cplx Ts[QB_NB][QB_NB];
  __shared__ cplx part[QB_NB][QB_T / 16];
  __shared__ cplx red[QB_NB];
  __shared__ double sh[QB_T / 64];
  __shared__ cplx alsh;
  const int tid = threadIdx.x;
  for (int e = tid; e < QB_NB * QB_NB; e += QB_T) Ts[e / QB_NB][e % QB_NB] = czero();
  for (int k = nbw; k < QB_NB; ++k)
    for (int i = j0 + tid; i < m; i += QB_T) V[(int64_t)(j0 + k) * ld + i] = czero();

  for (int jj = 0; jj < nbw; ++jj) {
    const int j = j0 + jj;
    cplx* colj = M + (int64_t)j * ld;
    double sig = 0.0;
    for (int i = j0 + tid; i < m; i += QB_T) {
      const cplx v = colj[i];
      if (i > j) sig += cabs2(v);
      else if (i == j) alsh = v;
    }
    sig = qb_block_sum(sig, sh);   // its barriers also publish alsh
    const cplx al = alsh;
    // reflector: beta = -e^{i arg(al)} ||x||, u = x / (al - beta), t = 1 + |al| / ||x||
    const double a2 = cabs2(al), x2 = a2 + sig;
    double t;
    cplx beta, iu0;
    if (x2 == 0.0) {
      t = 0.0; beta = al; iu0 = czero();
    } else {
      const double xn = sqrt(x2);
      const double aa = sqrt(a2);
      const cplx ph = a2 > 0.0 ? make_double2(al.x / aa, al.y / aa) : make_double2(1.0, 0.0);
      beta = make_double2(-ph.x * xn, -ph.y * xn);
      const cplx u0 = csub(al, beta);
      // 1 / u0 with u0 scaled by its larger component first (|u0|^2 can
      // leave the double range for numerically vanishing columns)
      const double sc = fmax(fabs(u0.x), fabs(u0.y));
      const cplx v = make_double2(u0.x / sc, u0.y / sc);
      const double d = cabs2(v) * sc;
      iu0 = make_double2(v.x / d, -v.y / d);
      t = 1.0 + aa / xn;
    }
    cplx* vj = V + (int64_t)j * ld;
    // acc[k]: u^H a_k (slot k > jj, dot for the update) or v_k^H u (k < jj, for
    // T); two passes of QB_NB / 2 slots each keep the accumulators in registers
    const int l16 = tid & 15, rg = tid >> 4;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      constexpr int HS = QB_NB / 2;
      cplx acc[HS];
#pragma unroll
      for (int k = 0; k < HS; ++k) acc[k] = czero();
      for (int i = j0 + tid; i < m; i += QB_T) {
        cplx u;
        if (h == 0) {
          if (i < j) u = czero();
          else if (i == j) u = make_double2(1.0, 0.0);
          else u = cmul(colj[i], iu0);
          vj[i] = u;
          if (i == j) colj[i] = beta;
        } else {
          u = vj[i];
        }
        if (i < j) continue;
#pragma unroll
        for (int kk = 0; kk < HS; ++kk) {
          const int k = h * HS + kk;
          if (k > jj) {
            if (j0 + k < pend) cfma(acc[kk], cconj(u), M[(int64_t)(j0 + k) * ld + i]);
          } else if (k < jj) {
            cfma(acc[kk], cconj(V[(int64_t)(j0 + k) * ld + i]), u);
          }
        }
      }
#pragma unroll
      for (int kk = 0; kk < HS; ++kk) {
        const cplx v = row16_sum(acc[kk]);
        if (l16 == 0) part[h * HS + kk][rg] = v;
      }
    }
    __syncthreads();
    {
      // QB_NB slots x 16 lanes; each lane adds two of the slot's QB_T / 16 partials
      const int k = tid >> 4, l = tid & 15;
      cplx v = cadd(part[k][2 * l], part[k][2 * l + 1]);
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) {
        v.x += __shfl_xor(v.x, off, 64);
        v.y += __shfl_xor(v.y, off, 64);
      }
      if (l == 0) red[k] = v;   // one lane's sum is the value every thread uses
    }
    __syncthreads();
    // T column jj: T[a][jj] = -t sum_{c=a}^{jj-1} T[a][c] z_c, T[jj][jj] = t
    if (tid < jj) {
      cplx sacc = czero();
      for (int c = tid; c < jj; ++c) cfma(sacc, Ts[tid][c], red[c]);
      Ts[tid][jj] = cscale(sacc, -t);
    } else if (tid == jj) {
      Ts[jj][jj] = make_double2(t, 0.0);
      tau[j] = t;
    }
    // apply H_j to the later panel columns (own rows)
    if (t != 0.0) {
      for (int i = j0 + tid; i < m; i += QB_T) {
        if (i < j) continue;
        const cplx tu = cscale(vj[i], t);
        for (int k = jj + 1; k < QB_NB; ++k) {
          if (j0 + k >= pend) break;
          cplx* a = M + (int64_t)(j0 + k) * ld + i;
          *a = csub(*a, cmul(tu, red[k]));
        }
      }
    }
    // the next step's reductions rewrite part/red only after its first barrier
  }
  __syncthreads();
  for (int e = tid; e < QB_NB * QB_NB; e += QB_T) T[e] = Ts[e / QB_NB][e % QB_NB];
}

// Sum over a group of GL = 8, 16 or 32 consecutive lanes; every lane of the
// group gets the same bits (each step adds two values that the partner lane
// adds in the other order): quad_perm [1,0,3,2], [2,3,0,1], then
// row_half_mirror (lanes i and 7 - i of each 8-lane half), then for 16 lanes
// row_mirror, then for 32 lanes a swap of the two 16-lane halves.
template <int GL>
__device__ inline double grp_sum(double v) {
  static_assert(GL == 8 || GL == 16 || GL == 32, "group of 8, 16 or 32 lanes");
  if (GL == 16) return row16_sum(v);
  if (GL == 32) {   // the two 16-lane halves add each other's sums (commutes)
    v = row16_sum(v);
    return v + __shfl_xor(v, 16, 64);
  }
#define QP_DPP_STEP(ctrl)                                                           \
  {                                                                                 \
    int lo = __double2loint(v), hi = __double2hiint(v);                             \
    int l2 = __builtin_amdgcn_update_dpp(0, lo, ctrl, 0xF, 0xF, false);             \
    int h2 = __builtin_amdgcn_update_dpp(0, hi, ctrl, 0xF, 0xF, false);             \
    v += __hiloint2double(h2, l2);                                                  \
  }
  QP_DPP_STEP(0xB1)
  QP_DPP_STEP(0x4E)
  QP_DPP_STEP(0x141)
#undef QP_DPP_STEP
  return v;
}
template <int GL>
__device__ inline cplx grp_sum(cplx v) {
  v.x = grp_sum<GL>(v.x);
  v.y = grp_sum<GL>(v.y);
  return v;
}

// Register-resident panel factorization: NB = NT / GL columns
// [j0, j0 + NB) of M (rows j0..m-1, m - j0 <= GL RPL).  Group c of GL lanes
// holds panel column c, lane l its rows j0 + l + GL r, for the whole panel.
// Step jj: the owner of column jj forms its reflector (the same Householder
// coefficients as the one-workgroup QRs), keeps beta and the reflector below
// the diagonal in its registers and publishes the reflector in LDS; after
// one barrier every later column applies it (group sums), and every earlier
// column c forms z_c = u_c^H u_jj, from which the next step builds T's
// column jj: T[a][jj] = -t_jj sum_{c=a}^{jj-1} T[a][c] z_c, T[jj][jj] = t_jj.
// One barrier per column; reflector and z buffers alternate between steps.
// Writes the panel back (R on and above the diagonal), V (explicit, zero
// above the diagonal, one on it, zero columns past the last reflector) and T.
constexpr int QP_CH = 6;

// Column q of the panel's T: T[a][q] = -t_q sum_{c=a}^{q-1} T[a][c] z_c for
// a < q, T[q][q] = t_q.  Eight consecutive threads share a row a (strided
// partial sums, then an 8-lane sum), so the step's critical path holds about
// q / 8 LDS reads instead of q.  Rows a <= q need 8 (q + 1) <= NT threads.
template <int NT, int NB>
__device__ inline void qp_t_column(int q, int tid, cplx (*Ts)[NB], const cplx* z,
                                   const double* tl) {
  const int a = tid >> 3, l8 = tid & 7;
  if (a > q) return;          // whole 8-lane groups leave together
  cplx acc = czero();
  for (int c = a + l8; c < q; c += 8) cfma(acc, Ts[a][c], z[c]);
  acc.x = grp_sum<8>(acc.x);
  acc.y = grp_sum<8>(acc.y);
  if (l8 == 0) Ts[a][q] = (a == q) ? make_double2(tl[q], 0.0) : cscale(acc, -tl[q]);
}

template <int NT, int GL, int RPL>
__global__ __launch_bounds__(NT) void k_qrp_panel(int j0, Dim Md, Dim Nd, cplx* __restrict__ M,
                                                    int64_t sM, int ld, cplx* __restrict__ V,
                                                    int64_t sV, double* __restrict__ tau,
                                                    int64_t sTau, cplx* __restrict__ T,
                                                    int64_t sT) {
  constexpr int NB = NT / GL;
  constexpr int MP = GL * RPL;
  static_assert(8 * NB <= NT, "T columns take eight threads per row");
  const int b = blockIdx.x;
  const int m = dimv(Md, b), n = dimv(Nd, b), s = min(m, n);
  if (j0 >= s) return;
  const int nbw = min(NB, s - j0), ncol = min(NB, n - j0);
  M += b * sM;
  V += b * sV;
  tau += b * sTau;
  T += b * sT + (int64_t)(j0 / NB) * NB * NB;
  __shared__ cplx ush[2][MP];
  __shared__ cplx zsh[2][NB];
  __shared__ double tl[NB];
  __shared__ cplx Ts[NB][NB];
  const int tid = threadIdx.x, grp = tid / GL, l = tid % GL;
  for (int e = tid; e < NB * NB; e += NT) Ts[e / NB][e % NB] = czero();
  const int c = j0 + grp;
  const bool have = grp < ncol;
  cplx a[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int i = j0 + l + GL * r;
    a[r] = (have && i < m) ? M[(int64_t)c * ld + i] : czero();
  }
  for (int jj = 0; jj < nbw; ++jj) {
    const int j = j0 + jj, buf = jj & 1;
    if (grp == jj) {
      double s0 = 0.0, s1 = 0.0;
      cplx al = czero();
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int i = j0 + l + GL * r;
        if (i > j && i < m) {
          if (r & 1) s1 += cabs2(a[r]);
          else s0 += cabs2(a[r]);
        }
        if (i == j) al = a[r];
      }
      const double sig2 = grp_sum<GL>(s0 + s1);
      al = grp_sum<GL>(al);   // one lane contributes
      double t;
      cplx beta, iu0;
      {
        double sc = 1.0, s2 = sig2;
        const double x2 = cabs2(al) + sig2;
        if (x2 > 0.0 && x2 < QR_TINY) {   // uniform over the group
          sc = QR_SCALE;
          s2 = 0.0;
#pragma unroll
          for (int r = 0; r < RPL; ++r) {
            const int i = j0 + l + GL * r;
            if (i > j && i < m) s2 += cabs2(cscale(a[r], sc));
          }
          s2 = grp_sum<GL>(s2);
        }
        house_coef(cscale(al, sc), s2, sc, t, beta, iu0);
      }
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int i = j0 + l + GL * r;
        cplx u;
        if (i < j || i >= m) u = czero();
        else if (i == j) u = make_double2(1.0, 0.0);
        else u = cmul(a[r], iu0);
        ush[buf][l + GL * r] = u;
        if (i == j) a[r] = beta;
        else if (i > j) a[r] = u;
      }
      if (l == 0) {
        tl[jj] = t;
        tau[j] = t;
      }
    }
    __syncthreads();
    const double t = tl[jj];
    // T column jj - 1 from the previous step's z (published by the barrier)
    if (jj >= 1) qp_t_column<NT>(jj - 1, tid, Ts, zsh[(jj - 1) & 1], tl);
    const cplx* u = ush[buf];
    // the reflector is read from LDS in chunks of QP_CH rows (the empty asm
    // statements keep the compiler from loading all of it at once: the
    // registers hold the column)
    if (grp > jj && have && t != 0.0) {
      // two interleaved partial sums halve the dependent FMA chain
      cplx w0 = czero(), w1 = czero();
#pragma unroll
      for (int r0 = 0; r0 < RPL; r0 += QP_CH) {
        asm volatile("" ::: "memory");
#pragma unroll
        for (int r = r0; r < r0 + QP_CH && r < RPL; ++r) {
          if (r & 1) cfma(w1, cconj(u[l + GL * r]), a[r]);
          else cfma(w0, cconj(u[l + GL * r]), a[r]);
        }
      }
      cplx w = grp_sum<GL>(cadd(w0, w1));
      const cplx f = cscale(w, -t);
#pragma unroll
      for (int r0 = 0; r0 < RPL; r0 += QP_CH) {
        asm volatile("" ::: "memory");
#pragma unroll
        for (int r = r0; r < r0 + QP_CH && r < RPL; ++r) cfma(a[r], u[l + GL * r], f);
      }
    } else if (grp < jj) {
      // rows i >= j > c: a holds this column's reflector there
      cplx z0 = czero(), z1 = czero();
#pragma unroll
      for (int r0 = 0; r0 < RPL; r0 += QP_CH) {
        asm volatile("" ::: "memory");
#pragma unroll
        for (int r = r0; r < r0 + QP_CH && r < RPL; ++r) {
          const int i = j0 + l + GL * r;
          if (i < j) continue;
          if (r & 1) cfma(z1, cconj(a[r]), u[l + GL * r]);
          else cfma(z0, cconj(a[r]), u[l + GL * r]);
        }
      }
      const cplx z = grp_sum<GL>(cadd(z0, z1));
      if (l == 0) zsh[buf][grp] = z;
    }
  }
  __syncthreads();
  qp_t_column<NT>(nbw - 1, tid, Ts, zsh[(nbw - 1) & 1], tl);
  // the panel back (R part) and the explicit reflectors
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int i = j0 + l + GL * r;
    if (i >= m) continue;
    if (have) M[(int64_t)c * ld + i] = (grp < nbw && i > c) ? czero() : a[r];
    cplx v;
    if (grp >= nbw || i < c) v = czero();
    else if (i == c) v = make_double2(1.0, 0.0);
    else v = a[r];
    V[(int64_t)c * ld + i] = v;
  }
  __syncthreads();
  for (int e = tid; e < NB * NB; e += NT) T[e] = Ts[e / NB][e % NB];
}

// Panel width and kernel of the blocked QR for a column capacity of mcap
// rows: 64 columns in 8-lane groups of a 512-thread workgroup up to 192
// rows; 32 columns in 32-lane groups of 1024 threads up to 288 rows (8 or 9
// rows per lane: a column step's dependent chain is about proportional to
// the rows per lane, 1.9 us per column at 8 against 4.6 at 24, measured on
// 256 x 128); 32 columns in 16-lane groups of 512 threads up to 384; 16
// columns in 32-lane groups up to 576; else the 32-column global-memory
// panel.
static int qrb_nb(int mcap) {
  if (mcap <= 8 * 24) return 64;
  if (mcap <= 16 * 24) return 32;
  if (mcap <= 32 * 18) return 16;
  return QB_NB;
}

static void qrb_panel(hipStream_t st, int batch, int mcap, int j0, Dim m, Dim n, cplx* Mw,
                      int64_t sM, int ld, const QrBlkWs& ws) {
#define QP_LAUNCH(NT, GL, RPL)                                                             \
  k_qrp_panel<NT, GL, RPL><<<batch, NT, 0, st>>>(j0, m, n, Mw, sM, ld, ws.V, ws.v_stride, \
                                                 ws.tau, ws.tau_stride, ws.T, ws.t_stride)
  if (mcap <= 8 * 12) QP_LAUNCH(512, 8, 12);
  else if (mcap <= 8 * 24) QP_LAUNCH(512, 8, 24);
  else if (mcap <= 32 * 8) QP_LAUNCH(1024, 32, 8);
  else if (mcap <= 32 * 9) QP_LAUNCH(1024, 32, 9);
  else if (mcap <= 16 * 24) QP_LAUNCH(512, 16, 24);
  else if (mcap <= 32 * 18) QP_LAUNCH(512, 32, 18);
  else
    k_qrb_panel<<<batch, QB_T, 0, st>>>(j0, m, n, Mw, sM, ld, ws.V, ws.v_stride, ws.tau,
                                        ws.tau_stride, ws.T, ws.t_stride);
#undef QP_LAUNCH
}

int64_t qr_blocked_tau_elems(int mcap, int ncap) {
  const int NB = qrb_nb(mcap);
  return (int64_t)((std::min(mcap, ncap) + NB - 1) / NB) * NB;
}

size_t qr_blocked_ws_elems(int mcap, int ncap, int64_t* v_elems, int64_t* t_elems,
                           int64_t* w_elems) {
  const int scap = std::min(mcap, ncap);
  const int NB = qrb_nb(mcap);
  const int P = (scap + NB - 1) / NB;
  *v_elems = (int64_t)mcap * P * NB;
  *t_elems = (int64_t)P * NB * NB;
  *w_elems = (int64_t)NB * ncap;
  return (size_t)(*v_elems + *t_elems + 2 * *w_elems);
}

// Matrices beyond registers and LDS: up to 576 rows the register-resident
// panels (one barrier per column) make the blocked form faster than the
// one-workgroup global-memory QR, whose every column step streams the trailing
// matrix through one CU; above 576 rows the global-memory panel is slow per
// column and the blocked form wins from 8 panels on (4x at 1024 x 512).
bool qr_blocked_wanted(int mcap, int ncap) {
  if (qr_reg_fits(mcap, ncap) || qr_lds_fits(mcap, ncap)) return false;
  if (mcap <= 32 * 18) return true;   // register-resident panels
  return std::min(mcap, ncap) >= 8 * QB_NB;
}

// Sizes of the factored matrix per instance when oriented: rows max(m, n),
// columns min(m, n), and whether it is A^H.
__global__ void k_qrb_dims(int batch, Dim Md, Dim Nd, int32_t* dims) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const int m = dimv(Md, b), n = dimv(Nd, b);
  dims[(int64_t)b * 3 + 0] = max(m, n);
  dims[(int64_t)b * 3 + 1] = min(m, n);
  dims[(int64_t)b * 3 + 2] = m < n ? 1 : 0;
}

void qr_blocked(hipStream_t st, int batch, int mcap, int ncap, Dim m0, Dim n0, const cplx* A,
                int64_t sA, cplx* Mw, int64_t sM, const QrBlkWs& ws, cplx* Q, int64_t sQ,
                cplx* R, int64_t sR, int32_t* s_out, int s_stride, bool orient) {
  // oriented: mcap, ncap are the capacities of the factored matrix (rows
  // >= columns) and m, n below its sizes per instance
  if (orient) k_qrb_dims<<<(batch + 127) / 128, 128, 0, st>>>(batch, m0, n0, ws.dims);
  const Dim m = orient ? dref(ws.dims, 3) : m0, n = orient ? dref(ws.dims + 1, 3) : n0;
  // live timing: the QR class covers this file's kernels; the products time
  // themselves as the GEMM class (regions do not nest)
  const bool prof = prof_on(PROF_QR);
  auto pb = [&]() { if (prof) g_prof->begin(); };
  auto pe = [&]() { if (prof) g_prof->end(); };
  const int ld = mcap;
  const int scap = std::min(mcap, ncap);
  const int NB = qrb_nb(mcap);
  const int P = (scap + NB - 1) / NB;
  const int64_t sV = ws.v_stride, sT = ws.t_stride, sW = ws.w_stride;
  const int ldw = ncap;
  const cplx one = make_double2(1.0, 0.0), mone = make_double2(-1.0, 0.0);
  auto cs = [](int64_t v) { return Str{nullptr, 0, 0, v}; };
  auto shift = [](Dim d, int by) { d.cst -= by; return d; };
  {
    const int tr = (mcap + QB_TILE - 1) / QB_TILE, tc = (ncap + QB_TILE - 1) / QB_TILE;
    pb();
    k_qrb_load<<<batch * tr * tc, 256, 0, st>>>(tr, tc, m0, n0, orient ? ws.dims : nullptr, A,
                                                sA, Mw, sM, ld, ws.s_dev);
    pe();
  }
  const Dim sd = dref(ws.s_dev, 1);
  for (int p = 0; p < P; ++p) {
    const int j0 = p * NB;
    pb();
    qrb_panel(st, batch, mcap, j0, m, n, Mw, sM, ld, ws);
    pe();
    const int ncap_t = ncap - j0 - NB;
    if (ncap_t <= 0) continue;
    const Dim nt = shift(n, j0 + NB), mt = shift(m, j0);
    // W1 (NB x n') = V^H A_trail
    gemm_ex(st, batch, 1, 1, dconst(NB), nt, mt, NB, ncap_t,
            mat(ws.V + (int64_t)j0 * ld + j0, sV, cs(ld), cs(1)), true,
            mat(Mw + (int64_t)(j0 + NB) * ld + j0, sM, cs(1), cs(ld)), false,
            mat(ws.W1, sW, cs(ldw), cs(1)), one, false, Dim{nullptr, 0, 0, 1 << 30}, mcap - j0);
    // W2 = T^H W1
    gemm_ex(st, batch, 1, 1, dconst(NB), nt, dconst(NB), NB, ncap_t,
            mat(ws.T + (int64_t)p * NB * NB, sT, cs(1), cs(NB)), true,
            mat(ws.W1, sW, cs(ldw), cs(1)), false, mat(ws.W2, sW, cs(ldw), cs(1)), one, false);
    // A_trail^T -= W2^T V^T  (the transposed form writes M along its columns)
    gemm_ex(st, batch, 1, 1, nt, mt, dconst(NB), ncap_t, mcap - j0,
            mat(ws.W2, sW, cs(1), cs(ldw)), false,
            mat(ws.V + (int64_t)j0 * ld + j0, sV, cs(ld), cs(1)), false,
            mat(Mw + (int64_t)(j0 + NB) * ld + j0, sM, cs(ld), cs(1)), mone, true);
  }
  {
    const int tr = (scap + QB_TILE - 1) / QB_TILE, tc = (ncap + QB_TILE - 1) / QB_TILE;
    pb();
    k_qrb_rout<<<batch * tr * tc, 256, 0, st>>>(tr, tc, m, n, Mw, sM, ld, R, sR);
    pe();
  }
  if (Q) {
    const int64_t cap_elems = (int64_t)ld * scap;
    const int per = (int)std::min<int64_t>((cap_elems + 255) / 256, 1024);
    pb();
    k_qrb_qinit<<<batch * per, 256, 0, st>>>(per, cap_elems, m, n, Mw, sM, ld);
    pe();
    for (int p = P - 1; p >= 0; --p) {
      const int j0 = p * NB;
      const int scap_t = scap - j0;
      const Dim st_ = shift(sd, j0), mt = shift(m, j0);
      // W1 (NB x (s - j0)) = V^H Q[j0:, j0:]
      gemm_ex(st, batch, 1, 1, dconst(NB), st_, mt, NB, scap_t,
              mat(ws.V + (int64_t)j0 * ld + j0, sV, cs(ld), cs(1)), true,
              mat(Mw + (int64_t)j0 * ld + j0, sM, cs(1), cs(ld)), false,
              mat(ws.W1, sW, cs(ldw), cs(1)), one, false, Dim{nullptr, 0, 0, 1 << 30}, mcap - j0);
      // W2 = T W1
      gemm_ex(st, batch, 1, 1, dconst(NB), st_, dconst(NB), NB, scap_t,
              mat(ws.T + (int64_t)p * NB * NB, sT, cs(NB), cs(1)), false,
              mat(ws.W1, sW, cs(ldw), cs(1)), false, mat(ws.W2, sW, cs(ldw), cs(1)), one, false);
      // Q[j0:, j0:]^T -= W2^T V^T
      gemm_ex(st, batch, 1, 1, st_, mt, dconst(NB), scap_t, mcap - j0,
              mat(ws.W2, sW, cs(1), cs(ldw)), false,
              mat(ws.V + (int64_t)j0 * ld + j0, sV, cs(ld), cs(1)), false,
              mat(Mw + (int64_t)j0 * ld + j0, sM, cs(ld), cs(1)), mone, true);
    }
    const int tr = (mcap + QB_TILE - 1) / QB_TILE, tc = (scap + QB_TILE - 1) / QB_TILE;
    pb();
    k_qrb_qout<<<batch * tr * tc, 256, 0, st>>>(tr, tc, m, n, Mw, sM, ld, Q, sQ, s_out, s_stride);
    pe();
  } else if (s_out) {
    k_qrb_sout<<<(batch + 255) / 256, 256, 0, st>>>(batch, ws.s_dev, s_out, s_stride);
  }
}

}  // namespace qt
