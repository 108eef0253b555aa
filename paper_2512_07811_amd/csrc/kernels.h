// Host-side launchers of the qtthom kernels (internal; not part of the C ABI).
#pragma once

#include "common.h"

namespace qt {

void enter(qt_ctx ctx);

// C_b = alpha * op(A_b) op(B_b) (+ C_b when accumulate), complex double,
// row-major packed matrices whose sizes M, N, K are read from device memory.
//   A stored M x K (conjA = false) or K x M (conjA = true, A^dagger used)
//   B stored K x N (conjB = false) or N x K (conjB = true, B^dagger used)
// Grid covers the capacities Mcap x Ncap; instances b = 0..batch-1 use base
// pointers advanced by the element strides sA, sB, sC (0 broadcasts).
void gemm(hipStream_t st, int batch, Dim M, Dim N, Dim K, int Mcap, int Ncap, bool conjA,
          const cplx* A, int64_t sA, bool conjB, const cplx* B, int64_t sB, cplx* C, int64_t sC,
          cplx alpha, bool accumulate);

// General strided batched GEMM: for every instance b and batch item (b1, b2)
// with b1 < nb1, b2 < nb2:  C = alpha * op(A) op(B) (+ C when accumulate),
// op = identity or conjugate (the transpose is expressed through strides).
// A is M x K, B is K x N, C is M x N, each addressed through its Mat strides.
// Batch items with b1 >= lim1 (a device size) are skipped.
// Kcap (optional, host bound on K): when the output has few tiles and K is
// long, K is split over workgroups whose partial tiles go to the context's
// split-K buffer and are summed in a fixed order by a second kernel.
void gemm_ex(hipStream_t st, int batch, int nb1, int nb2, Dim M, Dim N, Dim K, int Mcap, int Ncap,
             Mat A, bool conjA, Mat B, bool conjB, Mat C, cplx alpha, bool accumulate,
             Dim lim1 = Dim{nullptr, 0, 0, 1 << 30}, int64_t Kcap = 0);

// Householder QR of the packed m x n matrix A (one workgroup per instance):
// A = Q R with Q (m x s) and R (s x n) packed, s = min(m, n) written to s_out.
// W is an m x n scratch matrix per instance (stride sW), tau a scratch vector.
void qr(hipStream_t st, int batch, Dim m, Dim n, const cplx* A, int64_t sA, cplx* W, int64_t sW,
        double* tau, int64_t sTau, cplx* Q, int64_t sQ, cplx* R, int64_t sR, int32_t* s_out,
        int s_stride);

// Register-resident variant for m <= 256, n <= 96 (returns false when the
// capacities do not fit); qr_auto picks it when possible.
// orient = true factors B = A when m >= n and B = A^H otherwise (mcap/ncap
// must then bound max(m, n) and min(m, n)).
bool qr_reg(hipStream_t st, int batch, int mcap, int ncap, Dim m, Dim n, const cplx* A, int64_t sA,
            cplx* U, int64_t sU, double* tau, int64_t sTau, cplx* Q, int64_t sQ, cplx* R,
            int64_t sR, int32_t* s_out, int s_stride, bool orient = false);
// Memory-resident QR (LDS when the matrix fits, else the global scratch W).
void qr_mem(hipStream_t st, int batch, int mcap, int ncap, Dim m, Dim n, const cplx* A,
            int64_t sA, cplx* W, int64_t sW, double* tau, int64_t sTau, cplx* Q, int64_t sQ,
            cplx* R, int64_t sR, int32_t* s_out, int s_stride, bool orient = false);
void qr_auto(hipStream_t st, int batch, int mcap, int ncap, Dim m, Dim n, const cplx* A,
             int64_t sA, cplx* W, int64_t sW, double* tau, int64_t sTau, cplx* Q, int64_t sQ,
             cplx* R, int64_t sR, int32_t* s_out, int s_stride);
// Capacities that the register-resident / LDS-resident kernels cover.
bool qr_reg_fits(int mcap, int ncap);
bool qr_lds_fits(int mcap, int ncap);

// Blocked Householder QR (panels of 64, 32 or 16 columns factored in
// registers by one workgroup, or 32-column panels in global memory above 576
// rows; trailing updates and Q formation on the MFMA GEMM) for unfoldings
// beyond one workgroup's registers and LDS.
// Same contract as qr (Q may be null: R and s_out only).  Mw is the m x n work
// matrix (column-major, leading dimension mcap, stride sM >= mcap * ncap).
// orient: factor A^H where an instance's A is wide, as qr_reg does (mcap and
// ncap are then the capacities of the factored matrix, rows >= columns, and
// ws.dims must hold batch x 3 ints).
struct QrBlkWs {
  cplx* V;            // reflectors, mcap x (panels * NB) per instance
  int64_t v_stride;
  cplx* T;            // panels x NB x NB per instance
  int64_t t_stride;
  cplx* W1;           // NB x ncap per instance
  cplx* W2;
  int64_t w_stride;
  double* tau;        // panels * NB per instance (qr_blocked_tau_elems)
  int64_t tau_stride;
  int32_t* s_dev;     // batch
  int32_t* dims;      // batch x 3, for oriented factorizations (may be null otherwise)
};
bool qr_blocked_wanted(int mcap, int ncap);
// element counts per instance of V, T and one W buffer; returns V + T + 2 W
size_t qr_blocked_ws_elems(int mcap, int ncap, int64_t* v_elems, int64_t* t_elems,
                           int64_t* w_elems);
// reflector scalars per instance (QrBlkWs::tau_stride)
int64_t qr_blocked_tau_elems(int mcap, int ncap);
void qr_blocked(hipStream_t st, int batch, int mcap, int ncap, Dim m, Dim n, const cplx* A,
                int64_t sA, cplx* Mw, int64_t sM, const QrBlkWs& ws, cplx* Q, int64_t sQ,
                cplx* R, int64_t sR, int32_t* s_out, int s_stride, bool orient = false);

// Truncated SVD of the packed m x c matrix A by one-sided (Hestenes) Jacobi:
// keeps the smallest l >= 1 whose discarded tail does not exceed delta[b],
// l <= lmax; writes V^dagger[:l] (l x c) to core, U Sigma[:, :l] (m x l) to
// carry, l to l_out, adds the squared discarded tail to disc2[b].  svlog (may
// be null) receives the sorted singular values (stride svstride).
// Truncated SVD by QR, a second QR of R^H when A is wide, then one-sided
// Jacobi on the conjugate transpose of the triangle without accumulating its
// rotations: the matrix in LDS up to order 100, in global memory (Xw) up to
// 1024; core and carry = A core^H finished by the MFMA GEMM; returns false
// above order 1024.  Scratch: Qw, Uw (max x min, stride sQ), Rw, Xw (min^2,
// stride sR), tau (stride sT >= min + 4); qb (may be null): blocked-QR
// workspace for blocks where qr_blocked_wanted(max, min), whose QRs then run
// blocked.  A must not alias core.
bool svd_trunc_fast(hipStream_t st, int batch, int mcap, int ccap, Dim m, Dim c, const cplx* A,
                    int64_t sA, cplx* Qw, cplx* Uw, int64_t sQ, cplx* Rw, cplx* Xw, int64_t sR,
                    double* tau, int64_t sT, const QrBlkWs* qb, cplx* core, int64_t sCore, cplx* carry,
                    int64_t sCarry, int32_t* l_out, int l_stride, const double* delta,
                    double* disc2, int lmax, int max_sweeps, int32_t* status, double* svlog,
                    int64_t svstride, unsigned long long* counters, bool exact = false);

// Frobenius norm of a packed rows x cols matrix per instance; also sets
// delta[b] = eps * norm / sqrt(nb_bonds) (0 when nb_bonds == 0) and disc2[b] = 0.
void norm_delta(hipStream_t st, int batch, Dim rows, Dim cols, const cplx* X, int64_t sX,
                double* norm, double* delta, double* disc2, double eps, int nb_bonds);

// dst = src for a packed block of rows*cols elements per instance.
void copy(hipStream_t st, int batch, Dim rows, Dim cols, int64_t cap_elems, const cplx* src,
          int64_t sS, cplx* dst, int64_t sD);

// err[b] = sqrt(disc2[b]) / norm[b];  optional norm_out[b] = norm[b].
void finalize_err(hipStream_t st, int batch, const double* disc2, const double* norm, double* err,
                  double* norm_out);

// r[b] = scale_b * value[b] for residual bookkeeping (scale from host array uploaded to dev).
void scale_vec(hipStream_t st, int batch, const double* in, const double* scale, double* out);

// dst[i] = src[i] for i < count (a kernel, so that graphs hold no copy nodes).
void copy_i32(hipStream_t st, int64_t count, const int32_t* src, int32_t* dst);

}  // namespace qt
