// Exact TT algebra on device (Sec. 2.1 of arXiv 2512.07811): Hadamard
// product, TT x TTO contraction, scaled addition, and the dot product.
#include "kernels.h"
#include "round.h"

namespace qt {

// out ranks = product (or sum) of the input ranks, per instance.
struct OpRanks {
  int32_t v[QT_MAX_CORES + 1];
};

__global__ void k_rank_combine(int n, int batch, const int32_t* ra, int sa, const int32_t* rb,
                               int sb, OpRanks opr, int32_t* out, int mode) {
  int b = blockIdx.x;
  if (b >= batch) return;
  for (int k = threadIdx.x; k <= n; k += blockDim.x) {
    int a = ra ? ra[(int64_t)b * sa + k] : opr.v[k];
    int c = rb[(int64_t)b * sb + k];
    int v;
    if (mode == 0) v = a * c;                          // product
    else v = (k == 0 || k == n) ? 1 : a + c;           // block-diagonal sum
    out[(int64_t)b * (n + 1) + k] = v;
  }
}

// C[(a*rb0 + b), i, (a2*rb1 + b2)] = A[a, i, a2] * B[b, i, b2]
__global__ void k_hadamard(Dim ra0, Dim ra1, Dim rb0, Dim rb1, int p, const cplx* __restrict__ A,
                           int64_t sA, const cplx* __restrict__ B, int64_t sB, cplx* __restrict__ C,
                           int64_t sC) {
  const int bi = blockIdx.y;
  const int a0 = dimv(ra0, bi), a1 = dimv(ra1, bi), b0 = dimv(rb0, bi), b1 = dimv(rb1, bi);
  const int64_t total = (int64_t)a0 * b0 * p * a1 * b1;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int64_t t = e;
  const int jb = (int)(t % b1); t /= b1;
  const int ja = (int)(t % a1); t /= a1;
  const int i = (int)(t % p); t /= p;
  const int ib = (int)(t % b0); t /= b0;
  const int ia = (int)t;
  cplx x = A[bi * sA + ((int64_t)ia * p + i) * a1 + ja];
  cplx y = B[bi * sB + ((int64_t)ib * p + i) * b1 + jb];
  C[bi * sC + e] = cmul(x, y);
}

// C[(a*rx0 + b), i, (a2*rx1 + b2)] = sum_j D[a, i, j, a2] * X[b, j, b2]
__global__ void k_mpo(int d0, int d1, int po, int pi, int diag, Dim rx0, Dim rx1,
                      const cplx* __restrict__ D, const cplx* __restrict__ X, int64_t sX,
                      cplx* __restrict__ C, int64_t sC) {
  const int bi = blockIdx.y;
  const int x0 = dimv(rx0, bi), x1 = dimv(rx1, bi);
  const int64_t total = (int64_t)d0 * x0 * po * d1 * x1;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int64_t t = e;
  const int jb = (int)(t % x1); t /= x1;
  const int ja = (int)(t % d1); t /= d1;
  const int i = (int)(t % po); t /= po;
  const int ib = (int)(t % x0); t /= x0;
  const int ia = (int)t;
  const cplx* Xb = X + bi * sX;
  cplx acc;
  if (diag) {
    acc = cmul(D[((int64_t)ia * po + i) * d1 + ja], Xb[((int64_t)ib * pi + i) * x1 + jb]);
  } else {
    acc = make_double2(0.0, 0.0);
    for (int j = 0; j < pi; ++j)
      cfma(acc, D[(((int64_t)ia * po + i) * pi + j) * d1 + ja], Xb[((int64_t)ib * pi + j) * x1 + jb]);
  }
  C[bi * sC + e] = acc;
}

// Block-diagonal sum core; first core [al*X, be*Y], last [X; Y], middle diag(X, Y).
__global__ void k_add(int pos, Dim rx0, Dim rx1, Dim ry0, Dim ry1, int p, const cplx* __restrict__ X,
                      int64_t sX, const cplx* __restrict__ Y, int64_t sY, cplx* __restrict__ C,
                      int64_t sC, cplx al, cplx be) {
  // pos: 0 first, 1 middle, 2 last, 3 single core
  const int bi = blockIdx.y;
  const int x0 = dimv(rx0, bi), x1 = dimv(rx1, bi), y0 = dimv(ry0, bi), y1 = dimv(ry1, bi);
  int c0, c1;
  if (pos == 0) { c0 = 1; c1 = x1 + y1; }
  else if (pos == 2) { c0 = x0 + y0; c1 = 1; }
  else if (pos == 3) { c0 = 1; c1 = 1; }
  else { c0 = x0 + y0; c1 = x1 + y1; }
  const int64_t total = (int64_t)c0 * p * c1;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int j = (int)(e % c1);
  const int i = (int)((e / c1) % p);
  const int r = (int)(e / ((int64_t)c1 * p));
  const cplx* Xb = X + bi * sX;
  const cplx* Yb = Y + bi * sY;
  cplx v = make_double2(0.0, 0.0);
  if (pos == 3) {
    v = cadd(cmul(al, Xb[i]), cmul(be, Yb[i]));
  } else if (pos == 0) {
    if (j < x1) v = cmul(al, Xb[(int64_t)i * x1 + j]);
    else v = cmul(be, Yb[(int64_t)i * y1 + (j - x1)]);
  } else if (pos == 2) {
    if (r < x0) v = Xb[(int64_t)r * p + i];
    else v = Yb[(int64_t)(r - x0) * p + i];
  } else {
    if (r < x0 && j < x1) v = Xb[((int64_t)r * p + i) * x1 + j];
    else if (r >= x0 && j >= x1) v = Yb[((int64_t)(r - x0) * p + i) * y1 + (j - x1)];
  }
  C[bi * sC + e] = v;
}

// 1x1 final environment -> out[b] = (re, im)
__global__ void k_store_scalar(int batch, const cplx* E, int64_t sE, double* out) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < batch) {
    out[2 * b] = E[b * sE].x;
    out[2 * b + 1] = E[b * sE].y;
  }
}

__global__ void k_set_one(int batch, cplx* E, int64_t sE) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < batch) E[b * sE] = make_double2(1.0, 0.0);
}

}  // namespace qt

using namespace qt;


namespace qt {
qt_status hadamard_impl(qt_ctx ctx, const qt_tt* a, const qt_tt* b, qt_tt* out) {
  QT_CHECK(ctx && a && b && out, QT_EINVAL, "tt_hadamard: null argument");
  QT_TRY(tt_validate(a, "a"));
  QT_TRY(tt_validate(b, "b"));
  QT_TRY(tt_validate(out, "out"));
  QT_CHECK(a->n == b->n && b->n == out->n, QT_EINVAL, "tt_hadamard: core counts differ");
  QT_CHECK(a->batch == b->batch || a->batch == 1, QT_EINVAL, "tt_hadamard: batch mismatch");
  QT_CHECK(out->batch == b->batch, QT_EINVAL, "tt_hadamard: output batch mismatch");
  QT_CHECK(out->data != a->data && out->data != b->data, QT_EINVAL, "tt_hadamard: out aliases input");
  const int n = a->n, B = b->batch;
  for (int k = 0; k < n; ++k) {
    QT_CHECK(a->modes[k] == b->modes[k] && b->modes[k] == out->modes[k], QT_EINVAL,
             "tt_hadamard: modes differ");
  }
  for (int k = 0; k <= n; ++k)
    QT_CHECK((int64_t)out->cap[k] >= (int64_t)a->cap[k] * b->cap[k], QT_ECAPACITY,
             "tt_hadamard: output capacity below product of input capacities");
  hipStream_t st = ctx->stream;
  const int64_t sA = a->batch == 1 ? 0 : a->inst_stride;
  const int sra = a->batch == 1 ? 0 : n + 1;
  auto* A = (const cplx*)a->data;
  auto* Bd = (const cplx*)b->data;
  auto* C = (cplx*)out->data;
  for (int k = 0; k < n; ++k) {
    const int p = a->modes[k];
    int64_t cap = (int64_t)a->cap[k] * b->cap[k] * p * a->cap[k + 1] * b->cap[k + 1];
    dim3 grid((unsigned)((cap + 255) / 256), B);
    k_hadamard<<<grid, 256, 0, st>>>(dref(a->ranks + k, sra), dref(a->ranks + k + 1, sra),
                                     dref(b->ranks + k, n + 1), dref(b->ranks + k + 1, n + 1), p,
                                     A + a->offsets[k], sA, Bd + b->offsets[k], b->inst_stride,
                                     C + out->offsets[k], out->inst_stride);
  }
  k_rank_combine<<<B, 64, 0, st>>>(n, B, a->ranks, sra, b->ranks, n + 1, OpRanks{}, out->ranks, 0);
  QT_HIP(hipGetLastError());
  return QT_OK;
}

qt_status mpo_impl(qt_ctx ctx, const qt_mpo* A, const qt_tt* x, qt_tt* out) {
  QT_CHECK(ctx && A && x && out, QT_EINVAL, "tt_mpo_apply: null argument");
  QT_TRY(tt_validate(x, "x"));
  QT_TRY(tt_validate(out, "out"));
  QT_CHECK(A->n == x->n && x->n == out->n, QT_EINVAL, "tt_mpo_apply: core counts differ");
  QT_CHECK(out->batch == x->batch, QT_EINVAL, "tt_mpo_apply: batch mismatch");
  QT_CHECK(out->data != x->data, QT_EINVAL, "tt_mpo_apply: out aliases x");
  QT_CHECK(A->inst_stride == 0, QT_EINVAL,
           "tt_mpo_apply: per-instance operators are read by the sketch modes only");
  const int n = x->n, B = x->batch;
  for (int k = 0; k < n; ++k) {
    QT_CHECK(A->modes_in[k] == x->modes[k] && A->modes_out[k] == out->modes[k], QT_EINVAL,
             "tt_mpo_apply: modes differ");
    QT_CHECK(!A->diag[k] || A->modes_in[k] == A->modes_out[k], QT_EINVAL,
             "tt_mpo_apply: diagonal core with unequal modes");
  }
  QT_CHECK(A->ranks[0] == 1 && A->ranks[n] == 1, QT_EINVAL, "tt_mpo_apply: boundary ranks");
  for (int k = 0; k <= n; ++k)
    QT_CHECK((int64_t)out->cap[k] >= (int64_t)A->ranks[k] * x->cap[k], QT_ECAPACITY,
             "tt_mpo_apply: output capacity below r_A * cap_x");
  hipStream_t st = ctx->stream;
  auto* D = (const cplx*)A->data;
  auto* X = (const cplx*)x->data;
  auto* C = (cplx*)out->data;
  for (int k = 0; k < n; ++k) {
    const int po = A->modes_out[k], pi = A->modes_in[k];
    int64_t cap = (int64_t)A->ranks[k] * x->cap[k] * po * A->ranks[k + 1] * x->cap[k + 1];
    dim3 grid((unsigned)((cap + 255) / 256), B);
    k_mpo<<<grid, 256, 0, st>>>(A->ranks[k], A->ranks[k + 1], po, pi, A->diag[k],
                                dref(x->ranks + k, n + 1), dref(x->ranks + k + 1, n + 1),
                                D + A->offsets[k], X + x->offsets[k], x->inst_stride,
                                C + out->offsets[k], out->inst_stride);
  }
  OpRanks opr{};
  for (int k = 0; k <= n; ++k) opr.v[k] = A->ranks[k];
  k_rank_combine<<<B, 64, 0, st>>>(n, B, nullptr, 0, x->ranks, n + 1, opr, out->ranks, 0);
  QT_HIP(hipGetLastError());
  return QT_OK;
}

qt_status add_impl(qt_ctx ctx, double are, double aim, const qt_tt* x, double bre, double bim,
                   const qt_tt* y, qt_tt* out) {
  QT_CHECK(ctx && x && y && out, QT_EINVAL, "tt_add: null argument");
  QT_TRY(tt_validate(x, "x"));
  QT_TRY(tt_validate(y, "y"));
  QT_TRY(tt_validate(out, "out"));
  QT_CHECK(x->n == y->n && y->n == out->n, QT_EINVAL, "tt_add: core counts differ");
  QT_CHECK(x->batch == out->batch && (y->batch == out->batch || y->batch == 1), QT_EINVAL,
           "tt_add: batch mismatch");
  QT_CHECK(out->data != x->data && out->data != y->data, QT_EINVAL, "tt_add: out aliases input");
  const int n = x->n, B = out->batch;
  for (int k = 0; k < n; ++k)
    QT_CHECK(x->modes[k] == y->modes[k] && y->modes[k] == out->modes[k], QT_EINVAL,
             "tt_add: modes differ");
  for (int k = 1; k < n; ++k)
    QT_CHECK(out->cap[k] >= x->cap[k] + y->cap[k], QT_ECAPACITY, "tt_add: output capacity");
  hipStream_t st = ctx->stream;
  const int64_t sY = y->batch == 1 ? 0 : y->inst_stride;
  const int sry = y->batch == 1 ? 0 : n + 1;
  cplx al = make_double2(are, aim), be = make_double2(bre, bim);
  for (int k = 0; k < n; ++k) {
    const int p = x->modes[k];
    int pos = (n == 1) ? 3 : (k == 0 ? 0 : (k == n - 1 ? 2 : 1));
    int64_t cap = (int64_t)out->cap[k] * p * out->cap[k + 1];
    dim3 grid((unsigned)((cap + 255) / 256), B);
    k_add<<<grid, 256, 0, st>>>(pos, dref(x->ranks + k, n + 1), dref(x->ranks + k + 1, n + 1),
                                dref(y->ranks + k, sry), dref(y->ranks + k + 1, sry), p,
                                (const cplx*)x->data + x->offsets[k], x->inst_stride,
                                (const cplx*)y->data + y->offsets[k], sY,
                                (cplx*)out->data + out->offsets[k], out->inst_stride, al, be);
  }
  k_rank_combine<<<B, 64, 0, st>>>(n, B, x->ranks, n + 1, y->ranks, sry, OpRanks{}, out->ranks, 1);
  QT_HIP(hipGetLastError());
  return QT_OK;
}

}  // namespace qt

extern "C" qt_status tt_hadamard(qt_ctx ctx, const qt_tt* a, const qt_tt* b, qt_tt* out) {
  qt::enter(ctx);
  if (ctx) ctx->ws_top = 0;
  return qt::hadamard_impl(ctx, a, b, out);
}
extern "C" qt_status tt_mpo_apply(qt_ctx ctx, const qt_mpo* A, const qt_tt* x, qt_tt* out) {
  qt::enter(ctx);
  if (ctx) ctx->ws_top = 0;
  return qt::mpo_impl(ctx, A, x, out);
}
extern "C" qt_status tt_add(qt_ctx ctx, double are, double aim, const qt_tt* x, double bre,
                            double bim, const qt_tt* y, qt_tt* out) {
  qt::enter(ctx);
  if (ctx) ctx->ws_top = 0;
  return qt::add_impl(ctx, are, aim, x, bre, bim, y, out);
}

// Environment sweep: E_{k+1} = sum_i A_k(i)^H E_k B_k(i), done as two
// structured MFMA GEMMs per core: T = E * B_k (right unfolding),
// E' = A_k(left unfolding)^H * T.
namespace qt {
qt_status dot_impl(qt_ctx ctx, const qt_tt* a, const qt_tt* b, double* out, bool reserve) {
  const int n = a->n, B = b->batch;
  const int64_t sA = a->batch == 1 ? 0 : a->inst_stride;
  const int sra = a->batch == 1 ? 0 : n + 1;
  int64_t env = 1, tcap = 1;
  for (int k = 0; k <= n; ++k) env = std::max<int64_t>(env, (int64_t)a->cap[k] * b->cap[k]);
  for (int k = 0; k < n; ++k)
    tcap = std::max<int64_t>(tcap, (int64_t)a->cap[k] * b->modes[k] * b->cap[k + 1]);
  size_t need = sizeof(cplx) * B * (2 * env + tcap) + 4096;
  if (reserve) QT_TRY(ws_reserve(ctx, need));
  cplx* E0 = (cplx*)ws_take(ctx, sizeof(cplx) * B * env);
  cplx* E1 = (cplx*)ws_take(ctx, sizeof(cplx) * B * env);
  cplx* Tb = (cplx*)ws_take(ctx, sizeof(cplx) * B * tcap);
  QT_CHECK(E0 && E1 && Tb, QT_ENOMEM, "tt_dot: workspace too small");
  hipStream_t st = ctx->stream;
  k_set_one<<<(B + 127) / 128, 128, 0, st>>>(B, E0, env);
  auto* Ad = (const cplx*)a->data;
  auto* Bd = (const cplx*)b->data;
  cplx one = make_double2(1.0, 0.0);
  for (int k = 0; k < n; ++k) {
    const int p = b->modes[k];
    // T (ra_k x p rb_{k+1}) = E (ra_k x rb_k) * Bk (rb_k x p rb_{k+1})
    gemm_ex(st, B, 1, 1, dref(a->ranks + k, sra), dref(b->ranks + k + 1, n + 1, p),
            dref(b->ranks + k, n + 1), a->cap[k], p * b->cap[k + 1],
            mat(E0, env, sref(b->ranks + k, n + 1), sconst(1)), false,
            mat(Bd + b->offsets[k], b->inst_stride, sref(b->ranks + k + 1, n + 1, p), sconst(1)),
            false, mat(Tb, tcap, sref(b->ranks + k + 1, n + 1, p), sconst(1)), one, false,
            Dim{nullptr, 0, 0, 1 << 30}, b->cap[k]);
    // E' (ra_{k+1} x rb_{k+1}) = Ak^H (ra_{k+1} x ra_k p) * T (ra_k p x rb_{k+1})
    gemm_ex(st, B, 1, 1, dref(a->ranks + k + 1, sra), dref(b->ranks + k + 1, n + 1),
            dref(a->ranks + k, sra, p), a->cap[k + 1], b->cap[k + 1],
            mat(Ad + a->offsets[k], sA, sconst(1), sref(a->ranks + k + 1, sra)), true,
            mat(Tb, tcap, sref(b->ranks + k + 1, n + 1), sconst(1)), false,
            mat(E1, env, sref(b->ranks + k + 1, n + 1), sconst(1)), one, false,
            Dim{nullptr, 0, 0, 1 << 30}, (int64_t)a->cap[k] * p);
    std::swap(E0, E1);
  }
  k_store_scalar<<<(B + 127) / 128, 128, 0, st>>>(B, E0, env, out);
  QT_HIP(hipGetLastError());
  return QT_OK;
}
}  // namespace qt

extern "C" qt_status tt_dot(qt_ctx ctx, const qt_tt* a, const qt_tt* b, double* out) {
  qt::enter(ctx);
  QT_CHECK(ctx && a && b && out, QT_EINVAL, "tt_dot: null argument");
  QT_TRY(tt_validate(a, "a"));
  QT_TRY(tt_validate(b, "b"));
  QT_CHECK(a->n == b->n, QT_EINVAL, "tt_dot: core counts differ");
  QT_CHECK(a->batch == b->batch || a->batch == 1, QT_EINVAL, "tt_dot: batch mismatch");
  for (int k = 0; k < a->n; ++k) QT_CHECK(a->modes[k] == b->modes[k], QT_EINVAL, "tt_dot: modes differ");
  ctx->ws_top = 0;
  return dot_impl(ctx, a, b, out, true);
}
