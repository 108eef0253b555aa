// Rank-predictor MLP: three hidden layers of 64 tanh units, FP32.
//
// Parameters are one flat float array: W0 (F x 64), b0, W1 (64 x 64), b1,
// W2 (64 x 64), b2, W3 (64 x C), b3, each W row-major [in][out].
// Loss per sample (under-prediction triggers a fallback, over-prediction only
// costs work, so the loss is biased upward):
//   CE(z, y) + beta * sum_c softmax(z)_c w(c, y),
//   w(c, y) = (c - y)/C for c > y, gamma for c < y, 0 for c = y.
// Training step = full-batch gradient (samples processed in chunks of 64 by
// one 1024-thread workgroup, gradients kept in registers) + Adam (Kingma and
// Ba 2015) with bias correction.  Class c stands for rank 8 (c + 1): the
// coarse rank lattice r_c = n r_0 of Sec. 5.1 of arXiv 2512.07811 with r_0 = 8.
#include "kernels.h"

namespace qt {

constexpr int MH = 64;       // hidden width
constexpr int MCH = 64;      // samples per chunk
constexpr int MF_MAX = 32;   // max input features
constexpr int MC_MAX = 32;   // max classes

__host__ __device__ inline int mlp_nparams(int F, int C) {
  return F * MH + MH + 2 * (MH * MH + MH) + MH * C + C;
}

struct MlpOff {
  int W0, b0, W1, b1, W2, b2, W3, b3;
};
__host__ __device__ inline MlpOff mlp_off(int F, int C) {
  MlpOff o;
  o.W0 = 0; o.b0 = o.W0 + F * MH;
  o.W1 = o.b0 + MH; o.b1 = o.W1 + MH * MH;
  o.W2 = o.b1 + MH; o.b2 = o.W2 + MH * MH;
  o.W3 = o.b2 + MH; o.b3 = o.W3 + MH * C;
  return o;
}

// y[s][o] = act(sum_i x[s][i] W[i][o] + b[o]) for a chunk in LDS
__device__ inline void dense_chunk(const float* __restrict__ x, int nin, const float* __restrict__ W,
                                   const float* __restrict__ bias, int nout, float* y, int ns,
                                   bool act) {
  for (int e = threadIdx.x; e < ns * nout; e += blockDim.x) {
    const int s = e / nout, o = e % nout;
    float a = bias[o];
    for (int i = 0; i < nin; ++i) a = fmaf(x[s * nin + i], W[i * nout + o], a);
    y[e] = act ? tanhf(a) : a;
  }
}

__global__ __launch_bounds__(1024) void k_mlp_train(float* __restrict__ P, float* __restrict__ Mo,
                                                    float* __restrict__ Vo, int t,
                                                    const float* __restrict__ X,
                                                    const int32_t* __restrict__ Y, int B, int F,
                                                    int C, float lr, float beta, float gamma,
                                                    float* __restrict__ loss_out,
                                                    float* __restrict__ grad_out) {
  __shared__ float xs[MCH * MF_MAX];
  __shared__ float h1[MCH * MH], h2[MCH * MH], h3[MCH * MH];
  __shared__ float z[MCH * MC_MAX];
  __shared__ float d0[MCH * MH], d1[MCH * MH];
  __shared__ float lsum[32];
  const MlpOff o = mlp_off(F, C);
  const int np = mlp_nparams(F, C);
  constexpr int PPT = 16;  // parameters per thread (np <= 16384)
  float g[PPT];
#pragma unroll
  for (int r = 0; r < PPT; ++r) g[r] = 0.f;
  float loss = 0.f;
  for (int s0 = 0; s0 < B; s0 += MCH) {
    const int ns = min(MCH, B - s0);
    for (int e = threadIdx.x; e < ns * F; e += blockDim.x) xs[e] = X[(int64_t)s0 * F + e];
    __syncthreads();
    dense_chunk(xs, F, P + o.W0, P + o.b0, MH, h1, ns, true);
    __syncthreads();
    dense_chunk(h1, MH, P + o.W1, P + o.b1, MH, h2, ns, true);
    __syncthreads();
    dense_chunk(h2, MH, P + o.W2, P + o.b2, MH, h3, ns, true);
    __syncthreads();
    dense_chunk(h3, MH, P + o.W3, P + o.b3, C, z, ns, false);
    __syncthreads();
    // softmax, loss, dZ (scaled by 1/B) in place of z
    if (threadIdx.x < ns) {
      const int s = threadIdx.x;
      const int y = min(max(Y[s0 + s], 0), C - 1);
      float mx = -1e30f;
      for (int c = 0; c < C; ++c) mx = fmaxf(mx, z[s * C + c]);
      float se = 0.f;
      for (int c = 0; c < C; ++c) se += expf(z[s * C + c] - mx);
      float ec = 0.f;
      for (int c = 0; c < C; ++c) {
        const float p = expf(z[s * C + c] - mx) / se;
        const float w = c > y ? (float)(c - y) / C : (c < y ? gamma : 0.f);
        ec += p * w;
      }
      loss += -(z[s * C + y] - mx - logf(se)) + beta * ec;
      for (int c = 0; c < C; ++c) {
        const float p = expf(z[s * C + c] - mx) / se;
        const float w = c > y ? (float)(c - y) / C : (c < y ? gamma : 0.f);
        z[s * C + c] = ((p - (c == y ? 1.f : 0.f)) + beta * p * (w - ec)) / (float)B;
      }
    }
    __syncthreads();
    // dH3 = (dZ W3^T) (1 - h3^2) -> d0
    for (int e = threadIdx.x; e < ns * MH; e += blockDim.x) {
      const int s = e / MH, i = e % MH;
      float a = 0.f;
      for (int c = 0; c < C; ++c) a = fmaf(z[s * C + c], P[o.W3 + i * C + c], a);
      d0[e] = a * (1.f - h3[e] * h3[e]);
    }
    __syncthreads();
    // dH2 = (dH3 W2^T)(1 - h2^2) -> d1
    for (int e = threadIdx.x; e < ns * MH; e += blockDim.x) {
      const int s = e / MH, i = e % MH;
      float a = 0.f;
      for (int c = 0; c < MH; ++c) a = fmaf(d0[s * MH + c], P[o.W2 + i * MH + c], a);
      d1[e] = a * (1.f - h2[e] * h2[e]);
    }
    __syncthreads();
    // parameter gradients of layers 3 and 2 (inputs h3, h2; deltas z, d0)
#pragma unroll
    for (int r = 0; r < PPT; ++r) {
      const int p = threadIdx.x + 1024 * r;
      if (p >= np) continue;
      float a = 0.f;
      if (p >= o.W3 && p < o.b3) {
        const int i = (p - o.W3) / C, c = (p - o.W3) % C;
        for (int s = 0; s < ns; ++s) a = fmaf(h3[s * MH + i], z[s * C + c], a);
      } else if (p >= o.b3) {
        const int c = p - o.b3;
        for (int s = 0; s < ns; ++s) a += z[s * C + c];
      } else if (p >= o.W2 && p < o.b2) {
        const int i = (p - o.W2) / MH, c = (p - o.W2) % MH;
        for (int s = 0; s < ns; ++s) a = fmaf(h2[s * MH + i], d0[s * MH + c], a);
      } else if (p >= o.b2 && p < o.W3) {
        const int c = p - o.b2;
        for (int s = 0; s < ns; ++s) a += d0[s * MH + c];
      } else {
        continue;
      }
      g[r] += a;
    }
    __syncthreads();
    // dH1 = (dH2 W1^T)(1 - h1^2) -> d0
    for (int e = threadIdx.x; e < ns * MH; e += blockDim.x) {
      const int s = e / MH, i = e % MH;
      float a = 0.f;
      for (int c = 0; c < MH; ++c) a = fmaf(d1[s * MH + c], P[o.W1 + i * MH + c], a);
      d0[e] = a * (1.f - h1[e] * h1[e]);
    }
    __syncthreads();
    // layers 1 and 0 (inputs h1, xs; deltas d1, d0)
#pragma unroll
    for (int r = 0; r < PPT; ++r) {
      const int p = threadIdx.x + 1024 * r;
      if (p >= np) continue;
      float a = 0.f;
      if (p >= o.W1 && p < o.b1) {
        const int i = (p - o.W1) / MH, c = (p - o.W1) % MH;
        for (int s = 0; s < ns; ++s) a = fmaf(h1[s * MH + i], d1[s * MH + c], a);
      } else if (p >= o.b1 && p < o.W2) {
        const int c = p - o.b1;
        for (int s = 0; s < ns; ++s) a += d1[s * MH + c];
      } else if (p >= o.W0 && p < o.b0) {
        const int i = (p - o.W0) / MH, c = (p - o.W0) % MH;
        for (int s = 0; s < ns; ++s) a = fmaf(xs[s * F + i], d0[s * MH + c], a);
      } else if (p >= o.b0 && p < o.W1) {
        const int c = p - o.b0;
        for (int s = 0; s < ns; ++s) a += d0[s * MH + c];
      } else {
        continue;
      }
      g[r] += a;
    }
    __syncthreads();
  }
  // loss reduction
  for (int off = 32; off > 0; off >>= 1) loss += __shfl_xor(loss, off, 64);
  if ((threadIdx.x & 63) == 0) lsum[threadIdx.x >> 6] = loss;
  __syncthreads();
  if (threadIdx.x == 0) {
    float l = 0.f;
    for (int i = 0; i < 16; ++i) l += lsum[i];
    if (loss_out) *loss_out = l / (float)B;
  }
  // gradients out and Adam update
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
#pragma unroll
  for (int r = 0; r < PPT; ++r) {
    const int p = threadIdx.x + 1024 * r;
    if (p >= np) continue;
    if (grad_out) grad_out[p] = g[r];
    if (lr > 0.f) {
      const float m = b1 * Mo[p] + (1.f - b1) * g[r];
      const float v = b2 * Vo[p] + (1.f - b2) * g[r] * g[r];
      Mo[p] = m;
      Vo[p] = v;
      P[p] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
    }
  }
}

// Per-sample forward pass and class choice: the smallest class whose
// cumulative softmax probability reaches `quantile`; rank = 8 (class + 1),
// capped by cap[s] (natural and product bounds) and at least 1.
__global__ void k_mlp_infer(const float* __restrict__ P, const float* __restrict__ X, int B, int F,
                            int C, float quantile, float* __restrict__ logits,
                            int32_t* __restrict__ rank_out, const int32_t* __restrict__ cap) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= B) return;
  const MlpOff o = mlp_off(F, C);
  float a[MH], b[MH];
  for (int j = 0; j < MH; ++j) {
    float v = P[o.b0 + j];
    for (int i = 0; i < F; ++i) v = fmaf(X[(int64_t)s * F + i], P[o.W0 + i * MH + j], v);
    a[j] = tanhf(v);
  }
  for (int j = 0; j < MH; ++j) {
    float v = P[o.b1 + j];
    for (int i = 0; i < MH; ++i) v = fmaf(a[i], P[o.W1 + i * MH + j], v);
    b[j] = tanhf(v);
  }
  for (int j = 0; j < MH; ++j) {
    float v = P[o.b2 + j];
    for (int i = 0; i < MH; ++i) v = fmaf(b[i], P[o.W2 + i * MH + j], v);
    a[j] = tanhf(v);
  }
  float zc[MC_MAX];
  float mx = -1e30f;
  for (int c = 0; c < C; ++c) {
    float v = P[o.b3 + c];
    for (int i = 0; i < MH; ++i) v = fmaf(a[i], P[o.W3 + i * C + c], v);
    zc[c] = v;
    mx = fmaxf(mx, v);
    if (logits) logits[(int64_t)s * C + c] = v;
  }
  float se = 0.f;
  for (int c = 0; c < C; ++c) se += expf(zc[c] - mx);
  float cdf = 0.f;
  int cls = C - 1;
  for (int c = 0; c < C; ++c) {
    cdf += expf(zc[c] - mx) / se;
    if (cdf >= quantile) { cls = c; break; }
  }
  if (rank_out) {
    int r = 8 * (cls + 1);
    if (cap) r = min(r, cap[s]);
    rank_out[s] = max(r, 1);
  }
}

}  // namespace qt

using namespace qt;

extern "C" int32_t qt_mlp_num_params(int32_t n_in, int32_t n_cls) {
  return mlp_nparams(n_in, n_cls);
}

extern "C" qt_status qt_mlp_train_step(qt_ctx ctx, float* params, float* adam_m, float* adam_v,
                                       int32_t step, const float* X, const int32_t* labels,
                                       int32_t n, int32_t n_in, int32_t n_cls, float lr,
                                       float beta, float gamma, float* loss_out,
                                       float* grad_out) {
  QT_CHECK(ctx && params && X && labels, QT_EINVAL, "qt_mlp_train_step: null argument");
  QT_CHECK(n >= 1 && n_in >= 1 && n_in <= MF_MAX && n_cls >= 2 && n_cls <= MC_MAX, QT_EINVAL,
           "qt_mlp_train_step: sizes out of range");
  QT_CHECK(mlp_nparams(n_in, n_cls) <= 16 * 1024, QT_EINVAL, "qt_mlp_train_step: too many params");
  QT_CHECK(lr <= 0.f || (adam_m && adam_v && step >= 1), QT_EINVAL,
           "qt_mlp_train_step: Adam state missing");
  enter(ctx);
  k_mlp_train<<<1, 1024, 0, ctx->stream>>>(params, adam_m, adam_v, step, X, labels, n, n_in, n_cls,
                                           lr, beta, gamma, loss_out, grad_out);
  QT_HIP(hipGetLastError());
  return QT_OK;
}

extern "C" qt_status qt_mlp_infer(qt_ctx ctx, const float* params, const float* X, int32_t n,
                                  int32_t n_in, int32_t n_cls, float quantile, float* logits,
                                  int32_t* ranks, const int32_t* rank_cap) {
  QT_CHECK(ctx && params && X, QT_EINVAL, "qt_mlp_infer: null argument");
  QT_CHECK(n >= 0 && n_in >= 1 && n_in <= MF_MAX && n_cls >= 2 && n_cls <= MC_MAX, QT_EINVAL,
           "qt_mlp_infer: sizes out of range");
  enter(ctx);
  if (n == 0) return QT_OK;
  k_mlp_infer<<<(n + 63) / 64, 64, 0, ctx->stream>>>(params, X, n, n_in, n_cls, quantile, logits,
                                                    ranks, rank_cap);
  QT_HIP(hipGetLastError());
  return QT_OK;
}
