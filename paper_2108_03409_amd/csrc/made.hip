// Masked autoregressive proposal network (MADE, Germain et al. 2015) in
// float64: log q, minibatch NLL gradients, Adam training and autoregressive
// sampling.  Not part of the paper's method; it is the learned global
// Metropolis-Hastings proposal of VMC_PROP_MADE_MIX.
//
//   degrees   m(k) = k mod (N-1) + 1 (hidden), d + 1 (site d)
//   masks     M1[k][d] = [m(k) >= d+1],  M2[d][k] = [d+1 > m(k)]
//   logits    l = (W2*M2) relu((W1*M1) x + b1) + b2,   log q = sum_d x_d l_d - softplus(l_d)
// Parameters [W1 (H x N), b1 (H), W2 (N x H), b2 (N)].  Batched forward and
// backward passes are float64 GEMMs on the matrix cores (gemm64.hip); sampling
// runs one wavefront per row with the hidden units across lanes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.h"

using namespace dev;

namespace {

__device__ __forceinline__ int hdeg(int k, int N) { return k % (N - 1) + 1; }
__device__ __forceinline__ double softplus(double x) { return fmax(x, 0.0) + log1p(exp(-fabs(x))); }

// masked weights: W1m (H x N), W1mT (N x H), W2m (N x H)
__global__ void k_masks(const double* __restrict__ p, int N, int H, double* __restrict__ W1m,
                        double* __restrict__ W1mT, double* __restrict__ W2m) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)N * H) return;
  {
    const int k = (int)(e / N), d = (int)(e % N);
    const double w = hdeg(k, N) >= d + 1 ? p[e] : 0.0;
    W1m[e] = w;
    W1mT[(int64_t)d * H + k] = w;
  }
  {
    const int d = (int)(e / H), k = (int)(e % H);
    W2m[e] = (d + 1 > hdeg(k, N)) ? p[(int64_t)H * N + H + e] : 0.0;
  }
}

__global__ void k_unpack(const uint64_t* __restrict__ s, int64_t B, int N, int W, double* __restrict__ X) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= B * N) return;
  const int64_t b = e / N;
  const int d = (int)(e % N);
  X[e] = (double)((s[b * W + (d >> 6)] >> (d & 63)) & 1ull);
}

__global__ void k_bias_relu(double* __restrict__ A1, const double* __restrict__ b1, int64_t B, int H,
                            double* __restrict__ Hd) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= B * H) return;
  const double a = A1[e] + b1[e % H];
  A1[e] = a;
  Hd[e] = fmax(a, 0.0);
}

// L += b2; G = (sigmoid(L) - X) / B; nll += sum(softplus(L) - X L) / B
__global__ __launch_bounds__(256) void k_out_grad(double* __restrict__ L, const double* __restrict__ b2,
                                                  const double* __restrict__ X, int64_t B, int N, double inv_b,
                                                  double* __restrict__ G, double* __restrict__ nll) {
  __shared__ double red[4];
  const int64_t e = blockIdx.x * 256ll + threadIdx.x;
  double c = 0.0;
  if (e < B * N) {
    const double l = L[e] + b2[e % N];
    L[e] = l;
    const double x = X[e];
    G[e] = (1.0 / (1.0 + exp(-l)) - x) * inv_b;
    c = (softplus(l) - x * l) * inv_b;
  }
  c = wave_sum(c);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0 && nll) atomicAdd(nll, red[0] + red[1] + red[2] + red[3]);
}

// log q per row: sum_d x l - softplus(l) (L already holds the biased logits)
__global__ __launch_bounds__(64) void k_logq_rows(const double* __restrict__ L, const double* __restrict__ b2,
                                                  const double* __restrict__ X, int64_t B, int N,
                                                  double* __restrict__ logq) {
  const int64_t b = blockIdx.x;
  if (b >= B) return;
  double acc = 0.0;
  for (int d = threadIdx.x; d < N; d += 64) {
    const double l = L[b * N + d] + b2[d];
    acc += X[b * N + d] * l - softplus(l);
  }
  acc = wave_sum(acc);
  if (threadIdx.x == 0) logq[b] = acc;
}

__global__ void k_relu_mask(double* __restrict__ dH, const double* __restrict__ A1, int64_t n) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < n && !(A1[e] > 0.0)) dH[e] = 0.0;
}

__global__ void k_mask_grad(double* __restrict__ g, int N, int H) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)N * H) return;
  {
    const int k = (int)(e / N), d = (int)(e % N);
    if (!(hdeg(k, N) >= d + 1)) g[e] = 0.0;
  }
  {
    const int d = (int)(e / H), k = (int)(e % H);
    if (!(d + 1 > hdeg(k, N))) g[(int64_t)H * N + H + e] = 0.0;
  }
}

// column sums: a group takes 16 columns; its 16 row lanes sum every 16th row
// (eight independent partial sums each), then the lanes combine in a fixed order
__global__ __launch_bounds__(256) void k_colsum(const double* __restrict__ M, int64_t rows, int cols,
                                                double* __restrict__ out) {
  __shared__ double part[16][17];
  const int cl = threadIdx.x & 15, rl = threadIdx.x >> 4;
  const int c = blockIdx.x * 16 + cl;
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (c < cols) {
    int64_t r = rl;
    for (; r + 7 * 16 < rows; r += 8 * 16)
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] += M[(r + 16 * u) * cols + c];
    for (; r < rows; r += 16) acc[0] += M[r * cols + c];
  }
  part[rl][cl] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  __syncthreads();
  if (rl == 0 && c < cols) {
    double s = 0.0;
    for (int q = 0; q < 16; ++q) s += part[q][cl];
    out[c] = s;
  }
}

__global__ void k_adam(double* __restrict__ p, const double* __restrict__ g, double* __restrict__ m,
                       double* __restrict__ v, int64_t n, double lr, double bc1, double bc2) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double gi = g[e];
  const double mi = 0.9 * m[e] + 0.1 * gi;
  const double vi = 0.999 * v[e] + 0.001 * gi * gi;
  m[e] = mi;
  v[e] = vi;
  p[e] -= lr * (mi / bc1) / (sqrt(vi / bc2) + 1e-8);
}

// Autoregressive sampling, one wave per row; hidden units k = lane + 64 q.
// The W2 and W1^T rows of site d are loaded one site ahead (they do not depend
// on the decisions); the arithmetic order is that of the plain loop.
template <int QH>
__global__ __launch_bounds__(64) void k_made_sample(const double* __restrict__ W1mT, const double* __restrict__ W2m,
                                                    const double* __restrict__ b1, const double* __restrict__ b2,
                                                    int N, int H, int W, int64_t B, uint2 key, uint32_t lo,
                                                    uint32_t hi, uint64_t* __restrict__ s_out,
                                                    double* __restrict__ logq) {
  __shared__ uint64_t sb[64];
  const int64_t c = blockIdx.x;
  if (c >= B) return;
  const int lane = threadIdx.x;
  for (int w = lane; w < W; w += 64) sb[w] = 0ull;
  double a[QH], w2c[QH], w2n[QH], w1c[QH];
#pragma unroll
  for (int q = 0; q < QH; ++q) {
    const int k = lane + 64 * q;
    a[q] = k < H ? b1[k] : 0.0;
    w2n[q] = k < H ? W2m[k] : 0.0;
  }
  __syncthreads();
  double lq = 0.0;
  uint4 x4 = make_uint4(0, 0, 0, 0);
  for (int d = 0; d < N; ++d) {
#pragma unroll
    for (int q = 0; q < QH; ++q) {
      const int k = lane + 64 * q;
      w2c[q] = w2n[q];
      w1c[q] = k < H ? W1mT[(int64_t)d * H + k] : 0.0;
      w2n[q] = (k < H && d + 1 < N) ? W2m[(int64_t)(d + 1) * H + k] : 0.0;
    }
    if ((d & 3) == 0) x4 = philox(make_uint4((uint32_t)c, lo, hi, 1u + 256u * (uint32_t)(d >> 2)), key);
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < QH; ++q) {
      const int k = lane + 64 * q;
      if (k < H) part += w2c[q] * fmax(a[q], 0.0);
    }
    const double l = wave_sum_uniform(part) + b2[d];
    const double p = 1.0 / (1.0 + exp(-l));
    const uint32_t xr = (d & 3) == 0 ? x4.x : (d & 3) == 1 ? x4.y : (d & 3) == 2 ? x4.z : x4.w;
    const bool up = (double)xr * 0x1.0p-32 < p;
    lq += (up ? l : 0.0) - softplus(l);
    if (up) {
#pragma unroll
      for (int q = 0; q < QH; ++q) {
        const int k = lane + 64 * q;
        if (k < H) a[q] += w1c[q];
      }
      if (lane == 0) sb[d >> 6] |= 1ull << (d & 63);
    }
  }
  __syncthreads();
  for (int w = lane; w < W; w += 64) s_out[c * W + w] = sb[w];
  if (lane == 0 && logq) logq[c] = lq;
}

// The same sampling with one row per lane, for narrow hidden layers (H <= HM):
// each lane keeps its H pre-activations in registers, the weights of site d are
// the same for every lane (scalar loads), and no cross-lane reduction is
// needed.  Same Philox stream and decisions as k_made_sample.
template <int HM>
__global__ __launch_bounds__(64) void k_made_sample_lane(const double* __restrict__ W1mT,
                                                         const double* __restrict__ W2m,
                                                         const double* __restrict__ b1,
                                                         const double* __restrict__ b2, int N, int H, int W,
                                                         int64_t B, uint2 key, uint32_t lo, uint32_t hi,
                                                         uint64_t* __restrict__ s_out, double* __restrict__ logq) {
  const int64_t c = blockIdx.x * 64ll + threadIdx.x;
  const bool live = c < B;
  double a[HM];
#pragma unroll
  for (int k = 0; k < HM; ++k) a[k] = k < H ? b1[k] : 0.0;
  double lq = 0.0;
  uint64_t word = 0ull;
  uint4 x4 = make_uint4(0, 0, 0, 0);
  for (int d = 0; d < N; ++d) {
    double l = 0.0;
#pragma unroll
    for (int k = 0; k < HM; ++k)
      if (k < H) l = fma(W2m[(int64_t)d * H + k], fmax(a[k], 0.0), l);
    l += b2[d];
    if ((d & 3) == 0) x4 = philox(make_uint4((uint32_t)c, lo, hi, 1u + 256u * (uint32_t)(d >> 2)), key);
    const double p = 1.0 / (1.0 + exp(-l));
    const uint32_t xr = (d & 3) == 0 ? x4.x : (d & 3) == 1 ? x4.y : (d & 3) == 2 ? x4.z : x4.w;
    const bool up = (double)xr * 0x1.0p-32 < p;
    lq += (up ? l : 0.0) - softplus(l);
    const double u = up ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < HM; ++k)
      if (k < H) a[k] = fma(W1mT[(int64_t)d * H + k], u, a[k]);
    word |= (up ? 1ull : 0ull) << (d & 63);
    if ((d & 63) == 63 || d == N - 1) {
      if (live) s_out[c * W + (d >> 6)] = word;
      word = 0ull;
    }
  }
  if (live && logq) logq[c] = lq;
}

struct made_ws {
  double *X, *A1, *Hd, *L, *G, *dH, *grad, *nll;
};

size_t made_ws_bytes(const vmc_made* md, int64_t rows, int nll_slots) {
  const size_t N = md->N, H = md->H;
  return ws_round(sizeof(double) * rows * N) * 3 + ws_round(sizeof(double) * rows * H) * 3 +
         ws_round(sizeof(double) * md->P) + ws_round(sizeof(double) * std::max(1, nll_slots));
}

made_ws made_take(vmc_made* md, int64_t rows, int nll_slots) {
  vmc_ctx* ctx = md->ctx;
  made_ws w;
  w.X = (double*)ws_take(ctx, sizeof(double) * rows * md->N);
  w.L = (double*)ws_take(ctx, sizeof(double) * rows * md->N);
  w.G = (double*)ws_take(ctx, sizeof(double) * rows * md->N);
  w.A1 = (double*)ws_take(ctx, sizeof(double) * rows * md->H);
  w.Hd = (double*)ws_take(ctx, sizeof(double) * rows * md->H);
  w.dH = (double*)ws_take(ctx, sizeof(double) * rows * md->H);
  w.grad = (double*)ws_take(ctx, sizeof(double) * md->P);
  w.nll = (double*)ws_take(ctx, sizeof(double) * std::max(1, nll_slots));
  return w;
}

void refresh_masks(vmc_made* md) {
  const int64_t n = (int64_t)md->N * md->H;
  k_masks<<<grid_for(n, 256), 256, 0, md->ctx->stream>>>(md->params, md->N, md->H, md->W1m, md->W1mT, md->W2m);
  VMC_HIP(hipGetLastError());
}

// forward of rows [s, s + nb): X, A1 (biased), Hd, L (unbiased logits)
void forward(vmc_made* md, const uint64_t* s, int64_t nb, const made_ws& w) {
  vmc_ctx* ctx = md->ctx;
  const int N = md->N, H = md->H;
  k_unpack<<<grid_for(nb * N, 256), 256, 0, ctx->stream>>>(s, nb, N, md->W, w.X);
  dgemm(ctx, dgemm_args{w.X, N, 1, md->W1m, 1, N, w.A1, H, nb, H, N, 0.0});
  k_bias_relu<<<grid_for(nb * H, 256), 256, 0, ctx->stream>>>(w.A1, md->params + (int64_t)H * N, nb, H, w.Hd);
  dgemm(ctx, dgemm_args{w.Hd, H, 1, md->W2m, 1, H, w.L, N, nb, N, H, 0.0});
  VMC_HIP(hipGetLastError());
}

// gradient of the mean NLL over nb rows into w.grad; adds the mean NLL into *nll_slot
void backward(vmc_made* md, int64_t nb, const made_ws& w, double* nll_slot, double nll_scale) {
  vmc_ctx* ctx = md->ctx;
  const int N = md->N, H = md->H;
  const double* b2 = md->params + (int64_t)H * N + H + (int64_t)N * H;
  k_out_grad<<<grid_for(nb * N, 256), 256, 0, ctx->stream>>>(w.L, b2, w.X, nb, N, 1.0 / (double)nb, w.G, nll_slot);
  (void)nll_scale;
  double* gW1 = w.grad;
  double* gb1 = w.grad + (int64_t)H * N;
  double* gW2 = gb1 + H;
  double* gb2 = gW2 + (int64_t)N * H;
  dgemm(ctx, dgemm_args{w.G, 1, N, w.Hd, H, 1, gW2, H, N, H, nb, 0.0});
  dgemm(ctx, dgemm_args{w.G, N, 1, md->W2m, H, 1, w.dH, H, nb, H, N, 0.0});
  k_relu_mask<<<grid_for(nb * H, 256), 256, 0, ctx->stream>>>(w.dH, w.A1, nb * H);
  dgemm(ctx, dgemm_args{w.dH, 1, H, w.X, N, 1, gW1, N, H, N, nb, 0.0});
  k_mask_grad<<<grid_for((int64_t)N * H, 256), 256, 0, ctx->stream>>>(w.grad, N, H);
  k_colsum<<<grid_for(H, 16), 256, 0, ctx->stream>>>(w.dH, nb, H, gb1);
  k_colsum<<<grid_for(N, 16), 256, 0, ctx->stream>>>(w.G, nb, N, gb2);
  VMC_HIP(hipGetLastError());
}

void made_free(vmc_made* md) {
  for (double* p : {md->params, md->adam_m, md->adam_v, md->W1m, md->W1mT, md->W2m})
    if (p) (void)hipFree(p);
}

}  // namespace

void made_refresh(vmc_made* md) { refresh_masks(md); }

void made_sample_impl(vmc_made* md, int64_t B, uint64_t seed, uint64_t counter, uint64_t* s_out, double* logq) {
  const int QH = (md->H + 63) / 64;
  const uint2 key = make_uint2((uint32_t)seed, (uint32_t)(seed >> 32));
  const double* b1 = md->params + (int64_t)md->H * md->N;
  const double* b2 = b1 + md->H + (int64_t)md->N * md->H;
  hipStream_t st = md->ctx->stream;
  const uint32_t lo = (uint32_t)counter, hi = (uint32_t)(counter >> 32);
  if (md->H <= 64) {
    const unsigned g = (unsigned)((B + 63) / 64);
    if (md->H <= 32)
      k_made_sample_lane<32><<<g, 64, 0, st>>>(md->W1mT, md->W2m, b1, b2, md->N, md->H, md->W, B, key, lo, hi, s_out,
                                               logq);
    else
      k_made_sample_lane<64><<<g, 64, 0, st>>>(md->W1mT, md->W2m, b1, b2, md->N, md->H, md->W, B, key, lo, hi, s_out,
                                               logq);
    VMC_HIP(hipGetLastError());
    return;
  }
#define MADE_LAUNCH(Q) \
  k_made_sample<Q><<<(unsigned)B, 64, 0, st>>>(md->W1mT, md->W2m, b1, b2, md->N, md->H, md->W, B, key, lo, hi, s_out, logq)
  if (QH <= 1)
    MADE_LAUNCH(1);
  else if (QH <= 2)
    MADE_LAUNCH(2);
  else if (QH <= 4)
    MADE_LAUNCH(4);
  else if (QH <= 8)
    MADE_LAUNCH(8);
  else
    MADE_LAUNCH(16);
#undef MADE_LAUNCH
  VMC_HIP(hipGetLastError());
}

extern "C" int vmc_made_create(vmc_ctx* ctx, int n_in, int n_hidden, vmc_made** out) {
  return guard(ctx, [&] {
    VMC_REQUIRE(ctx && out, "NULL argument");
    VMC_REQUIRE(n_in >= 2 && n_in <= 4096, "n_in must be in [2, 4096]");
    VMC_REQUIRE(n_hidden >= 1 && n_hidden <= 1024, "n_hidden must be in [1, 1024]");
    VMC_HIP(hipSetDevice(ctx->device));
    auto* md = new vmc_made;
    md->ctx = ctx;
    md->N = n_in;
    md->H = n_hidden;
    md->W = (n_in + 63) / 64;
    md->P = 2ll * n_in * n_hidden + n_hidden + n_in;
    const size_t nh = sizeof(double) * (size_t)n_in * n_hidden;
    bool ok = hipMalloc(&md->params, sizeof(double) * md->P) == hipSuccess &&
              hipMalloc(&md->adam_m, sizeof(double) * md->P) == hipSuccess &&
              hipMalloc(&md->adam_v, sizeof(double) * md->P) == hipSuccess &&
              hipMalloc(&md->W1m, nh) == hipSuccess && hipMalloc(&md->W1mT, nh) == hipSuccess &&
              hipMalloc(&md->W2m, nh) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      made_free(md);
      delete md;
      throw vmc_error{VMC_ERR_OOM, "MADE allocation failed"};
    }
    VMC_HIP(hipMemsetAsync(md->params, 0, sizeof(double) * md->P, ctx->stream));
    VMC_HIP(hipMemsetAsync(md->adam_m, 0, sizeof(double) * md->P, ctx->stream));
    VMC_HIP(hipMemsetAsync(md->adam_v, 0, sizeof(double) * md->P, ctx->stream));
    refresh_masks(md);
    ctx_retain(ctx);
    *out = md;
  });
}

extern "C" int vmc_made_num_params(const vmc_made* md, int64_t* P) {
  if (!md || !P) return VMC_ERR_INVALID_ARG;
  *P = md->P;
  return VMC_OK;
}

extern "C" int vmc_made_set_params(vmc_made* md, const double* params_dev) {
  return guard(md ? md->ctx : nullptr, [&] {
    VMC_REQUIRE(md && params_dev, "NULL argument");
    VMC_HIP(hipSetDevice(md->ctx->device));
    VMC_HIP(hipMemcpyAsync(md->params, params_dev, sizeof(double) * md->P, hipMemcpyDeviceToDevice, md->ctx->stream));
    VMC_HIP(hipMemsetAsync(md->adam_m, 0, sizeof(double) * md->P, md->ctx->stream));
    VMC_HIP(hipMemsetAsync(md->adam_v, 0, sizeof(double) * md->P, md->ctx->stream));
    md->adam_t = 0;
    refresh_masks(md);
  });
}

extern "C" int vmc_made_get_params(const vmc_made* md, double* params_dev) {
  return guard(md ? md->ctx : nullptr, [&] {
    VMC_REQUIRE(md && params_dev, "NULL argument");
    VMC_HIP(hipSetDevice(md->ctx->device));
    VMC_HIP(hipMemcpyAsync(params_dev, md->params, sizeof(double) * md->P, hipMemcpyDeviceToDevice, md->ctx->stream));
  });
}

extern "C" int vmc_made_log_q(vmc_made* md, const uint64_t* s, int64_t B, double* logq) {
  return guard(md ? md->ctx : nullptr, [&] {
    VMC_REQUIRE(md, "NULL MADE");
    VMC_REQUIRE(B >= 0, "B < 0");
    if (B == 0) return;
    VMC_REQUIRE(s && logq, "NULL buffer");
    VMC_HIP(hipSetDevice(md->ctx->device));
    phase_scope ps(md->ctx, "made.log_q");
    const int64_t chunk = std::min<int64_t>(B, 1 << 16);
    ws_reserve(md->ctx, made_ws_bytes(md, chunk, 1));
    made_ws w = made_take(md, chunk, 1);
    const double* b2 = md->params + (int64_t)md->H * md->N + md->H + (int64_t)md->N * md->H;
    for (int64_t b0 = 0; b0 < B; b0 += chunk) {
      const int64_t nb = std::min(chunk, B - b0);
      forward(md, s + b0 * md->W, nb, w);
      k_logq_rows<<<(unsigned)nb, 64, 0, md->ctx->stream>>>(w.L, b2, w.X, nb, md->N, logq + b0);
    }
    VMC_HIP(hipGetLastError());
  });
}

extern "C" int vmc_made_nll_grad(vmc_made* md, const uint64_t* s, int64_t B, double* grad, double* nll_host) {
  return guard(md ? md->ctx : nullptr, [&] {
    VMC_REQUIRE(md, "NULL MADE");
    VMC_REQUIRE(B >= 1 && B <= (1 << 20), "B must be in [1, 2^20]");
    VMC_REQUIRE(s && grad, "NULL buffer");
    vmc_ctx* ctx = md->ctx;
    VMC_HIP(hipSetDevice(ctx->device));
    ws_reserve(ctx, made_ws_bytes(md, B, 1));
    made_ws w = made_take(md, B, 1);
    VMC_HIP(hipMemsetAsync(w.nll, 0, sizeof(double), ctx->stream));
    forward(md, s, B, w);
    backward(md, B, w, w.nll, 1.0);
    VMC_HIP(hipMemcpyAsync(grad, w.grad, sizeof(double) * md->P, hipMemcpyDeviceToDevice, ctx->stream));
    if (nll_host) {
      double* h = (double*)pinned_host(ctx, sizeof(double));
      VMC_HIP(hipMemcpyAsync(h, w.nll, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
      VMC_HIP(hipStreamSynchronize(ctx->stream));
      *nll_host = *h;
    }
  });
}

extern "C" int vmc_made_train(vmc_made* md, const uint64_t* s, int64_t B, int epochs, int batch, double lr,
                              double* nll_host) {
  return guard(md ? md->ctx : nullptr, [&] {
    VMC_REQUIRE(md, "NULL MADE");
    VMC_REQUIRE(B >= 1 && epochs >= 1 && batch >= 1 && batch <= (1 << 16), "bad training sizes");
    VMC_REQUIRE(std::isfinite(lr) && lr > 0, "lr must be positive");
    VMC_REQUIRE(s, "NULL samples");
    vmc_ctx* ctx = md->ctx;
    VMC_HIP(hipSetDevice(ctx->device));
    phase_scope ps(ctx, "made.train");
    const int64_t bs = std::min<int64_t>(batch, B);
    ws_reserve(ctx, made_ws_bytes(md, bs, epochs));
    made_ws w = made_take(md, bs, epochs);
    VMC_HIP(hipMemsetAsync(w.nll, 0, sizeof(double) * epochs, ctx->stream));
    const int64_t nmb = (B + bs - 1) / bs;
    for (int ep = 0; ep < epochs; ++ep) {
      for (int64_t b0 = 0; b0 < B; b0 += bs) {
        const int64_t nb = std::min(bs, B - b0);
        forward(md, s + b0 * md->W, nb, w);
        backward(md, nb, w, w.nll + ep, 1.0);
        md->adam_t += 1;
        const double bc1 = 1.0 - std::pow(0.9, (double)md->adam_t);
        const double bc2 = 1.0 - std::pow(0.999, (double)md->adam_t);
        k_adam<<<grid_for(md->P, 256), 256, 0, ctx->stream>>>(md->params, w.grad, md->adam_m, md->adam_v, md->P, lr,
                                                              bc1, bc2);
        refresh_masks(md);
      }
    }
    VMC_HIP(hipGetLastError());
    if (nll_host) {
      double* h = (double*)pinned_host(ctx, sizeof(double));
      VMC_HIP(hipMemcpyAsync(h, w.nll + epochs - 1, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
      VMC_HIP(hipStreamSynchronize(ctx->stream));
      *nll_host = *h / (double)nmb;
    }
  });
}

extern "C" int vmc_made_sample(vmc_made* md, int64_t B, uint64_t seed, uint64_t counter, uint64_t* s_out,
                               double* logq) {
  return guard(md ? md->ctx : nullptr, [&] {
    VMC_REQUIRE(md, "NULL MADE");
    VMC_REQUIRE(B >= 0 && B <= ((int64_t)1 << 31) - 1, "B out of range");
    if (B == 0) return;
    VMC_REQUIRE(s_out, "NULL s_out");
    VMC_REQUIRE(md->W <= 64, "up to 4096 sites");
    VMC_HIP(hipSetDevice(md->ctx->device));
    phase_scope ps(md->ctx, "made.sample");
    made_sample_impl(md, B, seed, counter, s_out, logq);
  });
}

extern "C" int vmc_made_destroy(vmc_made* md) {
  if (!md) return VMC_ERR_INVALID_ARG;
  (void)hipSetDevice(md->ctx->device);
  (void)hipStreamSynchronize(md->ctx->stream);
  made_free(md);
  vmc_ctx* ctx = md->ctx;
  delete md;
  ctx_release(ctx);
  return VMC_OK;
}
