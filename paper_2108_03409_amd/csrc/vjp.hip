// Vector-Jacobian product of log psi for reverse-mode autodiff:
//   out_k = sum_n g_n conj(O_nk),   O_nk = d log psi(s_n) / d theta_k,
// the backward of a holomorphic map in the conjugate-Wirtinger convention.
// O is recomputed chunk by chunk by the model's gradient kernels (no
// activations are kept between forward and backward) and reduced in float64.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"

using namespace dev;

namespace {

constexpr int kRows = 256;  // samples per partial sum

__global__ __launch_bounds__(256) void k_vjp_partial(const double2* __restrict__ O, const double2* __restrict__ g,
                                                     int64_t B, int64_t K, double2* __restrict__ part) {
  const int64_t k = blockIdx.x * 256ll + threadIdx.x;
  if (k >= K) return;
  const int64_t n0 = (int64_t)blockIdx.y * kRows, n1 = min(B, n0 + kRows);
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t n = n0; n < n1; ++n) acc = cadd(acc, cmul(g[n], cconj(O[n * K + k])));
  part[(int64_t)blockIdx.y * K + k] = acc;
}

__global__ void k_vjp_finish(const double2* __restrict__ part, int np, int64_t K, double2* __restrict__ out,
                             int accumulate) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= K) return;
  double2 acc = accumulate ? out[k] : make_double2(0.0, 0.0);
  for (int q = 0; q < np; ++q) acc = cadd(acc, part[(int64_t)q * K + k]);
  out[k] = acc;
}

}  // namespace

void log_psi_vjp_impl(vmc_model* m, const uint64_t* s, int64_t B, const double2* g, double2* out) {
  vmc_ctx* ctx = m->ctx;
  const int64_t K = m->K;
  const int64_t chunk = std::max<int64_t>(kRows, std::min<int64_t>(B, ((int64_t)1 << 30) / (16 * K) / kRows * kRows));
  const int np = (int)((chunk + kRows - 1) / kRows);
  // the gradient kernels carve their own scratch from the arena, so O and the
  // partial sums live in a separate allocation owned by this call
  void* buf = nullptr;
  const size_t obytes = sizeof(double2) * (size_t)chunk * K, pbytes = sizeof(double2) * (size_t)np * K;
  VMC_HIP(hipMalloc(&buf, obytes + pbytes));
  double2* O = (double2*)buf;
  double2* part = (double2*)((char*)buf + obytes);
  try {
    for (int64_t b0 = 0; b0 < B; b0 += chunk) {
      const int64_t nb = std::min(chunk, B - b0);
      if (m->kind == MODEL_RBM)
        rbm_grad(m, s + b0 * m->W, nb, O, VMC_DT_C128);
      else
        cnn_grad(m, s + b0 * m->W, nb, O, VMC_DT_C128);
      const int npp = (int)((nb + kRows - 1) / kRows);
      k_vjp_partial<<<dim3(grid_for(K, 256), npp), 256, 0, ctx->stream>>>(O, g + b0, nb, K, part);
      k_vjp_finish<<<grid_for(K, 256), 256, 0, ctx->stream>>>(part, npp, K, out, b0 > 0);
      VMC_HIP(hipGetLastError());
    }
  } catch (...) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(buf);
    throw;
  }
  VMC_HIP(hipStreamSynchronize(ctx->stream));
  VMC_HIP(hipFree(buf));
}
