// Vector-Jacobian product of log psi for reverse-mode autodiff:
//   out_k = sum_n g_n conj(O_nk),   O_nk = d log psi(s_n) / d theta_k,
// the backward of a holomorphic map in the conjugate-Wirtinger convention.
// Nothing of the forward pass is kept; and O itself is never stored:
//
//  RBM: with U_nj = g_n conj(tanh theta_nj) and sigma_ni = +-1,
//         out_W[j][i] = sum_n U_nj sigma_ni,  out_b[j] = sum_n U_nj,
//         out_a[i]    = sum_n g_n sigma_ni,
//       i.e. one product [N_h + 1 rows: U and g] x [N + 1 columns: sigma and
//       1] over the samples, two real float64 matrix-core GEMMs (Re and Im of
//       U) split over sample ranges, the slices added in a fixed order.
//  CNN: the gradient kernel recomputes both layers per sample and each
//       work-group accumulates g_n conj(O_n) over its samples into one row of
//       partial sums, which a second kernel adds in a fixed order.
//
// Scratch: the context's workspace (vmc_log_psi_vjp), or, for callers that
// cannot allocate, a fixed device array owned by this file
// (vmc_log_psi_vjp_noalloc).  Either way the work is chunked over samples to
// fit the scratch it is given.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "internal.h"

using namespace dev;

namespace {

constexpr int kSplit = 32;     // sample ranges of the RBM product
constexpr int kCnnGroups = 256;  // work-groups (partial rows) of the CNN product

// U'[n][j] = g_n conj(tanh theta_nj) (j < N_h), U'[n][N_h] = g_n; S'[n][i] = sigma_ni (i < N), S'[n][N] = 1.
__global__ __launch_bounds__(256) void k_vjp_rbm_prep(const double2* __restrict__ theta, const uint64_t* __restrict__ s,
                                                      const double2* __restrict__ g, int64_t B, int N, int W, int Nh,
                                                      double2* __restrict__ U, double* __restrict__ Sg) {
  const int64_t n = blockIdx.x;
  if (n >= B) return;
  const double2 gn = g[n];
  const uint64_t* sn = s + n * W;
  for (int j = threadIdx.x; j <= Nh; j += 256)
    U[n * (Nh + 1) + j] = j < Nh ? cmul(gn, cconj(ctanh(theta[n * Nh + j]))) : gn;
  for (int i = threadIdx.x; i <= N; i += 256) Sg[n * (N + 1) + i] = i < N ? (get_bit(sn, i) ? 1.0 : -1.0) : 1.0;
}

// out from the kSplit slices of C_re, C_im ([N_h + 1][N + 1] each): fixed order
__global__ void k_vjp_rbm_out(const double* __restrict__ Cre, const double* __restrict__ Cim, int N, int Nh,
                              int64_t slice, int nsplit, double2* __restrict__ out) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t K = (int64_t)N + Nh + (int64_t)Nh * N;
  if (e >= K) return;
  int64_t c;  // entry of the [N_h + 1][N + 1] product
  if (e < N)
    c = (int64_t)Nh * (N + 1) + e;  // a_i: row of g
  else if (e < N + Nh)
    c = (e - N) * (N + 1) + N;  // b_j: column of ones
  else {
    const int64_t r = e - N - Nh;  // W[j][i]
    c = (r / N) * (N + 1) + r % N;
  }
  double re = 0.0, im = 0.0;
  for (int z = 0; z < nsplit; ++z) {
    re += Cre[z * slice + c];
    im += Cim[z * slice + c];
  }
  out[e] = make_double2(re, im);
}

__global__ void k_zero2(double2* __restrict__ out, int64_t K) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < K) out[k] = make_double2(0.0, 0.0);
}

__global__ void k_vjp_rows(const double2* __restrict__ part, int rows, int64_t K, double2* __restrict__ out) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= K) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int q = 0; q < rows; ++q) acc = cadd(acc, part[(int64_t)q * K + k]);
  out[k] = acc;
}

// bytes of the fixed part of the RBM scratch, and per sample of a chunk
size_t rbm_fixed_bytes(const vmc_model* m) {
  return ws_round(sizeof(double) * 2 * (size_t)kSplit * (m->Nh + 1) * (m->N + 1));
}
size_t rbm_per_sample_bytes(const vmc_model* m) {
  return sizeof(double2) * (size_t)m->Nh + sizeof(double2) * (m->Nh + 1) + sizeof(double) * (m->N + 1);
}

void vjp_rbm(vmc_model* m, const uint64_t* s, int64_t B, const double2* g, double2* out, char* scratch,
             size_t bytes) {
  vmc_ctx* ctx = m->ctx;
  const int N = m->N, Nh = m->Nh;
  const size_t fixed = rbm_fixed_bytes(m);
  const int64_t chunk =
      std::min<int64_t>(B, (int64_t)((bytes - fixed - 3 * 256) / rbm_per_sample_bytes(m)));
  const int64_t slice = (int64_t)(Nh + 1) * (N + 1);
  double* Cre = (double*)scratch;
  double* Cim = Cre + (size_t)kSplit * slice;
  char* p = scratch + fixed;
  double2* theta = (double2*)p;
  p += ws_round(sizeof(double2) * (size_t)chunk * Nh);
  double2* U = (double2*)p;
  p += ws_round(sizeof(double2) * (size_t)chunk * (Nh + 1));
  double* Sg = (double*)p;
  for (int64_t b0 = 0; b0 < B; b0 += chunk) {
    const int64_t nb = std::min(chunk, B - b0);
    rbm_theta(m, s + b0 * m->W, nb, theta);
    k_vjp_rbm_prep<<<(unsigned)nb, 256, 0, ctx->stream>>>(theta, s + b0 * m->W, g + b0, nb, N, m->W, Nh, U, Sg);
    VMC_HIP(hipGetLastError());
    const int64_t kc = (nb + kSplit - 1) / kSplit;
    const double beta = b0 == 0 ? 0.0 : 1.0;
    // C[j][i] (+)= sum_n A(j, n) Sg[n][i], A = Re U' / Im U' read in place (stride 2 doubles)
    dgemm_args re{(const double*)U, 2, 2 * (int64_t)(Nh + 1), Sg, N + 1, 1, Cre, N + 1, Nh + 1, N + 1, nb, beta,
                  kc, slice};
    dgemm_args im = re;
    im.A = (const double*)U + 1;
    im.C = Cim;
    dgemm(ctx, re, kSplit);
    dgemm(ctx, im, kSplit);
  }
  const int64_t K = m->K;
  k_vjp_rbm_out<<<grid_for(K, 256), 256, 0, ctx->stream>>>(Cre, Cim, N, Nh, slice, kSplit, out);
  VMC_HIP(hipGetLastError());
}

void vjp_cnn(vmc_model* m, const uint64_t* s, int64_t B, const double2* g, double2* out, char* scratch,
             size_t bytes) {
  vmc_ctx* ctx = m->ctx;
  const int64_t K = m->K;
  const int groups = (int)std::min<int64_t>({B, (int64_t)kCnnGroups, (int64_t)(bytes / (sizeof(double2) * K))});
  double2* part = (double2*)scratch;
  cnn_vjp_partial(m, s, B, g, groups, part);
  k_vjp_rows<<<grid_for(K, 256), 256, 0, ctx->stream>>>(part, groups, K, out);
  VMC_HIP(hipGetLastError());
}

void vjp_run(vmc_model* m, const uint64_t* s, int64_t B, const double2* g, double2* out, char* scratch,
             size_t bytes) {
  if (m->kind == MODEL_RBM)
    vjp_rbm(m, s, B, g, out, scratch, bytes);
  else
    vjp_cnn(m, s, B, g, out, scratch, bytes);
}

// the smallest scratch that lets a model run (one sample per chunk / one partial row)
size_t min_scratch(const vmc_model* m) {
  if (m->kind == MODEL_RBM) return rbm_fixed_bytes(m) + 3 * 256 + rbm_per_sample_bytes(m);
  return sizeof(double2) * (size_t)m->K;
}

// ---- fixed scratch for callers that cannot allocate ------------------------
constexpr size_t kNoAllocBytes = (size_t)32 << 20;  // 32 MiB per device
__device__ __align__(256) char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

// Device address of `scratch` on the current device, looked up once per device
// with that device current (each device holds its own copy of the array; in
// host code the array's name is only a stand-in, never a device address).
char* noalloc_scratch() {
  int dev = 0;
  VMC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) throw vmc_error{VMC_ERR_UNSUPPORTED, "device index above 63"};
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    VMC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = p;
  }
  return (char*)g_scratch_ptr[dev];
}

}  // namespace

void log_psi_vjp_impl(vmc_model* m, const uint64_t* s, int64_t B, const double2* g, double2* out) {
  vmc_ctx* ctx = m->ctx;
  if (B == 0) {
    k_zero2<<<grid_for(m->K, 256), 256, 0, ctx->stream>>>(out, m->K);
    VMC_HIP(hipGetLastError());
    return;
  }
  size_t bytes;
  if (m->kind == MODEL_RBM) {
    const int64_t chunk = std::min<int64_t>(B, 65536);
    bytes = rbm_fixed_bytes(m) + 3 * 256 + (size_t)chunk * rbm_per_sample_bytes(m);
  } else {
    bytes = sizeof(double2) * (size_t)std::min<int64_t>(B, kCnnGroups) * m->K;
  }
  bytes = ws_round(bytes);
  ws_reserve(ctx, bytes);
  char* ws = (char*)ws_take(ctx, bytes);
  vjp_run(m, s, B, g, out, ws, bytes);
}

void log_psi_vjp_noalloc_impl(vmc_model* m, const uint64_t* s, int64_t B, const double2* g, double2* out) {
  const size_t need = min_scratch(m);
  if (need > kNoAllocBytes)
    throw vmc_error{VMC_ERR_WORKSPACE, "model needs " + std::to_string(need) + " bytes of scratch; the fixed " +
                                           "no-allocation scratch holds " + std::to_string(kNoAllocBytes)};
  char* sc = noalloc_scratch();
  if (B == 0) {
    k_zero2<<<grid_for(m->K, 256), 256, 0, m->ctx->stream>>>(out, m->K);
    VMC_HIP(hipGetLastError());
    return;
  }
  vjp_run(m, s, B, g, out, sc, kNoAllocBytes);
}
