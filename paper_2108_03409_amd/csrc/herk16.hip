// S = Obar^H Obar from split float16 products on the matrix cores.
//
// Each float32 value x of the centred Obar is scaled by a power of two 2^e_k
// per complex column k (so that the column maximum lies in [2^13, 2^14)) and
// written as x 2^e_k = hi + lo with hi = fp16(x 2^e_k), lo = fp16(x 2^e_k - hi):
// 22 significant bits.  Products use three terms, hi hi' + hi lo' + lo hi'
// (the dropped lo lo' and the split residuals are below 2^-21 relative), on
// v_mfma_f32_16x16x32_f16 with float32 accumulation, and the epilogue removes
// the scale 2^-(e_k + e_k').  Relative to the float32 Gram this is 3 x 2.5
// PFLOP/s-class products instead of 157 TFLOP/s-class ones.
//
// Layout for the matrix cores: the reduction runs over samples, so the split
// data are stored column-major in groups of 8 samples: for column k and sample
// group g, 4 x 8 halves [re_hi, re_lo, im_hi, im_lo] (64 bytes), which is one
// lane's fragment set.  The Gram kernel stages 128 + 128 columns x 32 samples
// of these sets in LDS per step (see k_herk16).
#include <hip/hip_runtime.h>

#include "internal.h"

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

// column maxima of |Re|, |Im| (as float bits; values are non-negative)
__global__ __launch_bounds__(256) void k_colmax(const float2* __restrict__ X, int64_t N, int64_t K,
                                                unsigned* __restrict__ cmax) {
  const int64_t k = blockIdx.x * 256ll + threadIdx.x;
  if (k >= K) return;
  const int64_t n0 = (int64_t)blockIdx.y * 256, n1 = min(N, n0 + 256);
  float m = 0.f;
  for (int64_t n = n0; n < n1; ++n) {
    const float2 v = X[n * K + k];
    m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
  }
  atomicMax(cmax + k, __float_as_uint(m));
}

// scale exponents: column max * 2^e in [2^13, 2^14)
__global__ void k_colscale(const unsigned* __restrict__ cmax, int64_t K, int* __restrict__ ex) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= K) return;
  const float m = __uint_as_float(cmax[k]);
  int e = 0;
  if (m > 0.f) {
    int em;
    frexpf(m, &em);  // m in [2^(em-1), 2^em)
    e = 14 - em;
  }
  ex[k] = e;
}

// split + transpose through LDS: tile of 64 samples x 64 columns
__global__ __launch_bounds__(256) void k_split16(const float2* __restrict__ X, int64_t N, int64_t K,
                                                 const int* __restrict__ ex, int64_t ngroups,
                                                 halfx8* __restrict__ H) {
  __shared__ float2 tile[64][65];
  const int64_t n0 = (int64_t)blockIdx.y * 64, k0 = (int64_t)blockIdx.x * 64;
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * 64; e += 256) {
    const int nn = e >> 6, kk = e & 63;
    const int64_t n = n0 + nn, k = k0 + kk;
    tile[nn][kk] = (n < N && k < K) ? X[n * K + k] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  // 64 columns x 8 groups of 8 samples = 512 fragment sets; two per thread
  for (int e = tid; e < 64 * 8; e += 256) {
    const int kk = e >> 3, gg = e & 7;
    const int64_t k = k0 + kk, g = n0 / 8 + gg;
    if (k >= K || g >= ngroups) continue;
    const float sc = ldexpf(1.f, ex[k]);
    halfx8 rh, rl, ih, il;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const float2 v = tile[gg * 8 + q][kk];
      const float xr = v.x * sc, xi = v.y * sc;
      const _Float16 hr = (_Float16)xr, hi = (_Float16)xi;
      rh[q] = hr;
      rl[q] = (_Float16)(xr - (float)hr);
      ih[q] = hi;
      il[q] = (_Float16)(xi - (float)hi);
    }
    halfx8* dst = H + (k * ngroups + g) * 4;
    dst[0] = rh;
    dst[1] = rl;
    dst[2] = ih;
    dst[3] = il;
  }
}

struct h16_args {
  const halfx8* H;  // [K][ngroups][4]
  const int* ex;
  int64_t ngroups, K;
  int mode;
  double nu, eps;
  double2* S;
  double2* diag;
  int64_t n_tiles;
};

constexpr int TB = 128;  // tile edge (complex rows = columns)

// 128 x 128 complex tile per 256-thread group (2 x 2 waves of 64 x 64, i.e.
// 4 x 4 blocks of 16 x 16 per wave).  Each stage covers 32 samples (4 groups
// of 8): the group stores the 128 + 128 columns' fragments (32 KB + 32 KB) in
// LDS and every wave reads its fragments from there, so each value is fetched
// from memory once per tile and stage.  The next stage's values are loaded
// into registers while the current one is multiplied.
__global__ __launch_bounds__(256, 1) void k_herk16(h16_args a) {
  __shared__ halfx8 As[TB * 4 * 4];  // [col][group][Rh, Rl, Ih, Il]
  __shared__ halfx8 Bs[TB * 4 * 4];
  const int64_t nb = a.n_tiles;
  const int64_t per = (nb + 7) / 8;
  const int64_t lin = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (lin >= nb) return;
  int tr = (int)((sqrt(8.0 * (double)lin + 1.0) - 1.0) * 0.5);
  while ((int64_t)(tr + 1) * (tr + 2) / 2 <= lin) ++tr;
  while ((int64_t)tr * (tr + 1) / 2 > lin) --tr;
  const int tc = (int)(lin - (int64_t)tr * (tr + 1) / 2);
  const int64_t row0 = (int64_t)tr * TB, col0 = (int64_t)tc * TB;
  const int64_t K = a.K;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int li = lane & 15, lk = lane >> 4;
  floatx4 acc[4][4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[i][j][0] = floatx4{0.f, 0.f, 0.f, 0.f};
      acc[i][j][1] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
  const halfx8 z = {0, 0, 0, 0, 0, 0, 0, 0};
  // 128 columns x 4 groups x 4 vectors = 2048 vectors per operand, 8 per thread
  halfx8 pa[8], pb[8];
  auto gload = [&](int64_t g0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int id = tid + 256 * q;
      const int col = id >> 4, gg = (id >> 2) & 3, v = id & 3;
      const int64_t g = g0 + gg;
      const int64_t ka = row0 + col, kb = col0 + col;
      pa[q] = (ka < K && g < a.ngroups) ? a.H[(ka * a.ngroups + g) * 4 + v] : z;
      pb[q] = (kb < K && g < a.ngroups) ? a.H[(kb * a.ngroups + g) * 4 + v] : z;
    }
  };
  gload(0);
  for (int64_t g0 = 0; g0 < a.ngroups; g0 += 4) {
    __syncthreads();  // previous stage's fragments are consumed
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      As[tid + 256 * q] = pa[q];
      Bs[tid + 256 * q] = pb[q];
    }
    __syncthreads();
    if (g0 + 4 < a.ngroups) gload(g0 + 4);
    halfx8 A[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int col = wr * 64 + i * 16 + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) A[i][v] = As[(col * 4 + lk) * 4 + v];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = wc * 64 + j * 16 + li;
      halfx8 Bf[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) Bf[v] = Bs[(col * 4 + lk) * 4 + v];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const halfx8 nih = -A[i][2], nil = -A[i][3];
        // re += re re' + im im',  im += re im' - im re';  each product hi hi + hi lo + lo hi
#define P3(acc_, xh, xl, y)                                                        \
  acc_ = __builtin_amdgcn_mfma_f32_16x16x32_f16(xh, Bf[y], acc_, 0, 0, 0);         \
  acc_ = __builtin_amdgcn_mfma_f32_16x16x32_f16(xh, Bf[y + 1], acc_, 0, 0, 0);     \
  acc_ = __builtin_amdgcn_mfma_f32_16x16x32_f16(xl, Bf[y], acc_, 0, 0, 0);
        P3(acc[i][j][0], A[i][0], A[i][1], 0);
        P3(acc[i][j][0], A[i][2], A[i][3], 2);
        P3(acc[i][j][1], A[i][0], A[i][1], 2);
        P3(acc[i][j][1], nih, nil, 0);
#undef P3
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t k = row0 + wr * 64 + i * 16 + 4 * lk + r;
        const int64_t kp = col0 + wc * 64 + j * 16 + li;
        if (k >= K || kp >= K || kp > k) continue;
        const double sc = ldexp(1.0, -(a.ex[k] + a.ex[kp]));
        double re = (double)acc[i][j][0][r] * sc;
        double im = (double)acc[i][j][1][r] * sc;
        if (a.mode == VMC_SR_REAL) im = 0.0;
        if (a.mode == VMC_SR_IMAG) re = 0.0;  // i Im S
        if (k == kp) {
          const double2 d = make_double2(re * (1.0 + a.nu) + a.eps, 0.0);
          a.diag[k] = d;
          a.S[k * K + k] = d;
        } else {
          a.S[k * K + kp] = make_double2(re, im);
          a.S[kp * K + k] = make_double2(re, -im);
        }
      }
}

}  // namespace

size_t herk16_ws_bytes(int64_t N, int64_t K) {
  const int64_t ng = (N + 7) / 8;
  return ws_round(sizeof(_Float16) * 32 * (size_t)ng * K) + ws_round(sizeof(unsigned) * K) + ws_round(sizeof(int) * K);
}

void herk_split16(vmc_ctx* ctx, const float2* X, int64_t N, int64_t K, int mode, double nu, double eps, double2* S,
                  double2* diag, void* ws) {
  hipStream_t st = ctx->stream;
  const int64_t ng = (N + 7) / 8;
  char* p = (char*)ws;
  halfx8* H = (halfx8*)p;
  p += ws_round(sizeof(_Float16) * 32 * (size_t)ng * K);
  unsigned* cmax = (unsigned*)p;
  p += ws_round(sizeof(unsigned) * K);
  int* ex = (int*)p;
  VMC_HIP(hipMemsetAsync(cmax, 0, sizeof(unsigned) * K, st));
  k_colmax<<<dim3(grid_for(K, 256), (unsigned)((N + 255) / 256)), 256, 0, st>>>(X, N, K, cmax);
  k_colscale<<<grid_for(K, 256), 256, 0, st>>>(cmax, K, ex);
  k_split16<<<dim3((unsigned)((K + 63) / 64), (unsigned)((N + 63) / 64)), 256, 0, st>>>(X, N, K, ex, ng, H);
  h16_args a{};
  a.H = H;
  a.ex = ex;
  a.ngroups = ng;
  a.K = K;
  a.mode = mode;
  a.nu = nu;
  a.eps = eps;
  a.S = S;
  a.diag = diag;
  const int64_t rt = (K + TB - 1) / TB;
  a.n_tiles = rt * (rt + 1) / 2;  // lower-triangle tiles, diagonal included
  k_herk16<<<(unsigned)(((a.n_tiles + 7) / 8) * 8), 256, 0, st>>>(a);
  VMC_HIP(hipGetLastError());
}
