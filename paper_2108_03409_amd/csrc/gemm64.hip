// Real float64 GEMM on the matrix cores with arbitrary strides:
//   C[m][n] = beta * C[m][n] + sum_k A(m, k) B(k, n),
//   A(m, k) = A[m * sam + k * sak],  B(k, n) = B[k * sbk + n * sbn].
// 64 x 64 output tile per 256-thread group (2 x 2 waves of 32 x 32, each
// 2 x 2 blocks of v_mfma_f64_16x16x4), the reduction staged 16 deep through
// two LDS buffers: the next stage's global loads are issued into registers
// before the current stage is used.  Loads are coalesced along whichever
// stride of each operand is 1.
// Split-K (nsplit > 1): grid z reduces over its own range of k and writes its
// own C slice (C + z cz); the caller adds the slices.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_dgemm(dgemm_args g) {
  __shared__ double As[2][16][65];
  __shared__ double Bs[2][16][65];
  const int64_t m0 = (int64_t)blockIdx.y * 64, n0 = (int64_t)blockIdx.x * 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int li = lane & 15, lk = lane >> 4;
  doublex4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
  const bool a_k_fast = g.sak == 1;
  const bool b_n_fast = g.sbn == 1;
  const int64_t kz0 = (int64_t)blockIdx.z * g.kchunk;
  const int64_t kz1 = g.kchunk ? min(g.K, kz0 + g.kchunk) : g.K;
  double* const Cz = g.C + (int64_t)blockIdx.z * g.cz;
  // the stage at k0: element q = tid + 256 j of the 64 x 16 A and 16 x 64 B tiles
  // (along whichever stride of the operand is 1), read into registers; the next
  // stage's loads are in flight while the current one is used from LDS
  double ra[4], rb[4];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = tid + 256 * j;
      const int mm = a_k_fast ? q >> 4 : q & 63, kk = a_k_fast ? q & 15 : q >> 6;
      const int64_t m = m0 + mm, k = k0 + kk;
      ra[j] = (m < g.M && k < kz1) ? g.A[m * g.sam + k * g.sak] : 0.0;
      const int nn = b_n_fast ? q & 63 : q >> 4, kb = b_n_fast ? q >> 6 : q & 15;
      const int64_t n = n0 + nn, kq = k0 + kb;
      rb[j] = (n < g.N && kq < kz1) ? g.B[kq * g.sbk + n * g.sbn] : 0.0;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = tid + 256 * j;
      As[buf][a_k_fast ? q & 15 : q >> 6][a_k_fast ? q >> 4 : q & 63] = ra[j];
      Bs[buf][b_n_fast ? q >> 6 : q & 15][b_n_fast ? q & 63 : q >> 4] = rb[j];
    }
  };
  if (kz0 < kz1) {
    gload(kz0);
    sstore(0);
  }
  __syncthreads();
  int buf = 0;
  for (int64_t k0 = kz0; k0 < kz1; k0 += 16) {
    const bool more = k0 + 16 < kz1;
    if (more) gload(k0 + 16);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int kk = ks * 4 + lk;
      double fa[2], fb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) fa[i] = As[buf][kk][wr * 32 + i * 16 + li];
#pragma unroll
      for (int j = 0; j < 2; ++j) fb[j] = Bs[buf][kk][wc * 32 + j * 16 + li];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
    if (more) sstore(buf ^ 1);  // the other buffer: its last readers passed the previous barrier
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // float64 accumulator layout: register r of lane l holds D[l/16 + 4r][l%16]
        const int64_t m = m0 + wr * 32 + i * 16 + lk + 4 * r;
        const int64_t n = n0 + wc * 32 + j * 16 + li;
        if (m < g.M && n < g.N) {
          double* c = Cz + m * g.ldc + n;
          *c = (g.beta == 0.0 ? 0.0 : g.beta * *c) + acc[i][j][r];
        }
      }
}

}  // namespace

void dgemm(vmc_ctx* ctx, const dgemm_args& g, int nsplit) {
  if (g.M <= 0 || g.N <= 0) return;
  dim3 grid((unsigned)((g.N + 63) / 64), (unsigned)((g.M + 63) / 64), (unsigned)std::max(1, nsplit));
  k_dgemm<<<grid, 256, 0, ctx->stream>>>(g);
  VMC_HIP(hipGetLastError());
}
