// Measurement utilities: a plain device copy (HBM bandwidth, and the byte
// count that hardware traffic counters read for a known transfer) and
// matrix-core loops (sustained MFMA rate per data type).  Not part of the
// method; the rooflines of the hot-path kernels are quoted against both the
// nominal peaks and these measured ones.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// 16-byte vector copy, grid-stride
__global__ __launch_bounds__(256) void k_calib_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                    int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

// Each wave runs `iters` rounds of 8 independent MFMA chains; the sum of the
// accumulators is written so the work cannot be removed.
__global__ __launch_bounds__(256) void k_calib_mfma_f32(int iters, float* __restrict__ out) {
  const float a = 1e-3f * (threadIdx.x & 7), b = 1e-3f;
  floatx4 acc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int i = 0; i < iters; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[j], 0, 0, 0);
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < 8; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_calib_mfma_f64(int iters, double* __restrict__ out) {
  const double a = 1e-3 * (threadIdx.x & 7), b = 1e-3;
  doublex4 acc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] = doublex4{0.0, 0.0, 0.0, 0.0};
  for (int i = 0; i < iters; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < 8; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_calib_mfma_bf16(int iters, float* __restrict__ out) {
  bf16x8 a, b;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    a[q] = (__bf16)(1e-3f * ((threadIdx.x + q) & 7));
    b[q] = (__bf16)1e-3f;
  }
  floatx4 acc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int i = 0; i < iters; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < 8; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

}  // namespace

extern "C" int vmc_calib_copy(vmc_ctx* ctx, const void* src, void* dst, int64_t bytes) {
  return guard(ctx, [&] {
    VMC_REQUIRE(ctx && src && dst, "NULL argument");
    VMC_REQUIRE(bytes > 0 && bytes % 16 == 0, "bytes must be a positive multiple of 16");
    VMC_REQUIRE(((uintptr_t)src | (uintptr_t)dst) % 16 == 0, "buffers must be 16-byte aligned");
    set_device(ctx);
    phase_scope ps(ctx, "calib.copy");
    const int64_t n16 = bytes / 16;
    const int64_t blocks = std::min<int64_t>((n16 + 255) / 256, 256 * 64);
    k_calib_copy<<<(unsigned)blocks, 256, 0, ctx->stream>>>((const uint4*)src, (uint4*)dst, n16);
    VMC_HIP(hipGetLastError());
  });
}

extern "C" int vmc_calib_mfma(vmc_ctx* ctx, int kind, int n_groups, int iters, void* out, double* flops_host) {
  return guard(ctx, [&] {
    VMC_REQUIRE(ctx && out && flops_host, "NULL argument");
    VMC_REQUIRE(n_groups >= 1 && n_groups <= 65536 && iters >= 1, "n_groups in [1, 65536], iters >= 1");
    set_device(ctx);
    phase_scope ps(ctx, "calib.mfma");
    // flops per MFMA: 2 M N K; 8 chains per wave, 4 waves per group
    const double per = kind == VMC_DT_F64 ? 2.0 * 16 * 16 * 4 : kind == VMC_DT_F32 ? 2.0 * 16 * 16 * 4
                                                                                      : 2.0 * 16 * 16 * 32;
    if (kind == VMC_DT_F64)
      k_calib_mfma_f64<<<(unsigned)n_groups, 256, 0, ctx->stream>>>(iters, (double*)out);
    else if (kind == VMC_DT_F32)
      k_calib_mfma_f32<<<(unsigned)n_groups, 256, 0, ctx->stream>>>(iters, (float*)out);
    else if (kind == VMC_CALIB_BF16)
      k_calib_mfma_bf16<<<(unsigned)n_groups, 256, 0, ctx->stream>>>(iters, (float*)out);
    else
      throw vmc_error{VMC_ERR_INVALID_ARG, "kind must be VMC_DT_F64, VMC_DT_F32 or VMC_CALIB_BF16"};
    VMC_HIP(hipGetLastError());
    *flops_host = per * 8.0 * 4.0 * (double)n_groups * (double)iters;
  });
}
