// Measurement utilities: a plain device copy (HBM bandwidth, and the byte
// count that hardware traffic counters read for a known transfer) and
// matrix-core loops (sustained MFMA rate per data type).  Not part of the
// method; the rooflines of the hot-path kernels are quoted against both the
// nominal peaks and these measured ones.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace {

constexpr int kCalibReadGroups = 256 * 32;

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// 16-byte vector copy, grid-stride
__global__ __launch_bounds__(256) void k_calib_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                    int64_t n16) {
  // four 16-byte loads in flight per thread per round
  const int64_t stride = (int64_t)gridDim.x * 256;
  int64_t i = blockIdx.x * 256ll + threadIdx.x;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    dst[i] = a;
    dst[i + stride] = b;
    dst[i + 2 * stride] = c;
    dst[i + 3 * stride] = d;
  }
  for (; i < n16; i += stride) dst[i] = src[i];
}

// Read-only stream: every 16-byte word is loaded once (four loads in flight per
// thread per round) and folded with xor; one word per group is written.
__global__ __launch_bounds__(256) void k_calib_read(const uint4* __restrict__ src, int64_t n16,
                                                    uint4* __restrict__ out) {
  __shared__ uint4 red[4];
  const int64_t stride = (int64_t)gridDim.x * 256;
  int64_t i = blockIdx.x * 256ll + threadIdx.x;
  uint4 acc = make_uint4(0u, 0u, 0u, 0u);
  for (; i + 3 * stride < n16; i += 4 * stride) {
    const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    acc.x ^= a.x ^ b.x ^ c.x ^ d.x;
    acc.y ^= a.y ^ b.y ^ c.y ^ d.y;
    acc.z ^= a.z ^ b.z ^ c.z ^ d.z;
    acc.w ^= a.w ^ b.w ^ c.w ^ d.w;
  }
  for (; i < n16; i += stride) {
    const uint4 a = src[i];
    acc.x ^= a.x;
    acc.y ^= a.y;
    acc.z ^= a.z;
    acc.w ^= a.w;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    acc.x ^= __shfl_xor(acc.x, o, 64);
    acc.y ^= __shfl_xor(acc.y, o, 64);
    acc.z ^= __shfl_xor(acc.z, o, 64);
    acc.w ^= __shfl_xor(acc.w, o, 64);
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint4 r = red[0];
    for (int q = 1; q < 4; ++q) {
      r.x ^= red[q].x;
      r.y ^= red[q].y;
      r.z ^= red[q].z;
      r.w ^= red[q].w;
    }
    out[blockIdx.x] = r;
  }
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
    const int64_t blocks = std::min<int64_t>((n16 + 255) / 256, 256 * 32);
    k_calib_copy<<<(unsigned)blocks, 256, 0, ctx->stream>>>((const uint4*)src, (uint4*)dst, n16);
    VMC_HIP(hipGetLastError());
  });
}

extern "C" int vmc_calib_read(vmc_ctx* ctx, const void* src, int64_t bytes, void* out) {
  return guard(ctx, [&] {
    VMC_REQUIRE(ctx && src && out, "NULL argument");
    VMC_REQUIRE(bytes > 0 && bytes % 16 == 0, "bytes must be a positive multiple of 16");
    VMC_REQUIRE(((uintptr_t)src | (uintptr_t)out) % 16 == 0, "buffers must be 16-byte aligned");
    set_device(ctx);
    phase_scope ps(ctx, "calib.read");
    k_calib_read<<<(unsigned)kCalibReadGroups, 256, 0, ctx->stream>>>((const uint4*)src, bytes / 16, (uint4*)out);
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
