// S = Obar^H Obar on the float32 matrix cores (eq:qfm with centred data).
//
// Obar is N_s x K complex64, sample-major.  For a complex 16x16 output block
// (rows k, columns k') the products conj(O_nk) O_nk' take three real products
// per sample (Gauss's identity, as in the 3M complex GEMM): three float32 MFMA
// accumulators at the same lane positions hold
//   A = sum Re O_nk Re O_nk',  B = sum Im O_nk Im O_nk',
//   C = sum (Re O_nk - Im O_nk)(Re O_nk' + Im O_nk'),
// and S_kk' = (A + B) + i (C - A + B), combined in float64 (three MFMAs per 4
// samples instead of four; the error bound of Im S grows by at most a factor
// of about 2).  One v_mfma_f32_16x16x4_f32 consumes 4 samples; a lane's A and B
// fragments are one float2 (re, im) each, read from LDS.
//
// Work-group tile: 128 complex rows x 64 complex columns, 4 waves (2 x 2),
// each wave 64 x 32 (4 x 2 blocks of 16 x 16, 96 accumulator registers).
// With K even and Obar 16-byte aligned (k_herk_c_dma) the samples are loaded
// 12 at a time straight from global memory into double-buffered LDS
// (global_load_lds_dwordx4, no staging registers), three groups per compute
// unit; otherwise (k_herk_mfma_f32) 16 at a time through registers into
// double-buffered LDS, two groups per compute unit.  Only tiles
// that touch the lower triangle are launched; the linear tile index is
// remapped so that consecutive tiles of one row stripe run on the same XCD
// (shared L2).  The epilogue writes S~ (float64, projection and diagonal shift
// applied) to the lower triangle and its conjugate to the upper triangle; for
// the Im projection it writes the Hermitian matrix i Im S (purely imaginary,
// zero diagonal) in place of the real antisymmetric Im S.
//
// Real mode (only Re S is used) keeps one accumulator, A + B, half the
// matrix-core work per sample of the conventional complex product; with the
// registers that frees it takes square
// 128 x 128 tiles (each wave 64 x 64), so the matrix-core work per staged sample
// and per barrier stays that of the complex tile and the operand traffic per
// flop halves.  When the tiles alone cannot fill the chip (small K, many
// samples) the sample range is split over blockIdx.y; each split stores its
// float32 accumulators in register order and a second kernel adds the splits in
// float64 (fixed order, so the result is reproducible) before the epilogue.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int BM = 128;  // complex rows per tile
constexpr int BK = 16;   // samples per LDS stage
constexpr int PAD = 2;   // float2 padding per LDS row

// complex mode: 128 x 64 tiles, three accumulators; real mode: 128 x 128, one
template <bool REAL>
struct herk_shape {
  static constexpr int BN = REAL ? 128 : 64;  // columns per tile
  static constexpr int JN = REAL ? 4 : 2;     // 16-column blocks per wave
  static constexpr int QN = REAL ? 1 : 3;     // accumulators per block
  static constexpr int ACC = 4 * JN * QN * 4; // accumulator values per thread
};

struct herk_args {
  const float2* X;  // [N][K]
  int64_t N, K;
  int mode;
  double nu, eps;
  double2* S;
  double2* diag;
  int n_row_tiles;
  int64_t n_tiles;
  int ksplit;        // sample-range splits (1 = none)
  float* part;       // [ksplit][n_tiles][ACC][256] partial accumulators when ksplit > 1
};

__device__ __forceinline__ int64_t remap_tile(int64_t bid, int64_t nb) {
  // XCD-aware remap: hardware places block i on XCD i % 8
  const int64_t per = (nb + 7) / 8;
  return (bid % 8) * per + bid / 8;
}

// lower-triangle tile (tr, tc) of linear index b: complex mode has 2 t + 2 column
// tiles in row tile t (cumulative t (t + 1)), real mode t + 1 (cumulative t (t + 1) / 2)
template <bool REAL>
__device__ __forceinline__ void tile_of(int64_t b, int& tr, int& tc) {
  if (REAL) {
    int t = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while ((int64_t)(t + 1) * (t + 2) / 2 <= b) ++t;
    while ((int64_t)t * (t + 1) / 2 > b) --t;
    tr = t;
    tc = (int)(b - (int64_t)t * (t + 1) / 2);
  } else {
    int t = (int)((sqrt(4.0 * (double)b + 1.0) - 1.0) * 0.5);
    while ((int64_t)(t + 1) * (t + 2) <= b) ++t;
    while ((int64_t)t * (t + 1) > b) --t;
    tr = t;
    tc = (int)(b - (int64_t)t * (t + 1));
  }
}

__device__ __forceinline__ int acc_index(int i, int j, int q, int r, int JN, int QN) {
  return ((i * JN + j) * QN + q) * 4 + r;
}

// writes one lane's values of the 16 x 16 blocks; get(i, j, q, r) returns accumulator q
template <bool REAL, typename Get>
__device__ __forceinline__ void herk_epilogue(const herk_args& a, int64_t row0, int64_t col0, int wr, int wc, int li,
                                              int lk, Get get) {
  using sh = herk_shape<REAL>;
  const int64_t K = a.K;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < sh::JN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t k = row0 + wr * 64 + i * 16 + 4 * lk + r;
        const int64_t kp = col0 + wc * (16 * sh::JN) + j * 16 + li;
        if (k >= K || kp >= K || kp > k) continue;
        double re, im = 0.0;
        if constexpr (REAL) {
          re = get(i, j, 0, r);
        } else {
          const double A = get(i, j, 0, r), B = get(i, j, 1, r);
          re = A + B;
          im = (get(i, j, 2, r) - A) + B;
          if (a.mode == VMC_SR_IMAG) re = 0.0;  // i Im S (Hermitian; zero diagonal)
        }
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

template <bool REAL>
__global__ __launch_bounds__(256, 2) void k_herk_mfma_f32(herk_args a) {
  using sh = herk_shape<REAL>;
  constexpr int BN = sh::BN, JN = sh::JN, QN = sh::QN;
  constexpr int NA = BK * BM / 256, NB = BK * BN / 256;  // float2 per thread per stage
  // complex mode: two LDS stages (one barrier per stage); real mode: one stage
  // (two barriers per stage) so that its square tiles leave room for four
  // resident groups per compute unit
  constexpr int NBUF = REAL ? 1 : 2;
  __shared__ float2 As[NBUF][BK][BM + PAD];
  __shared__ float2 Bs[NBUF][BK][BN + PAD];

  const int64_t nb = a.n_tiles;
  const int64_t lin = remap_tile(blockIdx.x, nb);
  if (lin >= nb) return;
  int tr, tc;
  tile_of<REAL>(lin, tr, tc);
  const int64_t row0 = (int64_t)tr * BM, col0 = (int64_t)tc * BN;
  const int64_t K = a.K, N = a.N;
  if (col0 >= K) return;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;  // wave position in the 2 x 2 grid

  floatx4 acc[4][JN][QN];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j)
#pragma unroll
      for (int q = 0; q < QN; ++q) acc[i][j][q] = floatx4{0.f, 0.f, 0.f, 0.f};

  // global -> register staging of one stage: A BK x BM, B BK x BN float2.
  // Out-of-range elements load X[0] (always valid) and are replaced by zero,
  // so the loads need no branches.
  float2 ra[NA], rb[NB];
  auto gload = [&](int64_t n0) {
#pragma unroll
    for (int r = 0; r < NA; ++r) {
      const int q = tid + 256 * r;
      const int nn = q / BM, cc = q % BM;
      const int64_t n = n0 + nn, c = row0 + cc;
      const bool ok = n < N && c < K;
      const float2 v = a.X[ok ? n * K + c : 0];
      ra[r] = ok ? v : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int r = 0; r < NB; ++r) {
      const int q = tid + 256 * r;
      const int nn = q / BN, cc = q % BN;
      const int64_t n = n0 + nn, c = col0 + cc;
      const bool ok = n < N && c < K;
      const float2 v = a.X[ok ? n * K + c : 0];
      rb[r] = ok ? v : make_float2(0.f, 0.f);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int r = 0; r < NA; ++r) {
      const int q = tid + 256 * r;
      As[buf][q / BM][q % BM] = ra[r];
    }
#pragma unroll
    for (int r = 0; r < NB; ++r) {
      const int q = tid + 256 * r;
      Bs[buf][q / BN][q % BN] = rb[r];
    }
  };

  const int64_t n_stages = (N + BK - 1) / BK;
  const int64_t sp = (n_stages + a.ksplit - 1) / a.ksplit;
  const int64_t st0 = blockIdx.y * sp, st1 = min(n_stages, st0 + sp);
  const int li = lane & 15, lk = lane >> 4;
  if (st0 < st1) {  // uniform over the group
    gload(st0 * BK);
    sstore(0);
    __syncthreads();
    for (int64_t st = st0; st < st1; ++st) {
      const int buf = NBUF == 2 ? (int)((st - st0) & 1) : 0;
      if (st + 1 < st1) gload((st + 1) * BK);
      // MFMA fragments double-buffered in registers: the LDS reads of step
      // ks + 1 are issued before the matrix-core work of step ks
      float2 fr[2][4], fc[2][JN];
      auto fload = [&](int p, int ks) {
        const int n = ks * 4 + lk;
#pragma unroll
        for (int i = 0; i < 4; ++i) fr[p][i] = As[buf][n][wr * 64 + i * 16 + li];
#pragma unroll
        for (int j = 0; j < JN; ++j) fc[p][j] = Bs[buf][n][wc * (16 * JN) + j * 16 + li];
      };
      fload(0, 0);
#pragma unroll
      for (int ks = 0; ks < BK / 4; ++ks) {
        const int p = ks & 1;
        if (ks + 1 < BK / 4) fload(p ^ 1, ks + 1);
        __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the products
        const float2* fa = fr[p];
        const float2* fb = fc[p];
        if constexpr (REAL) {
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < JN; ++j) {
              acc[i][j][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i].x, fb[j].x, acc[i][j][0], 0, 0, 0);
              acc[i][j][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i].y, fb[j].y, acc[i][j][0], 0, 0, 0);
            }
        } else {
          float da[4], sb[JN];
#pragma unroll
          for (int i = 0; i < 4; ++i) da[i] = fa[i].x - fa[i].y;
#pragma unroll
          for (int j = 0; j < JN; ++j) sb[j] = fb[j].x + fb[j].y;
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < JN; ++j) {
              acc[i][j][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i].x, fb[j].x, acc[i][j][0], 0, 0, 0);
              acc[i][j][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i].y, fb[j].y, acc[i][j][1], 0, 0, 0);
              acc[i][j][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(da[i], sb[j], acc[i][j][2], 0, 0, 0);
            }
        }
      }
      if constexpr (NBUF == 2) {
        if (st + 1 < st1) sstore(buf ^ 1);
        __syncthreads();
      } else {
        __syncthreads();  // every wave is done with the stage
        if (st + 1 < st1) {
          sstore(0);
          __syncthreads();
        }
      }
    }
  }

  if (a.ksplit > 1) {  // partial accumulators in register order, coalesced over threads
    float* dst = a.part + ((int64_t)blockIdx.y * nb + lin) * (sh::ACC * 256) + tid;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < JN; ++j)
#pragma unroll
        for (int q = 0; q < QN; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r) dst[acc_index(i, j, q, r, JN, QN) * 256] = acc[i][j][q][r];
    return;
  }
  // epilogue: lane holds D[4 * (lane / 16) + r][lane % 16] of each block
  herk_epilogue<REAL>(a, row0, col0, wr, wc, li, lk,
                      [&](int i, int j, int q, int r) { return (double)acc[i][j][q][r]; });
}

// Complex mode with the operand tiles loaded straight from global memory into
// LDS (global_load_lds_dwordx4: 16 bytes per lane, two complex values), no
// register staging.  A row of the A tile (128 complex) is one wave
// instruction, two rows of the B tile (64 complex each) are one.  Lanes
// outside the matrix load a 16-byte zero word instead.  Needs K even and Obar
// 16-byte aligned, so that a lane's two values are both inside or both outside.
__device__ float4 g_zero16 = {0.f, 0.f, 0.f, 0.f};

// samples per stage of the direct-to-LDS kernel and its resident waves per SIMD
constexpr int kDmaStage = 12, kDmaOcc = 3;

typedef __attribute__((address_space(1))) const void* gptr_t;
typedef __attribute__((address_space(3))) void* lptr_t;

using accs_c = floatx4[4][herk_shape<false>::JN][herk_shape<false>::QN];

// One stage of the complex DMA kernel: (if COMPUTE) reads every MFMA fragment
// of the current stage from (Ac, Bc) into registers, then issues the next
// stage's tile loads into (An, Bn), then runs the stage's matrix-core work.
// The compiler makes any LDS read that follows a direct-to-LDS load wait for
// it; with the reads first, that wait falls on the next stage's first read,
// after the barrier, so the loads overlap the whole stage's products.
template <int SD, bool COMPUTE>
__device__ __forceinline__ void herk_c_stage(const float2* Ac, const float2* Bc, float2* An, float2* Bn,
                                             const float2* __restrict__ X, int64_t N, int64_t K, int64_t n0,
                                             bool load_next, int64_t row0, int64_t col0, int wave, int lane,
                                             accs_c& acc) {
  using sh = herk_shape<false>;
  constexpr int BN = sh::BN, JN = sh::JN, NKS = SD / 4;
  const int wr = wave >> 1, wc = wave & 1, li = lane & 15, lk = lane >> 4;
  float2 fa[NKS][4], fb[NKS][JN];
  if constexpr (COMPUTE) {
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const int n = ks * 4 + lk;
#pragma unroll
      for (int i = 0; i < 4; ++i) fa[ks][i] = Ac[n * BM + wr * 64 + i * 16 + li];
#pragma unroll
      for (int j = 0; j < JN; ++j) fb[ks][j] = Bc[n * BN + wc * (16 * JN) + j * 16 + li];
    }
  }
  if (load_next) {
    // wave w loads A rows w, w + 4, ... (one per instruction) and B row pairs
    // w, w + 4, ... (two rows per instruction) of the stage starting at sample n0
    const float2* zero = (const float2*)&g_zero16;
#pragma unroll
    for (int n = wave; n < SD; n += 4) {
      const int64_t gn = n0 + n, c = row0 + 2 * lane;
      const float2* src = (gn < N && c < K) ? X + gn * K + c : zero;
      __builtin_amdgcn_global_load_lds((gptr_t)src, (lptr_t)(An + n * BM), 16, 0, 0);
    }
#pragma unroll
    for (int pr = wave; pr < SD / 2; pr += 4) {
      const int n = 2 * pr;
      const int64_t gn = n0 + n + (lane >> 5), c = col0 + 2 * (lane & 31);
      const float2* src = (gn < N && c < K) ? X + gn * K + c : zero;
      __builtin_amdgcn_global_load_lds((gptr_t)src, (lptr_t)(Bn + n * BN), 16, 0, 0);
    }
  }
  if constexpr (COMPUTE) {
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      float da[4], sb[JN];
#pragma unroll
      for (int i = 0; i < 4; ++i) da[i] = fa[ks][i].x - fa[ks][i].y;
#pragma unroll
      for (int j = 0; j < JN; ++j) sb[j] = fb[ks][j].x + fb[ks][j].y;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < JN; ++j) {
          acc[i][j][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[ks][i].x, fb[ks][j].x, acc[i][j][0], 0, 0, 0);
          acc[i][j][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[ks][i].y, fb[ks][j].y, acc[i][j][1], 0, 0, 0);
          acc[i][j][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(da[i], sb[j], acc[i][j][2], 0, 0, 0);
        }
    }
  }
}

template <int SD, int OCC>
__global__ __launch_bounds__(256, OCC) void k_herk_c_dma(herk_args a) {
  using sh = herk_shape<false>;
  constexpr int BN = sh::BN, JN = sh::JN, QN = sh::QN;
  __shared__ float2 As[2][SD * BM];
  __shared__ float2 Bs[2][SD * BN];

  const int64_t nb = a.n_tiles;
  const int64_t lin = remap_tile(blockIdx.x, nb);
  if (lin >= nb) return;
  int tr, tc;
  tile_of<false>(lin, tr, tc);
  const int64_t row0 = (int64_t)tr * BM, col0 = (int64_t)tc * BN;
  const int64_t K = a.K, N = a.N;
  if (col0 >= K) return;

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave >> 1, wc = wave & 1, li = lane & 15, lk = lane >> 4;

  accs_c acc;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j)
#pragma unroll
      for (int q = 0; q < QN; ++q) acc[i][j][q] = floatx4{0.f, 0.f, 0.f, 0.f};

  // the sample range of this split, as in the register-staged kernel (stages
  // of BK samples), walked in stages of SD samples
  const int64_t n_stages = (N + BK - 1) / BK;
  const int64_t sp = (n_stages + a.ksplit - 1) / a.ksplit;
  const int64_t s0 = min(N, blockIdx.y * sp * BK), s1 = min(N, (blockIdx.y + 1) * sp * BK);
  const int64_t st0 = 0, st1 = (s1 - s0 + SD - 1) / SD;
  if (st0 < st1) {  // uniform over the group
    // first stage into buffer 0 (loads only)
    herk_c_stage<SD, false>(As[1], Bs[1], As[0], Bs[0], a.X, s1, K, s0, true, row0, col0, wave, lane, acc);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int64_t st = st0; st < st1; ++st) {
      const int buf = (int)((st - st0) & 1);
      // the other buffer was released by every wave at the previous barrier
      herk_c_stage<SD, true>(As[buf], Bs[buf], As[buf ^ 1], Bs[buf ^ 1], a.X, s1, K, s0 + (st + 1) * SD, st + 1 < st1,
                             row0, col0, wave, lane, acc);
      __builtin_amdgcn_sched_barrier(0);  // the wait below stays after the products
      __builtin_amdgcn_s_waitcnt(0);      // this wave's rows of the next stage have landed
      __syncthreads();                // and every wave is done with this stage
    }
  }

  if (a.ksplit > 1) {
    float* dst = a.part + ((int64_t)blockIdx.y * nb + lin) * (sh::ACC * 256) + tid;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < JN; ++j)
#pragma unroll
        for (int q = 0; q < QN; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r) dst[acc_index(i, j, q, r, JN, QN) * 256] = acc[i][j][q][r];
    return;
  }
  herk_epilogue<false>(a, row0, col0, wr, wc, li, lk,
                       [&](int i, int j, int q, int r) { return (double)acc[i][j][q][r]; });
}

// adds the split partial accumulators (float64, split order) and writes S~
template <bool REAL>
__global__ __launch_bounds__(256) void k_herk_reduce(herk_args a) {
  using sh = herk_shape<REAL>;
  constexpr int JN = sh::JN, QN = sh::QN;
  const int64_t nb = a.n_tiles;
  const int64_t lin = remap_tile(blockIdx.x, nb);
  if (lin >= nb) return;
  int tr, tc;
  tile_of<REAL>(lin, tr, tc);
  const int64_t row0 = (int64_t)tr * BM, col0 = (int64_t)tc * sh::BN;
  if (col0 >= a.K) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  double acc[4][JN][QN][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j)
#pragma unroll
      for (int q = 0; q < QN; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          double s = 0.0;
          for (int sp = 0; sp < a.ksplit; ++sp)
            s += (double)a.part[((int64_t)sp * nb + lin) * (sh::ACC * 256) + acc_index(i, j, q, r, JN, QN) * 256 + tid];
          acc[i][j][q][r] = s;
        }
  herk_epilogue<REAL>(a, row0, col0, wr, wc, lane & 15, lane >> 4,
                      [&](int i, int j, int q, int r) { return acc[i][j][q][r]; });
}

int64_t herk_tiles(int64_t K, bool real) {
  const int64_t rt = (K + BM - 1) / BM;
  return real ? rt * (rt + 1) / 2 : rt * (rt + 1);
}

}  // namespace

int herk_splits(int64_t N, int64_t K, int mode) {
  const int64_t n_tiles = herk_tiles(K, mode == VMC_SR_REAL);
  const int64_t n_stages = (N + BK - 1) / BK;
  // at most 1024 groups (whole rounds of resident groups, no thin last round),
  // keeping at least 64 stages per split
  int64_t s = 1024 / n_tiles;
  s = std::min<int64_t>(s, n_stages / 64);
  return (int)std::max<int64_t>(1, std::min<int64_t>(s, 64));
}

size_t herk_ws_bytes(int64_t N, int64_t K, int mode) {
  const int s = herk_splits(N, K, mode);
  if (s <= 1) return 0;
  const bool real = mode == VMC_SR_REAL;
  const int acc = real ? herk_shape<true>::ACC : herk_shape<false>::ACC;
  return sizeof(float) * (size_t)s * (size_t)herk_tiles(K, real) * acc * 256;
}

void herk_mfma_f32(vmc_ctx* ctx, const float2* X, int64_t N, int64_t K, int mode, double nu, double eps, double2* S,
                   double2* diag, void* ws) {
  herk_args a{};
  a.X = X;
  a.N = N;
  a.K = K;
  a.mode = mode;
  a.nu = nu;
  a.eps = eps;
  a.S = S;
  a.diag = diag;
  a.n_row_tiles = (int)((K + BM - 1) / BM);
  const bool real = mode == VMC_SR_REAL;
  a.n_tiles = herk_tiles(K, real);
  a.ksplit = herk_splits(N, K, mode);
  a.part = (float*)ws;
  if (a.ksplit > 1 && !ws) throw vmc_error{VMC_ERR_WORKSPACE, "internal: split Gram without workspace"};
  const int64_t grid = ((a.n_tiles + 7) / 8) * 8;
  const dim3 g((unsigned)grid, (unsigned)a.ksplit);
  if (real)
    k_herk_mfma_f32<true><<<g, 256, 0, ctx->stream>>>(a);
  else if (K % 2 == 0 && (uintptr_t)X % 16 == 0)
    k_herk_c_dma<kDmaStage, kDmaOcc><<<g, 256, 0, ctx->stream>>>(a);
  else
    k_herk_mfma_f32<false><<<g, 256, 0, ctx->stream>>>(a);
  VMC_HIP(hipGetLastError());
  if (a.ksplit > 1) {
    if (real)
      k_herk_reduce<true><<<(unsigned)grid, 256, 0, ctx->stream>>>(a);
    else
      k_herk_reduce<false><<<(unsigned)grid, 256, 0, ctx->stream>>>(a);
    VMC_HIP(hipGetLastError());
  }
}
