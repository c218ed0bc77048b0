// RBM network evaluation in float32 or bfloat16 (vmc_model_set_precision):
//   theta = b + W sigma as a GEMM over the sample batch on the matrix cores
//   (v_mfma_f32_16x16x4_f32, or v_mfma_f32_16x16x32_bf16 with parameters
//   rounded to bfloat16; sigma = +-1 is exact in both; float32 accumulation),
//   log cosh / tanh and the per-slot ratio products of the local energy
//   (identity of rbm.hip) in float32, and every sum over hidden units, sites
//   and slots accumulated in float64.  The O_k kernels and the sampler always
//   run in float64.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"

using namespace dev;

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ float round_prec(double x, int prec) {
  const float f = (float)x;
  return prec == VMC_BF16 ? bf16_round(f) : f;
}

__global__ void k_lowp_params(const double2* __restrict__ p, int N, int Nh, int prec, float2* __restrict__ Wt32,
                              float2* __restrict__ ab32) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < (int64_t)N * Nh) {
    const int j = (int)(e / N), i = (int)(e % N);
    const double2 w = p[N + Nh + e];
    Wt32[(int64_t)i * Nh + j] = make_float2(round_prec(w.x, prec), round_prec(w.y, prec));
  }
  if (e < N + Nh) ab32[e] = make_float2(round_prec(p[e].x, prec), round_prec(p[e].y, prec));
}

// theta32 [B][2 N_h] (re, im interleaved) = b + sigma W^T; tile 64 samples x 64 real columns,
// wave w takes samples 16 w .. 16 w + 15 and four 16-column blocks
template <int PREC>
__global__ __launch_bounds__(256) void k_theta_mfma(const float* __restrict__ Wf /*[N][2Nh]*/,
                                                    const float* __restrict__ bf /*b as [2Nh]*/,
                                                    const uint64_t* __restrict__ s, int64_t B, int N, int W,
                                                    int Nh, float* __restrict__ theta) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t row = (int64_t)blockIdx.y * 64 + wave * 16 + li;  // sample of this lane's A fragment
  const int col0 = blockIdx.x * 64;
  const int ncol = 2 * Nh;
  const uint64_t* sr = s + (row < B ? row : 0) * W;
  floatx4 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};
  if (PREC == VMC_F32) {
    for (int k0 = 0; k0 < N; k0 += 4) {
      const int k = k0 + lk;
      const float a = (row < B && k < N) ? (((sr[k >> 6] >> (k & 63)) & 1ull) ? 1.f : -1.f) : 0.f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int c = col0 + j * 16 + li;
        const float b = (k < N && c < ncol) ? Wf[(int64_t)k * ncol + c] : 0.f;
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[j], 0, 0, 0);
      }
    }
  } else {
    for (int k0 = 0; k0 < N; k0 += 32) {
      bf16x8 a;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = k0 + 8 * lk + e;
        const float v = (row < B && k < N) ? (((sr[k >> 6] >> (k & 63)) & 1ull) ? 1.f : -1.f) : 0.f;
        a[e] = (__bf16)v;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int c = col0 + j * 16 + li;
        bf16x8 b;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int k = k0 + 8 * lk + e;
          b[e] = (__bf16)((k < N && c < ncol) ? Wf[(int64_t)k * ncol + c] : 0.f);
        }
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
      }
    }
  }
  // float32 accumulator layout: register r of lane l holds D[4 (l / 16) + r][l % 16]
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t b = (int64_t)blockIdx.y * 64 + wave * 16 + 4 * lk + r;
      const int c = col0 + j * 16 + li;
      if (b < B && c < ncol) theta[b * ncol + c] = acc[j][r] + bf[c];
    }
}

__global__ __launch_bounds__(64) void k_logpsi_lowp(const float2* __restrict__ ab32, const float2* __restrict__ th,
                                                    const uint64_t* __restrict__ s, int64_t B, int N, int W, int Nh,
                                                    double2* __restrict__ logpsi) {
  const int64_t n = blockIdx.x;
  if (n >= B) return;
  const int lane = threadIdx.x;
  const uint64_t* sn = s + n * W;
  double2 acc = make_double2(0.0, 0.0);
  for (int i = lane; i < N; i += 64) {
    const float2 a = ab32[i];
    const double sg = get_bit(sn, i) ? 1.0 : -1.0;
    acc.x += sg * a.x;
    acc.y += sg * a.y;
  }
  for (int j = lane; j < Nh; j += 64) {
    const float2 l = fclogcosh(th[n * Nh + j]);
    acc.x += l.x;
    acc.y += l.y;
  }
  acc = wave_sum(acc);
  if (lane == 0) logpsi[n] = acc;
}

// T [Nhp][n_moves], the rows past N_h (up to Nhp, a multiple of 16) zero
__global__ __launch_bounds__(64) void k_tables_lowp(const float2* __restrict__ Wt32, const float2* __restrict__ ab32,
                                                    const int2* __restrict__ bonds, int move_kind, int n_moves, int N,
                                                    int Nh, int Nhp, float2* __restrict__ T, float2* __restrict__ LC,
                                                    float2* __restrict__ alpha) {
  const int m = blockIdx.x;
  if (m >= n_moves) return;
  const int lane = threadIdx.x;
  int i, k = -1;
  if (move_kind == 0) {
    i = m;
  } else {
    i = bonds[m].x;
    k = bonds[m].y;
  }
  double2 lc = make_double2(0.0, 0.0);
  for (int j = lane; j < Nh; j += 64) {
    float2 d = Wt32[(int64_t)i * Nh + j];
    if (k >= 0) {
      const float2 d2 = Wt32[(int64_t)k * Nh + j];
      d = make_float2(d.x - d2.x, d.y - d2.y);
    }
    const float2 dd = make_float2(2.f * d.x, 2.f * d.y);
    T[(int64_t)j * n_moves + m] = fctanh(dd);
    const float2 l = fclogcosh(dd);
    lc.x += l.x;
    lc.y += l.y;
  }
  for (int j = Nh + lane; j < Nhp; j += 64) T[(int64_t)j * n_moves + m] = make_float2(0.f, 0.f);
  lc = wave_sum(lc);
  if (lane == 0) {
    LC[m] = make_float2((float)lc.x, (float)lc.y);
    const float2 ai = ab32[i];
    alpha[m] = k >= 0 ? make_float2(ai.x - ab32[k].x, ai.y - ab32[k].y) : ai;
  }
}

__global__ __launch_bounds__(64) void k_eloc_lowp(const float2* __restrict__ theta, const uint64_t* __restrict__ s,
                                                  int64_t B, int N, int W, int Nh, int ham_kind, double J, double h,
                                                  const int2* __restrict__ bonds, int n_bonds,
                                                  const float2* __restrict__ T, const float2* __restrict__ LC,
                                                  const float2* __restrict__ alpha, int n_moves, int Nhp,
                                                  double2* __restrict__ eloc) {
  // sigma t_j for both spins: tpm[0][j] = -t_j, tpm[1][j] = t_j, zero past N_h
  // (up to Nhp, a multiple of 16, where the table rows are zero as well)
  extern __shared__ float2 lds32[];
  float2* tpm = lds32;                   // [2][Nhp]
  int* moves = (int*)(lds32 + 2 * Nhp);  // [n_moves]
  const int64_t n = blockIdx.x;
  if (n >= B) return;
  const int lane = threadIdx.x;
  const uint64_t* sn = s + n * W;
  for (int j = lane; j < Nhp; j += 64) {
    const float2 tj = j < Nh ? fctanh(theta[n * Nh + j]) : make_float2(0.f, 0.f);
    tpm[j] = make_float2(-tj.x, -tj.y);
    tpm[Nhp + j] = tj;
  }
  int n_al = 0;
  for (int b = lane; b < n_bonds; b += 64) n_al += get_bit(sn, bonds[b].x) == get_bit(sn, bonds[b].y);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) n_al += __shfl_xor(n_al, o, 64);
  const int n_anti = n_bonds - n_al;
  const double diag = ham_kind == HAM_TFIM ? -J * (double)(n_al - n_anti) : J * (double)(n_al - n_anti);
  int n_slots = 0;
  double mel;
  if (ham_kind == HAM_TFIM) {
    mel = -h;
    if (h != 0.0) {
      for (int l = lane; l < N; l += 64) moves[l] = l;
      n_slots = N;
    }
  } else {
    mel = 2.0 * J;
    if (J != 0.0)
      for (int b0 = 0; b0 < n_bonds; b0 += 64) {
        const int b = b0 + lane;
        bool anti = false;
        if (b < n_bonds) anti = get_bit(sn, bonds[b].x) != get_bit(sn, bonds[b].y);
        const uint64_t mask = __ballot(anti);
        const int pos = n_slots + __popcll(mask & ((1ull << lane) - 1ull));
        if (anti) moves[pos] = b;
        n_slots += __popcll(mask);
      }
  }
  __syncthreads();
  double2 acc = make_double2(0.0, 0.0);
  for (int q0 = 0; q0 < n_slots; q0 += 64) {
    const int q = q0 + lane;
    if (q < n_slots) {
      const int m = moves[q];
      const int site = ham_kind == HAM_TFIM ? m : bonds[m].x;
      const int up = get_bit(sn, site);
      const float sg = up ? 1.f : -1.f;
      const float2* st = tpm + (up ? Nhp : 0);  // sigma t of this slot's spin
      const float2* Tm = T + m;                 // column m; rows n_moves apart (fewer than 2^31 entries)
      float2 P = make_float2(1.f, 0.f);
      int e2 = 0;
      for (int j0 = 0; j0 < Nhp; j0 += 16) {
#pragma unroll
        for (int jb = j0; jb < j0 + 16; jb += 8) {
          float2 Tv[8];  // eight table loads in flight before their products
#pragma unroll
          for (int u = 0; u < 8; ++u) Tv[u] = Tm[(jb + u) * n_moves];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const float2 tt = fcmul(st[jb + u], Tv[u]);  // sigma t_j T_jm
            P = fcmul(P, make_float2(1.f - tt.x, -tt.y));
          }
        }
        int e;
        frexpf(fmaxf(fabsf(P.x), fabsf(P.y)), &e);
        P.x = ldexpf(P.x, -e);
        P.y = ldexpf(P.y, -e);
        e2 += e;
      }
      const float2 a = alpha[m], lc = LC[m];
      const float2 lp = fclog(P);
      const float2 lr = make_float2(-2.f * sg * a.x + lc.x + lp.x + (float)e2 * 0.69314718f,
                                    -2.f * sg * a.y + lc.y + lp.y);
      const float2 r = fcexp(lr);
      acc.x += mel * (double)r.x;
      acc.y += mel * (double)r.y;
    }
  }
  acc = wave_sum(acc);
  if (lane == 0) eloc[n] = make_double2(acc.x + diag, acc.y);
}

constexpr int64_t kChunk = 1 << 16;

int nh_pad(int Nh) { return (Nh + 15) / 16 * 16; }

void ensure_params(vmc_model* m) {
  if (m->Wt32 && m->lowp_version == m->version && m->lowp_prec == m->prec) return;
  if (!m->Wt32) {
    VMC_HIP(hipMalloc(&m->Wt32, sizeof(float2) * (size_t)m->N * m->Nh));
    VMC_HIP(hipMalloc(&m->ab32, sizeof(float2) * (size_t)(m->N + m->Nh)));
  }
  const int64_t n = std::max<int64_t>((int64_t)m->N * m->Nh, m->N + m->Nh);
  k_lowp_params<<<grid_for(n, 256), 256, 0, m->ctx->stream>>>(m->params, m->N, m->Nh, m->prec, m->Wt32, m->ab32);
  VMC_HIP(hipGetLastError());
  m->lowp_version = m->version;
  m->lowp_prec = m->prec;
}

void theta_lowp(vmc_model* m, const uint64_t* s, int64_t B, float2* th) {
  // b as interleaved floats: ab32 + N viewed as float[2 Nh]
  const float* bf = (const float*)(m->ab32 + m->N);
  dim3 grid((unsigned)((2 * m->Nh + 63) / 64), (unsigned)((B + 63) / 64));
  if (m->prec == VMC_F32)
    k_theta_mfma<VMC_F32><<<grid, 256, 0, m->ctx->stream>>>((const float*)m->Wt32, bf, s, B, m->N, m->W, m->Nh,
                                                            (float*)th);
  else
    k_theta_mfma<VMC_BF16><<<grid, 256, 0, m->ctx->stream>>>((const float*)m->Wt32, bf, s, B, m->N, m->W, m->Nh,
                                                             (float*)th);
  VMC_HIP(hipGetLastError());
}

}  // namespace

void rbm_lowp_free(vmc_model* m) {
  if (m->Wt32) (void)hipFree(m->Wt32);
  if (m->ab32) (void)hipFree(m->ab32);
  for (auto& t : m->tab32) {
    if (t.T) (void)hipFree(t.T);
    if (t.LC) (void)hipFree(t.LC);
    if (t.alpha) (void)hipFree(t.alpha);
  }
}

void rbm_lowp_log_psi(vmc_model* m, const uint64_t* s, int64_t B, double2* logpsi) {
  vmc_ctx* ctx = m->ctx;
  ensure_params(m);
  const int64_t chunk = std::min<int64_t>(B, kChunk);
  ws_reserve(ctx, ws_round(sizeof(float2) * chunk * m->Nh));
  float2* th = (float2*)ws_take(ctx, sizeof(float2) * chunk * m->Nh);
  for (int64_t b0 = 0; b0 < B; b0 += chunk) {
    const int64_t nb = std::min(chunk, B - b0);
    theta_lowp(m, s + b0 * m->W, nb, th);
    k_logpsi_lowp<<<(unsigned)nb, 64, 0, ctx->stream>>>(m->ab32, th, s + b0 * m->W, nb, m->N, m->W, m->Nh,
                                                       logpsi + b0);
    VMC_HIP(hipGetLastError());
  }
}

void rbm_lowp_local_energy(vmc_model* m, vmc_ham* H, const uint64_t* s, int64_t B, double2* eloc) {
  vmc_ctx* ctx = m->ctx;
  ensure_params(m);
  const int move_kind = H->kind == HAM_TFIM ? 0 : 1;
  auto& tb = m->tab32[move_kind];
  const int n_moves = move_kind == 0 ? m->N : H->n_bonds;
  if (!tb.T || tb.n_moves != n_moves) {
    VMC_HIP(hipStreamSynchronize(ctx->stream));
    if (tb.T) VMC_HIP(hipFree(tb.T));
    if (tb.LC) VMC_HIP(hipFree(tb.LC));
    if (tb.alpha) VMC_HIP(hipFree(tb.alpha));
    tb.T = tb.LC = tb.alpha = nullptr;
    VMC_HIP(hipMalloc(&tb.T, sizeof(float2) * (size_t)nh_pad(m->Nh) * std::max(1, n_moves)));
    VMC_HIP(hipMalloc(&tb.LC, sizeof(float2) * std::max(1, n_moves)));
    VMC_HIP(hipMalloc(&tb.alpha, sizeof(float2) * std::max(1, n_moves)));
    tb.version = 0;
  }
  if (tb.version != m->version || tb.prec != m->prec || tb.n_moves != n_moves || (move_kind == 1 && tb.ham_uid != H->uid)) {
    if (n_moves > 0)
      k_tables_lowp<<<n_moves, 64, 0, ctx->stream>>>(m->Wt32, m->ab32, H->bonds, move_kind, n_moves, m->N, m->Nh,
                                                     nh_pad(m->Nh), tb.T, tb.LC, tb.alpha);
    VMC_HIP(hipGetLastError());
    tb.version = m->version;
    tb.prec = m->prec;
    tb.n_moves = n_moves;
    tb.ham_uid = H->uid;
  }
  const int64_t chunk = std::min<int64_t>(B, kChunk);
  ws_reserve(ctx, ws_round(sizeof(float2) * chunk * m->Nh));
  float2* th = (float2*)ws_take(ctx, sizeof(float2) * chunk * m->Nh);
  const int Nhp = nh_pad(m->Nh);
  const size_t lds = sizeof(float2) * 2 * Nhp + sizeof(int) * std::max(1, n_moves);
  VMC_REQUIRE(lds <= 64 * 1024, "model too large for the local-energy kernel's LDS budget");
  VMC_REQUIRE((int64_t)Nhp * std::max(1, n_moves) < ((int64_t)1 << 31), "move table too large");
  for (int64_t b0 = 0; b0 < B; b0 += chunk) {
    const int64_t nb = std::min(chunk, B - b0);
    theta_lowp(m, s + b0 * m->W, nb, th);
    k_eloc_lowp<<<(unsigned)nb, 64, lds, ctx->stream>>>(th, s + b0 * m->W, nb, m->N, m->W, m->Nh, H->kind, H->J,
                                                       H->h, H->bonds, H->n_bonds, tb.T, tb.LC, tb.alpha, n_moves, Nhp,
                                                       eloc + b0);
    VMC_HIP(hipGetLastError());
  }
}
