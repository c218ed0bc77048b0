// Global moves of the learned-proposal sampler (VMC_PROP_MADE_MIX): every
// sweep starts with global Metropolis-Hastings steps in which all chains
// propose together an independent sample s' ~ q of the frozen masked network
// (MADE), accepted with
//   r = 2 Re(log psi(s') - log psi(s)) + log q(s) - log q(s'),
// an independence-sampler kernel that keeps |psi|^2 invariant (Hastings 1970);
// the sweep's single-spin flips follow (sampler.hip).
//
// A global step g has two parts:
//  * the proposals, which do not depend on the chains: k_made_block draws
//    s' ~ q for every chain with its log q (Philox stream of step g), and
//    theta' = b + W sigma' follows on the matrix cores (rbm_theta).  Those of
//    step g + 1 are formed on a second stream while the main stream runs the
//    sweep after step g (two buffers, b = g & 1);
//  * on the main stream, log q of every chain state by teacher forcing, as
//    the plain masked forward pass (two float64 matrix-core products), and
//    k_mix_accept: the ratio from the chain's theta (kept between launches)
//    and theta', the uniform of Philox((c, g_lo, g_hi, 3)), and on acceptance
//    the proposal's bits and theta replace the chain's.
// The autoregressive draw is blocked: sites are taken MP = 16 at a time, and
// for each block
//   - the logits' part from hidden units whose inputs are all known (degree
//     m(k) <= d0) is a float64 matrix-core product [16 chains x H] . [H x 16 sites];
//   - the units whose degree falls inside the block (about 1.3 per site for
//     H = 512, N = 400) are finished site by site, 16 lanes per chain;
//   - the block's bits update the pre-activations of the later units as a
//     second product [16 chains x 16 sites] . [16 sites x H].
// The sequential dependence per sample is then 16 short site steps per block
// instead of one H-wide reduction per site.  The two evaluations of log q (the
// draw's, for s', and the forward pass, for s) sum in different orders, so the
// q of a state differs between them by rounding (about 1e-14 relative); the
// draw itself resolves each conditional to 2^-32 (32-bit uniforms), so the
// acceptance ratio is as consistent with the distribution actually sampled as
// a single evaluation would make it.
#include "internal.h"

using namespace dev;

namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int MC = 16;    // chains per work-group (rows of v_mfma_f64_16x16x4)
constexpr int MP = 16;    // sites per block (columns of the logits product)
constexpr int UCAP = 32;  // in-block units whose weights are staged in LDS
constexpr int CH = 16;    // matrix-core steps whose operand loads are issued together

struct made_block_args {
  const double* W1mT;  // [N][H] masked W1, transposed (row d: W1m[k][d] over k)
  const double* W2m;   // [N][H] masked W2 (row i: W2m[i][k] over k)
  const double* b1;    // [H]
  const double* b2;    // [N]
  const int* perm;     // [H] hidden units sorted by degree m(k) (ascending k within a degree)
  const int* mstart;   // [N + 1] first position in perm with degree >= v
  int N, H, W;
  int n_chains;
  uint64_t* prop;       // [n_chains][W] proposals
  double* lq_prop;      // [n_chains] their log q
  uint2 key;
  uint32_t lo, hi;
};

__device__ __forceinline__ int degree(int k, int N) { return k % (N - 1) + 1; }

// At most 128 registers per lane (four waves per SIMD): the kernel then fits
// beside a local-sweep wave of the RBM sampler (up to 376 registers), whose
// sweep it overlaps on the proposals' stream.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_made_block(made_block_args a) {
  extern __shared__ double smem[];
  const int N = a.N, H = a.H, W = a.W;
  const int Hs = H + 1;
  double* as_ = smem;                                 // [MC][Hs] pre-activations
  double* un_ = as_ + MC * Hs;                        // union: [4][256] partial logits | staged weights
  double* red_ = un_;
  double* w2s = un_;                                  // [MP][UCAP]
  double* w1s = un_ + MP * UCAP;                      // [MP][UCAP]
  double* Ls_ = un_ + 4 * 256;                        // [MC][MP] logits from the finished units (+ b2)
  uint64_t* bits_ = (uint64_t*)(Ls_ + MC * MP);       // [MC][W]
  int* us_ = (int*)(bits_ + MC * W);                  // [UCAP]
  int* deg_ = us_ + UCAP;                             // [H] degree m(k)

  const int c0 = blockIdx.x * MC;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;

  for (int e = tid; e < MC * H; e += 256) {
    const int c = e / H, k = e % H;
    as_[c * Hs + k] = a.b1[k];
  }
  for (int k = tid; k < H; k += 256) deg_[k] = degree(k, N);
  for (int e = tid; e < MC * W; e += 256) {
    const int c = e / W, w = e % W;
    bits_[e] = 0ull;
  }
  __syncthreads();

  // phase B lane roles: chain cl of this wave, 16 lanes per chain
  const int cl = wave * 4 + lk;
  const int sub = li;
  const uint32_t cg = (uint32_t)(c0 + cl);
  double lq = 0.0;
  uint4 x4 = make_uint4(0, 0, 0, 0);
  const int Hq = ((H + 15) / 16) * 4;  // hidden units per wave in phase A (a multiple of 4)

  for (int d0 = 0; d0 < N; d0 += MP) {
    const int P = min(MP, N - d0);
    // ---- phase A: logits of the block's sites from the finished units ----
    if (d0 > 0) {
      doublex4 acc = {0.0, 0.0, 0.0, 0.0};
      const int kb = wave * Hq, ke = min(H, kb + Hq);
      const double* w2row = a.W2m + (int64_t)(d0 + li) * H;
      const bool site_in = d0 + li < N;
      for (int kc = kb; kc < ke; kc += 4 * CH) {
        double bv[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) {  // operand loads of CH steps in flight together
          const int k = kc + 4 * q + lk;
          bv[q] = (site_in && k < ke) ? w2row[k] : 0.0;  // B[unit k][site li]
        }
#pragma unroll
        for (int q = 0; q < CH; ++q) {
          const int k = kc + 4 * q + lk;
          const double av = (k < ke && deg_[k] <= d0) ? fmax(as_[li * Hs + k], 0.0) : 0.0;  // A[chain li][unit k]
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[q], acc, 0, 0, 0);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) red_[wave * 256 + (lk + 4 * r) * 16 + li] = acc[r];
    }
    __syncthreads();
    {
      const int c = tid >> 4, i = tid & 15;
      double v = 0.0;
      if (d0 + i < N) {
        v = a.b2[d0 + i];
        if (d0 > 0) v += ((red_[tid] + red_[256 + tid]) + red_[512 + tid]) + red_[768 + tid];
      }
      Ls_[c * MP + i] = v;
    }
    __syncthreads();
    // ---- stage the weights of the units whose degree lies inside the block ----
    const int j0 = a.mstart[d0 + 1];
    const int nU = a.mstart[d0 + P] - j0;
    const bool staged = nU <= UCAP;
    if (staged) {
      for (int e = tid; e < MP * nU; e += 256) {
        const int i = e / nU, j = e % nU;
        const int u = a.perm[j0 + j];
        const bool in = i < P;
        w2s[i * UCAP + j] = in ? a.W2m[(int64_t)(d0 + i) * H + u] : 0.0;
        w1s[i * UCAP + j] = in ? a.W1mT[(int64_t)(d0 + i) * H + u] : 0.0;
        if (i == 0) us_[j] = u;
      }
    }
    __syncthreads();
    // ---- phase B: the block's sites one by one, 16 lanes per chain ----
    for (int i = 0; i < P; ++i) {
      const int d = d0 + i;
      double part = 0.0;
      if (staged) {
        for (int j = sub; j < nU; j += 16) {
          const int u = us_[j];
          if (deg_[u] <= d) part += w2s[i * UCAP + j] * fmax(as_[cl * Hs + u], 0.0);
        }
      } else {
        for (int j = sub; j < nU; j += 16) {
          const int u = a.perm[j0 + j];
          if (deg_[u] <= d) part += a.W2m[(int64_t)d * H + u] * fmax(as_[cl * Hs + u], 0.0);
        }
      }
      part = row16_sum(part);  // the same value in the chain's 16 lanes: a uniform decision
      const double l = Ls_[cl * MP + i] + part;
      const double e = exp(-fabs(l));  // p = sigmoid(l) and softplus(l) from one exponential
      if ((d & 3) == 0) x4 = philox(make_uint4(cg, a.lo, a.hi, 1u + 256u * (uint32_t)(d >> 2)), a.key);
      const uint32_t xr = (d & 3) == 0 ? x4.x : (d & 3) == 1 ? x4.y : (d & 3) == 2 ? x4.z : x4.w;
      const double p = (l >= 0.0 ? 1.0 : e) / (1.0 + e);
      const bool up = (double)xr * 0x1.0p-32 < p;
      lq += (up ? l : 0.0) - (fmax(l, 0.0) + log1p(e));
      if (up) {
        if (staged) {
          for (int j = sub; j < nU; j += 16) {
            const int u = us_[j];
            if (deg_[u] > d) as_[cl * Hs + u] += w1s[i * UCAP + j];
          }
        } else {
          for (int j = sub; j < nU; j += 16) {
            const int u = a.perm[j0 + j];
            if (deg_[u] > d) as_[cl * Hs + u] += a.W1mT[(int64_t)d * H + u];
          }
        }
        if (sub == 0) bits_[cl * W + (d >> 6)] |= 1ull << (d & 63);
      }
    }
    __syncthreads();
    // ---- phase C: the block's inputs into the units of higher degree ----
    if (d0 + P < N) {
      const int ntile = (H + 15) / 16;
      double av[4];  // A[chain li][site 4 ks + lk]: the same for every tile
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int i = ks * 4 + lk;
        av[ks] = i < P ? (double)((bits_[li * W + ((d0 + i) >> 6)] >> ((d0 + i) & 63)) & 1ull) : 0.0;
      }
      for (int t0 = wave; t0 < ntile; t0 += 4 * (CH / 4)) {
        double bv[CH / 4][4];
#pragma unroll
        for (int q = 0; q < CH / 4; ++q) {  // B[site][unit] of CH / 4 tiles in flight together
          const int k = (t0 + 4 * q) * 16 + li;
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) {
            const int i = ks * 4 + lk;
            bv[q][ks] = (i < P && k < H) ? a.W1mT[(int64_t)(d0 + i) * H + k] : 0.0;
          }
        }
#pragma unroll
        for (int q = 0; q < CH / 4; ++q) {
          const int k = (t0 + 4 * q) * 16 + li;
          doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ks], bv[q][ks], acc, 0, 0, 0);
          if (k < H && deg_[k] >= d0 + P) {
#pragma unroll
            for (int r = 0; r < 4; ++r) as_[(lk + 4 * r) * Hs + k] += acc[r];
          }
        }
      }
    }
    __syncthreads();
  }
  if (c0 + cl < a.n_chains && sub == 0) a.lq_prop[c0 + cl] = lq;
  for (int e = tid; e < MC * W; e += 256) {
    const int c = e / W;
    if (c0 + c < a.n_chains) a.prop[(int64_t)c0 * W + e] = bits_[e];
  }
}

// ---- teacher forcing of the chain states (the plain masked forward pass) ----
// A[c][k] = relu(b1[k] + sum_d s_d(c) W1m[k][d]) on the float64 matrix cores,
// the inputs 0 / 1 taken from the bits in LDS: 64 chains x 64 units per group,
// wave w the chains 16 w .. 16 w + 15 against four 16-unit tiles
// (v_mfma_f64_16x16x4f64: lane l holds A[l % 16][l / 16], B[l / 16][l % 16] and,
// in register r, D[l / 16 + 4 r][l % 16]).
constexpr int TF_KB = 4;  // k steps (4 sites each) whose operand loads are issued together
__global__ __launch_bounds__(256) void k_mix_hidden(const uint64_t* __restrict__ bits, int64_t nc, int N, int W,
                                                    int H, const double* __restrict__ W1mT,
                                                    const double* __restrict__ b1, double* __restrict__ A) {
  extern __shared__ uint64_t sbits[];  // [64][W]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t c0 = (int64_t)blockIdx.y * 64;
  const int k0c = blockIdx.x * 64;
  for (int e = tid; e < 64 * W; e += 256) {
    const int64_t c = c0 + e / W;
    sbits[e] = c < nc ? bits[c * W + e % W] : 0ull;
  }
  __syncthreads();
  const uint64_t* myb = sbits + (wave * 16 + li) * W;
  doublex4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = doublex4{0.0, 0.0, 0.0, 0.0};
  for (int d0 = 0; d0 < N; d0 += 4 * TF_KB) {
    double bv[TF_KB][4];
#pragma unroll
    for (int kb = 0; kb < TF_KB; ++kb) {
      const int d = d0 + 4 * kb + lk;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int k = k0c + 16 * t + li;
        bv[kb][t] = (d < N && k < H) ? W1mT[(int64_t)d * H + k] : 0.0;
      }
    }
#pragma unroll
    for (int kb = 0; kb < TF_KB; ++kb) {
      const int d = d0 + 4 * kb + lk;
      const double x = d < N ? (double)((myb[d >> 6] >> (d & 63)) & 1ull) : 0.0;
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, bv[kb][t], acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int k = k0c + 16 * t + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t c = c0 + wave * 16 + lk + 4 * r;
      if (c < nc && k < H) A[c * H + k] = fmax(acc[t][r] + b1[k], 0.0);
    }
  }
}

// log q of chain c: sum_d s_d l_d - softplus(l_d), l = L + b2; one wave per chain
__global__ __launch_bounds__(64) void k_mix_logq(const double* __restrict__ L, const double* __restrict__ b2,
                                                 const uint64_t* __restrict__ bits, int64_t nc, int N, int W,
                                                 double* __restrict__ lq) {
  const int64_t c = blockIdx.x;
  if (c >= nc) return;
  const uint64_t* sc = bits + c * W;
  double acc = 0.0;
  for (int d = threadIdx.x; d < N; d += 64) {
    const double l = L[c * N + d] + b2[d];
    acc += (get_bit(sc, d) ? l : 0.0) - (fmax(l, 0.0) + log1p(exp(-fabs(l))));
  }
  acc = wave_sum(acc);
  if (threadIdx.x == 0) lq[c] = acc;
}

struct mix_accept_args {
  const double2* params;  // RBM [a (N) | b | W]
  int N, W, Nh;
  int n_chains;
  uint64_t* bits;         // [n_chains][W]
  const uint64_t* prop;   // [n_chains][W]
  double2* theta;         // [n_chains][Nh]
  const double2* theta_prop;
  const double* lq_cur;
  const double* lq_prop;
  uint2 key;
  uint32_t lo, hi;
  unsigned long long* acc;  // [3][n_chains]: accepted (all), accepted global, global proposals
};

template <int Q>
__global__ __launch_bounds__(64) void k_mix_accept(mix_accept_args a) {
  const int c = blockIdx.x;
  if (c >= a.n_chains) return;
  const int lane = threadIdx.x;
  const int N = a.N, W = a.W, Nh = a.Nh;
  const uint64_t* sc = a.bits + (int64_t)c * W;
  const uint64_t* sp = a.prop + (int64_t)c * W;
  double dre = 0.0;  // 2 Re(log psi(s') - log psi(s)), lane partial
  for (int i = lane; i < N; i += 64) {
    const double sn = get_bit(sp, i) ? 1.0 : -1.0;
    const double so = get_bit(sc, i) ? 1.0 : -1.0;
    dre += 2.0 * a.params[i].x * (sn - so);
  }
  double2 thn[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int j = lane + 64 * q;
    thn[q] = j < Nh ? a.theta_prop[(int64_t)c * Nh + j] : make_double2(0.0, 0.0);
    if (j < Nh) dre += 2.0 * (clogcosh(thn[q]).x - clogcosh(a.theta[(int64_t)c * Nh + j]).x);
  }
  double dr = wave_sum(dre);
  dr = __shfl(dr, 0, 64);
  const double r = dr + a.lq_cur[c] - a.lq_prop[c];
  const uint4 x = philox(make_uint4((uint32_t)c, a.lo, a.hi, 3u), a.key);
  const double u = to_uniform(x.y, x.z);
  const bool acc = (r >= 0.0) || (u < exp(r));
  if (acc) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int j = lane + 64 * q;
      if (j < Nh) a.theta[(int64_t)c * Nh + j] = thn[q];
    }
    for (int w = lane; w < W; w += 64) a.bits[(int64_t)c * W + w] = sp[w];
  }
  if (lane == 0) {
    a.acc[c] += acc ? 1ull : 0ull;
    a.acc[a.n_chains + c] += acc ? 1ull : 0ull;
    a.acc[2 * (int64_t)a.n_chains + c] += 1ull;
  }
}

static_assert(2 * MP * UCAP <= 4 * 256, "staged weights share the partial-logit buffer");

size_t made_block_lds(int H, int W) {
  return sizeof(double) * ((size_t)MC * (H + 1) + 4 * 256 + MC * MP) + sizeof(uint64_t) * MC * (size_t)W +
         sizeof(int) * (UCAP + (size_t)H);
}

}  // namespace

// units sorted by degree m(k) = k mod (N - 1) + 1 and the first position of
// each degree (host side, once per proposal network)
void mix_made_layout(int N, int H, std::vector<int>& perm, std::vector<int>& mstart) {
  perm.resize(H);
  mstart.assign(N + 1, 0);
  std::vector<int> cnt(N + 1, 0);
  for (int k = 0; k < H; ++k) ++cnt[k % (N - 1) + 1];
  for (int v = 1; v <= N; ++v) mstart[v] = mstart[v - 1] + cnt[v - 1];
  std::vector<int> pos(mstart.begin(), mstart.end());
  for (int k = 0; k < H; ++k) perm[pos[k % (N - 1) + 1]++] = k;
}

bool mix_made_fits(int H, int W) {
  int dev = 0, lds = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return false;
  return made_block_lds(H, W) <= (size_t)lds;
}

namespace {

// proposals of global step g into buffer b, on stream st
void mix_proposals(vmc_sampler* S, uint64_t g, int b, hipStream_t st) {
  vmc_model* m = S->model;
  const int nc = S->opts.n_chains;
  const int N = m->N, H = S->made_H, W = m->W;
  const int64_t nh = (int64_t)N * H;
  made_block_args a{};
  a.W1mT = S->made_buf;
  a.W2m = S->made_buf + nh;
  a.b1 = S->made_buf + 2 * nh;
  a.b2 = S->made_buf + 2 * nh + H;
  a.perm = S->mix_perm;
  a.mstart = S->mix_perm + H;
  a.N = N;
  a.H = H;
  a.W = W;
  a.n_chains = nc;
  a.prop = S->mix_prop + (int64_t)b * nc * W;
  a.lq_prop = S->mix_lq + (int64_t)(1 + b) * nc;
  a.key = make_uint2((uint32_t)S->opts.seed, (uint32_t)(S->opts.seed >> 32));
  a.lo = (uint32_t)g;
  a.hi = (uint32_t)(g >> 32);
  k_made_block<<<(unsigned)((nc + MC - 1) / MC), 256, made_block_lds(H, W), st>>>(a);
  VMC_HIP(hipGetLastError());
  rbm_theta(m, a.prop, nc, S->mix_theta_prop + (int64_t)b * nc * m->Nh, st);
  S->mix_pg[b] = g;
  S->mix_pver[b] = m->version;
}

// log q of the chain states into mix_lq[0 .. nc) (main stream)
void mix_teacher(vmc_sampler* S) {
  vmc_ctx* ctx = S->ctx;
  hipStream_t st = ctx->stream;
  const int64_t nc = S->opts.n_chains;
  const int N = S->N, H = S->made_H;
  const int64_t nh = (int64_t)N * H;
  const double* W1mT = S->made_buf;
  const double* W2m = S->made_buf + nh;
  const double* b1 = S->made_buf + 2 * nh;
  const double* b2 = b1 + H;
  VMC_REQUIRE((nc + 63) / 64 <= 65535, "too many chains for the teacher-forcing grid");
  double* A = S->mix_tf;
  double* L = A + nc * H;
  // A = relu(b1 + s W1m^T), with W1m^T stored as [N][H]
  k_mix_hidden<<<dim3((unsigned)((H + 63) / 64), (unsigned)((nc + 63) / 64)), 256, sizeof(uint64_t) * 64 * S->W, st>>>(
      S->bits, nc, N, S->W, H, W1mT, b1, A);
  // L[c][i] = sum_k A[c][k] W2m[i][k]   (W2m stored as [N][H])
  dgemm(ctx, dgemm_args{A, H, 1, W2m, 1, H, L, N, nc, N, H, 0.0});
  k_mix_logq<<<(unsigned)nc, 64, 0, st>>>(L, b2, S->bits, nc, N, S->W, S->mix_lq);
  VMC_HIP(hipGetLastError());
}

}  // namespace

void mix_global_step(vmc_sampler* S, uint64_t g) {
  vmc_model* m = S->model;
  hipStream_t st = S->ctx->stream;
  const int nc = S->opts.n_chains;
  const int N = m->N, W = m->W;
  const int b = (int)(g & 1);
  mix_teacher(S);
  if (S->mix_pg[b] == g && S->mix_pver[b] == m->version) {
    VMC_HIP(hipStreamWaitEvent(st, S->mix_ev_prop[b], 0));  // formed ahead on the proposals' stream
  } else {
    mix_proposals(S, g, b, st);  // first step of a call, or the parameters changed
  }
  mix_accept_args c{};
  c.params = m->params;
  c.N = N;
  c.W = W;
  c.Nh = m->Nh;
  c.n_chains = nc;
  c.bits = S->bits;
  c.prop = S->mix_prop + (int64_t)b * nc * W;
  c.theta = S->mix_theta;
  c.theta_prop = S->mix_theta_prop + (int64_t)b * nc * m->Nh;
  c.lq_cur = S->mix_lq;
  c.lq_prop = S->mix_lq + (int64_t)(1 + b) * nc;
  c.key = make_uint2((uint32_t)S->opts.seed, (uint32_t)(S->opts.seed >> 32));
  c.lo = (uint32_t)g;
  c.hi = (uint32_t)(g >> 32);
  c.acc = S->acc;
  const int Q = (m->Nh + 63) / 64;
  if (Q <= 1)
    k_mix_accept<1><<<nc, 64, 0, st>>>(c);
  else if (Q <= 2)
    k_mix_accept<2><<<nc, 64, 0, st>>>(c);
  else if (Q <= 4)
    k_mix_accept<4><<<nc, 64, 0, st>>>(c);
  else if (Q <= 8)
    k_mix_accept<8><<<nc, 64, 0, st>>>(c);
  else
    k_mix_accept<16><<<nc, 64, 0, st>>>(c);
  VMC_HIP(hipGetLastError());
  // the proposals of step g + 1 go into the other buffer, whose last reader
  // (the acceptance of step g - 1) precedes this point of the main stream
  VMC_HIP(hipEventRecord(S->mix_ev_main, st));
  VMC_HIP(hipStreamWaitEvent(S->mix_side, S->mix_ev_main, 0));
  mix_proposals(S, g + 1, b ^ 1, S->mix_side);
  VMC_HIP(hipEventRecord(S->mix_ev_prop[b ^ 1], S->mix_side));
  S->mix_side_buf = b ^ 1;
}

void mix_wait_side(vmc_sampler* S) {
  // later work on the main stream (new parameters, freed buffers) is ordered
  // after the proposals formed ahead
  if (S->mix_side_buf >= 0) VMC_HIP(hipStreamWaitEvent(S->ctx->stream, S->mix_ev_prop[S->mix_side_buf], 0));
  S->mix_side_buf = -1;
}
