// Translation-symmetric single-layer network with ELU activation on a ring of
// L sites: the ground-state ansatz of the paper's example (Sec. 5.1,
// eq:gs_nqs), with real parameters [W (alpha x L), b (alpha)]:
//     theta_{a,w} = b_a + sum_l W_{a,l} sigma_{(l + w) mod L},
//     log psi(s)  = sum_{a,w} ELU(theta_{a,w}),   sigma = 2 s - 1.
// One wave per configuration (or chain) keeps the alpha L pre-activations in
// LDS; the filters are staged once per group.  Flipping site j changes every
// theta_{a,w} by -2 sigma_j W_{a,(j-w) mod L}, so a local energy or a
// Metropolis proposal costs alpha L activations instead of a full pass.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.h"

using namespace dev;

namespace {

constexpr int SE_NT = 256;
constexpr int SE_WAVES = SE_NT / 64;

__device__ __forceinline__ double elu(double x) { return x > 0.0 ? x : expm1(x); }
__device__ __forceinline__ double elu_d(double x) { return x > 0.0 ? 1.0 : exp(x); }

__device__ __forceinline__ void se_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// filters (real parts of the parameters) into LDS: Ws [alpha][L], bs [alpha]
__device__ void se_stage(const double2* __restrict__ p, int L, int alpha, double* Ws, double* bs) {
  for (int e = threadIdx.x; e < alpha * L; e += SE_NT) Ws[e] = p[e].x;
  for (int a = threadIdx.x; a < alpha; a += SE_NT) bs[a] = p[alpha * L + a].x;
  __syncthreads();
}

// sigma of one configuration into the wave's LDS, then theta (lanes over (a, w))
__device__ void se_theta(const uint64_t* __restrict__ srow, int L, int alpha, const double* Ws, const double* bs,
                         double* sig, double* th, int lane) {
  for (int l = lane; l < L; l += 64) sig[l] = ((srow[l >> 6] >> (l & 63)) & 1ull) ? 1.0 : -1.0;
  se_wave_sync();
  for (int q = lane; q < alpha * L; q += 64) {
    const int a = q / L, w = q - a * L;
    const double* Wa = Ws + a * L;
    double acc = bs[a];
    int l = 0;
    for (; l < L - w; ++l) acc = fma(Wa[l], sig[l + w], acc);
    for (; l < L; ++l) acc = fma(Wa[l], sig[l + w - L], acc);
    th[q] = acc;
  }
  se_wave_sync();
}

__global__ __launch_bounds__(SE_NT) void k_se_log_psi(const uint64_t* __restrict__ s, int64_t B, int W, int L,
                                                      int alpha, const double2* __restrict__ p,
                                                      double2* __restrict__ out) {
  extern __shared__ double lds[];
  double* Ws = lds;
  double* bs = Ws + alpha * L;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* sig = bs + alpha + wave * (L + alpha * L);
  double* th = sig + L;
  se_stage(p, L, alpha, Ws, bs);
  for (int64_t b = (int64_t)blockIdx.x * SE_WAVES + wave; b < B; b += (int64_t)gridDim.x * SE_WAVES) {
    se_theta(s + b * W, L, alpha, Ws, bs, sig, th, lane);
    double acc = 0.0;
    for (int q = lane; q < alpha * L; q += 64) acc += elu(th[q]);
    acc = wave_sum(acc);
    if (lane == 0) out[b] = make_double2(acc, 0.0);
    se_wave_sync();
  }
}

// E_loc: lanes over connected moves (TFIM: every site; Heisenberg: anti-aligned
// bonds in bond order), each lane sums the change of all alpha L activations
__global__ __launch_bounds__(SE_NT) void k_se_eloc(const uint64_t* __restrict__ s, int64_t B, int W, int L, int alpha,
                                                   const double2* __restrict__ p, int kind, double J, double hx,
                                                   const int2* __restrict__ bonds, int n_bonds,
                                                   double2* __restrict__ eloc) {
  extern __shared__ double lds[];
  double* Ws = lds;
  double* bs = Ws + alpha * L;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* sig = bs + alpha + wave * (L + 2 * alpha * L);
  double* th = sig + L;
  double* ev = th + alpha * L;
  se_stage(p, L, alpha, Ws, bs);
  const int AL = alpha * L;
  const double mel = kind == HAM_TFIM ? -hx : 2.0 * J;
  const bool offdiag = kind == HAM_TFIM ? hx != 0.0 : J != 0.0;
  for (int64_t b = (int64_t)blockIdx.x * SE_WAVES + wave; b < B; b += (int64_t)gridDim.x * SE_WAVES) {
    const uint64_t* srow = s + b * W;
    se_theta(srow, L, alpha, Ws, bs, sig, th, lane);
    for (int q = lane; q < AL; q += 64) ev[q] = elu(th[q]);
    se_wave_sync();
    int n_al = 0;
    for (int q0 = 0; q0 < n_bonds; q0 += 64) {
      const int q = q0 + lane;
      bool al = false;
      if (q < n_bonds) al = sig[bonds[q].x] == sig[bonds[q].y];
      n_al += __popcll(__ballot(q < n_bonds && al));
    }
    double e = 0.0;
    const int M = !offdiag ? 0 : (kind == HAM_TFIM ? L : n_bonds);
    for (int m0 = 0; m0 < M; m0 += 64) {
      const int m = m0 + lane;
      double r = 0.0;
      if (m < M) {
        int i = m, j = -1;
        bool live = true;
        if (kind != HAM_TFIM) {
          i = bonds[m].x;
          j = bonds[m].y;
          live = sig[i] != sig[j];
        }
        if (live) {
          const double ci = -2.0 * sig[i], cj = j >= 0 ? -2.0 * sig[j] : 0.0;
          double d = 0.0;
          for (int a = 0; a < alpha; ++a) {
            const double* Wa = Ws + a * L;
            const double* ta = th + a * L;
            const double* ea = ev + a * L;
            for (int w = 0; w < L; ++w) {
              const int li = i - w < 0 ? i - w + L : i - w;
              double t = fma(ci, Wa[li], ta[w]);
              if (j >= 0) {
                const int lj = j - w < 0 ? j - w + L : j - w;
                t = fma(cj, Wa[lj], t);
              }
              d += elu(t) - ea[w];
            }
          }
          r = mel * exp(d);
        }
      }
      e += wave_sum(r);
    }
    if (lane == 0) {
      const double diag = (kind == HAM_TFIM ? -J : J) * (double)(n_al - (n_bonds - n_al));
      eloc[b] = make_double2(diag + e, 0.0);
    }
    se_wave_sync();
  }
}

// O_k: d/dW_{a,l} = sum_w g_{a,w} sigma_{(l+w) mod L}, d/db_a = sum_w g_{a,w}, g = ELU'(theta)
template <typename OutT>
__global__ __launch_bounds__(SE_NT) void k_se_grad(const uint64_t* __restrict__ s, int64_t B, int W, int L, int alpha,
                                                   const double2* __restrict__ p, OutT* __restrict__ O) {
  extern __shared__ double lds[];
  double* Ws = lds;
  double* bs = Ws + alpha * L;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* sig = bs + alpha + wave * (L + alpha * L);
  double* th = sig + L;
  se_stage(p, L, alpha, Ws, bs);
  const int AL = alpha * L;
  const int64_t K = (int64_t)AL + alpha;
  for (int64_t b = (int64_t)blockIdx.x * SE_WAVES + wave; b < B; b += (int64_t)gridDim.x * SE_WAVES) {
    se_theta(s + b * W, L, alpha, Ws, bs, sig, th, lane);
    for (int q = lane; q < AL; q += 64) th[q] = elu_d(th[q]);
    se_wave_sync();
    OutT* row = O + b * K;
    for (int k = lane; k < K; k += 64) {
      double v = 0.0;
      if (k < AL) {
        const int a = k / L, l = k - a * L;
        const double* ga = th + a * L;
        int w = 0;
        for (; w < L - l; ++w) v = fma(ga[w], sig[l + w], v);
        for (; w < L; ++w) v = fma(ga[w], sig[l + w - L], v);
      } else {
        const double* ga = th + (k - AL) * L;
        for (int w = 0; w < L; ++w) v += ga[w];
      }
      if constexpr (std::is_same<OutT, double2>::value)
        row[k] = make_double2(v, 0.0);
      else if constexpr (std::is_same<OutT, float2>::value)
        row[k] = make_float2((float)v, 0.0f);
      else
        row[k] = (OutT)v;
    }
    se_wave_sync();
  }
}

struct se_samp_args {
  const double2* p;
  int L, alpha, W;
  int64_t nc;
  uint2 key;
  uint64_t t0;
  int init;
  int64_t therm_steps, sweep, n_record;
  uint64_t* bits;
  uint64_t* s_out;
  double2* lp_out;
  unsigned long long* acc;
};

// Metropolis chains, one wave per chain, single-site flips with the Philox
// stream of the network samplers: proposal t of chain c uses counter
// (c, t_lo, t_hi, 0): site idx(x0, L), u = unif(x1, x2); initial bits from
// counter (c, w / 2, 0, 2).  theta is updated additively on acceptance and
// recomputed from sigma at every recorded sample.
__global__ __launch_bounds__(SE_NT) void k_se_metropolis(se_samp_args a) {
  extern __shared__ double lds[];
  const int L = a.L, alpha = a.alpha, AL = alpha * L;
  double* Ws = lds;
  double* bs = Ws + AL;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* sig = bs + alpha + wave * (L + 2 * AL);
  double* th = sig + L;
  double* ev = th + AL;
  se_stage(a.p, L, alpha, Ws, bs);
  const int64_t c = (int64_t)blockIdx.x * SE_WAVES + wave;
  if (c >= a.nc) return;  // no group barrier after this point
  uint64_t word = 0ull;  // lane w < W holds word w of the configuration
  if (a.init) {
    if (lane < a.W) {
      const uint4 x = philox(make_uint4((uint32_t)c, (uint32_t)(lane >> 1), 0u, 2u), a.key);
      word = (lane & 1) == 0 ? ((uint64_t)x.x | ((uint64_t)x.y << 32)) : ((uint64_t)x.z | ((uint64_t)x.w << 32));
      const int rem = L - 64 * lane;
      if (rem < 64) word &= (1ull << rem) - 1ull;
    }
  } else if (lane < a.W) {
    word = a.bits[c * a.W + lane];
  }
  // sigma and theta from the words
  for (int l = lane; l < L; l += 64) {
    const uint64_t wv = __shfl(word, l >> 6, 64);
    sig[l] = ((wv >> (l & 63)) & 1ull) ? 1.0 : -1.0;
  }
  se_wave_sync();
  auto full = [&]() {
    for (int q = lane; q < AL; q += 64) {
      const int aa = q / L, w = q - aa * L;
      const double* Wa = Ws + aa * L;
      double acc = bs[aa];
      int l = 0;
      for (; l < L - w; ++l) acc = fma(Wa[l], sig[l + w], acc);
      for (; l < L; ++l) acc = fma(Wa[l], sig[l + w - L], acc);
      th[q] = acc;
      ev[q] = elu(acc);
    }
    se_wave_sync();
  };
  full();
  unsigned long long na = 0;
  uint64_t t = a.t0;
  auto step = [&]() {
    const uint4 x = philox(make_uint4((uint32_t)c, (uint32_t)t, (uint32_t)(t >> 32), 0u), a.key);
    const int j = (int)to_index(x.x, (uint32_t)L);
    const double u = to_uniform(x.y, x.z);
    const double cj = -2.0 * sig[j];
    double d = 0.0;
    for (int q = lane; q < AL; q += 64) {
      const int aa = q / L, w = q - aa * L;
      const int lj = j - w < 0 ? j - w + L : j - w;
      d += elu(fma(cj, Ws[aa * L + lj], th[q])) - ev[q];
    }
    d = wave_sum(d);
    const double r = 2.0 * d;
    if (r >= 0.0 || u < exp(r)) {  // uniform decision
      for (int q = lane; q < AL; q += 64) {
        const int aa = q / L, w = q - aa * L;
        const int lj = j - w < 0 ? j - w + L : j - w;
        const double tn = fma(cj, Ws[aa * L + lj], th[q]);
        th[q] = tn;
        ev[q] = elu(tn);
      }
      se_wave_sync();
      if (lane == 0) sig[j] = -sig[j];
      if (lane == (j >> 6)) word ^= 1ull << (j & 63);
      ++na;
      se_wave_sync();
    }
    ++t;
  };
  for (int64_t q = 0; q < a.therm_steps; ++q) step();
  for (int64_t k = 0; k < a.n_record; ++k) {
    for (int64_t q = 0; q < a.sweep; ++q) step();
    full();
    double lp = 0.0;
    for (int q = lane; q < AL; q += 64) lp += ev[q];
    lp = wave_sum(lp);
    if (lane < a.W) a.s_out[(k * a.nc + c) * a.W + lane] = word;
    if (lane == 0 && a.lp_out) a.lp_out[k * a.nc + c] = make_double2(lp, 0.0);
  }
  if (lane < a.W) a.bits[c * a.W + lane] = word;
  if (lane == 0) a.acc[c] = na;
}

size_t se_lds(int L, int alpha, int per_wave_arrays) {
  return sizeof(double) * ((size_t)alpha * L + alpha + (size_t)SE_WAVES * ((size_t)L + (size_t)per_wave_arrays * alpha * L));
}

int64_t se_groups(int64_t units, size_t lds) {
  const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(8, (int64_t)(160 * 1024) / (int64_t)lds));
  return std::max<int64_t>(1, std::min<int64_t>((units + SE_WAVES - 1) / SE_WAVES, 256 * per_cu));
}

constexpr size_t kSeLdsMax = 64 * 1024;

}  // namespace

void symelu_check(const vmc_model* m) {
  VMC_REQUIRE(se_lds(m->N, m->C, 2) <= kSeLdsMax, "alpha * L too large for the per-configuration tile");
}

void symelu_log_psi(vmc_model* m, const uint64_t* s, int64_t B, double2* out) {
  const size_t lds = se_lds(m->N, m->C, 1);
  k_se_log_psi<<<(unsigned)se_groups(B, lds), SE_NT, lds, m->ctx->stream>>>(s, B, m->W, m->N, m->C, m->params, out);
  VMC_HIP(hipGetLastError());
}

void symelu_local_energy(vmc_model* m, vmc_ham* H, const uint64_t* s, int64_t B, double2* eloc) {
  const size_t lds = se_lds(m->N, m->C, 2);
  k_se_eloc<<<(unsigned)se_groups(B, lds), SE_NT, lds, m->ctx->stream>>>(s, B, m->W, m->N, m->C, m->params, H->kind,
                                                                         H->J, H->h, H->bonds, H->n_bonds, eloc);
  VMC_HIP(hipGetLastError());
}

void symelu_grad(vmc_model* m, const uint64_t* s, int64_t B, void* O, int dtype) {
  const size_t lds = se_lds(m->N, m->C, 1);
  const unsigned g = (unsigned)se_groups(B, lds);
  hipStream_t st = m->ctx->stream;
  if (dtype == VMC_DT_C128)
    k_se_grad<double2><<<g, SE_NT, lds, st>>>(s, B, m->W, m->N, m->C, m->params, (double2*)O);
  else if (dtype == VMC_DT_C64)
    k_se_grad<float2><<<g, SE_NT, lds, st>>>(s, B, m->W, m->N, m->C, m->params, (float2*)O);
  else if (dtype == VMC_DT_F64)
    k_se_grad<double><<<g, SE_NT, lds, st>>>(s, B, m->W, m->N, m->C, m->params, (double*)O);
  else
    k_se_grad<float><<<g, SE_NT, lds, st>>>(s, B, m->W, m->N, m->C, m->params, (float*)O);
  VMC_HIP(hipGetLastError());
}

void symelu_sampler_run(vmc_sampler* S, int64_t n_per_chain, uint64_t* s_out, double2* logpsi_out) {
  vmc_model* m = S->model;
  se_samp_args a{};
  a.p = m->params;
  a.L = m->N;
  a.alpha = m->C;
  a.W = m->W;
  a.nc = S->opts.n_chains;
  a.key = make_uint2((uint32_t)S->opts.seed, (uint32_t)(S->opts.seed >> 32));
  a.t0 = S->t;
  a.init = !S->bits_valid;
  a.therm_steps = S->thermalized ? 0 : (int64_t)S->opts.therm_sweeps * S->opts.sweep_steps;
  a.sweep = S->opts.sweep_steps;
  a.n_record = n_per_chain;
  a.bits = S->bits;
  a.s_out = s_out;
  a.lp_out = logpsi_out;
  a.acc = S->acc;
  const size_t lds = se_lds(m->N, m->C, 2);
  k_se_metropolis<<<(unsigned)((a.nc + SE_WAVES - 1) / SE_WAVES), SE_NT, lds, S->ctx->stream>>>(a);
  VMC_HIP(hipGetLastError());
  S->t += (uint64_t)(a.therm_steps + n_per_chain * a.sweep);
  S->thermalized = 1;
  S->bits_valid = 1;
}
