// Tabulated wave function (test model, N <= 24): the parameters are the 2^N
// complex log-amplitudes themselves, theta_code = log psi(s) with code = the
// configuration's bits (site i = bit i).  Every quantity of the method is then
// exact: log psi is a lookup, O_k(s) = [k = code(s)], and the local energy of
// eq:Oloc reads the connected amplitudes from the table, so a table holding an
// exact eigenvector has E_loc(s) = E_0 for every s with psi(s) != 0 (Sec. 5.1).
// The Metropolis kernel follows the same Philox stream, proposals and
// acceptance rule as the network samplers (one chain per lane).
#include <hip/hip_runtime.h>

#include "internal.h"

using namespace dev;

namespace {

__device__ __forceinline__ double2 cexp_d(double2 z) {
  double s, c;
  sincos(z.y, &s, &c);
  const double m = exp(z.x);
  return make_double2(m * c, m * s);
}

__global__ void k_table_log_psi(const uint64_t* __restrict__ s, int64_t B, int W, uint32_t mask,
                                const double2* __restrict__ theta, double2* __restrict__ out) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b < B) out[b] = theta[(uint32_t)s[b * W] & mask];
}

// one configuration per thread, slots in the canonical order (diagonal, then
// flips of every site or swaps of every anti-aligned bond)
__global__ void k_table_eloc(const uint64_t* __restrict__ s, int64_t B, int W, int N, const double2* __restrict__ theta,
                             int kind, double J, double hx, const int2* __restrict__ bonds, int n_bonds,
                             double2* __restrict__ eloc) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= B) return;
  const uint32_t mask = N >= 32 ? 0xffffffffu : ((1u << N) - 1u);
  const uint32_t code = (uint32_t)s[b * W] & mask;
  const double2 lp = theta[code];
  int n_al = 0;
  for (int q = 0; q < n_bonds; ++q) {
    const int2 bd = bonds[q];
    n_al += (((code >> bd.x) ^ (code >> bd.y)) & 1u) == 0u;
  }
  const double diag = (kind == HAM_TFIM ? -J : J) * (double)(n_al - (n_bonds - n_al));
  double2 e = make_double2(diag, 0.0);
  if (kind == HAM_TFIM && hx != 0.0) {
    for (int l = 0; l < N; ++l) {
      const double2 r = cexp_d(csub(theta[code ^ (1u << l)], lp));
      e = cadd(e, make_double2(-hx * r.x, -hx * r.y));
    }
  } else if (kind == HAM_HEIS && J != 0.0) {
    for (int q = 0; q < n_bonds; ++q) {
      const int2 bd = bonds[q];
      if ((((code >> bd.x) ^ (code >> bd.y)) & 1u) == 0u) continue;
      const double2 r = cexp_d(csub(theta[code ^ (1u << bd.x) ^ (1u << bd.y)], lp));
      e = cadd(e, make_double2(2.0 * J * r.x, 2.0 * J * r.y));
    }
  }
  eloc[b] = e;
}

template <typename OutT>
__global__ void k_table_grad(const uint64_t* __restrict__ s, int64_t B, int W, uint32_t mask, int64_t K,
                             OutT* __restrict__ O) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= B * K) return;
  const int64_t b = e / K, k = e % K;
  const double v = ((uint32_t)s[b * W] & mask) == (uint32_t)k ? 1.0 : 0.0;
  if constexpr (sizeof(OutT) == sizeof(double2))
    O[e] = make_double2(v, 0.0);
  else
    O[e] = make_float2((float)v, 0.0f);
}

struct tab_args {
  const double2* theta;
  int N, n_bonds, move_kind, init;
  const int2* bonds;
  int64_t nc;
  uint2 key;
  uint64_t t0;
  int64_t therm_steps, sweep, n_record;
  uint64_t* bits;
  uint64_t* s_out;
  double2* lp_out;
  unsigned long long* acc;
};

__global__ __launch_bounds__(256) void k_table_metropolis(tab_args a) {
  const int64_t c = blockIdx.x * 256ll + threadIdx.x;
  if (c >= a.nc) return;
  const int N = a.N;
  const uint32_t mask = N >= 32 ? 0xffffffffu : ((1u << N) - 1u);
  uint32_t code;
  if (a.init) {
    if (a.move_kind == 0) {
      const uint4 x = philox(make_uint4((uint32_t)c, 0u, 0u, 2u), a.key);
      code = x.x & mask;
    } else {  // Sz = 0: sites 0 .. N/2-1 up, Fisher-Yates with j = idx(x0, i + 1)
      code = (1u << (N / 2)) - 1u;
      for (int i = N - 1; i >= 1; --i) {
        const uint4 x = philox(make_uint4((uint32_t)c, (uint32_t)i, 1u, 2u), a.key);
        const int j = (int)to_index(x.x, (uint32_t)(i + 1));
        const uint32_t bi = (code >> i) & 1u, bj = (code >> j) & 1u;
        if (bi != bj) code ^= (1u << i) | (1u << j);
      }
    }
  } else {
    code = (uint32_t)a.bits[c] & mask;
  }
  double2 lp = a.theta[code];
  unsigned long long na = 0;
  uint64_t t = a.t0;
  auto step = [&]() {
    const uint4 x = philox(make_uint4((uint32_t)c, (uint32_t)t, (uint32_t)(t >> 32), 0u), a.key);
    uint32_t sp;
    if (a.move_kind == 0) {
      sp = code ^ (1u << to_index(x.x, (uint32_t)N));
    } else {
      const int2 bd = a.bonds[to_index(x.x, (uint32_t)a.n_bonds)];
      sp = (((code >> bd.x) ^ (code >> bd.y)) & 1u) ? code ^ (1u << bd.x) ^ (1u << bd.y) : code;
    }
    const double u = to_uniform(x.y, x.z);
    const double2 lpn = a.theta[sp];
    const double r = 2.0 * (lpn.x - lp.x);
    if (r >= 0.0 || u < exp(r)) {
      code = sp;
      lp = lpn;
      ++na;
    }
    ++t;
  };
  for (int64_t q = 0; q < a.therm_steps; ++q) step();
  for (int64_t k = 0; k < a.n_record; ++k) {
    for (int64_t q = 0; q < a.sweep; ++q) step();
    a.s_out[k * a.nc + c] = code;
    if (a.lp_out) a.lp_out[k * a.nc + c] = lp;
  }
  a.bits[c] = code;
  a.acc[c] = na;
}

}  // namespace

void table_log_psi(vmc_model* m, const uint64_t* s, int64_t B, double2* out) {
  const uint32_t mask = (1u << m->N) - 1u;
  k_table_log_psi<<<grid_for(B, 256), 256, 0, m->ctx->stream>>>(s, B, m->W, mask, m->params, out);
  VMC_HIP(hipGetLastError());
}

void table_local_energy(vmc_model* m, vmc_ham* H, const uint64_t* s, int64_t B, double2* eloc) {
  k_table_eloc<<<grid_for(B, 128), 128, 0, m->ctx->stream>>>(s, B, m->W, m->N, m->params, H->kind, H->J, H->h,
                                                             H->bonds, H->n_bonds, eloc);
  VMC_HIP(hipGetLastError());
}

void table_grad(vmc_model* m, const uint64_t* s, int64_t B, void* O, int dtype) {
  const uint32_t mask = (1u << m->N) - 1u;
  if (dtype == VMC_DT_C128)
    k_table_grad<double2><<<grid_for(B * m->K, 256), 256, 0, m->ctx->stream>>>(s, B, m->W, mask, m->K, (double2*)O);
  else
    k_table_grad<float2><<<grid_for(B * m->K, 256), 256, 0, m->ctx->stream>>>(s, B, m->W, mask, m->K, (float2*)O);
  VMC_HIP(hipGetLastError());
}

void table_sampler_run(vmc_sampler* S, int64_t n_per_chain, uint64_t* s_out, double2* logpsi_out) {
  vmc_model* m = S->model;
  tab_args a{};
  a.theta = m->params;
  a.N = m->N;
  a.n_bonds = S->ham->n_bonds;
  a.bonds = S->ham->bonds;
  a.move_kind = S->opts.proposal == VMC_PROP_EXCHANGE ? 1 : 0;
  a.init = !S->bits_valid;
  a.nc = S->opts.n_chains;
  a.key = make_uint2((uint32_t)S->opts.seed, (uint32_t)(S->opts.seed >> 32));
  a.t0 = S->t;
  a.therm_steps = S->thermalized ? 0 : (int64_t)S->opts.therm_sweeps * S->opts.sweep_steps;
  a.sweep = S->opts.sweep_steps;
  a.n_record = n_per_chain;
  a.bits = S->bits;
  a.s_out = s_out;
  a.lp_out = logpsi_out;
  a.acc = S->acc;
  k_table_metropolis<<<(unsigned)((a.nc + 255) / 256), 256, 0, S->ctx->stream>>>(a);
  VMC_HIP(hipGetLastError());
  S->t += (uint64_t)(a.therm_steps + n_per_chain * a.sweep);
  S->thermalized = 1;
  S->bits_valid = 1;
}
