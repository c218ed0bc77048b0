// Metropolis sampler (Sec. 2.1 and Sec. 4.2 "Sampler"): all chains advance in
// sync, one wavefront per chain, the chain's hidden units spread over the 64
// lanes (theta_j and t_j = tanh theta_j live in registers).  A proposal costs
// N_h/64 complex multiply-adds per lane plus one wave reduction, using the
// move identity of rbm.hip:
//   2 Re(log psi(s') - log psi(s)) = 2 Re(-2 sigma_m alpha_m + LC_m)
//                                    + sum_j log|1 - sigma_m t_j T_jm|^2.
// On acceptance theta_j -= 2 sigma_m D_jm and t_j follows the tanh addition
// rule t' = (t - sigma T) / (1 - sigma t T); theta is rebuilt from the spins
// at the start of every call and t from theta at every recorded sample.
#include "internal.h"

using namespace dev;

namespace {

struct sampler_args {
  const double2* params;
  const double2* Wt;
  const double2* T;
  const double2* D;
  const double2* LC;
  const double2* alpha;
  const int2* bonds;
  int n_moves;
  int proposal;  // VMC_PROP_FLIP / VMC_PROP_EXCHANGE / VMC_PROP_MADE_MIX
  int N, W, Nh;
  int n_chains;
  uint64_t* bits;
  uint2 key;
  uint64_t t0;
  int init;             // draw initial states
  int64_t therm_steps;  // proposals before the first record
  int64_t n_record;
  int sweep;
  uint64_t* s_out;
  double2* logpsi_out;
  unsigned long long* acc;
};

template <int Q>
__global__ __launch_bounds__(64) void k_metropolis(sampler_args a) {
  __shared__ uint64_t cb[64];  // chain configuration, W <= 64 words
  const int c = blockIdx.x;
  if (c >= a.n_chains) return;
  const int lane = threadIdx.x;
  const int N = a.N, W = a.W, Nh = a.Nh;

  if (a.init) {
    if (lane == 0) {
      if (a.proposal != VMC_PROP_EXCHANGE) {
        for (int w = 0; w < W; ++w) {
          uint4 y = philox(make_uint4((uint32_t)c, (uint32_t)(w >> 1), 0u, 2u), a.key);
          uint64_t word = (w & 1) ? ((uint64_t)y.z | ((uint64_t)y.w << 32)) : ((uint64_t)y.x | ((uint64_t)y.y << 32));
          const int rem = N - 64 * w;
          if (rem < 64) word &= (1ull << rem) - 1ull;
          cb[w] = word;
        }
      } else {
        for (int w = 0; w < W; ++w) cb[w] = 0ull;
        for (int i = 0; i < N / 2; ++i) cb[i >> 6] |= 1ull << (i & 63);
        for (int i = N - 1; i >= 1; --i) {
          uint4 y = philox(make_uint4((uint32_t)c, (uint32_t)i, 1u, 2u), a.key);
          const int j = (int)to_index(y.x, (uint32_t)(i + 1));
          const uint64_t bi = (cb[i >> 6] >> (i & 63)) & 1ull, bj = (cb[j >> 6] >> (j & 63)) & 1ull;
          if (bi != bj) {
            cb[i >> 6] ^= 1ull << (i & 63);
            cb[j >> 6] ^= 1ull << (j & 63);
          }
        }
      }
    }
  } else {
    for (int w = lane; w < W; w += 64) cb[w] = a.bits[(int64_t)c * W + w];
  }
  __syncthreads();

  // theta_j = b_j + sum_i W_ji sigma_i for the lane's hidden units
  double2 th[Q], tt[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int j = lane + 64 * q;
    th[q] = j < Nh ? a.params[N + j] : make_double2(0.0, 0.0);
  }
  for (int i = 0; i < N; ++i) {
    const bool up = (cb[i >> 6] >> (i & 63)) & 1ull;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int j = lane + 64 * q;
      if (j < Nh) {
        const double2 w = a.Wt[(int64_t)i * Nh + j];
        th[q].x += up ? w.x : -w.x;
        th[q].y += up ? w.y : -w.y;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) tt[q] = ctanh(th[q]);

  unsigned long long accepted = 0;
  const int64_t total = a.therm_steps + a.n_record * a.sweep;
  for (int64_t step = 0; step < total; ++step) {
    const uint64_t t = a.t0 + (uint64_t)step;
    const uint4 x = philox(make_uint4((uint32_t)c, (uint32_t)t, (uint32_t)(t >> 32), 0u), a.key);
    const int m = (int)to_index(x.x, (uint32_t)a.n_moves);
    const double u = to_uniform(x.y, x.z);
    int site = m, site2 = -1;
    bool identity = false;
    if (a.proposal == VMC_PROP_EXCHANGE) {
      const int2 bd = a.bonds[m];
      site = bd.x;
      site2 = bd.y;
      identity = ((cb[site >> 6] >> (site & 63)) & 1ull) == ((cb[site2 >> 6] >> (site2 & 63)) & 1ull);
    }
    if (identity) {
      ++accepted;
    } else {
      const double sg = ((cb[site >> 6] >> (site & 63)) & 1ull) ? 1.0 : -1.0;
      double prod = 1.0;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int j = lane + 64 * q;
        if (j < Nh) {
          const double2 p = cmul(tt[q], a.T[(int64_t)j * a.n_moves + m]);
          const double fx = 1.0 - sg * p.x, fy = -sg * p.y;
          prod *= fx * fx + fy * fy;
        }
      }
      double L = wave_sum(log(prod));
      L = __shfl(L, 0, 64);  // one value for the whole wave: a uniform decision
      const double2 al = a.alpha[m], lc = a.LC[m];
      const double r = 2.0 * (-2.0 * sg * al.x + lc.x) + L;
      const bool acc = (r >= 0.0) || (u < exp(r));
      if (acc) {
        ++accepted;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int j = lane + 64 * q;
          if (j < Nh) {
            const double2 d = a.D[(int64_t)j * a.n_moves + m];
            const double2 Tm = a.T[(int64_t)j * a.n_moves + m];
            th[q].x -= 2.0 * sg * d.x;
            th[q].y -= 2.0 * sg * d.y;
            const double2 p = cmul(tt[q], Tm);
            tt[q] = cdiv(make_double2(tt[q].x - sg * Tm.x, tt[q].y - sg * Tm.y),
                         make_double2(1.0 - sg * p.x, -sg * p.y));
          }
        }
        __syncthreads();
        if (lane == 0) {
          cb[site >> 6] ^= 1ull << (site & 63);
          if (site2 >= 0) cb[site2 >> 6] ^= 1ull << (site2 & 63);
        }
        __syncthreads();
      }
    }
    // record after every completed sweep of the recording phase
    if (step >= a.therm_steps && ((step - a.therm_steps + 1) % a.sweep) == 0) {
      const int64_t k = (step - a.therm_steps + 1) / a.sweep - 1;
      const int64_t row = k * a.n_chains + c;
      for (int w = lane; w < W; w += 64) a.s_out[row * W + w] = cb[w];
      double2 lp = make_double2(0.0, 0.0);
      for (int i = lane; i < N; i += 64) {
        const double2 av = a.params[i];
        const double sgi = ((cb[i >> 6] >> (i & 63)) & 1ull) ? 1.0 : -1.0;
        lp = cadd(lp, cscale(av, sgi));
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int j = lane + 64 * q;
        if (j < Nh) {
          lp = cadd(lp, clogcosh(th[q]));
          tt[q] = ctanh(th[q]);
        }
      }
      lp = wave_sum(lp);
      if (lane == 0 && a.logpsi_out) a.logpsi_out[row] = lp;
    }
  }
  for (int w = lane; w < W; w += 64) a.bits[(int64_t)c * W + w] = cb[w];
  if (lane == 0) a.acc[c] = accepted;
}

template <int Q>
void launch(const sampler_args& a, hipStream_t st) {
  k_metropolis<Q><<<a.n_chains, 64, 0, st>>>(a);
}

}  // namespace

void sampler_run(vmc_sampler* S, int64_t n_per_chain, uint64_t* s_out, double2* logpsi_out) {
  vmc_model* m = S->model;
  VMC_REQUIRE(m->kind == MODEL_RBM, "sampler supports RBM models");
  VMC_REQUIRE(m->W <= 64, "sampler supports up to 4096 sites");
  VMC_REQUIRE(S->opts.proposal != VMC_PROP_MADE_MIX, "MADE proposals are handled by the mixed sampler");
  const int move_kind = S->opts.proposal == VMC_PROP_EXCHANGE ? 1 : 0;
  rbm_ensure_tables(m, S->ham, move_kind);
  const rbm_move_tables& tb = m->tab[move_kind];
  sampler_args a{};
  a.params = m->params;
  a.Wt = m->Wt;
  a.T = tb.T;
  a.D = tb.D;
  a.LC = tb.LC;
  a.alpha = tb.alpha;
  a.bonds = S->ham->bonds;
  a.n_moves = tb.n_moves;
  a.proposal = S->opts.proposal;
  a.N = m->N;
  a.W = m->W;
  a.Nh = m->Nh;
  a.n_chains = S->opts.n_chains;
  a.bits = S->bits;
  a.key = make_uint2((uint32_t)S->opts.seed, (uint32_t)(S->opts.seed >> 32));
  a.t0 = S->t;
  a.init = S->t == 0 && !S->thermalized;
  a.therm_steps = S->thermalized ? 0 : (int64_t)S->opts.therm_sweeps * S->opts.sweep_steps;
  a.n_record = n_per_chain;
  a.sweep = S->opts.sweep_steps;
  a.s_out = s_out;
  a.logpsi_out = logpsi_out;
  a.acc = S->acc;
  const int Q = (m->Nh + 63) / 64;
  hipStream_t st = S->ctx->stream;
  if (Q <= 1)
    launch<1>(a, st);
  else if (Q <= 2)
    launch<2>(a, st);
  else if (Q <= 4)
    launch<4>(a, st);
  else if (Q <= 8)
    launch<8>(a, st);
  else if (Q <= 16)
    launch<16>(a, st);
  else
    throw vmc_error{VMC_ERR_UNSUPPORTED, "sampler supports up to 1024 hidden units"};
  VMC_HIP(hipGetLastError());
  S->t += (uint64_t)(a.therm_steps + a.n_record * a.sweep);
  S->thermalized = 1;
}
