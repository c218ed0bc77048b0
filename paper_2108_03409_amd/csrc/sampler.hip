// Metropolis sampler (Sec. 2.1 and Sec. 4.2 "Sampler"): all chains advance in
// sync, one wavefront per chain (two when the chains leave SIMDs idle), the
// chain's hidden units spread over the lanes (t_j = tanh theta_j in registers,
// theta_j in lane-private LDS slots).  A proposal costs N_h/64 complex
// multiply-adds per lane plus one wave reduction, using the move identity of
// rbm.hip:
//   2 Re(log psi(s') - log psi(s)) = 2 Re(-2 sigma_m alpha_m + LC_m)
//                                    + sum_j log|1 - sigma_m t_j T_jm|^2.
// On acceptance theta_j -= 2 sigma_m D_jm and t_j follows the tanh addition
// rule t' = (t - sigma T) / (1 - sigma t T); theta is rebuilt from the spins
// at the start of every call and t from theta at every recorded sample.
//
// VMC_PROP_MADE_MIX: each sweep starts with global Metropolis-Hastings steps
// made by all chains together (mixsampler.hip; the proposals of the next step
// are formed on a second stream during the sweep); the sweep's single-spin
// flips then run here, one launch per sweep, with each chain's theta kept in
// device memory between the launches.
#include "internal.h"

using namespace dev;

namespace {

struct sampler_args {
  const double2* params;
  const double2* Wt;
  const double2* T;  // [n_moves][N_h]
  const double2* D;  // [n_moves][N_h]
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
  unsigned long long* acc;  // [n_chains] accepted proposals (added to)
  double2* theta_store;     // [n_chains][N_h] theta kept between launches (NULL: none)
  int theta_in;             // 1: start from theta_store instead of rebuilding theta from the spins
};

// One chain per work-group of NW waves.  With NW = 2 (chains fewer than the
// device's SIMDs, so that one wave per chain would leave SIMDs idle) wave w
// takes the hidden units j = 64 Q w + 64 q + lane; both waves keep their own
// copy of the configuration and of the step tables and reach the same
// decisions, exchanging only their partial ratio (mantissa and exponent)
// through LDS behind one barrier per proposal.  Up to four slots of hidden
// units the kernel is held to 256 registers, so that two waves share a SIMD
// (1 024 chains of two waves fill 2 048 wave slots on 1 024 SIMDs).
template <int Q, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(Q <= 4 ? 2 : 1))) void k_metropolis(sampler_args a) {
  __shared__ uint64_t cbs[NW][64];  // chain configuration, W <= 64 words (one copy per wave)
  // theta_j of the chain in lane-private LDS slots [q][lane]: registers hold
  // only t_j = tanh theta_j (theta in registers measured slower)
  __shared__ double2 thss[NW][Q * 64];
  __shared__ double pm_s[2][NW];  // partial ratios of the waves (double-buffered by step parity)
  __shared__ int pe_s[2][NW];
  __shared__ double2 lp_s[NW];
  const int c = blockIdx.x;
  if (c >= a.n_chains) return;
  const int lane = threadIdx.x & 63;
  const int wv = NW == 1 ? 0 : __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  uint64_t* cb = cbs[wv];
  double2* ths = thss[wv];
  const int jb = 64 * Q * wv;  // first hidden unit of this wave
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

  // theta_j = b_j + sum_i W_ji sigma_i for the lane's hidden units (or the
  // value kept from the previous launch of this call)
  double2 tt[Q];
  auto theta = [&](int q) -> double2& { return ths[q * 64 + lane]; };
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int j = jb + lane + 64 * q;
    double2 acc = j < Nh ? a.params[N + j] : make_double2(0.0, 0.0);
    if (j < Nh) {
      if (a.theta_in) {
        acc = a.theta_store[(int64_t)c * Nh + j];
      } else {
        for (int i = 0; i < N; ++i) {
          const bool up = (cb[i >> 6] >> (i & 63)) & 1ull;
          const double2 w = a.Wt[(int64_t)i * Nh + j];
          acc.x += up ? w.x : -w.x;
          acc.y += up ? w.y : -w.y;
        }
      }
    }
    theta(q) = acc;
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) tt[q] = ctanh(theta(q));

  unsigned long long accepted = 0;
  const int64_t total = a.therm_steps + a.n_record * a.sweep;
  // The move of step t + 1 is known from its counter before step t resolves:
  // its rows of T (the ratio) and D (the update on acceptance) are loaded one
  // step ahead (local-move kernels with up to 512 hidden units, where the
  // extra registers fit).
  constexpr bool PF = Q <= 8;
  // The counters of 64 consecutive steps are drawn together, one per lane, into
  // a table of moves and log u (the same Philox values as one per step; the
  // test u < exp(r) is decided from log u, below, alike away from |r - log u|
  // at the rounding level).
  __shared__ int mv_ss[NW][64];
  __shared__ double uv_ss[NW][64];
  int* mv_s = mv_ss[wv];
  double* uv_s = uv_ss[wv];
  // entry (m, lane + 64 q) of a [n_moves][N_h] table, zero past N_h: the
  // address is clamped and the value selected, so the proposal and the update
  // run without branches over the lane's units (a unit past N_h has t = 0 and
  // T = D = 0, hence f = 1 and no change)
  auto row_entry = [&](const double2* tab, int m, int q) {
    const int j = jb + lane + 64 * q;
    const double2 v = tab[(int64_t)m * Nh + (j < Nh ? j : Nh - 1)];
    return j < Nh ? v : make_double2(0.0, 0.0);
  };
  auto draw64 = [&](int64_t s0) {
    const uint64_t tl = a.t0 + (uint64_t)(s0 + lane);
    const uint4 y = philox(make_uint4((uint32_t)c, (uint32_t)tl, (uint32_t)(tl >> 32), 0u), a.key);
    __syncthreads();
    mv_s[lane] = (int)to_index(y.x, (uint32_t)a.n_moves);
    uv_s[lane] = log(to_uniform(y.y, y.z));
    __syncthreads();
  };
  draw64(0);
  // Two sets of prefetch registers, A and B, alternate between the current
  // step's rows and the next step's (the loop runs two steps per trip), so
  // that no step copies its prefetched rows from one set to the other.
  constexpr int QP = PF ? Q : 1;
  double2 TA[QP], DA[QP], TB[QP], DB[QP];
  double2 alA = make_double2(0.0, 0.0), lcA = alA;  // alpha and LC of the move
  int2 bdA = make_int2(0, 0);                       // its bond (exchange moves)
  double2 alB = alA, lcB = alA;
  int2 bdB = bdA;
  if (PF) {
    const int mn = mv_s[0];
    alA = a.alpha[mn];
    lcA = a.LC[mn];
    if (a.proposal == VMC_PROP_EXCHANGE) bdA = a.bonds[mn];
#pragma unroll
    for (int q = 0; q < QP; ++q) {
      TA[q] = row_entry(a.T, mn, q);
      DA[q] = row_entry(a.D, mn, q);
    }
  }
  constexpr int NSTEP = PF ? 2 : 1;  // proposals per trip of the loop (one without prefetch)
  for (int64_t s0 = 0; s0 < total; s0 += NSTEP) {
#pragma unroll
  for (int h = 0; h < NSTEP; ++h) {
    const int64_t step = s0 + h;
    if (h > 0 && step >= total) break;
    // the current move's prefetched rows in (Tc, Dc, alc, lcc, bdc), the
    // next move's loaded into (Tn, Dn, aln, lcn, bdn)
    const double2(&Tc)[QP] = h ? TB : TA;
    const double2(&Dc)[QP] = h ? DB : DA;
    const double2 alc = h ? alB : alA, lcc = h ? lcB : lcA;
    const int2 bdc = h ? bdB : bdA;
    double2(&Tn)[QP] = h ? TA : TB;
    double2(&Dn)[QP] = h ? DA : DB;
    double2& aln = h ? alA : alB;
    double2& lcn = h ? lcA : lcB;
    int2& bdn = h ? bdA : bdB;
    const int m = mv_s[step & 63];
    const double lu = uv_s[step & 63];
    if (step + 1 < total) {
      if (((step + 1) & 63) == 0) draw64(step + 1);
      if (PF) {
        const int mn = mv_s[(step + 1) & 63];
        aln = a.alpha[mn];
        lcn = a.LC[mn];
        if (a.proposal == VMC_PROP_EXCHANGE) bdn = a.bonds[mn];
#pragma unroll
        for (int q = 0; q < QP; ++q) {
          Tn[q] = row_entry(a.T, mn, q);
          Dn[q] = row_entry(a.D, mn, q);
        }
      }
    }
    {
    int site = m, site2 = -1;
    bool identity = false;
    if (a.proposal == VMC_PROP_EXCHANGE) {
      const int2 bd = PF ? bdc : a.bonds[m];
      site = bd.x;
      site2 = bd.y;
      identity = ((cb[site >> 6] >> (site & 63)) & 1ull) == ((cb[site2 >> 6] >> (site2 & 63)) & 1ull);
    }
    if (identity) {
      ++accepted;
    } else {
      const double sg = ((cb[site >> 6] >> (site & 63)) & 1ull) ? 1.0 : -1.0;
      double prod = 1.0;
      // per hidden unit the factor f = 1 - sigma t_j T_jm and |f|^2, kept for the update
      double2 fq[Q];
      double nq[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const double2 p = cmul(tt[q], PF ? Tc[PF ? q : 0] : row_entry(a.T, m, q));
        fq[q] = make_double2(1.0 - sg * p.x, -sg * p.y);
        nq[q] = fq[q].x * fq[q].x + fq[q].y * fq[q].y;
        prod *= nq[q];
      }
      // accept iff L = sum_j log |f_j|^2 > lu - c, c = 2 Re(-2 sigma alpha + LC), without a
      // logarithm on the chain's path: each lane's product as mantissa in [1/2, 1) and
      // exponent, the wave's product M 2^E (M >= 2^-64, no underflow), and M 2^E > e^(lu - c)
      // tested as ldexp(M, E - n) > 2^r with (lu - c) / ln 2 = n + r, n integer, r in [0, 1);
      // n and 2^r do not depend on the ratio and are formed beside it.  Decides as
      // lu < c + L except within rounding of a tie.
      const double2 al = PF ? alc : a.alpha[m], lc = PF ? lcc : a.LC[m];
      const double t2 = fmin(fmax((lu - 2.0 * (-2.0 * sg * al.x + lc.x)) * 1.4426950408889634074, -4096.0), 4096.0);
      const double n2 = floor(t2);
      const double p2 = exp2(t2 - n2);
      int ex;
      const double mt = frexp(prod, &ex);
      double M = wave_prod_uniform(mt);
      int E = wave_isum_uniform(ex);
      if constexpr (NW > 1) {  // the other waves' units: every wave forms the same product
        const int par = (int)(step & 1);
        if (lane == 0) {
          pm_s[par][wv] = M;
          pe_s[par][wv] = E;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
        M = pm_s[par][0];
        E = pe_s[par][0];
#pragma unroll
        for (int w = 1; w < NW; ++w) {
          M *= pm_s[par][w];
          E += pe_s[par][w];
        }
      }
      const bool acc = ldexp(M, E - (int)n2) > p2;  // one value for the work-group: a uniform decision
      if (acc) {
        ++accepted;
        double2 th[Q];  // all LDS reads first: one wait instead of one per unit
#pragma unroll
        for (int q = 0; q < Q; ++q) th[q] = theta(q);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const double2 d = PF ? Dc[PF ? q : 0] : row_entry(a.D, m, q);
          const double2 Tm = PF ? Tc[PF ? q : 0] : row_entry(a.T, m, q);
          theta(q) = make_double2(th[q].x - 2.0 * sg * d.x, th[q].y - 2.0 * sg * d.y);
          // t' = (t - sigma T) / f = (t - sigma T) conj(f) / |f|^2, with 1 / |f|^2
          // from the hardware reciprocal and two Newton steps (|f|^2 > 0 here:
          // a zero factor gives a zero ratio, which is never accepted)
          const double2 nu = make_double2(tt[q].x - sg * Tm.x, tt[q].y - sg * Tm.y);
          double inv = __builtin_amdgcn_rcp(nq[q]);
          inv = fma(inv, fma(-nq[q], inv, 1.0), inv);
          inv = fma(inv, fma(-nq[q], inv, 1.0), inv);
          tt[q] = make_double2((nu.x * fq[q].x + nu.y * fq[q].y) * inv, (nu.y * fq[q].x - nu.x * fq[q].y) * inv);
        }
        // one wavefront per work-group: LDS operations of the wave stay in
        // program order, so the flips need no barrier and no returned value
        if (lane == 0) {
          __hip_atomic_fetch_xor(&cb[site >> 6], 1ull << (site & 63), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          if (site2 >= 0)
            __hip_atomic_fetch_xor(&cb[site2 >> 6], 1ull << (site2 & 63), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
    }
    }
    // record after every completed sweep of the recording phase
    if (step >= a.therm_steps && ((step - a.therm_steps + 1) % a.sweep) == 0) {
      const int64_t k = (step - a.therm_steps + 1) / a.sweep - 1;
      const int64_t row = k * a.n_chains + c;
      if (wv == 0)
        for (int w = lane; w < W; w += 64) a.s_out[row * W + w] = cb[w];
      double2 lp = make_double2(0.0, 0.0);
      if (wv == 0)
        for (int i = lane; i < N; i += 64) {
          const double2 av = a.params[i];
          const double sgi = ((cb[i >> 6] >> (i & 63)) & 1ull) ? 1.0 : -1.0;
          lp = cadd(lp, cscale(av, sgi));
        }
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int j = jb + lane + 64 * q;
        if (j < Nh) {
          const double2 thv = theta(q);
          lp = cadd(lp, clogcosh(thv));
          tt[q] = ctanh(thv);
        }
      }
      lp = wave_sum(lp);
      if constexpr (NW > 1) {  // records are rare: plain barriers around the exchange
        if (lane == 0) lp_s[wv] = lp;
        __syncthreads();
        lp = lp_s[0];
#pragma unroll
        for (int w = 1; w < NW; ++w) lp = cadd(lp, lp_s[w]);
        __syncthreads();
      }
      if (wv == 0 && lane == 0 && a.logpsi_out) a.logpsi_out[row] = lp;
    }
  }
  }
  if (wv == 0)
    for (int w = lane; w < W; w += 64) a.bits[(int64_t)c * W + w] = cb[w];
  if (a.theta_store)
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int j = jb + lane + 64 * q;
      if (j < Nh) a.theta_store[(int64_t)c * Nh + j] = theta(q);
    }
  if (wv == 0 && lane == 0) a.acc[c] += accepted;
}

__global__ void k_zero_u64(unsigned long long* p, int64_t n) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < n) p[e] = 0ull;
}

template <int NW>
void launch_nw(const sampler_args& a, int Q, hipStream_t st) {
  const dim3 blk(64 * NW);
  if (Q <= 1)
    k_metropolis<1, NW><<<a.n_chains, blk, 0, st>>>(a);
  else if (Q <= 2)
    k_metropolis<2, NW><<<a.n_chains, blk, 0, st>>>(a);
  else if (Q <= 4)
    k_metropolis<4, NW><<<a.n_chains, blk, 0, st>>>(a);
  else if (Q <= 8)
    k_metropolis<8, NW><<<a.n_chains, blk, 0, st>>>(a);
  else if (Q <= 16)
    k_metropolis<16, NW><<<a.n_chains, blk, 0, st>>>(a);
  else
    throw vmc_error{VMC_ERR_UNSUPPORTED, "sampler supports up to 1024 hidden units"};
  VMC_HIP(hipGetLastError());
}

// Two waves per chain when the chains leave SIMDs idle (at most one chain per
// SIMD) and each wave keeps more than two slots of 64 hidden units: measured
// at 1 024 chains, N_h = 400 (exchanges) 1.38 -> 1.24 ms per 8 sweeps, while
// at N_h = 256 (flips) the barrier per proposal costs more than the halved
// per-unit work saves (1.27 -> 1.50 ms per 16 sweeps).
void launch(vmc_ctx* ctx, const sampler_args& a, hipStream_t st) {
  const bool two = a.n_chains <= 4 * cu_count(ctx) && a.Nh > 256;
  if (two)
    launch_nw<2>(a, (a.Nh + 127) / 128, st);
  else
    launch_nw<1>(a, (a.Nh + 63) / 64, st);
}

}  // namespace

void sampler_run(vmc_sampler* S, int64_t n_per_chain, uint64_t* s_out, double2* logpsi_out) {
  vmc_model* m = S->model;
  VMC_REQUIRE(m->kind == MODEL_RBM, "sampler supports RBM models");
  VMC_REQUIRE(m->W <= 64, "sampler supports up to 4096 sites");
  const int move_kind = S->opts.proposal == VMC_PROP_EXCHANGE ? 1 : 0;
  rbm_ensure_tables(m, S->ham, move_kind);
  const rbm_move_tables& tb = m->tab[move_kind];
  const int nc = S->opts.n_chains;
  hipStream_t st = S->ctx->stream;
  sampler_args a{};
  a.params = m->params;
  a.Wt = m->Wt;
  a.T = tb.Tt;
  a.D = tb.Dt;
  a.LC = tb.LC;
  a.alpha = tb.alpha;
  a.bonds = S->ham->bonds;
  a.n_moves = tb.n_moves;
  a.proposal = S->opts.proposal;
  a.N = m->N;
  a.W = m->W;
  a.Nh = m->Nh;
  a.n_chains = nc;
  a.bits = S->bits;
  a.key = make_uint2((uint32_t)S->opts.seed, (uint32_t)(S->opts.seed >> 32));
  a.acc = S->acc;
  a.sweep = S->opts.sweep_steps;
  k_zero_u64<<<grid_for(3 * (int64_t)nc, 256), 256, 0, st>>>(S->acc, 3 * (int64_t)nc);
  if (S->opts.proposal != VMC_PROP_MADE_MIX) {
    a.t0 = S->t;
    a.init = !S->bits_valid;
    a.therm_steps = S->thermalized ? 0 : (int64_t)S->opts.therm_sweeps * S->opts.sweep_steps;
    a.n_record = n_per_chain;
    a.s_out = s_out;
    a.logpsi_out = logpsi_out;
    launch(S->ctx, a, st);
    S->t += (uint64_t)(a.therm_steps + a.n_record * a.sweep);
    S->thermalized = 1;
    S->bits_valid = 1;
    return;
  }
  // MADE_MIX: per sweep, global_steps global steps of all chains, then one
  // launch of the sweep's flips; theta is rebuilt once per call and kept in
  // S->mix_theta between the launches
  mix_ensure(S);
  a.theta_store = S->mix_theta;
  a.t0 = S->t;
  a.init = !S->bits_valid;
  a.theta_in = 0;
  a.therm_steps = 0;
  a.n_record = 0;
  launch(S->ctx, a, st);  // initial states (first call) and theta, no proposals
  S->bits_valid = 1;
  a.init = 0;
  a.theta_in = 1;
  const int64_t n_therm = S->thermalized ? 0 : S->opts.therm_sweeps;
  for (int64_t sw = 0; sw < n_therm + n_per_chain; ++sw) {
    for (int gs = 0; gs < S->opts.global_steps; ++gs) mix_global_step(S, S->g++);
    const bool rec = sw >= n_therm;
    a.t0 = S->t;
    a.therm_steps = rec ? 0 : a.sweep;
    a.n_record = rec ? 1 : 0;
    a.s_out = rec ? s_out + (sw - n_therm) * (int64_t)nc * m->W : nullptr;
    a.logpsi_out = (rec && logpsi_out) ? logpsi_out + (sw - n_therm) * (int64_t)nc : nullptr;
    launch(S->ctx, a, st);
    S->t += (uint64_t)a.sweep;
  }
  mix_wait_side(S);
  S->thermalized = 1;
}

namespace {
__global__ void k_copy_made(const double* __restrict__ W1mT, const double* __restrict__ W2m,
                            const double* __restrict__ params, int N, int H, double* __restrict__ buf) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t nh = (int64_t)N * H;
  if (e < nh) {
    buf[e] = W1mT[e];
    buf[nh + e] = W2m[e];
  }
  if (e < H) buf[2 * nh + e] = params[nh + e];
  if (e < N) buf[2 * nh + H + e] = params[2 * nh + H + e];
}
}  // namespace

// work buffers of the global steps (allocated on first use)
void mix_ensure(vmc_sampler* S) {
  const int64_t nc = S->opts.n_chains;
  if (!S->mix_tf) {  // the teacher-forcing workspace depends on the proposal's hidden size
    VMC_HIP(hipMalloc(&S->mix_tf, sizeof(double) * nc * ((int64_t)S->N + S->made_H)));
  }
  if (S->mix_prop) return;
  VMC_HIP(hipMalloc(&S->mix_prop, sizeof(uint64_t) * 2 * nc * S->W));
  VMC_HIP(hipMalloc(&S->mix_lq, sizeof(double) * 3 * nc));
  VMC_HIP(hipMalloc(&S->mix_theta, sizeof(double2) * nc * S->model->Nh));
  VMC_HIP(hipMalloc(&S->mix_theta_prop, sizeof(double2) * 2 * nc * S->model->Nh));
  VMC_HIP(hipStreamCreateWithFlags(&S->mix_side, hipStreamNonBlocking));
  VMC_HIP(hipEventCreateWithFlags(&S->mix_ev_main, hipEventDisableTiming));
  for (auto& e : S->mix_ev_prop) VMC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
}

void mix_release(vmc_sampler* S) {
  if (S->mix_side) (void)hipStreamSynchronize(S->mix_side);
  for (void* p : {(void*)S->mix_prop, (void*)S->mix_lq, (void*)S->mix_theta, (void*)S->mix_theta_prop, (void*)S->mix_tf})
    if (p) (void)hipFree(p);
  S->mix_prop = nullptr;
  S->mix_lq = nullptr;
  S->mix_theta = S->mix_theta_prop = nullptr;
  S->mix_tf = nullptr;
  for (auto& e : S->mix_ev_prop)
    if (e) (void)hipEventDestroy(e);
  if (S->mix_ev_main) (void)hipEventDestroy(S->mix_ev_main);
  if (S->mix_side) (void)hipStreamDestroy(S->mix_side);
  S->mix_ev_prop[0] = S->mix_ev_prop[1] = S->mix_ev_main = nullptr;
  S->mix_side = nullptr;
  S->mix_pg[0] = S->mix_pg[1] = ~0ull;
}

extern "C" int vmc_sampler_set_proposal_made(vmc_sampler* S, const vmc_made* md) {
  if (!S || !md) return VMC_ERR_INVALID_ARG;
  try {
    VMC_REQUIRE(md->ctx == S->ctx, "MADE belongs to another context");
    VMC_REQUIRE(md->N == S->N, "MADE input size differs from the sampler's site count");
    VMC_REQUIRE(md->H <= 1024, "MADE hidden size above 1024");
    VMC_HIP(hipSetDevice(S->ctx->device));
    VMC_REQUIRE(mix_made_fits(md->H, md->W),
                "MADE proposal too large for the batched global step (its pre-activations for 16 chains must fit "
                "in one work-group's LDS)");
    const int64_t nh = (int64_t)md->N * md->H;
    const size_t bytes = sizeof(double) * (size_t)(2 * nh + md->H + md->N);
    std::vector<int> perm, mstart;
    mix_made_layout(md->N, md->H, perm, mstart);
    perm.insert(perm.end(), mstart.begin(), mstart.end());
    VMC_HIP(hipStreamSynchronize(S->ctx->stream));
    if (S->mix_side) VMC_HIP(hipStreamSynchronize(S->mix_side));
    S->mix_pg[0] = S->mix_pg[1] = ~0ull;  // proposals of the previous network
    if (S->mix_tf) VMC_HIP(hipFree(S->mix_tf));
    S->mix_tf = nullptr;
    if (S->made_buf) VMC_HIP(hipFree(S->made_buf));
    if (S->mix_perm) VMC_HIP(hipFree(S->mix_perm));
    S->made_buf = nullptr;
    S->mix_perm = nullptr;
    S->made_H = 0;
    VMC_HIP(hipMalloc(&S->made_buf, bytes));
    VMC_HIP(hipMalloc(&S->mix_perm, sizeof(int) * perm.size()));
    VMC_HIP(hipMemcpy(S->mix_perm, perm.data(), sizeof(int) * perm.size(), hipMemcpyHostToDevice));
    S->made_H = md->H;
    const int64_t n = std::max<int64_t>(nh, std::max(md->H, md->N));
    k_copy_made<<<grid_for(n, 256), 256, 0, S->ctx->stream>>>(md->W1mT, md->W2m, md->params, md->N, md->H,
                                                               S->made_buf);
    VMC_HIP(hipGetLastError());
    S->ctx->err.clear();
    return VMC_OK;
  } catch (vmc_error& e) {
    S->ctx->err = e.msg;
    return e.code;
  }
}
