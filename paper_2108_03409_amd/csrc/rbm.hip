// RBM network kernels: pre-activations theta = W sigma + b over sample
// batches, log psi, the fused connected-configuration / local-energy kernel,
// and the per-sample log-derivatives O_k.
//
// Local energies (eq:Oloc) need psi(s')/psi(s) on every connected s'.  For the
// RBM of eq:rbm_ex a connected configuration differs from s by one flipped spin
// (TFIM) or one exchanged anti-aligned pair (Heisenberg), i.e. by a "move" m
// that shifts every pre-activation by theta_j -> theta_j - 2 sigma_m D_jm with
//   flip of site l:           D_jm = W_jl,          sigma_m = sigma_l,
//   exchange of bond (i,k):   D_jm = W_ji - W_jk,   sigma_m = sigma_i (= -sigma_k).
// cosh(theta - 2 sigma D) = cosh(theta) cosh(2D) (1 - sigma tanh(theta) tanh(2D)),
// so, exactly,
//   log psi(s') - log psi(s) = -2 sigma_m alpha_m + LC_m + sum_j log(1 - sigma_m t_j T_jm)
// with t_j = tanh(theta_j(s)), T_jm = tanh(2 D_jm), LC_m = sum_j log cosh(2 D_jm)
// and alpha_m = a_l (flip) or a_i - a_k (exchange).  T, LC and alpha depend on
// the parameters only and are tabulated once per parameter version; each
// connected configuration then costs N_h complex multiply-adds and no
// transcendental, instead of a fresh N x N_h network evaluation.
#include "internal.h"

using namespace dev;

namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));

int nh_pad16(int Nh) { return (Nh + 15) / 16 * 16; }
constexpr int kThRows = 64;  // samples per group of the matrix-core theta
constexpr int kThCols = 64;  // real columns per group (32 hidden units, re and im)
constexpr int kThKB = 4;     // k steps (4 sites each) whose operand loads are issued together

// theta = b + W sigma on the float64 matrix cores.  With Wt viewed as reals
// [N][2 N_h] (column c = 2 j + re/im), theta[n][c] = b[c] + sum_i sigma_i(n) Wt[i][c]:
// a group takes 64 samples x 64 columns, wave w the samples 16 w .. 16 w + 15
// against four 16-column tiles.  v_mfma_f64_16x16x4f64: lane l holds
// A[l % 16][l / 16] (sample, site), B[l / 16][l % 16] (site, column) and, in
// register r, D[l / 16 + 4 r][l % 16].  sigma = +-1 is exact; the sums are
// float64 in the matrix core's order.
__global__ __launch_bounds__(256) void k_theta_mfma(const double* __restrict__ bre, const double* __restrict__ Wr,
                                                    const uint64_t* __restrict__ s, int64_t B, int N, int W, int Nh,
                                                    double* __restrict__ theta) {
  extern __shared__ uint64_t sbits[];  // [kThRows][W]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t n0 = (int64_t)blockIdx.y * kThRows;
  const int ncol = 2 * Nh;
  const int c0 = blockIdx.x * kThCols;
  for (int e = tid; e < kThRows * W; e += 256) {
    const int64_t n = n0 + e / W;
    sbits[e] = n < B ? s[n * W + e % W] : 0ull;
  }
  __syncthreads();
  const uint64_t* myb = sbits + (wave * 16 + li) * W;  // the bits of the lane's A row
  const bool row_ok = n0 + wave * 16 + li < B;
  doublex4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = doublex4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < N; k0 += 4 * kThKB) {
    double bv[kThKB][4];
#pragma unroll
    for (int kb = 0; kb < kThKB; ++kb) {
      const int k = k0 + 4 * kb + lk;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int c = c0 + 16 * t + li;
        bv[kb][t] = (k < N && c < ncol) ? Wr[(int64_t)k * ncol + c] : 0.0;
      }
    }
#pragma unroll
    for (int kb = 0; kb < kThKB; ++kb) {
      const int k = k0 + 4 * kb + lk;
      const double a = (k < N && row_ok) ? (((myb[k >> 6] >> (k & 63)) & 1ull) ? 1.0 : -1.0) : 0.0;
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv[kb][t], acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int c = c0 + 16 * t + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t n = n0 + wave * 16 + lk + 4 * r;
      if (n < B && c < ncol) theta[n * ncol + c] = acc[t][r] + bre[c];
    }
  }
}

// log psi(n) = sum_i a_i sigma_i + sum_j logcosh(theta_j); one wave per sample.
__global__ __launch_bounds__(64) void k_logpsi(const double2* __restrict__ params, const double2* __restrict__ theta,
                                               const uint64_t* __restrict__ s, int64_t B, int N, int W, int Nh,
                                               double2* __restrict__ logpsi) {
  const int64_t n = blockIdx.x;
  if (n >= B) return;
  const int lane = threadIdx.x;
  double2 acc = make_double2(0.0, 0.0);
  const uint64_t* sn = s + n * W;
  for (int i = lane; i < N; i += 64) {
    const double2 a = params[i];
    const double sg = get_bit(sn, i) ? 1.0 : -1.0;
    acc = cadd(acc, cscale(a, sg));
  }
  for (int j = lane; j < Nh; j += 64) acc = cadd(acc, clogcosh(theta[n * Nh + j]));
  acc = wave_sum(acc);
  if (lane == 0) logpsi[n] = acc;
}

// Move tables: one wave per move m.
// T and D [N_h][n_moves]; T holds zero rows past N_h up to Nhp (a multiple of 16)
__global__ __launch_bounds__(64) void k_tables(const double2* __restrict__ params, const int2* __restrict__ bonds,
                                               int move_kind, int n_moves, int N, int Nh, int Nhp, double2* __restrict__ T,
                                               double2* __restrict__ D, double2* __restrict__ LC,
                                               double2* __restrict__ alpha) {
  const int m = blockIdx.x;
  if (m >= n_moves) return;
  const int lane = threadIdx.x;
  const double2* Wm = params + N + Nh;
  int i, k = -1;
  if (move_kind == 0) {
    i = m;
  } else {
    i = bonds[m].x;
    k = bonds[m].y;
  }
  double2 lc = make_double2(0.0, 0.0);
  for (int j = lane; j < Nh; j += 64) {
    double2 d = Wm[(int64_t)j * N + i];
    if (k >= 0) d = csub(d, Wm[(int64_t)j * N + k]);
    const double2 d2 = cscale(d, 2.0);
    D[(int64_t)j * n_moves + m] = d;
    T[(int64_t)j * n_moves + m] = ctanh(d2);
    lc = cadd(lc, clogcosh(d2));
  }
  for (int j = Nh + lane; j < Nhp; j += 64) T[(int64_t)j * n_moves + m] = make_double2(0.0, 0.0);
  lc = wave_sum(lc);
  if (lane == 0) {
    LC[m] = lc;
    alpha[m] = k >= 0 ? csub(params[i], params[k]) : params[i];
  }
}

// Local energies, S samples per wavefront, for move sets shared by all samples
// (single-spin flips of the TFIM; the kernel also accepts bonds, masked per
// sample to the anti-aligned ones).  Lanes run over the moves, and every table
// entry T_jm read from memory serves the S samples, whose tanh theta_j sit in
// LDS.  For each (sample,
// move) the product prod_j (1 - sigma t_j T_jm) is kept with exact
// power-of-two rescaling, and
//   E_loc = diag + mel * sum_m exp(-2 sigma_m alpha_m + LC_m + log prod).
template <int S>
__global__ __launch_bounds__(64) void k_eloc(const double2* __restrict__ theta, const uint64_t* __restrict__ s,
                                             int64_t B, int N, int W, int Nh, int ham_kind, double J, double h,
                                             const int2* __restrict__ bonds, int n_bonds,
                                             const double2* __restrict__ T, const double2* __restrict__ LC,
                                             const double2* __restrict__ alpha, int n_moves,
                                             double2* __restrict__ eloc) {
  extern __shared__ double2 tl[];  // [S][Nh]
  const int64_t b0 = (int64_t)blockIdx.x * S;
  if (b0 >= B) return;
  const int lane = threadIdx.x;
  for (int e = lane; e < S * Nh; e += 64) {
    const int q = e / Nh, j = e - q * Nh;
    tl[e] = b0 + q < B ? ctanh(theta[(b0 + q) * Nh + j]) : make_double2(0.0, 0.0);
  }
  // diagonal element: coupling * (n_aligned - n_anti), exact integer count
  double diag[S];
#pragma unroll
  for (int q = 0; q < S; ++q) {
    int n_al = 0;
    if (b0 + q < B) {
      const uint64_t* sn = s + (b0 + q) * W;
      for (int b = lane; b < n_bonds; b += 64) {
        const int2 bd = bonds[b];
        n_al += get_bit(sn, bd.x) == get_bit(sn, bd.y);
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) n_al += __shfl_xor(n_al, o, 64);
    const int n_anti = n_bonds - n_al;
    diag[q] = ham_kind == HAM_TFIM ? -J * (double)(n_al - n_anti) : J * (double)(n_al - n_anti);
  }
  __syncthreads();
  const double mel = ham_kind == HAM_TFIM ? -h : 2.0 * J;
  const bool off = ham_kind == HAM_TFIM ? h != 0.0 : J != 0.0;
  double2 acc[S];
#pragma unroll
  for (int q = 0; q < S; ++q) acc[q] = make_double2(0.0, 0.0);
  if (off)
    for (int m0 = 0; m0 < n_moves; m0 += 64) {
      const int m = m0 + lane;
      if (m >= n_moves) continue;
      const int site = ham_kind == HAM_TFIM ? m : bonds[m].x;
      const int site2 = ham_kind == HAM_TFIM ? -1 : bonds[m].y;
      double sg[S];
      bool active[S];
      double2 P[S];
      int e2[S];
#pragma unroll
      for (int q = 0; q < S; ++q) {
        const bool in = b0 + q < B;
        const uint64_t* sn = s + (in ? b0 + q : b0) * W;
        const int bi = get_bit(sn, site);
        sg[q] = bi ? 1.0 : -1.0;
        active[q] = in && (site2 < 0 || bi != get_bit(sn, site2));
        P[q] = make_double2(1.0, 0.0);
        e2[q] = 0;
      }
      const double2* Tm = T + m;
      for (int j0 = 0; j0 < Nh; j0 += 32) {
        const int j1 = min(Nh, j0 + 32);
        for (int jb = j0; jb < j1; jb += 8) {
          // eight table loads in flight before the products that use them
          double2 Tv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u)
            Tv[u] = jb + u < j1 ? Tm[(int64_t)(jb + u) * n_moves] : make_double2(0.0, 0.0);
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            if (jb + u >= j1) break;
            const int j = jb + u;
#pragma unroll
            for (int q = 0; q < S; ++q) {
              const double2 tt = cmul(tl[q * Nh + j], Tv[u]);
              P[q] = cmul(P[q], make_double2(1.0 - sg[q] * tt.x, -sg[q] * tt.y));
            }
          }
        }
        // keep |P| near 1: exact power-of-two rescaling
#pragma unroll
        for (int q = 0; q < S; ++q) {
          int e;
          frexp(fmax(fabs(P[q].x), fabs(P[q].y)), &e);
          P[q].x = ldexp(P[q].x, -e);
          P[q].y = ldexp(P[q].y, -e);
          e2[q] += e;
        }
      }
      const double2 al = alpha[m], lcm = LC[m];
#pragma unroll
      for (int q = 0; q < S; ++q) {
        if (!active[q]) continue;
        double2 lr = cadd(cscale(al, -2.0 * sg[q]), lcm);
        const double2 lp = clog(P[q]);
        lr.x += lp.x + (double)e2[q] * 0.69314718055994530942;
        lr.y += lp.y;
        acc[q] = cadd(acc[q], cscale(cexp(lr), mel));
      }
    }
#pragma unroll
  for (int q = 0; q < S; ++q) {
    const double2 v = wave_sum(acc[q]);
    if (lane == 0 && b0 + q < B) eloc[b0 + q] = make_double2(v.x + diag[q], v.y);
  }
}

// Fused enumeration + evaluation + reduction of E_loc, one wave per sample, for
// move sets that depend on the sample (exchanges of anti-aligned bonds).
// LDS: t_j (Nh complex) and the compacted move list (<= n_moves ints).
__global__ __launch_bounds__(64) void k_eloc_compact(const double2* __restrict__ theta, const uint64_t* __restrict__ s,
                                             int64_t B, int N, int W, int Nh, int ham_kind, double J, double h,
                                             const int2* __restrict__ bonds, int n_bonds,
                                             const double2* __restrict__ T, const double2* __restrict__ LC,
                                             const double2* __restrict__ alpha, int n_moves, int Nhp,
                                             double2* __restrict__ eloc) {
  // sigma t_j for both spins: tpm[0][j] = -t_j, tpm[1][j] = t_j, zero past N_h up
  // to Nhp (a multiple of 16, where the table rows are zero as well)
  extern __shared__ double2 lds[];
  double2* tpm = lds;                            // [2][Nhp]
  int* moves = (int*)(lds + 2 * Nhp);            // [n_moves]
  const int64_t n = blockIdx.x;
  if (n >= B) return;
  const int lane = threadIdx.x;
  const uint64_t* sn = s + n * W;

  for (int j = lane; j < Nhp; j += 64) {
    const double2 tj = j < Nh ? ctanh(theta[n * Nh + j]) : make_double2(0.0, 0.0);
    tpm[j] = make_double2(-tj.x, -tj.y);
    tpm[Nhp + j] = tj;
  }

  // diagonal element: coupling * (n_aligned - n_anti), exact integer count
  int n_al = 0;
  for (int b = lane; b < n_bonds; b += 64) {
    const int2 bd = bonds[b];
    n_al += get_bit(sn, bd.x) == get_bit(sn, bd.y);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) n_al += __shfl_xor(n_al, o, 64);
  const int n_anti = n_bonds - n_al;
  const double diag = ham_kind == HAM_TFIM ? -J * (double)(n_al - n_anti) : J * (double)(n_al - n_anti);

  // compacted list of off-diagonal moves in slot order
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
    if (J != 0.0) {
      for (int b0 = 0; b0 < n_bonds; b0 += 64) {
        const int b = b0 + lane;
        bool anti = false;
        if (b < n_bonds) {
          const int2 bd = bonds[b];
          anti = get_bit(sn, bd.x) != get_bit(sn, bd.y);
        }
        const uint64_t mask = __ballot(anti);
        const int pos = n_slots + __popcll(mask & ((1ull << lane) - 1ull));
        if (anti) moves[pos] = b;
        n_slots += __popcll(mask);
      }
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
      const double sg = up ? 1.0 : -1.0;
      const double2* st = tpm + (up ? Nhp : 0);  // sigma t of this slot's spin
      double2 P = make_double2(1.0, 0.0);
      int e2 = 0;
      const double2* Tm = T + m;  // column m; rows n_moves apart (fewer than 2^31 entries)
      for (int j0 = 0; j0 < Nhp; j0 += 16) {
#pragma unroll
        for (int jb = j0; jb < j0 + 16; jb += 8) {
          double2 Tv[8];  // eight table loads in flight before their products
#pragma unroll
          for (int u = 0; u < 8; ++u) Tv[u] = Tm[(jb + u) * n_moves];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const double2 tt = cmul(st[jb + u], Tv[u]);  // sigma t_j T_jm
            P = cmul(P, make_double2(1.0 - tt.x, -tt.y));
          }
        }
        // keep |P| near 1: exact power-of-two rescaling
        int e;
        frexp(fmax(fabs(P.x), fabs(P.y)), &e);
        P.x = ldexp(P.x, -e);
        P.y = ldexp(P.y, -e);
        e2 += e;
      }
      const double2 a = alpha[m];
      double2 lr = cadd(cscale(a, -2.0 * sg), LC[m]);
      const double2 lp = clog(P);
      lr.x += lp.x + (double)e2 * 0.69314718055994530942;
      lr.y += lp.y;
      acc = cadd(acc, cscale(cexp(lr), mel));
    }
  }
  acc = wave_sum(acc);
  if (lane == 0) eloc[n] = make_double2(acc.x + diag, acc.y);
}

// O_k rows: [sigma (N), t (Nh), t_j sigma_i (Nh x N)]; one block per sample.
template <typename OutT>
__global__ __launch_bounds__(256) void k_grad(const double2* __restrict__ theta, const uint64_t* __restrict__ s,
                                              int64_t B, int N, int W, int Nh, int64_t K, OutT* __restrict__ O) {
  extern __shared__ double2 tl[];  // [Nh]
  const int64_t n = blockIdx.x;
  if (n >= B) return;
  const int tid = threadIdx.x;
  const uint64_t* sn = s + n * W;
  for (int j = tid; j < Nh; j += 256) tl[j] = ctanh(theta[n * Nh + j]);
  __syncthreads();
  OutT* row = O + n * K;
  auto put = [&](int64_t k, double2 v) {
    if constexpr (sizeof(OutT) == sizeof(double2))
      row[k] = v;
    else
      row[k] = make_float2((float)v.x, (float)v.y);
  };
  for (int i = tid; i < N; i += 256) put(i, make_double2(get_bit(sn, i) ? 1.0 : -1.0, 0.0));
  for (int j = tid; j < Nh; j += 256) put(N + j, tl[j]);
  const int64_t nw = (int64_t)N * Nh;
  for (int64_t e = tid; e < nw; e += 256) {
    const int j = (int)(e / N);
    const int i = (int)(e - (int64_t)j * N);
    const double2 v = tl[j];
    put(N + Nh + e, get_bit(sn, i) ? v : make_double2(-v.x, -v.y));
  }
}

// get_s_primes as a test export: one thread per sample.
__global__ void k_connected(const uint64_t* __restrict__ s, int64_t B, int N, int W, int ham_kind, double J,
                            double h, const int2* __restrict__ bonds, int n_bonds, int M_max,
                            uint64_t* __restrict__ sp, double* __restrict__ mel, int32_t* __restrict__ count) {
  const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (n >= B) return;
  const uint64_t* sn = s + n * W;
  int n_al = 0;
  for (int b = 0; b < n_bonds; ++b) n_al += get_bit(sn, bonds[b].x) == get_bit(sn, bonds[b].y);
  const int n_anti = n_bonds - n_al;
  uint64_t* out = sp + n * (int64_t)M_max * W;
  double* me = mel + n * (int64_t)M_max;
  auto copy_s = [&](int slot) {
    for (int w = 0; w < W; ++w) out[(int64_t)slot * W + w] = sn[w];
  };
  copy_s(0);
  me[0] = ham_kind == HAM_TFIM ? -J * (double)(n_al - n_anti) : J * (double)(n_al - n_anti);
  int c = 1;
  if (ham_kind == HAM_TFIM) {
    if (h != 0.0)
      for (int l = 0; l < N; ++l, ++c) {
        copy_s(c);
        out[(int64_t)c * W + (l >> 6)] ^= 1ull << (l & 63);
        me[c] = -h;
      }
  } else if (J != 0.0) {
    for (int b = 0; b < n_bonds; ++b) {
      const int i = bonds[b].x, k = bonds[b].y;
      if (get_bit(sn, i) == get_bit(sn, k)) continue;
      copy_s(c);
      out[(int64_t)c * W + (i >> 6)] ^= 1ull << (i & 63);
      out[(int64_t)c * W + (k >> 6)] ^= 1ull << (k & 63);
      me[c] = 2.0 * J;
      ++c;
    }
  }
  count[n] = c;
  for (int q = c; q < M_max; ++q) {
    copy_s(q);
    me[q] = 0.0;
  }
}

constexpr int64_t kChunk = 1 << 16;  // samples per theta chunk

}  // namespace

void rbm_theta(vmc_model* m, const uint64_t* s, int64_t B, double2* theta, hipStream_t st) {
  if (!st) st = m->ctx->stream;
  // at most 65535 row tiles per launch
  const int64_t chunk = (int64_t)65535 * kThRows;
  const unsigned gx = (unsigned)((2 * m->Nh + kThCols - 1) / kThCols);
  for (int64_t b0 = 0; b0 < B; b0 += chunk) {
    const int64_t nb = std::min(chunk, B - b0);
    k_theta_mfma<<<dim3(gx, (unsigned)((nb + kThRows - 1) / kThRows)), 256, sizeof(uint64_t) * kThRows * m->W,
                   st>>>((const double*)(m->params + m->N), (const double*)m->Wt, s + b0 * m->W, nb, m->N,
                                     m->W, m->Nh, (double*)(theta + b0 * m->Nh));
    VMC_HIP(hipGetLastError());
  }
}

namespace {
// [rows][cols] -> [cols][rows] for two tables at once (sampler layout)
__global__ void k_transpose2(const double2* __restrict__ A, const double2* __restrict__ B, int rows, int cols,
                             double2* __restrict__ At, double2* __restrict__ Bt) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)rows * cols) return;
  const int64_t r = e / cols, c = e % cols;
  At[c * rows + r] = A[e];
  Bt[c * rows + r] = B[e];
}
}  // namespace

void rbm_ensure_tables(vmc_model* m, const vmc_ham* H, int move_kind) {
  rbm_move_tables& tb = m->tab[move_kind];
  const int n_moves = move_kind == 0 ? m->N : H->n_bonds;
  if (tb.T && tb.param_version == m->version && tb.n_moves == n_moves && (move_kind == 0 || tb.ham_uid == H->uid)) return;
  if (tb.n_moves != n_moves || !tb.T) {
    VMC_HIP(hipStreamSynchronize(m->ctx->stream));
    if (tb.T) VMC_HIP(hipFree(tb.T));
    if (tb.D) VMC_HIP(hipFree(tb.D));
    if (tb.LC) VMC_HIP(hipFree(tb.LC));
    if (tb.alpha) VMC_HIP(hipFree(tb.alpha));
    if (tb.Tt) VMC_HIP(hipFree(tb.Tt));
    if (tb.Dt) VMC_HIP(hipFree(tb.Dt));
    tb.T = tb.D = tb.LC = tb.alpha = tb.Tt = tb.Dt = nullptr;
    size_t tsz = sizeof(double2) * (size_t)m->Nh * std::max(1, n_moves);
    VMC_HIP(hipMalloc(&tb.T, sizeof(double2) * (size_t)nh_pad16(m->Nh) * std::max(1, n_moves)));
    VMC_HIP(hipMalloc(&tb.D, tsz));
    VMC_HIP(hipMalloc(&tb.Tt, tsz));
    VMC_HIP(hipMalloc(&tb.Dt, tsz));
    VMC_HIP(hipMalloc(&tb.LC, sizeof(double2) * std::max(1, n_moves)));
    VMC_HIP(hipMalloc(&tb.alpha, sizeof(double2) * std::max(1, n_moves)));
  }
  tb.move_kind = move_kind;
  tb.n_moves = n_moves;
  tb.ham_uid = H->uid;
  if (n_moves > 0) {
    k_tables<<<n_moves, 64, 0, m->ctx->stream>>>(m->params, H->bonds, move_kind, n_moves, m->N, m->Nh,
                                                 nh_pad16(m->Nh), tb.T, tb.D, tb.LC, tb.alpha);
    const int64_t n = (int64_t)m->Nh * n_moves;
    k_transpose2<<<grid_for(n, 256), 256, 0, m->ctx->stream>>>(tb.T, tb.D, m->Nh, n_moves, tb.Tt, tb.Dt);
    VMC_HIP(hipGetLastError());
  }
  tb.param_version = m->version;
}

void rbm_log_psi(vmc_model* m, const uint64_t* s, int64_t B, double2* logpsi) {
  vmc_ctx* ctx = m->ctx;
  const int64_t chunk = std::min<int64_t>(B, kChunk);
  ws_reserve(ctx, ws_round(sizeof(double2) * chunk * m->Nh));
  double2* theta = (double2*)ws_take(ctx, sizeof(double2) * chunk * m->Nh);
  for (int64_t b0 = 0; b0 < B; b0 += chunk) {
    const int64_t nb = std::min(chunk, B - b0);
    rbm_theta(m, s + b0 * m->W, nb, theta);
    k_logpsi<<<(unsigned)nb, 64, 0, ctx->stream>>>(m->params, theta, s + b0 * m->W, nb, m->N, m->W, m->Nh,
                                                  logpsi + b0);
    VMC_HIP(hipGetLastError());
  }
}

void rbm_local_energy(vmc_model* m, vmc_ham* H, const uint64_t* s, int64_t B, double2* eloc) {
  vmc_ctx* ctx = m->ctx;
  const int move_kind = H->kind == HAM_TFIM ? 0 : 1;
  rbm_ensure_tables(m, H, move_kind);
  const rbm_move_tables& tb = m->tab[move_kind];
  const int64_t chunk = std::min<int64_t>(B, kChunk);
  ws_reserve(ctx, ws_round(sizeof(double2) * chunk * m->Nh));
  double2* theta = (double2*)ws_take(ctx, sizeof(double2) * chunk * m->Nh);
  // flips: 4 samples per wavefront share the table reads; exchanges: one
  // sample per wavefront over its compacted list of anti-aligned bonds
  const int S = m->Nh <= 1024 ? 4 : 2;
  const size_t lds = sizeof(double2) * (size_t)S * m->Nh;
  const int Nhp = nh_pad16(m->Nh);
  const size_t lds1 = sizeof(double2) * 2 * Nhp + sizeof(int) * std::max(1, tb.n_moves);
  VMC_REQUIRE((move_kind == 1 ? lds1 : lds) <= 64 * 1024, "model too large for the local-energy kernel's LDS budget");
  VMC_REQUIRE((int64_t)Nhp * std::max(1, tb.n_moves) < ((int64_t)1 << 31), "move table too large");
  for (int64_t b0 = 0; b0 < B; b0 += chunk) {
    const int64_t nb = std::min(chunk, B - b0);
    rbm_theta(m, s + b0 * m->W, nb, theta);
    if (move_kind == 1) {
      k_eloc_compact<<<(unsigned)nb, 64, lds1, ctx->stream>>>(theta, s + b0 * m->W, nb, m->N, m->W, m->Nh, H->kind,
                                                              H->J, H->h, H->bonds, H->n_bonds, tb.T, tb.LC, tb.alpha,
                                                              tb.n_moves, Nhp, eloc + b0);
      VMC_HIP(hipGetLastError());
      continue;
    }
    const unsigned grid = (unsigned)((nb + S - 1) / S);
#define ELOC_LAUNCH(SS)                                                                                             \
  k_eloc<SS><<<grid, 64, lds, ctx->stream>>>(theta, s + b0 * m->W, nb, m->N, m->W, m->Nh, H->kind, H->J, H->h,     \
                                             H->bonds, H->n_bonds, tb.T, tb.LC, tb.alpha, tb.n_moves, eloc + b0)
    if (S == 4)
      ELOC_LAUNCH(4);
    else
      ELOC_LAUNCH(2);
#undef ELOC_LAUNCH
    VMC_HIP(hipGetLastError());
  }
}

void rbm_grad(vmc_model* m, const uint64_t* s, int64_t B, void* O, int dtype) {
  vmc_ctx* ctx = m->ctx;
  const int64_t chunk = std::min<int64_t>(B, kChunk);
  ws_reserve(ctx, ws_round(sizeof(double2) * chunk * m->Nh));
  double2* theta = (double2*)ws_take(ctx, sizeof(double2) * chunk * m->Nh);
  const size_t esz = dtype == VMC_DT_C128 ? sizeof(double2) : sizeof(float2);
  for (int64_t b0 = 0; b0 < B; b0 += chunk) {
    const int64_t nb = std::min(chunk, B - b0);
    rbm_theta(m, s + b0 * m->W, nb, theta);
    void* out = (char*)O + (size_t)b0 * m->K * esz;
    if (dtype == VMC_DT_C128)
      k_grad<double2><<<(unsigned)nb, 256, sizeof(double2) * m->Nh, ctx->stream>>>(
          theta, s + b0 * m->W, nb, m->N, m->W, m->Nh, m->K, (double2*)out);
    else
      k_grad<float2><<<(unsigned)nb, 256, sizeof(double2) * m->Nh, ctx->stream>>>(
          theta, s + b0 * m->W, nb, m->N, m->W, m->Nh, m->K, (float2*)out);
    VMC_HIP(hipGetLastError());
  }
}

void ham_connected_impl(vmc_ham* H, const uint64_t* s, int64_t B, uint64_t* sp, double* mel, int32_t* cnt) {
  k_connected<<<grid_for(B, 128), 128, 0, H->ctx->stream>>>(s, B, H->N, H->W, H->kind, H->J, H->h, H->bonds,
                                                             H->n_bonds, H->M_max, sp, mel, cnt);
  VMC_HIP(hipGetLastError());
}
