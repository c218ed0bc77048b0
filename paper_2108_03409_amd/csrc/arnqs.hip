// Autoregressive neural quantum state with direct sampling (Sec. 2.4: the joint
// distribution factorises into conditionals p_i(s_i | s_<i), so a sample is drawn
// site by site with one network pass and no Markov chain).
//
// The state is psi(s) = sqrt(q(s)) with q a masked autoregressive network (MADE:
// one ReLU hidden layer, hidden degree m(k) = k mod (N - 1) + 1, W1 entry (k, d)
// live iff m(k) >= d + 1, W2 entry (i, k) live iff i + 1 > m(k)), so log psi =
// (1/2) sum_i [s_i l_i - softplus(l_i)] is real and psi is normalised over all 2^N
// configurations.  The parameter vector holds only the live entries, in the order
//   W1 (k ascending, then d < m(k)) | b1 (H) | W2 (i ascending, then k with m(k) <= i) | b2 (N),
// N H + H + N real numbers; masked weights are not parameters.
//
// Local energies (eq:Oloc) use the move structure of the network: flipping or
// swapping sites P changes the hidden pre-activations by the W1 columns of P, and
// only the logits i >= min P can change, so each connected configuration costs one
// sparse hidden update and one (N - min P) x H product instead of a full pass.
// O_k = d log psi / d theta_k is the per-sample backward pass of the same network.
#include <hip/hip_runtime.h>

#include <type_traits>
#include <vector>

#include "internal.h"

using namespace dev;

namespace {

constexpr int AR_NT = 256;
constexpr int AR_WAVES = AR_NT / 64;

__device__ __forceinline__ int ar_deg(int k, int N) { return k % (N - 1) + 1; }
__device__ __forceinline__ double ar_softplus(double x) { return fmax(x, 0.0) + log1p(exp(-fabs(x))); }

// value of `v` in lane `src` (src uniform across the wave); reads the register
// whatever the execution mask, so every lane must have written it
__device__ __forceinline__ double lane_bcast(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One configuration through the network, all threads of the group:
// x (N, 0/1), a (H, pre-activations), hh (H, ReLU), l (N, logits).
__device__ void ar_forward(const uint64_t* __restrict__ srow, int N, int H, const double* __restrict__ W1mT,
                           const double* __restrict__ W2t, const double* __restrict__ b1,
                           const double* __restrict__ b2, double* x, double* a, double* hh, double* l) {
  for (int d = threadIdx.x; d < N; d += AR_NT) x[d] = (double)((srow[d >> 6] >> (d & 63)) & 1ull);
  __syncthreads();
  for (int k = threadIdx.x; k < H; k += AR_NT) {
    double acc = b1[k];
    const int m = ar_deg(k, N);
    for (int d = 0; d < m; ++d) acc = fma(W1mT[(int64_t)d * H + k], x[d], acc);
    a[k] = acc;
    hh[k] = fmax(acc, 0.0);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < N; i += AR_NT) {
    double acc = b2[i];
    for (int k = 0; k < H; ++k) acc = fma(W2t[(int64_t)k * N + i], hh[k], acc);
    l[i] = acc;
  }
  __syncthreads();
}

__global__ __launch_bounds__(AR_NT) void k_ar_log_psi(const uint64_t* __restrict__ s, int N, int H, int W,
                                                      const double* __restrict__ W1mT, const double* __restrict__ W2t,
                                                      const double* __restrict__ b1, const double* __restrict__ b2,
                                                      double2* __restrict__ out) {
  extern __shared__ double lds[];
  __shared__ double red[AR_WAVES];
  double *x = lds, *a = x + N, *hh = a + H, *l = hh + H;
  const int64_t b = blockIdx.x;
  ar_forward(s + b * W, N, H, W1mT, W2t, b1, b2, x, a, hh, l);
  double acc = 0.0;
  for (int i = threadIdx.x; i < N; i += AR_NT) acc += x[i] * l[i] - ar_softplus(l[i]);
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < AR_WAVES; ++w) t += red[w];
    out[b] = make_double2(0.5 * t, 0.0);
  }
}

// E_loc of one configuration per group.  Wave 0 lists the connected moves in the
// canonical slot order (TFIM: every site when h != 0; Heisenberg: anti-aligned
// bonds in bond order when J != 0) and counts aligned bonds for the diagonal; the
// four waves then take moves round-robin, lanes over hidden units for the update
// of the pre-activations and over outputs i >= min P for the new logits.
template <int QH>
__global__ __launch_bounds__(AR_NT) void k_ar_eloc(const uint64_t* __restrict__ s, int N, int H, int W,
                                                   const double* __restrict__ W1mT, const double* __restrict__ W2t,
                                                   const double* __restrict__ b1, const double* __restrict__ b2,
                                                   int kind, double J, double hx, const int2* __restrict__ bonds,
                                                   int n_bonds, double2* __restrict__ eloc) {
  extern __shared__ double lds[];
  __shared__ double red[AR_WAVES];
  __shared__ int n_moves_s, n_al_s;
  double *x = lds, *a = x + N, *hh = a + H, *l = hh + H, *t = l + N;
  int* mv = (int*)(t + N);
  const int64_t b = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  ar_forward(s + b * W, N, H, W1mT, W2t, b1, b2, x, a, hh, l);
  for (int i = threadIdx.x; i < N; i += AR_NT) t[i] = x[i] * l[i] - ar_softplus(l[i]);
  if (wave == 0) {
    const uint64_t* srow = s + b * W;
    int n_al = 0, nm = 0;
    const bool list = kind == HAM_HEIS && J != 0.0;
    for (int b0 = 0; b0 < n_bonds; b0 += 64) {
      const int q = b0 + lane;
      bool al = false, anti = false;
      if (q < n_bonds) {
        const int2 bd = bonds[q];
        al = get_bit(srow, bd.x) == get_bit(srow, bd.y);
        anti = !al;
      }
      n_al += __popcll(__ballot(al));
      const unsigned long long am = __ballot(anti);
      if (list && anti) mv[nm + __popcll(am & ((1ull << lane) - 1ull))] = q;
      nm += __popcll(am);
    }
    if (lane == 0) {
      n_al_s = n_al;
      n_moves_s = kind == HAM_TFIM ? (hx != 0.0 ? N : 0) : (list ? nm : 0);
    }
  }
  __syncthreads();
  const int M = n_moves_s;
  const double mel = kind == HAM_TFIM ? -hx : 2.0 * J;
  double e_w = 0.0;
  for (int mi = wave; mi < M; mi += AR_WAVES) {
    int p0, p1;
    if (kind == HAM_TFIM) {
      p0 = mi;
      p1 = -1;
    } else {
      const int2 bd = bonds[mv[mi]];
      p0 = min(bd.x, bd.y);
      p1 = max(bd.x, bd.y);
    }
    const double d0 = 1.0 - 2.0 * x[p0];
    const double d1 = p1 >= 0 ? 1.0 - 2.0 * x[p1] : 0.0;
    double dh[QH];
#pragma unroll
    for (int q = 0; q < QH; ++q) {
      const int k = lane + 64 * q;
      dh[q] = 0.0;
      if (k < H) {
        double ap = fma(W1mT[(int64_t)p0 * H + k], d0, a[k]);
        if (p1 >= 0) ap = fma(W1mT[(int64_t)p1 * H + k], d1, ap);
        dh[q] = fmax(ap, 0.0) - hh[k];
      }
    }
    double acc = 0.0;
    for (int i0 = p0; i0 < N; i0 += 64) {  // uniform trip count
      const int i = i0 + lane;
      const bool ok = i < N;
      double lp = ok ? l[i] : 0.0;
#pragma unroll
      for (int q = 0; q < QH; ++q) {
        for (int kk = 0; kk < 64; ++kk) {
          const int k = 64 * q + kk;
          if (k >= H) break;
          const double d = lane_bcast(dh[q], kk);
          if (d != 0.0 && ok) lp = fma(W2t[(int64_t)k * N + i], d, lp);
        }
      }
      if (ok) {
        const double xi = (i == p0 || i == p1) ? 1.0 - x[i] : x[i];
        acc += (xi * lp - ar_softplus(lp)) - t[i];
      }
    }
    acc = wave_sum(acc);
    e_w += mel * exp(0.5 * acc);
  }
  if (lane == 0) red[wave] = e_w;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int n_anti = n_bonds - n_al_s;
    const double diag = (kind == HAM_TFIM ? -J : J) * (double)(n_al_s - n_anti);
    double e = diag;
    for (int w = 0; w < AR_WAVES; ++w) e += red[w];
    eloc[b] = make_double2(e, 0.0);
  }
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The same local energies with both masked weight matrices held in LDS (staged
// once per group) and one wave per configuration.  The connected moves are taken
// AR_CM at a time and their (move, output) pairs -- output i >= min P of the
// move -- are laid out over the lanes, so a wave instruction serves several
// moves when their triangles are short: for each chunk the changes of the
// hidden units (lanes over (move, unit)), then the new logit and its
// log-likelihood term per pair, then per-move sums over 16-lane groups.  Moves
// and pairs are summed in a fixed order (reproducible results).
constexpr int AR_CM = 4;  // moves per chunk (64 / AR_CM lanes per move in the sums)

template <int NT>
__global__ __launch_bounds__(NT) void k_ar_eloc_tri(const uint64_t* __restrict__ s, int64_t B, int N, int H,
                                                       int W, const double* __restrict__ W1mT,
                                                       const double* __restrict__ W2t, const double* __restrict__ b1,
                                                       const double* __restrict__ b2, int kind, double J, double hx,
                                                       const int2* __restrict__ bonds, int n_bonds,
                                                       double2* __restrict__ eloc) {
  extern __shared__ double lds[];
  double* W1s = lds;          // [N][H]
  double* W2s = W1s + N * H;  // [H][N]
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int per = (3 + AR_CM) * N + (2 + AR_CM) * H + (n_bonds + 1) / 2;  // doubles per wave
  double* x = W2s + H * N + wave * per;
  double* l = x + N;
  double* t = l + N;
  double* a = t + N;
  double* hh = a + H;
  double* DH = hh + H;         // [AR_CM][H] hidden-unit changes of the chunk's moves
  double* buf = DH + AR_CM * H;  // [AR_CM][N] per-pair log-likelihood changes
  int* mv = (int*)(buf + AR_CM * N);  // anti-aligned bonds (Heisenberg), bond order
  for (int e = threadIdx.x; e < N * H; e += NT) {
    W1s[e] = W1mT[e];
    W2s[e] = W2t[e];
  }
  __syncthreads();
  const double mel = kind == HAM_TFIM ? -hx : 2.0 * J;
  const bool offdiag = kind == HAM_TFIM ? hx != 0.0 : J != 0.0;
  const int grp = lane >> 4, gl = lane & 15;  // 16-lane group of the per-move sums
  for (int64_t b = (int64_t)blockIdx.x * (NT / 64) + wave; b < B; b += (int64_t)gridDim.x * (NT / 64)) {
    const uint64_t* srow = s + b * W;
    for (int i = lane; i < N; i += 64) x[i] = (double)((srow[i >> 6] >> (i & 63)) & 1ull);
    wave_sync();
    for (int k = lane; k < H; k += 64) {
      double acc = b1[k];
      for (int d = 0; d < N; ++d) acc = fma(W1s[d * H + k], x[d], acc);  // zero beyond the unit's degree
      a[k] = acc;
      hh[k] = fmax(acc, 0.0);
    }
    wave_sync();
    for (int i = lane; i < N; i += 64) {
      double acc = b2[i];
      for (int k = 0; k < H; ++k) acc = fma(W2s[k * N + i], hh[k], acc);
      l[i] = acc;
      t[i] = x[i] * acc - ar_softplus(acc);
    }
    // moves: diagonal count and the anti-aligned bond list
    int n_al = 0, M = 0;
    for (int q0 = 0; q0 < n_bonds; q0 += 64) {
      const int q = q0 + lane;
      bool al = false, anti = false;
      if (q < n_bonds) {
        const int2 bd = bonds[q];
        al = get_bit(srow, bd.x) == get_bit(srow, bd.y);
        anti = !al;
      }
      n_al += __popcll(__ballot(al));
      const unsigned long long am = __ballot(anti);
      if (kind == HAM_HEIS && anti) mv[M + __popcll(am & ((1ull << lane) - 1ull))] = q;
      M += __popcll(am);
    }
    if (kind == HAM_TFIM) M = N;
    if (!offdiag) M = 0;
    wave_sync();
    auto move_sites = [&](int m, int& p0, int& p1) {
      if (kind == HAM_TFIM) {
        p0 = m;
        p1 = -1;
      } else {
        const int2 bd = bonds[mv[m]];
        p0 = min(bd.x, bd.y);
        p1 = max(bd.x, bd.y);
      }
    };
    double e = 0.0;
    for (int m0 = 0; m0 < M; m0 += AR_CM) {
      const int cm = min(AR_CM, M - m0);
      int p0s[AR_CM], p1s[AR_CM], off[AR_CM + 1];
      off[0] = 0;
#pragma unroll
      for (int mm = 0; mm < AR_CM; ++mm) {
        int p0 = N, p1 = -1;
        if (mm < cm) move_sites(m0 + mm, p0, p1);
        p0s[mm] = p0;
        p1s[mm] = p1;
        off[mm + 1] = off[mm] + (mm < cm ? N - p0 : 0);
      }
      // hidden-unit changes, lanes over (move, unit)
      for (int q = lane; q < cm * H; q += 64) {
        const int mm = q / H, k = q - mm * H;
        int p0 = p0s[0], p1 = p1s[0];
#pragma unroll
        for (int r = 1; r < AR_CM; ++r)
          if (mm == r) {
            p0 = p0s[r];
            p1 = p1s[r];
          }
        double ap = fma(W1s[p0 * H + k], 1.0 - 2.0 * x[p0], a[k]);
        if (p1 >= 0) ap = fma(W1s[p1 * H + k], 1.0 - 2.0 * x[p1], ap);
        DH[q] = fmax(ap, 0.0) - hh[k];  // exactly 0 for units of degree <= p0
      }
      wave_sync();
      // (move, output) pairs over the lanes
      const int total = off[AR_CM];  // moves past cm add nothing
      for (int q0 = 0; q0 < total; q0 += 64) {
        const int q = q0 + lane;
        if (q < total) {
          int mm = 0;
#pragma unroll
          for (int r = 1; r < AR_CM; ++r) mm += q >= off[r] ? 1 : 0;
          int p0 = p0s[0], p1 = p1s[0], o = off[0];
#pragma unroll
          for (int r = 1; r < AR_CM; ++r)
            if (mm == r) {
              p0 = p0s[r];
              p1 = p1s[r];
              o = off[r];
            }
          const int i = p0 + (q - o);
          const double* dh = DH + mm * H;
          double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
          int k = 0;
          for (; k + 4 <= H; k += 4) {
            s0 = fma(W2s[k * N + i], dh[k], s0);
            s1 = fma(W2s[(k + 1) * N + i], dh[k + 1], s1);
            s2 = fma(W2s[(k + 2) * N + i], dh[k + 2], s2);
            s3 = fma(W2s[(k + 3) * N + i], dh[k + 3], s3);
          }
          for (; k < H; ++k) s0 = fma(W2s[k * N + i], dh[k], s0);
          const double lp = l[i] + ((s0 + s1) + (s2 + s3));
          const double xi = (i == p0 || i == p1) ? 1.0 - x[i] : x[i];
          buf[mm * N + i] = (xi * lp - ar_softplus(lp)) - t[i];
        }
      }
      wave_sync();
      // per-move sums: 16 lanes per move, fixed order
      double acc = 0.0;
      int p0g = p0s[0];
#pragma unroll
      for (int r = 1; r < AR_CM; ++r)
        if (grp == r) p0g = p0s[r];
      if (grp < cm)
        for (int i = p0g + gl; i < N; i += 16) acc += buf[grp * N + i];
      acc = row16_sum(acc);
      const double r = grp < cm ? mel * exp(0.5 * acc) : 0.0;
#pragma unroll
      for (int mm = 0; mm < AR_CM; ++mm) e += lane_bcast(r, 16 * mm);
      wave_sync();  // DH and buf are rewritten by the next chunk
    }
    if (lane == 0) {
      const int n_anti = n_bonds - n_al;
      const double diag = (kind == HAM_TFIM ? -J : J) * (double)(n_al - n_anti);
      eloc[b] = make_double2(diag + e, 0.0);
    }
    wave_sync();  // per-wave arrays are rewritten by the next configuration
  }
}

// O_k = (1/2) d log q / d theta_k for SB configurations per group:
//   g_l[i] = s_i - sigmoid(l_i),  g_h[k] = [a_k > 0] sum_i (W2 * M2)[i, k] g_l[i],
//   W1 (k, d): g_h[k] s_d,  b1 k: g_h[k],  W2 (i, k): g_l[i] relu(a_k),  b2 i: g_l[i].
template <int SB, typename OutT>
__global__ __launch_bounds__(AR_NT) void k_ar_grad(const uint64_t* __restrict__ s, int64_t B, int N, int H, int W,
                                                   const double* __restrict__ W1mT, const double* __restrict__ W2t,
                                                   const double* __restrict__ W2m, const double* __restrict__ b1,
                                                   const double* __restrict__ b2, const int2* __restrict__ idx,
                                                   int64_t r1, int64_t r2, int64_t r3, int64_t K,
                                                   OutT* __restrict__ O) {
  extern __shared__ double lds[];
  const int per = 2 * N + 3 * H;
  const int64_t b0 = (int64_t)blockIdx.x * SB;
  for (int q = 0; q < SB; ++q) {
    double* x = lds + q * per;
    double *a = x + N, *hh = a + H, *l = hh + H, *gh = l + N;
    if (b0 + q < B) {  // uniform over the group
      ar_forward(s + (b0 + q) * W, N, H, W1mT, W2t, b1, b2, x, a, hh, l);
      for (int i = threadIdx.x; i < N; i += AR_NT) l[i] = x[i] - 1.0 / (1.0 + exp(-l[i]));
      __syncthreads();
      for (int k = threadIdx.x; k < H; k += AR_NT) {
        double acc = 0.0;
        for (int i = ar_deg(k, N); i < N; ++i) acc = fma(W2m[(int64_t)i * H + k], l[i], acc);
        gh[k] = a[k] > 0.0 ? acc : 0.0;
      }
      __syncthreads();
    }
  }
  for (int64_t j = threadIdx.x; j < K; j += AR_NT) {
    const int2 pr = idx[j];
    const int region = j < r1 ? 0 : j < r2 ? 1 : j < r3 ? 2 : 3;
#pragma unroll
    for (int q = 0; q < SB; ++q) {
      if (b0 + q >= B) break;
      const double* x = lds + q * per;
      const double *a = x + N, *hh = a + H, *gl = hh + H, *gh = gl + N;
      (void)a;
      double v;
      if (region == 0)
        v = gh[pr.x] * x[pr.y];
      else if (region == 1)
        v = gh[pr.x];
      else if (region == 2)
        v = gl[pr.x] * hh[pr.y];
      else
        v = gl[pr.x];
      v *= 0.5;
      OutT* row = O + (b0 + q) * K;
      if constexpr (std::is_same<OutT, double2>::value)
        row[j] = make_double2(v, 0.0);
      else if constexpr (std::is_same<OutT, float2>::value)
        row[j] = make_float2((float)v, 0.0f);
      else
        row[j] = (OutT)v;
    }
  }
}

// The same O_k with one wave per configuration and both masked weight matrices
// in LDS (staged once per group, configurations taken grid-stride): the forward
// pass, g_l and g_h with lanes over units, then the K outputs with lanes over the
// live parameters (coalesced row writes).
template <typename OutT>
__global__ __launch_bounds__(AR_NT) void k_ar_grad_w(const uint64_t* __restrict__ s, int64_t B, int N, int H, int W,
                                                     const double* __restrict__ W1mT,
                                                     const double* __restrict__ W2t, const double* __restrict__ b1,
                                                     const double* __restrict__ b2, const int2* __restrict__ idx,
                                                     int64_t r1, int64_t r2, int64_t r3, int64_t K,
                                                     OutT* __restrict__ O) {
  extern __shared__ double lds[];
  double* W1s = lds;          // [N][H]
  double* W2s = W1s + N * H;  // [H][N]
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* x = W2s + H * N + wave * (2 * N + 2 * H);
  double* gl = x + N;   // logits, then s_i - sigmoid(l_i)
  double* hh = gl + N;  // ReLU(a), with a kept as the sign of the gate below
  double* gh = hh + H;
  for (int e = threadIdx.x; e < N * H; e += AR_NT) {
    W1s[e] = W1mT[e];
    W2s[e] = W2t[e];
  }
  __syncthreads();
  for (int64_t b = (int64_t)blockIdx.x * AR_WAVES + wave; b < B; b += (int64_t)gridDim.x * AR_WAVES) {
    const uint64_t* srow = s + b * W;
    for (int i = lane; i < N; i += 64) x[i] = (double)((srow[i >> 6] >> (i & 63)) & 1ull);
    wave_sync();
    for (int k = lane; k < H; k += 64) {
      double acc = b1[k];
      for (int d = 0; d < N; ++d) acc = fma(W1s[d * H + k], x[d], acc);
      hh[k] = fmax(acc, 0.0);
      gh[k] = acc > 0.0 ? 1.0 : 0.0;  // ReLU gate
    }
    wave_sync();
    for (int i = lane; i < N; i += 64) {
      double acc = b2[i];
      for (int k = 0; k < H; ++k) acc = fma(W2s[k * N + i], hh[k], acc);
      gl[i] = x[i] - 1.0 / (1.0 + exp(-acc));
    }
    wave_sync();
    for (int k = lane; k < H; k += 64) {
      double acc = 0.0;
      for (int i = ar_deg(k, N); i < N; ++i) acc = fma(W2s[k * N + i], gl[i], acc);
      gh[k] *= acc;
    }
    wave_sync();
    OutT* row = O + b * K;
    for (int64_t j = lane; j < K; j += 64) {
      const int2 pr = idx[j];
      double v;
      if (j < r1)
        v = gh[pr.x] * x[pr.y];
      else if (j < r2)
        v = gh[pr.x];
      else if (j < r3)
        v = gl[pr.x] * hh[pr.y];
      else
        v = gl[pr.x];
      v *= 0.5;
      if constexpr (std::is_same<OutT, double2>::value)
        row[j] = make_double2(v, 0.0);
      else if constexpr (std::is_same<OutT, float2>::value)
        row[j] = make_float2((float)v, 0.0f);
      else
        row[j] = (OutT)v;
    }
    wave_sync();
  }
}

// compact live parameters -> dense masked layout [W1 (H x N) | b1 | W2 (N x H) | b2]
__global__ void k_ar_scatter(const double2* __restrict__ theta, const int2* __restrict__ idx, int64_t r1, int64_t r2,
                             int64_t r3, int64_t K, int N, int H, double* __restrict__ dense) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= K) return;
  const int2 pr = idx[j];
  const int64_t HN = (int64_t)H * N;
  int64_t at;
  if (j < r1)
    at = (int64_t)pr.x * N + pr.y;
  else if (j < r2)
    at = HN + pr.x;
  else if (j < r3)
    at = HN + H + (int64_t)pr.x * H + pr.y;
  else
    at = 2 * HN + H + pr.x;
  dense[at] = theta[j].x;
}

__global__ void k_ar_transpose(const double* __restrict__ W2m, int N, int H, double* __restrict__ W2t) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)N * H) return;
  const int i = (int)(e / H), k = (int)(e % H);
  W2t[(int64_t)k * N + i] = W2m[e];
}

__global__ void k_ar_half(const double* __restrict__ lq, int64_t B, double2* __restrict__ out) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < B) out[e] = make_double2(0.5 * lq[e], 0.0);
}

struct ar_ptrs {
  const double *W1mT, *W2m, *b1, *b2;
};

ar_ptrs ptrs(const vmc_model* m) {
  const vmc_made* md = m->made;
  const int64_t HN = (int64_t)m->Nh * m->N;
  return ar_ptrs{md->W1mT, md->W2m, md->params + HN, md->params + 2 * HN + m->Nh};
}

constexpr size_t kArLdsMax = 64 * 1024;

void* ar_alloc(size_t bytes) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    throw vmc_error{VMC_ERR_OOM, "device allocation failed"};
  }
  return p;
}

}  // namespace

void ar_init(vmc_model* m) {
  const int N = m->N, H = m->Nh;
  std::vector<int2> idx;
  idx.reserve((size_t)m->K);
  auto deg = [&](int k) { return k % (N - 1) + 1; };
  for (int k = 0; k < H; ++k)
    for (int d = 0; d < deg(k); ++d) idx.push_back(make_int2(k, d));
  m->ar_r1 = (int64_t)idx.size();
  for (int k = 0; k < H; ++k) idx.push_back(make_int2(k, 0));
  m->ar_r2 = (int64_t)idx.size();
  for (int i = 0; i < N; ++i)
    for (int k = 0; k < H; ++k)
      if (deg(k) <= i) idx.push_back(make_int2(i, k));
  m->ar_r3 = (int64_t)idx.size();
  for (int i = 0; i < N; ++i) idx.push_back(make_int2(i, 0));
  if ((int64_t)idx.size() != m->K) throw vmc_error{VMC_ERR_INVALID_ARG, "internal: live parameter count mismatch"};
  vmc_ctx* ctx = m->ctx;
  vmc_made* md = nullptr;
  if (vmc_made_create(ctx, N, H, &md) != VMC_OK) throw vmc_error{VMC_ERR_OOM, vmc_last_error(ctx)};
  m->made = md;
  m->ar_idx = (int2*)ar_alloc(sizeof(int2) * idx.size());
  m->ar_w2t = (double*)ar_alloc(sizeof(double) * (size_t)N * H);
  VMC_HIP(hipMemcpyAsync(m->ar_idx, idx.data(), sizeof(int2) * idx.size(), hipMemcpyHostToDevice, ctx->stream));
  VMC_HIP(hipStreamSynchronize(ctx->stream));
  ar_set_params(m);
}

void ar_free(vmc_model* m) {
  if (m->ar_idx) (void)hipFree(m->ar_idx);
  if (m->ar_w2t) (void)hipFree(m->ar_w2t);
  if (m->made) (void)vmc_made_destroy(m->made);
  m->ar_idx = nullptr;
  m->ar_w2t = nullptr;
  m->made = nullptr;
}

void ar_set_params(vmc_model* m) {
  vmc_made* md = m->made;
  hipStream_t st = m->ctx->stream;
  VMC_HIP(hipMemsetAsync(md->params, 0, sizeof(double) * md->P, st));
  k_ar_scatter<<<grid_for(m->K, 256), 256, 0, st>>>(m->params, m->ar_idx, m->ar_r1, m->ar_r2, m->ar_r3, m->K, m->N,
                                                    m->Nh, md->params);
  VMC_HIP(hipGetLastError());
  made_refresh(md);
  const int64_t n = (int64_t)m->N * m->Nh;
  k_ar_transpose<<<grid_for(n, 256), 256, 0, st>>>(md->W2m, m->N, m->Nh, m->ar_w2t);
  VMC_HIP(hipGetLastError());
}

void ar_log_psi(vmc_model* m, const uint64_t* s, int64_t B, double2* out) {
  const ar_ptrs p = ptrs(m);
  const size_t lds = sizeof(double) * (2 * (size_t)m->N + 2 * (size_t)m->Nh);
  for (int64_t b0 = 0; b0 < B; b0 += INT32_MAX) {
    const int64_t nb = std::min<int64_t>(INT32_MAX, B - b0);
    k_ar_log_psi<<<(unsigned)nb, AR_NT, lds, m->ctx->stream>>>(s + b0 * m->W, m->N, m->Nh, m->W, p.W1mT, m->ar_w2t,
                                                              p.b1, p.b2, out + b0);
    VMC_HIP(hipGetLastError());
  }
}

void ar_local_energy(vmc_model* m, vmc_ham* H, const uint64_t* s, int64_t B, double2* eloc) {
  const ar_ptrs p = ptrs(m);
  const size_t per_wave = (size_t)(3 + AR_CM) * m->N + (size_t)(2 + AR_CM) * m->Nh + ((size_t)H->n_bonds + 1) / 2;
  auto lds_of = [&](int waves) { return sizeof(double) * (2 * (size_t)m->N * m->Nh + (size_t)waves * per_wave); };
  // eight waves per group share one copy of the weights where it fits (more
  // resident waves per compute unit for the same LDS), else four
  const int nt = lds_of(8) <= kArLdsMax ? 512 : 256;
  const size_t lds_w = lds_of(nt / 64);
  if (lds_w <= kArLdsMax) {
    // one resident wave of groups: as many as the LDS of 256 compute units holds (at most 8 each)
    const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(8, (int64_t)(160 * 1024) / (int64_t)lds_w));
    const int64_t groups = std::min<int64_t>((B + nt / 64 - 1) / (nt / 64), 256 * per_cu);
    if (nt == 512)
      k_ar_eloc_tri<512><<<(unsigned)groups, 512, lds_w, m->ctx->stream>>>(
          s, B, m->N, m->Nh, m->W, p.W1mT, m->ar_w2t, p.b1, p.b2, H->kind, H->J, H->h, H->bonds, H->n_bonds, eloc);
    else
      k_ar_eloc_tri<256><<<(unsigned)groups, 256, lds_w, m->ctx->stream>>>(
          s, B, m->N, m->Nh, m->W, p.W1mT, m->ar_w2t, p.b1, p.b2, H->kind, H->J, H->h, H->bonds, H->n_bonds, eloc);
    VMC_HIP(hipGetLastError());
    return;
  }
  const size_t lds = sizeof(double) * (3 * (size_t)m->N + 2 * (size_t)m->Nh) + sizeof(int) * (size_t)H->n_bonds;
  VMC_REQUIRE(lds <= kArLdsMax, "network too large for the per-configuration local-energy tile");
  const int QH = (m->Nh + 63) / 64;
  for (int64_t b0 = 0; b0 < B; b0 += INT32_MAX) {
    const int64_t nb = std::min<int64_t>(INT32_MAX, B - b0);
#define AR_ELOC(Q)                                                                                                 \
  k_ar_eloc<Q><<<(unsigned)nb, AR_NT, lds, m->ctx->stream>>>(s + b0 * m->W, m->N, m->Nh, m->W, p.W1mT, m->ar_w2t, \
                                                             p.b1, p.b2, H->kind, H->J, H->h, H->bonds, H->n_bonds, \
                                                             eloc + b0)
    if (QH <= 1)
      AR_ELOC(1);
    else if (QH <= 2)
      AR_ELOC(2);
    else if (QH <= 4)
      AR_ELOC(4);
    else if (QH <= 8)
      AR_ELOC(8);
    else
      AR_ELOC(16);
#undef AR_ELOC
    VMC_HIP(hipGetLastError());
  }
}

void ar_grad(vmc_model* m, const uint64_t* s, int64_t B, void* O, int dtype) {
  const ar_ptrs p = ptrs(m);
  const size_t lds_w = sizeof(double) * (2 * (size_t)m->N * m->Nh + (size_t)AR_WAVES * (2 * (size_t)m->N + 2 * m->Nh));
  if (lds_w <= kArLdsMax) {
    const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(8, (int64_t)(160 * 1024) / (int64_t)lds_w));
    const unsigned g = (unsigned)std::min<int64_t>((B + AR_WAVES - 1) / AR_WAVES, 256 * per_cu);
    hipStream_t st = m->ctx->stream;
#define AR_GRAD_W(T)                                                                                           \
  k_ar_grad_w<T><<<g, AR_NT, lds_w, st>>>(s, B, m->N, m->Nh, m->W, p.W1mT, m->ar_w2t, p.b1, p.b2, m->ar_idx, \
                                          m->ar_r1, m->ar_r2, m->ar_r3, m->K, (T*)O)
    if (dtype == VMC_DT_C128)
      AR_GRAD_W(double2);
    else if (dtype == VMC_DT_C64)
      AR_GRAD_W(float2);
    else if (dtype == VMC_DT_F64)
      AR_GRAD_W(double);
    else
      AR_GRAD_W(float);
#undef AR_GRAD_W
    VMC_HIP(hipGetLastError());
    return;
  }
  const size_t per = sizeof(double) * (2 * (size_t)m->N + 3 * (size_t)m->Nh);
  const int sb = 4 * per <= kArLdsMax ? 4 : 1;
  VMC_REQUIRE(per <= kArLdsMax, "network too large for the per-configuration gradient tile");
  const int64_t groups = (B + sb - 1) / sb;
  VMC_REQUIRE(groups <= INT32_MAX, "too many configurations for one launch");
  hipStream_t st = m->ctx->stream;
#define AR_GRAD(S, T)                                                                                           \
  k_ar_grad<S, T><<<(unsigned)groups, AR_NT, S * per, st>>>(s, B, m->N, m->Nh, m->W, p.W1mT, m->ar_w2t, p.W2m, \
                                                            p.b1, p.b2, m->ar_idx, m->ar_r1, m->ar_r2, m->ar_r3, \
                                                            m->K, (T*)O)
  if (dtype == VMC_DT_C128) {
    if (sb == 4)
      AR_GRAD(4, double2);
    else
      AR_GRAD(1, double2);
  } else if (dtype == VMC_DT_C64) {
    if (sb == 4)
      AR_GRAD(4, float2);
    else
      AR_GRAD(1, float2);
  } else if (dtype == VMC_DT_F64) {
    if (sb == 4)
      AR_GRAD(4, double);
    else
      AR_GRAD(1, double);
  } else {
    if (sb == 4)
      AR_GRAD(4, float);
    else
      AR_GRAD(1, float);
  }
#undef AR_GRAD
  VMC_HIP(hipGetLastError());
}

void ar_sample(vmc_sampler* S, int64_t B, uint64_t* s_out, double2* logpsi_out) {
  vmc_model* m = S->model;
  vmc_ctx* ctx = S->ctx;
  VMC_REQUIRE(B <= INT32_MAX, "at most 2^31 - 1 direct samples per call");
  double* lq = nullptr;
  if (logpsi_out) {
    ws_reserve(ctx, ws_round(sizeof(double) * B));
    lq = (double*)ws_take(ctx, sizeof(double) * B);
  }
  made_sample_impl(m->made, B, S->opts.seed, S->t, s_out, lq);
  if (logpsi_out) {
    k_ar_half<<<grid_for(B, 256), 256, 0, ctx->stream>>>(lq, B, logpsi_out);
    VMC_HIP(hipGetLastError());
  }
  S->t += 1;
}
