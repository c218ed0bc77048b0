// Blocked right-looking Cholesky S~ = L L^H in float64 (lower triangle, row-major,
// in place) and the two triangular solves, block size 64.
//
// Two levels: 256-column panels, each factored as four 64-column blocks.
// Per 64-column block b:
//   k_chol_diag   one work-group factors the diagonal block in LDS (packed
//                 lower triangle), writes L_bb, inverts it and writes
//                 L_bb^{-1} (dense 64 x 64) to the Linv buffer;
//   k_zmfma<0>    rows below: L_rb = A_rb L_bb^{-H}, a complex GEMM on the
//                 float64 matrix cores (in place, one 64-row block per group);
//   k_zmfma<2>    the rest of the panel's columns: A_rc -= L_rb L_cb^H.
// Per panel p, once its four blocks are done:
//   k_zmfma<2>    lookahead: the next panel's columns -= L_rp L_cp^H;
//   k_zmfma<1>    trailing update A_rc -= L_rp L_cp^H (reduction depth 256) on
//                 the lower 64 x 64 tiles of the rest of the trailing matrix,
//                 on a second stream, overlapping the next panel's
//                 factorisation; the trailing matrix is read and written once
//                 per 256 columns.
// The complex products P conj(Q) take three real products per term (Gauss's
// identity, as in the 3M complex GEMM): with A = sum Pr Qr, B = sum Pi Qi and
// C = sum (Pr + Pi)(Qr - Qi), held in three accumulators at the same lanes,
//   Re = A + B,   Im = C - A + B,
// so a 16x16 complex block costs three float64 MFMAs per 4 reduction columns
// instead of four; the error bound of Im grows by at most a factor of about 2.
// A non-positive pivot sets the fail index; every later kernel then exits at
// once.  The upper triangle of S~ is never written.
//
// Triangular solves: one launch per direction, one group per 64-row block,
// blocks handed over through ready flags in the order of the solve.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"

using namespace dev;

namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int CB = 64;  // block size

__device__ __forceinline__ int pk(int r, int c) { return r * (r + 1) / 2 + c; }  // packed lower index

// Factor and invert the diagonal block at kb0 (nb <= 64 valid rows/cols; the
// rest is padded with the identity).  LDS holds the packed lower triangles of
// the block (L) and of its inverse (X).
constexpr int CD_NT = 512;         // threads of the diagonal-block kernel
constexpr int CD_RS = CD_NT / 16;  // row stride of a thread's entries
constexpr int CD_RA = CB / CD_RS;  // rows per thread

__global__ __launch_bounds__(CD_NT) void k_chol_diag(double2* __restrict__ A, int64_t K, int64_t kb0, int nb,
                                                   double2* __restrict__ Linv, long long* __restrict__ fail,
                                                   double* __restrict__ pivmin) {
  __shared__ double2 L[CB * (CB + 1) / 2];
  __shared__ double2 X[CB * (CB + 1) / 2];
  __shared__ double dpiv[CB];
  __shared__ double sq[CB], isq[CB];
  if (*fail >= 0) return;
  const int tid = threadIdx.x;
  // thread (ty, tx) owns rows ty + CD_RS a, columns tx + 16 b of both triangles
  const int ty = tid >> 4, tx = tid & 15;
  {
    double2 v[CD_RA][4];
#pragma unroll
    for (int aa = 0; aa < CD_RA; ++aa)
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) {
        const int r = ty + CD_RS * aa, c = tx + 16 * bb;
        v[aa][bb] = (c <= r && r < nb) ? A[(kb0 + r) * K + kb0 + c] : make_double2(r == c ? 1.0 : 0.0, 0.0);
      }
#pragma unroll
    for (int aa = 0; aa < CD_RA; ++aa)
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) {
        const int r = ty + CD_RS * aa, c = tx + 16 * bb;
        if (c <= r) {
          L[pk(r, c)] = v[aa][bb];
          X[pk(r, c)] = make_double2(r == c ? 1.0 : 0.0, 0.0);
        }
      }
  }
  __syncthreads();
  // Right-looking elimination on the unscaled Schur complement and the inverse
  // of the unit-lower factor together, one barrier per column j.  With
  // f_r = A_rj / A_jj (the multiplier of row r, which equals L_rj / L_jj):
  //   A_rc -= f_r conj(A_cj)   for j < c <= r   (elimination),
  //   B_rc -= f_r B_jc         for c <= j < r   (B = I at the start; row j of B
  //                                              is final after step j - 1).
  // Column j of A and row j of B are only read in step j, and the two updates
  // write disjoint entries.  Afterwards L_rc = A_rc / sqrt(d_c), L_cc = sqrt(d_c)
  // and L^{-1}_rc = B_rc / sqrt(d_r), with the pivots d_j = A_jj kept.
  int bad = -1;
  double pmin = INFINITY;
  for (int j = 0; j < CB; ++j) {
    const double d = L[pk(j, j)].x;  // the same value in every thread
    if (j < nb) {
      pmin = fmin(pmin, d);
      if (!(d > 0.0)) {
        bad = j;
        break;
      }
    }
    if (tid == 0) dpiv[j] = d;
    const double id = 1.0 / d;
#pragma unroll
    for (int aa = 0; aa < CD_RA; ++aa) {
      const int r = ty + CD_RS * aa;
      if (r <= j) continue;
      const double2 f = cscale(L[pk(r, j)], id);
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) {
        const int c = tx + 16 * bb;
        if (c > r) continue;
        if (c > j)
          L[pk(r, c)] = csub(L[pk(r, c)], cmul(f, cconj(L[pk(c, j)])));
        else
          X[pk(r, c)] = csub(X[pk(r, c)], cmul(f, X[pk(j, c)]));
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    pivmin[kb0 / CB] = pmin;
    if (bad >= 0) *fail = kb0 + bad;
  }
  if (bad >= 0) return;  // uniform: every thread saw the same pivot
  if (tid < CB) {
    const double t = sqrt(dpiv[tid]);
    sq[tid] = t;
    isq[tid] = 1.0 / t;
  }
  __syncthreads();
#pragma unroll
  for (int aa = 0; aa < CD_RA; ++aa)
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
      const int r = ty + CD_RS * aa, c = tx + 16 * bb;
      double2 lv = make_double2(0.0, 0.0), xv = make_double2(0.0, 0.0);
      if (c <= r) {
        lv = r == c ? make_double2(sq[c], 0.0) : cscale(L[pk(r, c)], isq[c]);
        xv = cscale(X[pk(r, c)], isq[r]);
        if (r < nb) A[(kb0 + r) * K + kb0 + c] = lv;
      }
      Linv[r * CB + c] = xv;
    }
}

struct zargs {
  double2* S;
  int64_t K;
  int64_t kb0;   // first panel column of the reduction
  int depth;     // valid panel columns (reduction length)
  int64_t rbase; // first output row
  int64_t cbase; // first output column
  int64_t cend;  // one past the last output column (MODE 2)
  int nct;       // column tiles (MODE 2)
  const double2* Linv;
  int64_t ntiles;
  const long long* fail;
};

// MODE 0 (panel solve):   S[R][kb0 + c] = sum_m S[R][kb0 + m] conj(Linv[c][m]),  R = rbase + 64 b + r
// MODE 1 (trailing):      S[R][C] -= sum_m S[R][kb0 + m] conj(S[C][kb0 + m]) on lower 64x64 tiles of
//                         the square region starting at (rbase, rbase), C <= R
// MODE 2 (inside panel):  as MODE 1 for R >= rbase, cbase <= C < cend, C <= R (rectangular tile grid)
// The reduction is staged 16 columns at a time through double-buffered LDS.
template <int MODE>
__global__ __launch_bounds__(256, 2) void k_zmfma(zargs a) {
  __shared__ double2 Ps[2][16][CB + 1];
  __shared__ double2 Qs[2][16][CB + 1];
  if (*a.fail >= 0) return;
  const int64_t K = a.K;
  int64_t r0, c0;
  if (MODE == 0) {
    r0 = a.rbase + (int64_t)blockIdx.x * CB;
    c0 = 0;
  } else if (MODE == 1) {
    const int64_t per = (a.ntiles + 7) / 8;
    const int64_t lin = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (lin >= a.ntiles) return;
    int tr = (int)((sqrt(8.0 * (double)lin + 1.0) - 1.0) * 0.5);
    while ((int64_t)(tr + 1) * (tr + 2) / 2 <= lin) ++tr;
    while ((int64_t)tr * (tr + 1) / 2 > lin) --tr;
    const int tc = (int)(lin - (int64_t)tr * (tr + 1) / 2);
    r0 = a.rbase + (int64_t)tr * CB;
    c0 = a.rbase + (int64_t)tc * CB;
  } else {
    r0 = a.rbase + (int64_t)(blockIdx.x / a.nct) * CB;
    c0 = a.cbase + (int64_t)(blockIdx.x % a.nct) * CB;
  }
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int li = lane & 15, lk = lane >> 4;

  doublex4 acc[2][2][3];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 3; ++q) acc[i][j][q] = doublex4{0.0, 0.0, 0.0, 0.0};

  double2 rp[4], rq[4];
  auto gload = [&](int m0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = tid + 256 * j;
      const int r = q >> 4, mm = q & 15;
      const int m = m0 + mm;
      const int64_t R = r0 + r;
      rp[j] = (R < K && m < a.depth) ? a.S[R * K + a.kb0 + m] : make_double2(0.0, 0.0);
      if (MODE == 0) {
        rq[j] = a.Linv[r * CB + m];
      } else {
        const int64_t C = c0 + r;
        rq[j] = (C < K && m < a.depth) ? a.S[C * K + a.kb0 + m] : make_double2(0.0, 0.0);
      }
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = tid + 256 * j;
      Ps[buf][q & 15][q >> 4] = rp[j];
      Qs[buf][q & 15][q >> 4] = rq[j];
    }
  };
  const int nst = (a.depth + 15) / 16;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    if (st + 1 < nst) gload((st + 1) * 16);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int m = ks * 4 + lk;
      double2 fa[2], fb[2];
      double sa[2], db[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        fa[i] = Ps[buf][m][wr * 32 + i * 16 + li];
        sa[i] = fa[i].x + fa[i].y;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        fb[j] = Qs[buf][m][wc * 32 + j * 16 + li];
        db[j] = fb[j].x - fb[j].y;
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[i][j][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i].x, fb[j].x, acc[i][j][0], 0, 0, 0);
          acc[i][j][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i].y, fb[j].y, acc[i][j][1], 0, 0, 0);
          acc[i][j][2] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa[i], db[j], acc[i][j][2], 0, 0, 0);
        }
    }
    if (st + 1 < nst) sstore(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // float64 MFMA accumulators interleave rows: register r of lane l holds
        // D[l / 16 + 4 r][l % 16] (float32 holds D[4 (l / 16) + r][l % 16])
        const int row = wr * 32 + i * 16 + lk + 4 * r;
        const int col = wc * 32 + j * 16 + li;
        const double re = acc[i][j][0][r] + acc[i][j][1][r];
        const double im = (acc[i][j][2][r] - acc[i][j][0][r]) + acc[i][j][1][r];
        const int64_t R = r0 + row;
        if (R >= K) continue;
        if (MODE == 0) {
          if (col < a.depth) a.S[R * K + a.kb0 + col] = make_double2(re, im);
        } else {
          const int64_t C = c0 + col;
          if (C < K && C <= R && (MODE == 1 || C < a.cend)) {
            const double2 v = a.S[R * K + C];
            a.S[R * K + C] = make_double2(v.x - re, v.y - im);
          }
        }
      }
}

__device__ __forceinline__ double2 shfl_xor2(double2 v, int o) {
  return make_double2(__shfl_xor(v.x, o, 64), __shfl_xor(v.y, o, 64));
}

// sum over the four lanes q = lane % 4 of a quad
__device__ __forceinline__ double2 quad_sum(double2 v) {
  v = cadd(v, shfl_xor2(v, 1));
  return cadd(v, shfl_xor2(v, 2));
}

// ---------------------------------------------------------------- solves --
// Each triangular solve is one launch with one group per 64-row block.  A group
// takes a ticket (an atomic counter) when it starts and solves the block with
// that rank in the order of the solve, so every block it waits for belongs to a
// group that started earlier: the waits end whatever the number of groups the
// device holds at once.  A block's solution is published by its group with a
// release store of a per-block ready flag; wave 0 of a consumer polls the flags
// (64 at a time, relaxed), then takes an acquire fence before it reads the
// solutions.  Off-diagonal products are accumulated in registers over all
// earlier blocks and reduced once, so the critical path per block is one flag
// hand-over, one 64-term update and the 64 x 64 product with L_bb^{-1}.
//
// sync layout (ints, zeroed before the forward solve): [0] forward ticket,
// [1, nblk] forward flags, [nblk + 1] backward ticket, [nblk + 2, 2 nblk + 1]
// backward flags, [2 nblk + 2] set when a wait exceeded its poll limit.
constexpr int kPollLimit = 1 << 22;  // polls (a global load and a short sleep each) before a wait gives up

__global__ void k_zero_ints(int* __restrict__ p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// Wave 0 of a group: wait until the flags of blocks j, j + d, j + 2d, ... up to
// (not including) `end` are set, at least block j; returns the first block
// past the leading run of set flags (d = +1 forward, -1 backward).
__device__ __forceinline__ int wait_ready(const int* __restrict__ flag, int j, int end, int d, int* __restrict__ err) {
  const int lane = threadIdx.x & 63;
  const int jl = j + d * lane;
  for (int polls = 0;; ++polls) {
    const bool in = d > 0 ? jl < end : jl > end;
    const int f = in ? __hip_atomic_load(flag + jl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
    const unsigned long long m = __ballot(f != 0);
    const int n = ~m == 0ull ? 64 : __builtin_ctzll(~m);
    if (n > 0) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      return j + d * n;
    }
    if (polls >= kPollLimit) {  // never reached when every group runs to its end
      if (lane == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return j + d;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// L y = rhs.  Group rank b: thread (r, q) = (tid / 4, tid % 4) accumulates
// sum_j L[R][64 j + m] y_j[m] over m = q, q + 4, ... for row R = 64 b + r
// (each quad reads 64 contiguous bytes of its row per load), then
// y_b = L_bb^{-1} (rhs_b - sum).  The row entries of the next two blocks are in
// flight while a block is applied (three register buffers in turn); L_bb^{-1}
// waits in LDS, so that two groups fit on a compute unit and every group of the
// launch is resident at once.
__global__ __launch_bounds__(256, 2) void k_fwd_chain(const double2* __restrict__ A, int64_t K, int nblk,
                                                      const double2* __restrict__ Linv, const double2* __restrict__ rhs,
                                                      double2* __restrict__ y, int* __restrict__ sync) {
  __shared__ int tk;
  __shared__ double2 li[CB * (CB + 1)];  // L_bb^{-1}, row stride 65
  __shared__ double2 yb[2][CB];
  __shared__ double2 rs[CB];
  __shared__ double2 ys[CB];
  const int tid = threadIdx.x;
  const int r = tid >> 2, q = tid & 3;
  if (tid == 0) tk = atomicAdd(sync, 1);
  __syncthreads();
  const int b = tk;
  int* flag = sync + 1;
  const int64_t R = (int64_t)b * CB + r;
  const bool row_ok = R < K;
  const int nb = (int)std::min<int64_t>(CB, K - (int64_t)b * CB);
  const double2 zero = make_double2(0.0, 0.0);
  const double2* Ar = A + (row_ok ? R : 0) * K + q;
  auto load_blk = [&](int j, double2(&v)[CB / 4]) {
#pragma unroll
    for (int t = 0; t < CB / 4; ++t) v[t] = row_ok ? Ar[(int64_t)j * CB + 4 * t] : zero;
  };
  double2 A0[CB / 4], A1[CB / 4], A2[CB / 4];
  if (b > 0) load_blk(0, A0);
  if (b > 1) load_blk(1, A1);
  const double2 rv = (row_ok && q == 0) ? rhs[R] : zero;
  for (int i = tid; i < CB * CB; i += 256) li[(i >> 6) * (CB + 1) + (i & 63)] = Linv[(size_t)b * CB * CB + i];
  double2 acc = zero;
  int ready = 0;  // wave 0: blocks [0, ready) are published
  // apply block j (entries in cur); the entries of block j + 2 go to pre
  auto step = [&](int j, double2(&cur)[CB / 4], double2(&pre)[CB / 4]) {
    if (tid < 64) {
      if (j >= ready) ready = wait_ready(flag, j, b, 1, sync + 2 * nblk + 2);
      yb[j & 1][tid] = y[(int64_t)j * CB + tid];  // block j < b is a full block
    }
    __syncthreads();
    if (j + 2 < b) load_blk(j + 2, pre);
#pragma unroll
    for (int t = 0; t < CB / 4; ++t) acc = cadd(acc, cmul(cur[t], yb[j & 1][4 * t + q]));
  };
  for (int j = 0; j < b; j += 3) {
    step(j, A0, A2);
    if (j + 1 < b) step(j + 1, A1, A0);
    if (j + 2 < b) step(j + 2, A2, A1);
  }
  acc = quad_sum(acc);
  if (q == 0) rs[r] = row_ok ? csub(rv, acc) : zero;
  __syncthreads();  // also orders the LDS copy of L_bb^{-1} before its reads
  double2 s = zero;
#pragma unroll
  for (int t = 0; t < CB / 4; ++t) {
    const int m = q + 4 * t;
    if (m <= r && m < nb) s = cadd(s, cmul(li[r * (CB + 1) + m], rs[m]));
  }
  s = quad_sum(s);
  if (q == 0) ys[r] = s;
  __syncthreads();
  if (tid < 64) {
    if (tid < nb) y[(int64_t)b * CB + tid] = ys[tid];
    __hip_atomic_store(flag + b, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// L^H x = y.  Group rank t solves block b = nblk - 1 - t: thread (w, c) =
// (tid / 64, tid % 64) accumulates sum_j sum_m conj(L[64 j + m][64 b + c]) x_j[m]
// over m = 16 w .. 16 w + 15 for j > b (each load reads 64 consecutive columns
// of one row), then x_b = L_bb^{-H} (y_b - sum).  Buffers as in the forward
// solve; here every step reads 64 rows not read before, so the two-block
// prefetch also covers their address-translation misses.
__global__ __launch_bounds__(256, 2) void k_bwd_chain(const double2* __restrict__ A, int64_t K, int nblk,
                                                      const double2* __restrict__ Linv, const double2* __restrict__ y,
                                                      double2* __restrict__ x, int* __restrict__ sync) {
  __shared__ int tk;
  __shared__ double2 li[CB * (CB + 1)];  // L_bb^{-1}, row stride 65
  __shared__ double2 xb[2][CB];
  __shared__ double2 part[4][CB];
  __shared__ double2 vs[CB];
  const int tid = threadIdx.x;
  const int w = tid >> 6, c = tid & 63;
  if (tid == 0) tk = atomicAdd(sync + nblk + 1, 1);
  __syncthreads();
  const int b = nblk - 1 - tk;
  int* flag = sync + nblk + 2;
  const int nb = (int)std::min<int64_t>(CB, K - (int64_t)b * CB);
  const double2 zero = make_double2(0.0, 0.0);
  auto nb_of = [&](int j) { return (int)std::min<int64_t>(CB, K - (int64_t)j * CB); };
  // column 64 b + c exists for every block b < nblk - 1, the only ones that load
  // (row addresses are wave-uniform: scalar bases plus the lane's column offset)
  const int wu = __builtin_amdgcn_readfirstlane(w);
  auto load_blk = [&](int j, double2(&v)[CB / 4]) {
    const int nbj = nb_of(j);
#pragma unroll
    for (int i = 0; i < CB / 4; ++i) {
      const int m = wu * (CB / 4) + i;
      const double2* row = A + ((int64_t)j * CB + m) * K + (int64_t)b * CB;
      v[i] = m < nbj ? cconj(row[c]) : zero;
    }
  };
  double2 A0[CB / 4], A1[CB / 4], A2[CB / 4];
  if (b < nblk - 1) load_blk(nblk - 1, A0);
  if (b < nblk - 2) load_blk(nblk - 2, A1);
  const double2 yv = tid < nb ? y[(int64_t)b * CB + tid] : zero;
  for (int i = tid; i < CB * CB; i += 256) li[(i >> 6) * (CB + 1) + (i & 63)] = Linv[(size_t)b * CB * CB + i];
  double2 acc = zero;
  int ready = nblk - 1;  // wave 0: blocks (ready, nblk) are published
  // apply block j (entries in cur); the entries of block j - 2 go to pre
  auto step = [&](int j, double2(&cur)[CB / 4], double2(&pre)[CB / 4]) {
    if (tid < 64) {
      if (j <= ready) ready = wait_ready(flag, j, b, -1, sync + 2 * nblk + 2);
      xb[j & 1][tid] = tid < nb_of(j) ? x[(int64_t)j * CB + tid] : zero;
    }
    __syncthreads();
    if (j - 2 > b) load_blk(j - 2, pre);
#pragma unroll
    for (int i = 0; i < CB / 4; ++i) acc = cadd(acc, cmul(cur[i], xb[j & 1][w * (CB / 4) + i]));
  };
  for (int j = nblk - 1; j > b; j -= 3) {
    step(j, A0, A2);
    if (j - 1 > b) step(j - 1, A1, A0);
    if (j - 2 > b) step(j - 2, A2, A1);
  }
  part[w][c] = acc;
  __syncthreads();  // also orders the LDS copy of L_bb^{-1} before its reads
  if (tid < 64)
    vs[tid] = tid < nb ? csub(yv, cadd(cadd(part[0][tid], part[1][tid]), cadd(part[2][tid], part[3][tid]))) : zero;
  __syncthreads();
  // x_b[c] = sum_{m >= c} conj(L_bb^{-1}[m][c]) v_b[m], wave w over m = w + 4 t
  double2 s = zero;
#pragma unroll
  for (int t = 0; t < CB / 4; ++t) {
    const int m = w + 4 * t;
    if (m >= c && m < nb) s = cadd(s, cmul(cconj(li[m * (CB + 1) + c]), vs[m]));
  }
  part[w][c] = s;  // every read of part above finished before the last barrier
  __syncthreads();
  if (tid < 64) {
    if (tid < nb) x[(int64_t)b * CB + tid] = cadd(cadd(part[0][tid], part[1][tid]), cadd(part[2][tid], part[3][tid]));
    __hip_atomic_store(flag + b, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

}  // namespace

size_t chol_linv_bytes(int64_t K) { return sizeof(double2) * (size_t)((K + CB - 1) / CB) * CB * CB; }
int chol_block() { return CB; }

void chol_factor(vmc_ctx* ctx, double2* S, int64_t K, double2* Linv, long long* fail, double* pivmin) {
  hipStream_t st = ctx->stream;
  constexpr int PW = 256;  // panel width of the trailing update
  // Lookahead: after panel P_p is factored, the next panel's columns are
  // updated by P_p on the main stream, while the rest of the trailing matrix
  // (columns from the panel after next on) is updated on the auxiliary stream,
  // overlapping the factorisation of the next panel.  The only conflict is
  // the next lookahead (it writes columns the previous auxiliary update also
  // writes), so it waits for that update.
  hipStream_t aux = aux_stream(ctx);
  bool aux_busy = false;
  for (int64_t p0 = 0; p0 < K; p0 += PW) {
    const int64_t pend = std::min<int64_t>(K, p0 + PW);
    for (int64_t c0 = p0; c0 < pend; c0 += CB) {
      const int nb = (int)std::min<int64_t>(CB, K - c0);
      double2* Lb = Linv + (size_t)(c0 / CB) * CB * CB;
      k_chol_diag<<<1, CD_NT, 0, st>>>(S, K, c0, nb, Lb, fail, pivmin);
      const int64_t rest = K - c0 - nb;
      if (rest <= 0) continue;
      zargs a{};
      a.S = S;
      a.K = K;
      a.kb0 = c0;
      a.depth = nb;
      a.rbase = c0 + nb;
      a.Linv = Lb;
      a.fail = fail;
      k_zmfma<0><<<(unsigned)((rest + CB - 1) / CB), 256, 0, st>>>(a);
      if (c0 + nb < pend) {  // remaining columns of this panel
        a.cbase = c0 + nb;
        a.cend = pend;
        a.nct = (int)((pend - a.cbase + CB - 1) / CB);
        const int64_t nrt = (rest + CB - 1) / CB;
        k_zmfma<2><<<(unsigned)(nrt * a.nct), 256, 0, st>>>(a);
      }
    }
    if (pend >= K) break;
    const int64_t pend2 = std::min<int64_t>(K, pend + PW);
    VMC_HIP(hipEventRecord(ctx->ev_main, st));  // panel P_p factored
    // lookahead: columns [pend, pend2), rows >= pend, reduction over P_p
    if (aux_busy) VMC_HIP(hipStreamWaitEvent(st, ctx->ev_aux, 0));
    {
      zargs a{};
      a.S = S;
      a.K = K;
      a.kb0 = p0;
      a.depth = (int)(pend - p0);
      a.rbase = pend;
      a.cbase = pend;
      a.cend = pend2;
      a.nct = (int)((pend2 - pend + CB - 1) / CB);
      a.fail = fail;
      const int64_t nrt = (K - pend + CB - 1) / CB;
      k_zmfma<2><<<(unsigned)(nrt * a.nct), 256, 0, st>>>(a);
    }
    // the rest of the trailing matrix on the auxiliary stream
    if (pend2 < K) {
      VMC_HIP(hipStreamWaitEvent(aux, ctx->ev_main, 0));
      zargs a{};
      a.S = S;
      a.K = K;
      a.kb0 = p0;
      a.depth = (int)(pend - p0);
      a.rbase = pend2;
      a.fail = fail;
      const int64_t nt = (K - pend2 + CB - 1) / CB;
      a.ntiles = nt * (nt + 1) / 2;
      k_zmfma<1><<<(unsigned)(((a.ntiles + 7) / 8) * 8), 256, 0, aux>>>(a);
      VMC_HIP(hipEventRecord(ctx->ev_aux, aux));
      aux_busy = true;
    }
  }
  if (aux_busy) VMC_HIP(hipStreamWaitEvent(st, ctx->ev_aux, 0));
  VMC_HIP(hipGetLastError());
}

size_t chol_sync_bytes(int64_t K) { return sizeof(int) * (size_t)(2 * ((K + CB - 1) / CB) + 3); }
int chol_sync_err_index(int64_t K) { return (int)(2 * ((K + CB - 1) / CB) + 2); }

// y and x are K-vectors; x receives the solution, rhs is left unchanged;
// sync holds chol_sync_bytes(K) (its error word is set if a wait gave up)
void chol_solve(vmc_ctx* ctx, const double2* S, int64_t K, const double2* Linv, const double2* rhs, double2* y,
                double2* x, int* sync) {
  hipStream_t st = ctx->stream;
  const int nblk = (int)((K + CB - 1) / CB);
  k_zero_ints<<<1, 256, 0, st>>>(sync, 2 * nblk + 3);
  k_fwd_chain<<<(unsigned)nblk, 256, 0, st>>>(S, K, nblk, Linv, rhs, y, sync);
  k_bwd_chain<<<(unsigned)nblk, 256, 0, st>>>(S, K, nblk, Linv, y, x, sync);
  VMC_HIP(hipGetLastError());
}
