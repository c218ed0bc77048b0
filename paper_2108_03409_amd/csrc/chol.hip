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
// Triangular solves: one launch per block.  Launch b updates the remaining
// right-hand side with block b's solution (64 rows or columns per group, a
// quad or a wave per 16 terms); the group that holds the next block's entries,
// final after its update, forms that block's solution from L_bb^{-1}.
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

// y_0 = Linv_0 rhs_0 (one group; thread (r, q) = (tid / 4, tid % 4) sums m = q, q + 4, ...)
__global__ __launch_bounds__(256) void k_fwd_first(const double2* __restrict__ Linv, const double2* __restrict__ rhs,
                                                   double2* __restrict__ y, int nb) {
  const int r = threadIdx.x >> 2, q = threadIdx.x & 3;
  double2 s = make_double2(0.0, 0.0);
  for (int m = q; m <= r && m < nb; m += 4) s = cadd(s, cmul(Linv[r * CB + m], rhs[m]));
  s = quad_sum(s);
  if (q == 0 && r < nb) y[r] = s;
}

// Forward update of block b (y_b in y): rhs[R] -= sum_m L[R][kb0 + m] y_b[m] for
// R >= kb0 + 64, 64 rows per group, thread (r, q) summing m = q, q + 4, ...
// (each quad reads 64 contiguous bytes of its row per step).  Group 0 holds the
// rows of block b + 1, which are then final: it also forms
// y_{b+1} = Linv_{b+1} rhs_{b+1}.
__global__ __launch_bounds__(256) void k_fwd_update(const double2* __restrict__ A, int64_t K, int64_t kb0,
                                                    const double2* __restrict__ Linv_next, int nb_next,
                                                    double2* __restrict__ rhs, double2* __restrict__ y) {
  __shared__ double2 yb[CB];
  __shared__ double2 rs[CB];
  const int tid = threadIdx.x;
  const int r = tid >> 2, q = tid & 3;
  // group 0: this thread's entries of Linv_{b+1} (m = q + 4 t <= r), loaded
  // first so that they arrive while the rows are updated
  double2 lv[CB / 4];
  if (blockIdx.x == 0) {
#pragma unroll
    for (int t = 0; t < CB / 4; ++t) {
      const int m = q + 4 * t;
      lv[t] = (m <= r && m < nb_next) ? Linv_next[r * CB + m] : make_double2(0.0, 0.0);
    }
  }
  // the row entries and the right-hand side do not depend on y_b: their loads
  // are issued before y_b is published through LDS
  const int64_t R = kb0 + CB + (int64_t)blockIdx.x * CB + r;
  double2 av[CB / 4];
#pragma unroll
  for (int j = 0; j < CB / 4; ++j) av[j] = R < K ? A[R * K + kb0 + 4 * j + q] : make_double2(0.0, 0.0);
  const double2 rv = (R < K && q == 0) ? rhs[R] : make_double2(0.0, 0.0);
  if (tid < CB) yb[tid] = y[kb0 + tid];
  __syncthreads();
  double2 acc = make_double2(0.0, 0.0);
#pragma unroll
  for (int j = 0; j < CB / 4; ++j) acc = cadd(acc, cmul(av[j], yb[4 * j + q]));
  acc = quad_sum(acc);
  double2 nv = make_double2(0.0, 0.0);
  if (R < K && q == 0) {
    nv = csub(rv, acc);
    rhs[R] = nv;
  }
  if (blockIdx.x != 0) return;  // uniform over the group
  if (q == 0) rs[r] = nv;
  __syncthreads();
  double2 s = make_double2(0.0, 0.0);
#pragma unroll
  for (int t = 0; t < CB / 4; ++t) s = cadd(s, cmul(lv[t], rs[q + 4 * t]));
  s = quad_sum(s);
  if (q == 0 && r < nb_next) y[kb0 + CB + r] = s;
}

// x_b = Linv_b^H v_b for the last block b (one group): (Linv^H)[r][m] = conj(Linv[m][r]), m >= r
__global__ __launch_bounds__(256) void k_bwd_first(const double2* __restrict__ Linv, const double2* __restrict__ v,
                                                   double2* __restrict__ x, int nb) {
  const int r = threadIdx.x >> 2, q = threadIdx.x & 3;
  double2 s = make_double2(0.0, 0.0);
  for (int m = r + q; m < nb; m += 4) s = cadd(s, cmul(cconj(Linv[m * CB + r]), v[m]));
  s = quad_sum(s);
  if (q == 0 && r < nb) x[r] = s;
}

// Backward update of block b (x_b in x): v[c] -= sum_m conj(L[kb0 + m][c]) x_b[m]
// for c < kb0, 64 columns per group, wave q summing m = 16 q .. 16 q + 15 (each
// step reads 64 consecutive columns of one row).  The last group holds the
// columns of block b - 1, which are then final: it also forms
// x_{b-1} = Linv_{b-1}^H v_{b-1}.
__global__ __launch_bounds__(256) void k_bwd_update(const double2* __restrict__ A, int64_t K, int64_t kb0, int nb,
                                                    const double2* __restrict__ Linv_prev, double2* __restrict__ v,
                                                    double2* __restrict__ x) {
  __shared__ double2 xb[CB];
  __shared__ double2 part[4][CB];
  __shared__ double2 vs[CB];
  const int tid = threadIdx.x;
  const int wv = tid >> 6, ln = tid & 63;
  // last group: wave w holds conj(Linv_{b-1}[m][ln]) for the rows m = w + 4 t
  // (each load one contiguous row; entries above the diagonal are stored as
  // zeros), loaded first so that they arrive while the columns are updated
  double2 lv[CB / 4];
  if (blockIdx.x == gridDim.x - 1) {
#pragma unroll
    for (int t = 0; t < CB / 4; ++t) lv[t] = cconj(Linv_prev[(wv + 4 * t) * CB + ln]);
  }
  // the column entries and v do not depend on x_b: their loads are issued
  // before x_b is published through LDS
  const int cl = tid & 63, q = tid >> 6;
  const int64_t c = (int64_t)blockIdx.x * CB + cl;  // < kb0: the grid covers kb0 / 64 column blocks
  double2 av[CB / 4];
#pragma unroll
  for (int j = 0; j < CB / 4; ++j) {
    const int m = q * (CB / 4) + j;
    av[j] = m < nb ? cconj(A[(kb0 + m) * K + c]) : make_double2(0.0, 0.0);
  }
  const double2 vc = tid < CB ? v[c] : make_double2(0.0, 0.0);
  if (tid < CB) xb[tid] = tid < nb ? x[kb0 + tid] : make_double2(0.0, 0.0);
  __syncthreads();
  double2 acc = make_double2(0.0, 0.0);
#pragma unroll
  for (int j = 0; j < CB / 4; ++j) acc = cadd(acc, cmul(av[j], xb[q * (CB / 4) + j]));
  part[q][cl] = acc;
  __syncthreads();
  if (tid < CB) {
    const double2 nv = csub(vc, cadd(cadd(part[0][tid], part[1][tid]), cadd(part[2][tid], part[3][tid])));
    v[c] = nv;
    vs[tid] = nv;
  }
  if (blockIdx.x != gridDim.x - 1) return;  // uniform over the group
  __syncthreads();
  // x_{b-1}[ln] = sum_m conj(Linv_{b-1}[m][ln]) v_{b-1}[m], wave w over m = w + 4 t
  double2 s = make_double2(0.0, 0.0);
#pragma unroll
  for (int t = 0; t < CB / 4; ++t) s = cadd(s, cmul(lv[t], vs[wv + 4 * t]));
  part[wv][ln] = s;  // the column update's reads of part finished before the barrier above
  __syncthreads();
  if (tid < CB) x[kb0 - CB + tid] = cadd(cadd(part[0][tid], part[1][tid]), cadd(part[2][tid], part[3][tid]));
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

// rhs is consumed; y and x are K-vectors; x receives the solution
void chol_solve(vmc_ctx* ctx, const double2* S, int64_t K, const double2* Linv, double2* rhs, double2* y, double2* x) {
  hipStream_t st = ctx->stream;
  const int nblk = (int)((K + CB - 1) / CB);
  auto nb_of = [&](int b) { return (int)std::min<int64_t>(CB, K - (int64_t)b * CB); };
  // L y = rhs: y_0 first; launch b updates the rows below block b and forms y_{b+1}
  k_fwd_first<<<1, 256, 0, st>>>(Linv, rhs, y, nb_of(0));
  for (int b = 0; b + 1 < nblk; ++b) {
    const int64_t kb0 = (int64_t)b * CB;
    const int64_t rows = K - kb0 - CB;
    k_fwd_update<<<(unsigned)((rows + CB - 1) / CB), 256, 0, st>>>(S, K, kb0, Linv + (size_t)(b + 1) * CB * CB,
                                                                    nb_of(b + 1), rhs, y);
  }
  // L^H x = y (in place in y): x of the last block first; launch b updates the
  // columns left of block b and forms x_{b-1}
  const int64_t kl = (int64_t)(nblk - 1) * CB;
  k_bwd_first<<<1, 256, 0, st>>>(Linv + (size_t)(nblk - 1) * CB * CB, y + kl, x + kl, nb_of(nblk - 1));
  for (int b = nblk - 1; b >= 1; --b) {
    const int64_t kb0 = (int64_t)b * CB;
    k_bwd_update<<<(unsigned)b, 256, 0, st>>>(S, K, kb0, nb_of(b), Linv + (size_t)(b - 1) * CB * CB, y, x);
  }
  VMC_HIP(hipGetLastError());
}
