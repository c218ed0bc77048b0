// Stochastic reconfiguration / TDVP solve (eq:qfm, eq:force_vector,
// eq:tdvp_util, Sec. 3.1 diagonal shift):
//   1. sample means <O_k>, <E> and Var E (float64 accumulation);
//   2. centred, weight-scaled Obar_nk = sqrt(w_n) (O_nk - <O_k>) and the force
//      F_k = sum_n w_n conj(O_nk - <O_k>) (E_n - <E>) in one pass over O;
//   3. S = Obar^H Obar (Hermitian, lower triangle computed, mirrored);
//      [[.]] projection and the shift S~ = S + nu diag(S) + eps I;
//   4. blocked right-looking Cholesky S~ = L L^H in float64 (lower triangle
//      overwritten; the upper triangle keeps S~ for the residual);
//   5. L y = -[[gamma F]], L^H x = y; residual ||S~ x + [[gamma F]]|| / ||[[gamma F]]||.
#include <algorithm>
#include <cmath>
#include <memory>

#include <type_traits>

#include "internal.h"

using namespace dev;

namespace {

constexpr int kColChunk = 256;  // samples per partial-sum chunk

template <typename InT>
__device__ __forceinline__ double2 load_c(const InT* p, int64_t i) {
  if constexpr (std::is_same<InT, double2>::value) {
    return p[i];
  } else if constexpr (std::is_same<InT, float2>::value) {
    const float2 f = p[i];
    return make_double2(f.x, f.y);
  } else {  // real O
    return make_double2((double)p[i], 0.0);
  }
}

// sum of weights (or N when w == NULL) and the energy statistics
__global__ __launch_bounds__(1024) void k_energy_stats(const double2* __restrict__ e, const double* __restrict__ w,
                                                       int64_t N, double* __restrict__ out /*wsum, mean re, im, var*/) {
  __shared__ double red[3][16];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double sw = 0, sr = 0, si = 0;
  for (int64_t n = tid; n < N; n += 1024) {
    const double wn = w ? w[n] : 1.0;
    sw += wn;
    sr += wn * e[n].x;
    si += wn * e[n].y;
  }
  sw = wave_sum(sw);
  sr = wave_sum(sr);
  si = wave_sum(si);
  if (lane == 0) {
    red[0][wv] = sw;
    red[1][wv] = sr;
    red[2][wv] = si;
  }
  __syncthreads();
  __shared__ double tot[3];
  if (tid == 0) {
    double a = 0, b = 0, c = 0;
    for (int q = 0; q < 16; ++q) {
      a += red[0][q];
      b += red[1][q];
      c += red[2][q];
    }
    tot[0] = a;
    tot[1] = b / a;
    tot[2] = c / a;
  }
  __syncthreads();
  const double wsum = tot[0], mr = tot[1], mi = tot[2];
  double sv = 0;
  for (int64_t n = tid; n < N; n += 1024) {
    const double wn = w ? w[n] : 1.0;
    const double dr = e[n].x - mr, di = e[n].y - mi;
    sv += wn * (dr * dr + di * di);
  }
  sv = wave_sum(sv);
  __syncthreads();
  if (lane == 0) red[0][wv] = sv;
  __syncthreads();
  if (tid == 0) {
    double a = 0;
    for (int q = 0; q < 16; ++q) a += red[0][q];
    out[0] = wsum;
    out[1] = mr;
    out[2] = mi;
    out[3] = a / wsum;
  }
}

// partial[chunk][k] = sum_{n in chunk} w_n O_nk
template <typename InT>
__global__ __launch_bounds__(256) void k_col_partial(const InT* __restrict__ O, const double* __restrict__ w, int64_t N,
                                                     int64_t K, double2* __restrict__ partial) {
  const int64_t k = blockIdx.x * 256ll + threadIdx.x;
  if (k >= K) return;
  const int64_t n0 = (int64_t)blockIdx.y * kColChunk, n1 = min(N, n0 + kColChunk);
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t n = n0; n < n1; ++n) {
    const double wn = w ? w[n] : 1.0;
    const double2 v = load_c(O, n * K + k);
    acc.x += wn * v.x;
    acc.y += wn * v.y;
  }
  partial[(int64_t)blockIdx.y * K + k] = acc;
}

// Column sums of the per-chunk partials: a group of 16 waves owns 64 columns;
// wave w adds chunks w, w + 16, ... in order and the 16 wave sums are combined
// in wave order (deterministic).  out[k] = scale * sum_c partial[c][k], scale =
// 1 / stats[0] when stats is given.
constexpr int kRedWaves = 16;

__global__ __launch_bounds__(64 * kRedWaves) void k_reduce_cols(const double2* __restrict__ partial, int nchunk,
                                                                int64_t K, const double* __restrict__ stats,
                                                                double2* __restrict__ out) {
  __shared__ double2 red[kRedWaves][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t k = blockIdx.x * 64ll + lane;
  double2 acc = make_double2(0.0, 0.0);
  if (k < K)
    for (int c = wave; c < nchunk; c += kRedWaves) acc = cadd(acc, partial[(int64_t)c * K + k]);
  red[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && k < K) {
    double2 s = red[0][lane];
    for (int w = 1; w < kRedWaves; ++w) s = cadd(s, red[w][lane]);
    out[k] = stats ? cscale(s, 1.0 / stats[0]) : s;
  }
}

// Xc[n][k] = sqrt(w_n / wsum) (O_nk - mean_k); Fpartial[chunk][k] = sum w_n conj(O_nk - mean_k) (E_n - Ebar)
template <typename InT, typename XT>
__global__ __launch_bounds__(256) void k_center_force(const InT* __restrict__ O, const double* __restrict__ w,
                                                      const double2* __restrict__ e, int64_t N, int64_t K,
                                                      const double2* __restrict__ mean,
                                                      const double* __restrict__ stats, XT* __restrict__ Xc,
                                                      double2* __restrict__ Fpartial) {
  const int64_t k = blockIdx.x * 256ll + threadIdx.x;
  if (k >= K) return;
  const int64_t n0 = (int64_t)blockIdx.y * kColChunk, n1 = min(N, n0 + kColChunk);
  const double wsum = stats[0];
  const double2 eb = make_double2(stats[1], stats[2]);
  const double2 mk = mean[k];
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t n = n0; n < n1; ++n) {
    const double wn = (w ? w[n] : 1.0) / wsum;
    const double2 d = csub(load_c(O, n * K + k), mk);
    const double sq = sqrt(wn);
    if constexpr (sizeof(XT) == sizeof(double2))
      Xc[n * K + k] = make_double2(sq * d.x, sq * d.y);
    else
      Xc[n * K + k] = make_float2((float)(sq * d.x), (float)(sq * d.y));
    const double2 de = csub(e[n], eb);
    const double2 p = cmul(cconj(d), de);
    acc.x += wn * p.x;
    acc.y += wn * p.y;
  }
  Fpartial[(int64_t)blockIdx.y * K + k] = acc;
}

// Real O: two consecutive samples share one complex row of the centred matrix,
//   Xc[m][k] = (sqrt(w_2m) (O_2m,k - mean_k), sqrt(w_2m+1) (O_2m+1,k - mean_k)),
// so that Re(Xc^H Xc) = sum_n w_n (O_n - mean)(O_n - mean)^T with half the rows
// (the imaginary part of that product is not S and is never formed).
template <typename InT, typename XT>
__global__ __launch_bounds__(256) void k_center_force_pair(const InT* __restrict__ O, const double* __restrict__ w,
                                                           const double2* __restrict__ e, int64_t N, int64_t K,
                                                           const double2* __restrict__ mean,
                                                           const double* __restrict__ stats, XT* __restrict__ Xc,
                                                           double2* __restrict__ Fpartial) {
  const int64_t k = blockIdx.x * 256ll + threadIdx.x;
  if (k >= K) return;
  const int64_t n0 = (int64_t)blockIdx.y * kColChunk, n1 = min(N, n0 + kColChunk);  // n0 even
  const double wsum = stats[0];
  const double2 eb = make_double2(stats[1], stats[2]);
  const double mk = mean[k].x;
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t n = n0; n < n1; n += 2) {
    double v[2] = {0.0, 0.0};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (n + h >= N) break;
      const double wn = (w ? w[n + h] : 1.0) / wsum;
      const double d = (double)O[(n + h) * K + k] - mk;
      v[h] = sqrt(wn) * d;
      const double2 de = csub(e[n + h], eb);
      acc.x += wn * d * de.x;
      acc.y += wn * d * de.y;
    }
    if constexpr (std::is_same<XT, double2>::value)
      Xc[(n >> 1) * K + k] = make_double2(v[0], v[1]);
    else
      Xc[(n >> 1) * K + k] = make_float2((float)v[0], (float)v[1]);
  }
  Fpartial[(int64_t)blockIdx.y * K + k] = acc;
}


// S[r][c] = sum_n conj(Xc[n][r]) Xc[n][c] for the 32x32 tile (r >= c block-wise),
// written to both triangles; projection and shift applied here.
template <typename XT>
__global__ __launch_bounds__(256) void k_herk_simple(const XT* __restrict__ X, int64_t N, int64_t K, int mode,
                                                     double nu, double eps, double2* __restrict__ S,
                                                     double2* __restrict__ diag) {
  const int tr = blockIdx.y, tc = blockIdx.x;
  if (tc > tr) return;
  __shared__ double2 xa[16][33], xb[16][33];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t r0 = (int64_t)tr * 32, c0 = (int64_t)tc * 32;
  double2 acc[2][2] = {};
  for (int64_t n0 = 0; n0 < N; n0 += 16) {
    for (int e = threadIdx.x; e < 16 * 32; e += 256) {
      const int nn = e >> 5, cc = e & 31;
      const int64_t n = n0 + nn;
      xa[nn][cc] = (n < N && r0 + cc < K) ? load_c(X, n * K + r0 + cc) : make_double2(0.0, 0.0);
      xb[nn][cc] = (n < N && c0 + cc < K) ? load_c(X, n * K + c0 + cc) : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int nn = 0; nn < 16; ++nn) {
      const double2 a0 = cconj(xa[nn][ty]), a1 = cconj(xa[nn][ty + 16]);
      const double2 b0 = xb[nn][tx], b1 = xb[nn][tx + 16];
      acc[0][0] = cadd(acc[0][0], cmul(a0, b0));
      acc[0][1] = cadd(acc[0][1], cmul(a0, b1));
      acc[1][0] = cadd(acc[1][0], cmul(a1, b0));
      acc[1][1] = cadd(acc[1][1], cmul(a1, b1));
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t r = r0 + ty + 16 * i, c = c0 + tx + 16 * j;
      if (r >= K || c >= K || c > r) continue;
      double2 v = acc[i][j];
      if (mode == VMC_SR_REAL) v.y = 0.0;
      if (mode == VMC_SR_IMAG) v.x = 0.0;  // i Im S
      if (r == c) {
        v = make_double2(v.x * (1.0 + nu) + eps, 0.0);
        diag[r] = v;
      }
      S[r * K + c] = v;
      if (r != c) S[c * K + r] = cconj(v);
    }
}

// rhs = -[[gamma F]]; for the Im projection the system Im[S~] x = -Im[gamma F]
// is held as (i Im S~) x = -i Im[gamma F], so rhs = (0, -Im[gamma F])
__global__ void k_rhs(const double2* __restrict__ F, int64_t K, double gr, double gi, int mode, double2* __restrict__ rhs) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= K) return;
  double2 v = cmul(make_double2(gr, gi), F[k]);
  if (mode == VMC_SR_REAL) v.y = 0.0;
  if (mode == VMC_SR_IMAG) v.x = 0.0;
  rhs[k] = make_double2(-v.x, -v.y);
}

// x <- Re x (the Im projection's solution is real)
__global__ void k_keep_real(double2* __restrict__ x, int64_t K) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < K) x[k].y = 0.0;
}

// r_k = sum_c S~[k][c] x_c - rhs_k, using the upper triangle (S~ itself) and
// the saved diagonal; one wave per row.
__global__ __launch_bounds__(64) void k_resid_upper(const double2* __restrict__ A, int64_t K,
                                                    const double2* __restrict__ diag, const double2* __restrict__ x,
                                                    double2* __restrict__ r) {
  const int64_t k = blockIdx.x;
  const int lane = threadIdx.x;
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t c = k + 1 + lane; c < K; c += 64) acc = cadd(acc, cmul(A[k * K + c], x[c]));
  acc = wave_sum(acc);
  if (lane == 0) r[k] = cadd(acc, cmul(diag[k], x[k]));
}

// part[chunk][c] = sum_{k in chunk, k < c} conj(S~[k][c]) x_k  (strictly lower part
// via the upper storage); rows split into chunks of 256 over blockIdx.y.
__global__ __launch_bounds__(256) void k_resid_lower_part(const double2* __restrict__ A, int64_t K,
                                                          const double2* __restrict__ x, double2* __restrict__ part) {
  const int64_t c = blockIdx.x * 256ll + threadIdx.x;
  if (c >= K) return;
  const int64_t k0 = (int64_t)blockIdx.y * 256, k1 = min(c, k0 + 256);
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t k = k0; k < k1; ++k) acc = cadd(acc, cmul(cconj(A[k * K + c]), x[k]));
  part[(int64_t)blockIdx.y * K + c] = acc;
}

__global__ void k_resid_finish(const double2* __restrict__ part, int nchunk, int64_t K,
                               const double2* __restrict__ rhs, double2* __restrict__ r) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= K) return;
  double2 acc = r[c];
  for (int q = 0; q < nchunk; ++q) acc = cadd(acc, part[(int64_t)q * K + c]);
  r[c] = csub(acc, rhs[c]);
}

__global__ __launch_bounds__(1024) void k_norms(const double2* __restrict__ a, const double2* __restrict__ b, int64_t K,
                                                double* __restrict__ out) {
  __shared__ double ra[16], rb[16];
  double sa = 0, sb = 0;
  for (int64_t k = threadIdx.x; k < K; k += 1024) {
    sa += a[k].x * a[k].x + a[k].y * a[k].y;
    sb += b[k].x * b[k].x + b[k].y * b[k].y;
  }
  sa = wave_sum(sa);
  sb = wave_sum(sb);
  if ((threadIdx.x & 63) == 0) {
    ra[threadIdx.x >> 6] = sa;
    rb[threadIdx.x >> 6] = sb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double x = 0, y = 0;
    for (int q = 0; q < 16; ++q) {
      x += ra[q];
      y += rb[q];
    }
    out[0] = x;
    out[1] = y;
  }
}

__global__ void k_init_fail(long long* f) { *f = -1; }

// ---- matrix-free conjugate gradient (diagonal shift + iterative solver) ----

// The centred, weight-scaled samples are applied without forming them:
//   (Obar v)_n   = sq_n (sum_k O_nk v_k - <O>.v),        sq_n = sqrt(w_n / sum w)
//   (Obar^H u)_k = sum_n conj(O_nk) sq_n u_n - conj(<O_k>) sum_n sq_n u_n
// so the operator is exactly that of the given O (float64 arithmetic).

__global__ void k_sqw(const double* __restrict__ w, int64_t N, const double* __restrict__ stats,
                      double* __restrict__ sq) {
  const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (n < N) sq[n] = sqrt((w ? w[n] : 1.0) / stats[0]);
}

// per column chunk: Fpart = sum sq^2 conj(O - <O>) (E - <E>), Dpart = (sum sq^2 |O - <O>|^2, 0)
template <typename InT>
__global__ __launch_bounds__(256) void k_force_diag(const InT* __restrict__ O, const double* __restrict__ sq,
                                                    const double2* __restrict__ e, int64_t N, int64_t K,
                                                    const double2* __restrict__ mean, const double* __restrict__ stats,
                                                    double2* __restrict__ Fpart, double2* __restrict__ Dpart) {
  const int64_t k = blockIdx.x * 256ll + threadIdx.x;
  if (k >= K) return;
  const int64_t n0 = (int64_t)blockIdx.y * kColChunk, n1 = min(N, n0 + kColChunk);
  const double2 eb = make_double2(stats[1], stats[2]);
  const double2 mk = mean[k];
  double2 f = make_double2(0.0, 0.0);
  double dd = 0.0;
  for (int64_t n = n0; n < n1; ++n) {
    const double wn = sq[n] * sq[n];
    const double2 d = csub(load_c(O, n * K + k), mk);
    const double2 p = cmul(cconj(d), csub(e[n], eb));
    f.x += wn * p.x;
    f.y += wn * p.y;
    dd += wn * (d.x * d.x + d.y * d.y);
  }
  Fpart[(int64_t)blockIdx.y * K + k] = f;
  Dpart[(int64_t)blockIdx.y * K + k] = make_double2(dd, 0.0);
}

// u_n = sq_n (sum_k O_nk v_k - mv[0]), one group per row
template <typename InT>
__global__ __launch_bounds__(256) void k_ov(const InT* __restrict__ O, int64_t N, int64_t K,
                                            const double2* __restrict__ v, const double* __restrict__ mv,
                                            const double* __restrict__ sq, double2* __restrict__ u) {
  __shared__ double2 red[4];
  const int64_t n = blockIdx.x;
  if (n >= N) return;
  const InT* row = O + n * K;
  double2 acc = make_double2(0.0, 0.0), acc2 = acc;
  int64_t k = threadIdx.x;
  // two independent accumulators, four loads in flight per thread
  for (; k + 3 * 256 < K; k += 4 * 256) {
    const double2 o0 = load_c(row, k), o1 = load_c(row, k + 256), o2 = load_c(row, k + 512),
                  o3 = load_c(row, k + 768);
    acc = cadd(acc, cmul(o0, v[k]));
    acc2 = cadd(acc2, cmul(o1, v[k + 256]));
    acc = cadd(acc, cmul(o2, v[k + 512]));
    acc2 = cadd(acc2, cmul(o3, v[k + 768]));
  }
  for (; k < K; k += 256) acc = cadd(acc, cmul(load_c(row, k), v[k]));
  acc = wave_sum(cadd(acc, acc2));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double2 s = cadd(cadd(red[0], red[1]), cadd(red[2], red[3]));
    u[n] = cscale(make_double2(s.x - mv[0], s.y - mv[1]), sq[n]);
  }
}

// partial[chunk][k] = sum_{n in chunk} conj(O_nk) sq_n u_n
template <typename InT>
__global__ __launch_bounds__(256) void k_ohu(const InT* __restrict__ O, int64_t N, int64_t K,
                                             const double2* __restrict__ u, const double* __restrict__ sq,
                                             double2* __restrict__ partial) {
  const int64_t k = blockIdx.x * 256ll + threadIdx.x;
  if (k >= K) return;
  const int64_t n0 = (int64_t)blockIdx.y * kColChunk, n1 = min(N, n0 + kColChunk);
  double2 acc = make_double2(0.0, 0.0), acc2 = acc;
  int64_t n = n0;
  for (; n + 3 < n1; n += 4) {
    const double2 o0 = load_c(O, n * K + k), o1 = load_c(O, (n + 1) * K + k), o2 = load_c(O, (n + 2) * K + k),
                  o3 = load_c(O, (n + 3) * K + k);
    acc = cadd(acc, cscale(cmul(cconj(o0), u[n]), sq[n]));
    acc2 = cadd(acc2, cscale(cmul(cconj(o1), u[n + 1]), sq[n + 1]));
    acc = cadd(acc, cscale(cmul(cconj(o2), u[n + 2]), sq[n + 2]));
    acc2 = cadd(acc2, cscale(cmul(cconj(o3), u[n + 3]), sq[n + 3]));
  }
  for (; n < n1; ++n) acc = cadd(acc, cscale(cmul(cconj(load_c(O, n * K + k)), u[n]), sq[n]));
  partial[(int64_t)blockIdx.y * K + k] = cadd(acc, acc2);
}

// out[0..1] = sum_n sq_n u_n
__global__ __launch_bounds__(1024) void k_wsum(const double* __restrict__ sq, const double2* __restrict__ u, int64_t N,
                                               double* __restrict__ out) {
  __shared__ double red[2][16];
  double sr = 0, si = 0;
  for (int64_t n = threadIdx.x; n < N; n += 1024) {
    sr += sq[n] * u[n].x;
    si += sq[n] * u[n].y;
  }
  sr = wave_sum(sr);
  si = wave_sum(si);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = sr;
    red[1][threadIdx.x >> 6] = si;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, b = 0;
    for (int q = 0; q < 16; ++q) {
      a += red[0][q];
      b += red[1][q];
    }
    out[0] = a;
    out[1] = b;
  }
}

// Ap_k = [[sum_chunks partial - conj(<O_k>) su]] + (nu dS_k + eps) p_k
__global__ void k_cg_apply(const double2* __restrict__ partial, int nchunk, int64_t K, const double2* __restrict__ p,
                           const double2* __restrict__ mean, const double* __restrict__ su,
                           const double* __restrict__ dS, double nu, double eps, int mode, double2* __restrict__ Ap) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= K) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int c = 0; c < nchunk; ++c) acc = cadd(acc, partial[(int64_t)c * K + k]);
  acc = csub(acc, cmul(cconj(mean[k]), make_double2(su[0], su[1])));
  if (mode == VMC_SR_REAL) acc.y = 0.0;
  const double sh = nu * dS[k] + eps;
  Ap[k] = make_double2(acc.x + sh * p[k].x, acc.y + sh * p[k].y);
}

__global__ void k_conj(const double2* __restrict__ a, int64_t K, double2* __restrict__ out) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < K) out[k] = cconj(a[k]);
}

// out[0..1] = sum conj(a_k) b_k; with c != NULL also out[2..3] = sum conj(c_k) c_k
__global__ __launch_bounds__(1024) void k_cg_dot(const double2* __restrict__ a, const double2* __restrict__ b,
                                                 const double2* __restrict__ c, int64_t K, double* __restrict__ out) {
  __shared__ double red[3][16];
  double sr = 0, si = 0, sc = 0;
  for (int64_t k = threadIdx.x; k < K; k += 1024) {
    const double2 p = cmul(cconj(a[k]), b[k]);
    sr += p.x;
    si += p.y;
    if (c) sc += c[k].x * c[k].x + c[k].y * c[k].y;
  }
  sr = wave_sum(sr);
  si = wave_sum(si);
  sc = wave_sum(sc);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = sr;
    red[1][w] = si;
    red[2][w] = sc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a0 = 0, a1 = 0, a2 = 0;
    for (int q = 0; q < 16; ++q) {
      a0 += red[0][q];
      a1 += red[1][q];
      a2 += red[2][q];
    }
    out[0] = a0;
    out[1] = a1;
    if (c) out[2] = a2;
  }
}

// scalars: sc[0..1] = r^H z, sc[2..3] = p^H A p, sc[4..5] = new r^H z, sc[6] = r^H r
__global__ void k_cg_step1(double2* __restrict__ x, double2* __restrict__ r, double2* __restrict__ z,
                           const double2* __restrict__ p, const double2* __restrict__ Ap,
                           const double* __restrict__ M, const double* __restrict__ sc, int64_t K) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= K) return;
  const double2 al = cdiv(make_double2(sc[0], sc[1]), make_double2(sc[2], sc[3]));
  x[k] = cadd(x[k], cmul(al, p[k]));
  const double2 rn = csub(r[k], cmul(al, Ap[k]));
  r[k] = rn;
  z[k] = cscale(rn, 1.0 / M[k]);
}

__global__ void k_cg_step2(double2* __restrict__ p, const double2* __restrict__ z, const double* __restrict__ sc,
                           int64_t K) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= K) return;
  const double2 be = cdiv(make_double2(sc[4], sc[5]), make_double2(sc[0], sc[1]));
  p[k] = cadd(z[k], cmul(be, p[k]));
}

__global__ void k_cg_rotate(double* __restrict__ sc) {
  sc[0] = sc[4];
  sc[1] = sc[5];
}

// M_k = (1 + nu) dS_k + eps (1 where that vanishes); z = b / M; p = z; x = 0; r = b
__global__ void k_cg_init(const double2* __restrict__ b, const double* __restrict__ dS, double nu, double eps,
                          int64_t K, double* __restrict__ M, double2* __restrict__ x, double2* __restrict__ r,
                          double2* __restrict__ z, double2* __restrict__ p) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= K) return;
  double m = (1.0 + nu) * dS[k] + eps;
  if (!(m > 0.0)) m = 1.0;
  M[k] = m;
  x[k] = make_double2(0.0, 0.0);
  r[k] = b[k];
  z[k] = cscale(b[k], 1.0 / m);
  p[k] = z[k];
}

__global__ void k_cg_resid(const double2* __restrict__ b, const double2* __restrict__ Ax, int64_t K,
                           double2* __restrict__ res) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < K) res[k] = csub(b[k], Ax[k]);
}

__global__ void k_take_real(const double2* __restrict__ a, int64_t K, double* __restrict__ out) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < K) out[k] = a[k].x;
}


// ---- eigen-decomposition regularisation (pseudo-inverse cutoffs, SNR) ----

// rho_j = sum_k conj(V_kj) b_k  (V row-major K x K)
__global__ void k_vh_mul(const double2* __restrict__ V, const double2* __restrict__ b, int64_t K,
                         double2* __restrict__ rho) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= K) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t k = 0; k < K; ++k) acc = cadd(acc, cmul(cconj(V[k * K + j]), b[k]));
  rho[j] = acc;
}

// x_k = sum_j V_kj y_j, one wave per row
__global__ __launch_bounds__(64) void k_v_mul(const double2* __restrict__ V, const double2* __restrict__ y, int64_t K,
                                              double2* __restrict__ x) {
  const int64_t k = blockIdx.x;
  const int lane = threadIdx.x;
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t j = lane; j < K; j += 64) acc = cadd(acc, cmul(V[k * K + j], y[j]));
  acc = wave_sum(acc);
  if (lane == 0) x[k] = acc;
}

// Y_nk = sqrt(w_n) conj(f_nk),  f_nk = [[gamma (E_n - Ebar) conj(O_nk - mean_k)]]: the per-sample
// terms whose weighted sum is [[gamma F]] (i Im[.] for the Im projection)
template <typename InT, typename XT>
__global__ __launch_bounds__(256) void k_force_terms(const InT* __restrict__ O, const double* __restrict__ w,
                                                     const double2* __restrict__ e, int64_t N, int64_t K,
                                                     const double2* __restrict__ mean, const double* __restrict__ stats,
                                                     double gr, double gi, int mode, XT* __restrict__ Y) {
  const int64_t k = blockIdx.x * 256ll + threadIdx.x;
  if (k >= K) return;
  const int64_t n0 = (int64_t)blockIdx.y * kColChunk, n1 = min(N, n0 + kColChunk);
  const double wsum = stats[0];
  const double2 eb = make_double2(stats[1], stats[2]);
  const double2 mk = mean[k];
  for (int64_t n = n0; n < n1; ++n) {
    const double sq = sqrt((w ? w[n] : 1.0) / wsum);
    const double2 d = csub(load_c(O, n * K + k), mk);
    double2 f = cmul(make_double2(gr, gi), cmul(csub(e[n], eb), cconj(d)));
    if (mode == VMC_SR_REAL) f.y = 0.0;
    if (mode == VMC_SR_IMAG) f.x = 0.0;  // i Im[.], the terms of the rhs held as i b
    const double2 y = make_double2(sq * f.x, -sq * f.y);
    if constexpr (std::is_same<XT, double2>::value)
      Y[n * K + k] = y;
    else
      Y[n * K + k] = make_float2((float)y.x, (float)y.y);
  }
}

// C = A B, K x K complex float64 (row-major), 32 x 32 tiles, 4 outputs per thread
__global__ __launch_bounds__(256) void k_zgemm_nn(const double2* __restrict__ A, const double2* __restrict__ B,
                                                  int64_t K, double2* __restrict__ C) {
  __shared__ double2 As[32][33], Bs[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // ty 0..7
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  double2 acc[4] = {};
  for (int64_t k0 = 0; k0 < K; k0 += 32) {
    for (int q = 0; q < 4; ++q) {
      const int rr = ty + 8 * q;
      As[rr][tx] = (r0 + rr < K && k0 + tx < K) ? A[(r0 + rr) * K + k0 + tx] : make_double2(0.0, 0.0);
      Bs[rr][tx] = (k0 + rr < K && c0 + tx < K) ? B[(k0 + rr) * K + c0 + tx] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int kk = 0; kk < 32; ++kk) {
      const double2 b = Bs[kk][tx];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = cadd(acc[q], cmul(As[ty + 8 * q][kk], b));
    }
    __syncthreads();
  }
  for (int q = 0; q < 4; ++q) {
    const int64_t r = r0 + ty + 8 * q, c = c0 + tx;
    if (r < K && c < K) C[r * K + c] = acc[q];
  }
}

// var_j = sum_k conj(V_kj) W_kj - |rho_j|^2  with W = H V (the weighted second moment
// of the eigen-basis components of the per-sample terms, minus the squared mean)
__global__ void k_snr_var(const double2* __restrict__ V, const double2* __restrict__ W, const double2* __restrict__ rho,
                          int64_t K, double* __restrict__ var) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= K) return;
  double acc = 0.0;
  for (int64_t k = 0; k < K; ++k) {
    const double2 v = V[k * K + j], q = W[k * K + j];
    acc += v.x * q.x + v.y * q.y;  // Re(conj(v) q)
  }
  const double2 r = rho[j];
  var[j] = acc - (r.x * r.x + r.y * r.y);
}

__global__ __launch_bounds__(1024) void k_absmax(const double* __restrict__ a, int64_t K, double* __restrict__ out) {
  __shared__ double red[16];
  double m = 0.0;
  for (int64_t k = threadIdx.x; k < K; k += 1024) m = fmax(m, fabs(a[k]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int q = 0; q < 16; ++q) r = fmax(r, red[q]);
    out[0] = r;
  }
}

// y_j = lambda_j^+ rho_j with the regularised inverse of the eigenvalue:
//   hard:  0 if |lambda_j / lambda_1| < eps_pinv, else 1 / lambda_j
//   soft:  1 / (lambda_j (1 + (eps_pinv / |lambda_j / lambda_1|)^6))
//   SNR:   times 1 / (1 + (eps_snr / SNR_j)^6),  SNR_j = |rho_j| / sqrt(var_j / N_s)
// and lambda_j^+ = 0 for lambda_j = 0.
__global__ void k_pinv_scale(const double* __restrict__ lam, const double* __restrict__ lmax,
                             const double2* __restrict__ rho, const double* __restrict__ var, int64_t K, double ns,
                             double eps_pinv, int soft, double eps_snr, double2* __restrict__ y,
                             double* __restrict__ snr_out) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= K) return;
  const double l = lam[j];
  const double rel = lmax[0] > 0.0 ? fabs(l) / lmax[0] : 0.0;
  double inv = 0.0;
  if (l != 0.0) {
    if (eps_pinv <= 0.0) {
      inv = 1.0 / l;
    } else if (soft) {
      const double q = eps_pinv / rel;
      const double q2 = q * q;
      inv = 1.0 / (l * (1.0 + q2 * q2 * q2));
    } else {
      inv = rel < eps_pinv ? 0.0 : 1.0 / l;
    }
  }
  double snr = INFINITY;
  if (var) {
    const double2 r = rho[j];
    const double sig = sqrt(fmax(var[j], 0.0) / ns);
    const double ar = sqrt(r.x * r.x + r.y * r.y);
    snr = sig > 0.0 ? ar / sig : (ar > 0.0 ? INFINITY : 0.0);
    if (eps_snr > 0.0) {
      if (snr == 0.0) {
        inv = 0.0;
      } else if (isfinite(snr)) {
        const double q = eps_snr / snr;
        const double q2 = q * q;
        inv /= 1.0 + q2 * q2 * q2;
      }
    }
  }
  if (snr_out) snr_out[j] = snr;
  y[j] = make_double2(inv * rho[j].x, inv * rho[j].y);
}

}  // namespace

void sr_solve_impl(vmc_ctx* ctx, const void* O, int dtype, const double2* eloc, const double* w, int64_t N, int64_t K,
                   const vmc_sr_opts* o, double2* x, vmc_sr_info* info, const vmc_eig_opts* eo, double* evals,
                   double* snr, int* sweeps, double2* S_out, double2* F_out) {
  hipStream_t st = ctx->stream;
  const int nchunk = (int)((N + kColChunk - 1) / kColChunk);
  const int kchunk = (int)((K + 255) / 256);
  const int npart = std::max(nchunk, kchunk);
  const int CB = chol_block();
  const int nblk = (int)((K + CB - 1) / CB);
  const bool real_o = dtype == VMC_DT_F32 || dtype == VMC_DT_F64;
  const bool f32 = dtype == VMC_DT_C64 || dtype == VMC_DT_F32;
  const int64_t Nx = real_o ? (N + 1) / 2 : N;     // rows of the centred matrix (real O: sample pairs)
  const int hmode = real_o ? VMC_SR_REAL : o->mode;  // S is real for real O
  const size_t xsz = (f32 ? sizeof(float2) : sizeof(double2)) * (size_t)Nx * K;
  const bool split16 = o->gram == 1;
  const bool eig = eo != nullptr;
  const bool use_snr = eig && (eo->eps_snr > 0.0 || snr);
  const size_t hws = (!split16 && f32) ? std::max(herk_ws_bytes(Nx, K, hmode),
                                                  use_snr ? herk_ws_bytes(N, K, o->mode) : (size_t)0)
                                       : 0;
  const size_t ysz = use_snr ? (f32 ? sizeof(float2) : sizeof(double2)) * (size_t)N * K : 0;
  const size_t kk = sizeof(double2) * (size_t)K * K;
  const size_t eig_extra = eig ? ws_round(eig_ws_bytes(K)) + ws_round(kk) + ws_round(sizeof(double) * K) * 3 +
                                     ws_round(sizeof(double2) * K) * 2 + ws_round(64) +
                                     (use_snr ? ws_round(ysz) + ws_round(kk) : 0)
                               : 0;
  size_t total = eig_extra + (split16 ? herk16_ws_bytes(Nx, K) : 0) + ws_round(hws) + ws_round(64) + ws_round(sizeof(double2) * npart * K) + ws_round(sizeof(double2) * K) * 7 +
                 ws_round(chol_linv_bytes(K)) +
                 ws_round(xsz) + ws_round(sizeof(double2) * (size_t)K * K) + ws_round(sizeof(double) * nblk) +
                 ws_round(sizeof(long long)) + ws_round(sizeof(double) * 4) + ws_round(chol_sync_bytes(K));
  ws_reserve(ctx, total);
  double* stats = (double*)ws_take(ctx, 64);
  double2* partial = (double2*)ws_take(ctx, sizeof(double2) * npart * K);
  double2* mean = (double2*)ws_take(ctx, sizeof(double2) * K);
  double2* F = (double2*)ws_take(ctx, sizeof(double2) * K);
  double2* rhs = (double2*)ws_take(ctx, sizeof(double2) * K);
  double2* sol = (double2*)ws_take(ctx, sizeof(double2) * K);
  double2* diag = (double2*)ws_take(ctx, sizeof(double2) * K);
  double2* res = (double2*)ws_take(ctx, sizeof(double2) * K);
  double2* yv = (double2*)ws_take(ctx, sizeof(double2) * K);
  double2* Linv = (double2*)ws_take(ctx, chol_linv_bytes(K));
  void* Xc = ws_take(ctx, xsz);
  double2* S = (double2*)ws_take(ctx, sizeof(double2) * (size_t)K * K);
  double* pivmin = (double*)ws_take(ctx, sizeof(double) * nblk);
  long long* fail = (long long*)ws_take(ctx, sizeof(long long));
  double* norms = (double*)ws_take(ctx, sizeof(double) * 4);
  int* tsync = (int*)ws_take(ctx, chol_sync_bytes(K));
  void* h16ws = split16 ? ws_take(ctx, herk16_ws_bytes(Nx, K)) : nullptr;
  void* hws_p = hws ? ws_take(ctx, hws) : nullptr;
  void* eig_ws = eig ? ws_take(ctx, eig_ws_bytes(K)) : nullptr;
  double2* Vm = eig ? (double2*)ws_take(ctx, kk) : nullptr;
  double* lam = eig ? (double*)ws_take(ctx, sizeof(double) * K) : nullptr;
  double* var = eig ? (double*)ws_take(ctx, sizeof(double) * K) : nullptr;
  double* snr_d = eig ? (double*)ws_take(ctx, sizeof(double) * K) : nullptr;
  double2* rho = eig ? (double2*)ws_take(ctx, sizeof(double2) * K) : nullptr;
  double2* yv2 = eig ? (double2*)ws_take(ctx, sizeof(double2) * K) : nullptr;
  double* lmax = eig ? (double*)ws_take(ctx, 64) : nullptr;
  void* Ysnr = use_snr ? ws_take(ctx, ysz) : nullptr;
  double2* Hm = use_snr ? (double2*)ws_take(ctx, kk) : nullptr;

  std::unique_ptr<phase_scope> ph(new phase_scope(ctx, "sr.center"));
  k_energy_stats<<<1, 1024, 0, st>>>(eloc, w, N, stats);
  dim3 cg(grid_for(K, 256), nchunk);
  if (dtype == VMC_DT_C64)
    k_col_partial<float2><<<cg, 256, 0, st>>>((const float2*)O, w, N, K, partial);
  else if (dtype == VMC_DT_C128)
    k_col_partial<double2><<<cg, 256, 0, st>>>((const double2*)O, w, N, K, partial);
  else if (dtype == VMC_DT_F32)
    k_col_partial<float><<<cg, 256, 0, st>>>((const float*)O, w, N, K, partial);
  else
    k_col_partial<double><<<cg, 256, 0, st>>>((const double*)O, w, N, K, partial);
  k_reduce_cols<<<(unsigned)((K + 63) / 64), 64 * kRedWaves, 0, st>>>(partial, nchunk, K, stats, mean);
  if (dtype == VMC_DT_C64)
    k_center_force<float2, float2><<<cg, 256, 0, st>>>((const float2*)O, w, eloc, N, K, mean, stats, (float2*)Xc,
                                                        partial);
  else if (dtype == VMC_DT_C128)
    k_center_force<double2, double2><<<cg, 256, 0, st>>>((const double2*)O, w, eloc, N, K, mean, stats,
                                                          (double2*)Xc, partial);
  else if (dtype == VMC_DT_F32)
    k_center_force_pair<float, float2><<<cg, 256, 0, st>>>((const float*)O, w, eloc, N, K, mean, stats,
                                                            (float2*)Xc, partial);
  else
    k_center_force_pair<double, double2><<<cg, 256, 0, st>>>((const double*)O, w, eloc, N, K, mean, stats,
                                                              (double2*)Xc, partial);
  k_reduce_cols<<<(unsigned)((K + 63) / 64), 64 * kRedWaves, 0, st>>>(partial, nchunk, K, nullptr, F);
  VMC_HIP(hipGetLastError());
  ph.reset();

  ph.reset(new phase_scope(ctx, "sr.herk"));
  const unsigned nb32 = (unsigned)((K + 31) / 32);
  dim3 hg(nb32, nb32);
  if (split16)
    herk_split16(ctx, (const float2*)Xc, Nx, K, hmode, o->nu_rel, o->eps_abs, S, diag, h16ws);
  else if (f32)
    herk_mfma_f32(ctx, (const float2*)Xc, Nx, K, hmode, o->nu_rel, o->eps_abs, S, diag, hws_p);
  else
    k_herk_simple<double2><<<hg, 256, 0, st>>>((const double2*)Xc, Nx, K, hmode, o->nu_rel, o->eps_abs, S, diag);
  VMC_HIP(hipGetLastError());
  ph.reset();

  if (S_out) {  // test export: S~ and F as formed for the solve, no factorisation
    VMC_HIP(hipMemcpyAsync(S_out, S, sizeof(double2) * (size_t)K * K, hipMemcpyDeviceToDevice, st));
    VMC_HIP(hipMemcpyAsync(F_out, F, sizeof(double2) * K, hipMemcpyDeviceToDevice, st));
    double* hs = (double*)pinned_host(ctx, sizeof(double) * 4);
    VMC_HIP(hipMemcpyAsync(hs, stats, sizeof(double) * 4, hipMemcpyDeviceToHost, st));
    VMC_HIP(hipStreamSynchronize(st));
    info->e_mean[0] = hs[1];
    info->e_mean[1] = hs[2];
    info->e_var = hs[3];
    info->fail_index = -1;
    info->residual = NAN;
    info->min_pivot = NAN;
    return;
  }

  if (eig) {
    info->fail_index = -1;
    // second moment of the per-sample force terms (SNR): H = Y^H Y
    if (use_snr) {
      ph.reset(new phase_scope(ctx, "sr.snr"));
      const int fmode = o->mode == VMC_SR_REAL ? VMC_SR_REAL : VMC_SR_COMPLEX;
      if (dtype == VMC_DT_C64)
        k_force_terms<float2, float2><<<cg, 256, 0, st>>>((const float2*)O, w, eloc, N, K, mean, stats, o->gamma_re,
                                                           o->gamma_im, o->mode, (float2*)Ysnr);
      else if (dtype == VMC_DT_F32)
        k_force_terms<float, float2><<<cg, 256, 0, st>>>((const float*)O, w, eloc, N, K, mean, stats, o->gamma_re,
                                                          o->gamma_im, o->mode, (float2*)Ysnr);
      else if (dtype == VMC_DT_C128)
        k_force_terms<double2, double2><<<cg, 256, 0, st>>>((const double2*)O, w, eloc, N, K, mean, stats,
                                                             o->gamma_re, o->gamma_im, o->mode, (double2*)Ysnr);
      else
        k_force_terms<double, double2><<<cg, 256, 0, st>>>((const double*)O, w, eloc, N, K, mean, stats, o->gamma_re,
                                                            o->gamma_im, o->mode, (double2*)Ysnr);
      VMC_HIP(hipGetLastError());
      if (f32)
        herk_mfma_f32(ctx, (const float2*)Ysnr, N, K, fmode, 0.0, 0.0, Hm, rho, hws_p);
      else
        k_herk_simple<double2><<<hg, 256, 0, st>>>((const double2*)Ysnr, N, K, fmode, 0.0, 0.0, Hm, rho);
      VMC_HIP(hipGetLastError());
      ph.reset();
    }
    ph.reset(new phase_scope(ctx, "sr.eig"));
    const int sw = eig_hermitian(ctx, S, K, eo->tol > 0.0 ? eo->tol : 1e-14, eo->max_sweeps > 0 ? eo->max_sweeps : 50,
                                 lam, Vm, eig_ws);
    if (sweeps) *sweeps = sw;
    ph.reset();
    ph.reset(new phase_scope(ctx, "sr.trsv"));
    k_rhs<<<grid_for(K, 256), 256, 0, st>>>(F, K, o->gamma_re, o->gamma_im, o->mode, rhs);
    k_vh_mul<<<grid_for(K, 256), 256, 0, st>>>(Vm, rhs, K, rho);
    if (use_snr) {
      double2* Wm = (double2*)eig_ws;  // the Jacobi workspace is free again
      const dim3 gg((unsigned)((K + 31) / 32), (unsigned)((K + 31) / 32));
      k_zgemm_nn<<<gg, 256, 0, st>>>(Hm, Vm, K, Wm);
      k_snr_var<<<grid_for(K, 256), 256, 0, st>>>(Vm, Wm, rho, K, var);
    }
    k_absmax<<<1, 1024, 0, st>>>(lam, K, lmax);
    k_pinv_scale<<<grid_for(K, 256), 256, 0, st>>>(lam, lmax, rho, use_snr ? var : nullptr, K, (double)N,
                                                   eo->eps_pinv, eo->soft, eo->eps_snr, yv2, snr_d);
    k_v_mul<<<(unsigned)K, 64, 0, st>>>(Vm, yv2, K, sol);
    if (o->mode == VMC_SR_IMAG) k_keep_real<<<grid_for(K, 256), 256, 0, st>>>(sol, K);
    VMC_HIP(hipGetLastError());
    ph.reset();
    if (evals) VMC_HIP(hipMemcpyAsync(evals, lam, sizeof(double) * K, hipMemcpyDeviceToDevice, st));
    if (snr) VMC_HIP(hipMemcpyAsync(snr, snr_d, sizeof(double) * K, hipMemcpyDeviceToDevice, st));
    // residual of the regularised solution against the unregularised (shifted) system
    ph.reset(new phase_scope(ctx, "sr.resid"));
    VMC_HIP(hipMemcpyAsync(res, rhs, sizeof(double2) * K, hipMemcpyDeviceToDevice, st));
    k_resid_upper<<<(unsigned)K, 64, 0, st>>>(S, K, diag, sol, res);
    k_resid_lower_part<<<dim3(grid_for(K, 256), kchunk), 256, 0, st>>>(S, K, sol, partial);
    k_resid_finish<<<grid_for(K, 256), 256, 0, st>>>(partial, kchunk, K, rhs, res);
    k_norms<<<1, 1024, 0, st>>>(res, rhs, K, norms);
    VMC_HIP(hipMemcpyAsync(x, sol, sizeof(double2) * K, hipMemcpyDeviceToDevice, st));
    VMC_HIP(hipGetLastError());
    ph.reset();
    const size_t hb = sizeof(double) * (6 + K);
    double* hh = (double*)pinned_host(ctx, hb);
    VMC_HIP(hipMemcpyAsync(hh, norms, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
    VMC_HIP(hipMemcpyAsync(hh + 2, stats, sizeof(double) * 4, hipMemcpyDeviceToHost, st));
    VMC_HIP(hipMemcpyAsync(hh + 6, lam, sizeof(double) * K, hipMemcpyDeviceToHost, st));
    VMC_HIP(hipStreamSynchronize(st));
    info->residual = hh[1] > 0 ? std::sqrt(hh[0] / hh[1]) : std::sqrt(hh[0]);
    info->e_mean[0] = hh[3];
    info->e_mean[1] = hh[4];
    info->e_var = hh[5];
    double pm = INFINITY;
    for (int64_t j = 0; j < K; ++j) pm = std::min(pm, hh[6 + j]);
    info->min_pivot = pm;  // smallest eigenvalue of the shifted S
    return;
  }

  ph.reset(new phase_scope(ctx, "sr.chol"));
  k_init_fail<<<1, 1, 0, st>>>(fail);
  chol_factor(ctx, S, K, Linv, fail, pivmin);
  VMC_HIP(hipGetLastError());
  ph.reset();

  // fail flag and pivots back to the host
  const size_t hbytes = sizeof(long long) + sizeof(double) * (nblk + 8);
  char* h = (char*)pinned_host(ctx, hbytes);
  VMC_HIP(hipMemcpyAsync(h, fail, sizeof(long long), hipMemcpyDeviceToHost, st));
  VMC_HIP(hipMemcpyAsync(h + sizeof(long long), pivmin, sizeof(double) * nblk, hipMemcpyDeviceToHost, st));
  VMC_HIP(hipMemcpyAsync(h + sizeof(long long) + sizeof(double) * nblk, stats, sizeof(double) * 4,
                         hipMemcpyDeviceToHost, st));
  VMC_HIP(hipStreamSynchronize(st));
  long long fidx;
  std::memcpy(&fidx, h, sizeof(fidx));
  const double* piv = (const double*)(h + sizeof(long long));
  const double* hs = piv + nblk;
  info->e_mean[0] = hs[1];
  info->e_mean[1] = hs[2];
  info->e_var = hs[3];
  info->fail_index = fidx;
  const int nb_done = fidx >= 0 ? (int)(fidx / CB) + 1 : nblk;
  double pm = INFINITY;
  for (int b = 0; b < nb_done; ++b) pm = std::min(pm, piv[b]);
  info->min_pivot = pm;
  info->residual = NAN;
  if (fidx >= 0) return;

  ph.reset(new phase_scope(ctx, "sr.trsv"));
  k_rhs<<<grid_for(K, 256), 256, 0, st>>>(F, K, o->gamma_re, o->gamma_im, o->mode, rhs);
  chol_solve(ctx, S, K, Linv, rhs, yv, sol, tsync);
  VMC_HIP(hipGetLastError());
  ph.reset();
  ph.reset(new phase_scope(ctx, "sr.resid"));
  k_resid_upper<<<(unsigned)K, 64, 0, st>>>(S, K, diag, sol, res);
  k_resid_lower_part<<<dim3(grid_for(K, 256), kchunk), 256, 0, st>>>(S, K, sol, partial);
  k_resid_finish<<<grid_for(K, 256), 256, 0, st>>>(partial, kchunk, K, rhs, res);
  k_norms<<<1, 1024, 0, st>>>(res, rhs, K, norms);
  VMC_HIP(hipMemcpyAsync(x, sol, sizeof(double2) * K, hipMemcpyDeviceToDevice, st));
  VMC_HIP(hipGetLastError());
  ph.reset();
  double* hn = (double*)pinned_host(ctx, sizeof(double) * 3);
  VMC_HIP(hipMemcpyAsync(hn, norms, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
  VMC_HIP(hipMemcpyAsync(hn + 2, tsync + chol_sync_err_index(K), sizeof(int), hipMemcpyDeviceToHost, st));
  VMC_HIP(hipStreamSynchronize(st));
  int wait_err;
  std::memcpy(&wait_err, hn + 2, sizeof(int));
  if (wait_err) throw vmc_error{VMC_ERR_HIP, "triangular solve: a block hand-over exceeded its poll limit"};
  info->residual = hn[1] > 0 ? std::sqrt(hn[0] / hn[1]) : std::sqrt(hn[0]);
}

namespace {
__global__ __launch_bounds__(1024) void k_wtotal(const double* __restrict__ w, int64_t N, double* __restrict__ stats) {
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t n = threadIdx.x; n < N; n += 1024) s += w ? w[n] : 1.0;
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int q = 0; q < 16; ++q) r += red[q];
    stats[0] = r;
  }
}
}  // namespace

// v^H S v = sum_n w_n |(O_n - <O>) . v|^2 (weights normalised), from the samples
double fisher_quad_impl(vmc_ctx* ctx, const void* O, int dtype, const double* w, int64_t N, int64_t K,
                        const double2* v) {
  hipStream_t st = ctx->stream;
  const int nchunk = (int)((N + kColChunk - 1) / kColChunk);
  ws_reserve(ctx, ws_round(64) + ws_round(sizeof(double2) * (size_t)nchunk * K) + ws_round(sizeof(double2) * K) * 2 +
                      ws_round(sizeof(double) * N) + ws_round(sizeof(double2) * N) + ws_round(sizeof(double) * 16));
  double* stats = (double*)ws_take(ctx, 64);
  double2* partial = (double2*)ws_take(ctx, sizeof(double2) * (size_t)nchunk * K);
  double2* mean = (double2*)ws_take(ctx, sizeof(double2) * K);
  double2* cmean = (double2*)ws_take(ctx, sizeof(double2) * K);
  double* sq = (double*)ws_take(ctx, sizeof(double) * N);
  double2* u = (double2*)ws_take(ctx, sizeof(double2) * N);
  double* sc = (double*)ws_take(ctx, sizeof(double) * 16);
  k_wtotal<<<1, 1024, 0, st>>>(w, N, stats);
  const dim3 cg(grid_for(K, 256), nchunk);
  if (dtype == VMC_DT_C64)
    k_col_partial<float2><<<cg, 256, 0, st>>>((const float2*)O, w, N, K, partial);
  else if (dtype == VMC_DT_C128)
    k_col_partial<double2><<<cg, 256, 0, st>>>((const double2*)O, w, N, K, partial);
  else if (dtype == VMC_DT_F32)
    k_col_partial<float><<<cg, 256, 0, st>>>((const float*)O, w, N, K, partial);
  else
    k_col_partial<double><<<cg, 256, 0, st>>>((const double*)O, w, N, K, partial);
  k_reduce_cols<<<(unsigned)((K + 63) / 64), 64 * kRedWaves, 0, st>>>(partial, nchunk, K, stats, mean);
  k_conj<<<grid_for(K, 256), 256, 0, st>>>(mean, K, cmean);
  k_cg_dot<<<1, 1024, 0, st>>>(cmean, v, nullptr, K, sc + 8);  // <O> . v
  k_sqw<<<grid_for(N, 256), 256, 0, st>>>(w, N, stats, sq);
  if (dtype == VMC_DT_C64)
    k_ov<float2><<<(unsigned)N, 256, 0, st>>>((const float2*)O, N, K, v, sc + 8, sq, u);
  else if (dtype == VMC_DT_C128)
    k_ov<double2><<<(unsigned)N, 256, 0, st>>>((const double2*)O, N, K, v, sc + 8, sq, u);
  else if (dtype == VMC_DT_F32)
    k_ov<float><<<(unsigned)N, 256, 0, st>>>((const float*)O, N, K, v, sc + 8, sq, u);
  else
    k_ov<double><<<(unsigned)N, 256, 0, st>>>((const double*)O, N, K, v, sc + 8, sq, u);
  k_norms<<<1, 1024, 0, st>>>(u, u, N, sc);
  VMC_HIP(hipGetLastError());
  double* h = (double*)pinned_host(ctx, sizeof(double) * 2);
  VMC_HIP(hipMemcpyAsync(h, sc, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
  VMC_HIP(hipStreamSynchronize(st));
  return h[0];
}

// Shifted SR solve by Jacobi-preconditioned conjugate gradient, with
// S v = Obar^H (Obar v) applied from the samples (S is never formed).
void sr_solve_cg_impl(vmc_ctx* ctx, const void* O, int dtype, const double2* eloc, const double* w, int64_t N,
                      int64_t K, const vmc_sr_opts* o, double tol, int max_iter, double2* x, vmc_sr_info* info,
                      int* iters) {
  hipStream_t st = ctx->stream;
  const int nchunk = (int)((N + kColChunk - 1) / kColChunk);
  const bool f32 = dtype == VMC_DT_C64;
  const size_t vk = ws_round(sizeof(double2) * K);
  const size_t pk = ws_round(sizeof(double2) * (size_t)nchunk * K);
  size_t total = ws_round(64) + 2 * pk + vk * 11 + ws_round(sizeof(double) * K) * 2 + ws_round(sizeof(double2) * N) +
                 ws_round(sizeof(double) * N) + ws_round(sizeof(double) * 16);
  ws_reserve(ctx, total);
  double* stats = (double*)ws_take(ctx, 64);
  double2* partial = (double2*)ws_take(ctx, sizeof(double2) * (size_t)nchunk * K);
  double2* partial2 = (double2*)ws_take(ctx, sizeof(double2) * (size_t)nchunk * K);
  double2* mean = (double2*)ws_take(ctx, sizeof(double2) * K);
  double2* cmean = (double2*)ws_take(ctx, sizeof(double2) * K);
  double2* F = (double2*)ws_take(ctx, sizeof(double2) * K);
  double2* b = (double2*)ws_take(ctx, sizeof(double2) * K);
  double2* xs = (double2*)ws_take(ctx, sizeof(double2) * K);
  double2* r = (double2*)ws_take(ctx, sizeof(double2) * K);
  double2* z = (double2*)ws_take(ctx, sizeof(double2) * K);
  double2* pv = (double2*)ws_take(ctx, sizeof(double2) * K);
  double2* Ap = (double2*)ws_take(ctx, sizeof(double2) * K);
  double2* dSc = (double2*)ws_take(ctx, sizeof(double2) * K);
  double2* spare = (double2*)ws_take(ctx, sizeof(double2) * K);
  double* dS = (double*)ws_take(ctx, sizeof(double) * K);
  double* M = (double*)ws_take(ctx, sizeof(double) * K);
  double2* u = (double2*)ws_take(ctx, sizeof(double2) * N);
  double* sq = (double*)ws_take(ctx, sizeof(double) * N);
  double* sc = (double*)ws_take(ctx, sizeof(double) * 16);  // [0..6] CG scalars, [8..9] <O>.v, [10..11] sum sq u
  (void)spare;

  std::unique_ptr<phase_scope> ph(new phase_scope(ctx, "sr.center"));
  k_energy_stats<<<1, 1024, 0, st>>>(eloc, w, N, stats);
  dim3 cg(grid_for(K, 256), nchunk);
  if (f32)
    k_col_partial<float2><<<cg, 256, 0, st>>>((const float2*)O, w, N, K, partial);
  else
    k_col_partial<double2><<<cg, 256, 0, st>>>((const double2*)O, w, N, K, partial);
  k_reduce_cols<<<(unsigned)((K + 63) / 64), 64 * kRedWaves, 0, st>>>(partial, nchunk, K, stats, mean);
  k_conj<<<grid_for(K, 256), 256, 0, st>>>(mean, K, cmean);
  k_sqw<<<grid_for(N, 256), 256, 0, st>>>(w, N, stats, sq);
  if (f32)
    k_force_diag<float2><<<cg, 256, 0, st>>>((const float2*)O, sq, eloc, N, K, mean, stats, partial, partial2);
  else
    k_force_diag<double2><<<cg, 256, 0, st>>>((const double2*)O, sq, eloc, N, K, mean, stats, partial, partial2);
  k_reduce_cols<<<(unsigned)((K + 63) / 64), 64 * kRedWaves, 0, st>>>(partial, nchunk, K, nullptr, F);
  k_reduce_cols<<<(unsigned)((K + 63) / 64), 64 * kRedWaves, 0, st>>>(partial2, nchunk, K, nullptr, dSc);
  k_take_real<<<grid_for(K, 256), 256, 0, st>>>(dSc, K, dS);
  k_rhs<<<grid_for(K, 256), 256, 0, st>>>(F, K, o->gamma_re, o->gamma_im, o->mode, b);
  VMC_HIP(hipGetLastError());
  ph.reset();

  auto matvec = [&](const double2* v, double2* out) {
    k_cg_dot<<<1, 1024, 0, st>>>(cmean, v, nullptr, K, sc + 8);  // <O>.v
    if (f32) {
      k_ov<float2><<<(unsigned)N, 256, 0, st>>>((const float2*)O, N, K, v, sc + 8, sq, u);
      k_ohu<float2><<<cg, 256, 0, st>>>((const float2*)O, N, K, u, sq, partial);
    } else {
      k_ov<double2><<<(unsigned)N, 256, 0, st>>>((const double2*)O, N, K, v, sc + 8, sq, u);
      k_ohu<double2><<<cg, 256, 0, st>>>((const double2*)O, N, K, u, sq, partial);
    }
    k_wsum<<<1, 1024, 0, st>>>(sq, u, N, sc + 10);
    k_cg_apply<<<grid_for(K, 256), 256, 0, st>>>(partial, nchunk, K, v, mean, sc + 10, dS, o->nu_rel, o->eps_abs,
                                                 o->mode, out);
  };

  ph.reset(new phase_scope(ctx, "sr.cg"));
  const unsigned gk = grid_for(K, 256);
  k_cg_init<<<gk, 256, 0, st>>>(b, dS, o->nu_rel, o->eps_abs, K, M, xs, r, z, pv);
  k_cg_dot<<<1, 1024, 0, st>>>(r, z, b, K, sc);  // sc[0..1] = r^H z, sc[2] = b^H b
  double* hsc = (double*)pinned_host(ctx, sizeof(double) * 16);
  VMC_HIP(hipMemcpyAsync(hsc, sc, sizeof(double) * 8, hipMemcpyDeviceToHost, st));
  VMC_HIP(hipStreamSynchronize(st));
  const double bb = hsc[2];
  int it = 0;
  if (bb > 0.0) {
    for (it = 0; it < max_iter;) {
      matvec(pv, Ap);
      k_cg_dot<<<1, 1024, 0, st>>>(pv, Ap, nullptr, K, sc + 2);
      k_cg_step1<<<gk, 256, 0, st>>>(xs, r, z, pv, Ap, M, sc, K);
      k_cg_dot<<<1, 1024, 0, st>>>(r, z, r, K, sc + 4);  // sc[4..5] = r^H z, sc[6] = r^H r
      k_cg_step2<<<gk, 256, 0, st>>>(pv, z, sc, K);
      k_cg_rotate<<<1, 1, 0, st>>>(sc);
      ++it;
      if (it % 8 == 0 || it == max_iter) {
        VMC_HIP(hipMemcpyAsync(hsc, sc, sizeof(double) * 8, hipMemcpyDeviceToHost, st));
        VMC_HIP(hipStreamSynchronize(st));
        if (!std::isfinite(hsc[6]) || std::sqrt(hsc[6] / bb) <= tol) break;
      }
    }
  }
  VMC_HIP(hipGetLastError());
  ph.reset();

  // true residual ||b - A x|| / ||b||
  ph.reset(new phase_scope(ctx, "sr.resid"));
  matvec(xs, Ap);
  k_cg_resid<<<gk, 256, 0, st>>>(b, Ap, K, z);
  k_norms<<<1, 1024, 0, st>>>(z, b, K, sc);
  VMC_HIP(hipMemcpyAsync(x, xs, sizeof(double2) * K, hipMemcpyDeviceToDevice, st));
  VMC_HIP(hipGetLastError());
  ph.reset();
  VMC_HIP(hipMemcpyAsync(hsc, sc, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
  VMC_HIP(hipMemcpyAsync(hsc + 2, stats, sizeof(double) * 4, hipMemcpyDeviceToHost, st));
  VMC_HIP(hipStreamSynchronize(st));
  info->residual = hsc[1] > 0 ? std::sqrt(hsc[0] / hsc[1]) : std::sqrt(hsc[0]);
  info->e_mean[0] = hsc[3];
  info->e_mean[1] = hsc[4];
  info->e_var = hsc[5];
  info->fail_index = -1;
  info->min_pivot = NAN;
  *iters = it;
}
