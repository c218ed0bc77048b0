// Hermitian eigendecomposition on the device (float64), for the pseudo-inverse
// and signal-to-noise regularisations of the TDVP equation (Sec. 3.3: the
// regularised inverse needs S = V diag(lambda) V^dagger).
//
// Two-sided block Jacobi.  The matrix (padded with decoupled zero rows and
// columns to Kp, a multiple of 2 BJ) is cut into nb = Kp / BJ index blocks; a
// sweep is nb - 1 rounds, and round r pairs every block once (circle ordering).
// For a pair (P, Q) the 2 BJ x 2 BJ Hermitian submatrix on the indices P u Q is
// diagonalised in LDS by cyclic Jacobi (below), giving a unitary U; then every
// block (i, j) of pairs becomes U_i^H A_ij U_j and V <- V diag(U).  The pairs
// of a round are disjoint, so the block transforms commute; each round reads
// the matrix it transforms from one buffer and writes the other.  Sweeps stop
// when the off-diagonal Frobenius norm is below tol times the full norm.
//
// Inner cyclic Jacobi on M (2 BJ indices, each round pairs every index once):
// for a pair (p, q) with M_pp = a, M_qq = b, M_pq = |z| e^{i phi}, the unitary
//     J = [[c, s], [-s e, c e]],  e = e^{-i phi},  t = s / c the smaller root of
//     t^2 + 2 tau t - 1 = 0,  tau = (b - a) / (2 |z|),
// zeroes M_pq (M <- J^H M J on rows and columns p, q; U <- U J).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.h"

using namespace dev;

namespace {

constexpr int BJ = 16;       // index block of the outer Jacobi
constexpr int BM = 2 * BJ;   // a pair's submatrix
constexpr int MAX_INNER = 1; // inner sweeps per submatrix and round (one measured fastest)
// a pair's submatrix is reduced below INNER_TOL x the outer tolerance, so that what the
// pairs leave on their own off-diagonals stays below the outer criterion
constexpr double INNER_TOL = 0.125;

struct jrot {
  int p, q;
  double c, s;
  double2 e;
  double a_new, b_new;  // diagonal after the rotation
  int active;
};

// circle ordering of n indices (n even), round r: pair i
__device__ __forceinline__ void circle_pair(int n, int r, int i, int& p, int& q) {
  const int m = n - 1;
  if (i == 0) {
    p = m;
    q = r;
  } else {
    p = (r + i) % m;
    q = (r - i + m) % m;
  }
}

// rotation of pair i of inner round r on the BM x BM matrix M (row-major in LDS)
__device__ __forceinline__ jrot make_rot(const double2* M, int i, int r) {
  int p, q;
  circle_pair(BM, r, i, p, q);
  const double a = M[p * BM + p].x, b = M[q * BM + q].x;
  const double2 z = M[p * BM + q];
  const double az = hypot(z.x, z.y);
  jrot R;
  R.p = p;
  R.q = q;
  // negligible coupling: no rotation (also for the decoupled padding indices)
  if (!(az > 0.0) || az <= 1e-300 || az < 1e-17 * sqrt(fabs(a) * fabs(b))) {
    R.c = 1.0;
    R.s = 0.0;
    R.e = make_double2(1.0, 0.0);
    R.a_new = a;
    R.b_new = b;
    R.active = 0;
  } else {
    const double tau = (b - a) / (2.0 * az);
    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
    R.c = 1.0 / sqrt(1.0 + t * t);
    R.s = t * R.c;
    R.e = make_double2(z.x / az, -z.y / az);  // e^{-i phi}
    R.a_new = a - t * az;
    R.b_new = b + t * az;
    R.active = 1;
  }
  return R;
}

// global index of local index l (0 .. BM - 1) of the pair (P, Q)
__device__ __forceinline__ int64_t gidx(int P, int Q, int l) {
  return l < BJ ? (int64_t)P * BJ + l : (int64_t)Q * BJ + (l - BJ);
}

// One group per block pair of outer round r: diagonalise the submatrix on P u Q
// by inner Jacobi sweeps (until its off-diagonal norm is below tol times its
// norm, max_inner at most) and write the accumulated unitary U (BM x BM,
// row-major) to Ub[i] and the rotated submatrix to Mb[i].
__global__ __launch_bounds__(256) void k_bj_solve(const double2* __restrict__ A, int64_t Kp, int nb, int r,
                                                  double tol, int max_inner, double2* __restrict__ Ub,
                                                  double2* __restrict__ Mb) {
  __shared__ double2 M[2][BM * BM];
  __shared__ double2 U[BM * BM];
  __shared__ double red[2][4];
  const int i = blockIdx.x, tid = threadIdx.x;
  int P, Q;
  circle_pair(nb, r, i, P, Q);
  for (int e = tid; e < BM * BM; e += 256) {
    const int a = e / BM, b = e % BM;
    M[0][e] = A[gidx(P, Q, a) * Kp + gidx(P, Q, b)];
    U[e] = make_double2(a == b ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  // thread (ii, jj): the 2 x 2 block of pair ii's rows and pair jj's columns,
  // and rows ii, ii + 16 of U in pair jj's columns
  const int ii = tid >> 4, jj = tid & 15;
  int cur = 0;
  for (int sw = 0; sw < max_inner; ++sw) {
    // off-diagonal and full norm of M
    double off = 0.0, all = 0.0;
    for (int e = tid; e < BM * BM; e += 256) {
      const double2 v = M[cur][e];
      const double m2 = v.x * v.x + v.y * v.y;
      all += m2;
      if (e / BM != e % BM) off += m2;
    }
    off = wave_sum(off);
    all = wave_sum(all);
    if ((tid & 63) == 0) {
      red[0][tid >> 6] = off;
      red[1][tid >> 6] = all;
    }
    __syncthreads();
    const double to = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    const double ta = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    __syncthreads();
    if (!(to > tol * tol * ta)) break;
    for (int rr = 0; rr < BM - 1; ++rr) {
      const double2* Mi = M[cur];
      double2* Mo = M[cur ^ 1];
      const jrot Ri = make_rot(Mi, ii, rr), Rj = make_rot(Mi, jj, rr);
      double2* w0 = Mo + Ri.p * BM;
      double2* w1 = Mo + Ri.q * BM;
      const double2* r0 = Mi + Ri.p * BM;
      const double2* r1 = Mi + Ri.q * BM;
      if (ii == jj) {
        if (Ri.active) {  // the pair's own 2 x 2 block: diagonal by construction
          w0[Ri.p] = make_double2(Ri.a_new, 0.0);
          w1[Ri.q] = make_double2(Ri.b_new, 0.0);
          w0[Ri.q] = make_double2(0.0, 0.0);
          w1[Ri.p] = make_double2(0.0, 0.0);
        } else {
          w0[Ri.p] = r0[Ri.p];
          w1[Ri.q] = r1[Ri.q];
          w0[Ri.q] = r0[Ri.q];
          w1[Ri.p] = r1[Ri.p];
        }
      } else {
        const double2 m00 = r0[Rj.p], m01 = r0[Rj.q], m10 = r1[Rj.p], m11 = r1[Rj.q];
        // T = M J_j:  T[:,0] = c M[:,0] - s e M[:,1],  T[:,1] = s M[:,0] + c e M[:,1]
        const double2 em01 = cmul(Rj.e, m01), em11 = cmul(Rj.e, m11);
        const double2 t00 = make_double2(Rj.c * m00.x - Rj.s * em01.x, Rj.c * m00.y - Rj.s * em01.y);
        const double2 t10 = make_double2(Rj.c * m10.x - Rj.s * em11.x, Rj.c * m10.y - Rj.s * em11.y);
        const double2 t01 = make_double2(Rj.s * m00.x + Rj.c * em01.x, Rj.s * m00.y + Rj.c * em01.y);
        const double2 t11 = make_double2(Rj.s * m10.x + Rj.c * em11.x, Rj.s * m10.y + Rj.c * em11.y);
        // M' = J_i^H T:  row 0 = c T[0,:] - s conj(e) T[1,:],  row 1 = s T[0,:] + c conj(e) T[1,:]
        const double2 ce = cconj(Ri.e);
        const double2 u10 = cmul(ce, t10), u11 = cmul(ce, t11);
        w0[Rj.p] = make_double2(Ri.c * t00.x - Ri.s * u10.x, Ri.c * t00.y - Ri.s * u10.y);
        w0[Rj.q] = make_double2(Ri.c * t01.x - Ri.s * u11.x, Ri.c * t01.y - Ri.s * u11.y);
        w1[Rj.p] = make_double2(Ri.s * t00.x + Ri.c * u10.x, Ri.s * t00.y + Ri.c * u10.y);
        w1[Rj.q] = make_double2(Ri.s * t01.x + Ri.c * u11.x, Ri.s * t01.y + Ri.c * u11.y);
      }
      // U <- U J_j on rows ii and ii + 16
      if (Rj.active)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          double2* row = U + (ii + 16 * h) * BM;
          const double2 v0 = row[Rj.p], v1 = row[Rj.q];
          const double2 ev1 = cmul(Rj.e, v1);
          row[Rj.p] = make_double2(Rj.c * v0.x - Rj.s * ev1.x, Rj.c * v0.y - Rj.s * ev1.y);
          row[Rj.q] = make_double2(Rj.s * v0.x + Rj.c * ev1.x, Rj.s * v0.y + Rj.c * ev1.y);
        }
      __syncthreads();
      cur ^= 1;
    }
  }
  // one Newton-Schulz step U <- U (3 I - U^H U) / 2: the product of the rotations is
  // unitary only to the rounding of each rotation; this takes U back to the rounding
  // of one step, so that V, which takes a U every round, stays orthonormal
  {
    const int a = tid >> 3, b0 = tid & 7;
    double2 g[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) g[k] = make_double2(0.0, 0.0);
    for (int m = 0; m < BM; ++m) {
      const double2 u = cconj(U[m * BM + a]);
#pragma unroll
      for (int k = 0; k < 4; ++k) g[k] = cadd(g[k], cmul(u, U[m * BM + b0 + 8 * k]));
    }
    // H = (3 I - G) / 2 into M[cur ^ 1]
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int b = b0 + 8 * k;
      M[cur ^ 1][a * BM + b] = make_double2((a == b ? 1.5 : 0.0) - 0.5 * g[k].x, -0.5 * g[k].y);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) g[k] = make_double2(0.0, 0.0);
    for (int m = 0; m < BM; ++m) {
      const double2 u = U[a * BM + m];
#pragma unroll
      for (int k = 0; k < 4; ++k) g[k] = cadd(g[k], cmul(u, M[cur ^ 1][m * BM + b0 + 8 * k]));
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) U[a * BM + b0 + 8 * k] = g[k];
    __syncthreads();
  }
  double2* out = Ub + (int64_t)i * BM * BM;
  double2* mout = Mb + (int64_t)i * BM * BM;
  for (int e = tid; e < BM * BM; e += 256) {
    out[e] = U[e];
    mout[e] = M[cur][e];
  }
}

// Groups with blockIdx.y < np: block (i = blockIdx.y, j = blockIdx.x) of pairs,
// Aout[P_i u Q_i, P_j u Q_j] = U_i^H Ain[...] U_j; a pair's own block (i = j)
// is the submatrix the rotations left (a product would put rounding noise back
// into its off-diagonal, where the sweeps could not remove it again).  The
// others: V <- V U_j on rows 32 x of V (in place; each group owns its rows and
// pair j's columns).
__global__ __launch_bounds__(256) void k_bj_apply(const double2* __restrict__ Ain, double2* __restrict__ Aout,
                                                  double2* __restrict__ Vm, int64_t Kp, int nb, int r,
                                                  const double2* __restrict__ Ub, const double2* __restrict__ Mb) {
  __shared__ double2 T[BM * (BM + 1)];
  __shared__ double2 Uj[BM * (BM + 1)];
  const int np = nb / 2;
  const int tid = threadIdx.x;
  const int j = blockIdx.x;
  int Pj, Qj;
  circle_pair(nb, r, j, Pj, Qj);
  for (int e = tid; e < BM * BM; e += 256) Uj[(e / BM) * (BM + 1) + e % BM] = Ub[(int64_t)j * BM * BM + e];
  if ((int)blockIdx.y == j) {
    for (int e = tid; e < BM * BM; e += 256)
      Aout[gidx(Pj, Qj, e / BM) * Kp + gidx(Pj, Qj, e % BM)] = Mb[(int64_t)j * BM * BM + e];
  } else if ((int)blockIdx.y < np) {
    const int i = blockIdx.y;
    int Pi, Qi;
    circle_pair(nb, r, i, Pi, Qi);
    for (int e = tid; e < BM * BM; e += 256) {
      const int a = e / BM, b = e % BM;
      T[a * (BM + 1) + b] = Ain[gidx(Pi, Qi, a) * Kp + gidx(Pj, Qj, b)];
    }
    __syncthreads();
    // thread: row a = tid / 8 of the block, columns b = (tid % 8) + 8 k
    const int a = tid >> 3, b0 = tid & 7;
    double2 x[4];  // (T U_j)[a][b]
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = make_double2(0.0, 0.0);
    for (int m = 0; m < BM; ++m) {
      const double2 t = T[a * (BM + 1) + m];
#pragma unroll
      for (int k = 0; k < 4; ++k) x[k] = cadd(x[k], cmul(t, Uj[m * (BM + 1) + b0 + 8 * k]));
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) T[a * (BM + 1) + b0 + 8 * k] = x[k];
    // U_i into Uj's place (U_j is no longer needed)
    for (int e = tid; e < BM * BM; e += 256) Uj[(e / BM) * (BM + 1) + e % BM] = Ub[(int64_t)i * BM * BM + e];
    __syncthreads();
    // out[a][b] = sum_m conj(U_i[m][a]) (T U_j)[m][b]
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = make_double2(0.0, 0.0);
    for (int m = 0; m < BM; ++m) {
      const double2 u = cconj(Uj[m * (BM + 1) + a]);
#pragma unroll
      for (int k = 0; k < 4; ++k) x[k] = cadd(x[k], cmul(u, T[m * (BM + 1) + b0 + 8 * k]));
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) Aout[gidx(Pi, Qi, a) * Kp + gidx(Pj, Qj, b0 + 8 * k)] = x[k];
  } else {
    const int64_t r0 = (int64_t)(blockIdx.y - np) * BM;
    for (int e = tid; e < BM * BM; e += 256) {
      const int a = e / BM, b = e % BM;
      T[a * (BM + 1) + b] = Vm[(r0 + a) * Kp + gidx(Pj, Qj, b)];
    }
    __syncthreads();
    const int a = tid >> 3, b0 = tid & 7;
    double2 x[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = make_double2(0.0, 0.0);
    for (int m = 0; m < BM; ++m) {
      const double2 t = T[a * (BM + 1) + m];
#pragma unroll
      for (int k = 0; k < 4; ++k) x[k] = cadd(x[k], cmul(t, Uj[m * (BM + 1) + b0 + 8 * k]));
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) Vm[(r0 + a) * Kp + gidx(Pj, Qj, b0 + 8 * k)] = x[k];
  }
}

// out[0] += sum of |A_ij|^2 off the diagonal, out[1] += sum of all |A_ij|^2 (per row, one wave)
__global__ __launch_bounds__(256) void k_offnorm(const double2* __restrict__ A, int64_t Kp, double* __restrict__ out) {
  const int64_t row = blockIdx.x * 4ll + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= Kp) return;
  double off = 0.0, all = 0.0;
  for (int64_t c = lane; c < Kp; c += 64) {
    const double2 v = A[row * Kp + c];
    const double m = v.x * v.x + v.y * v.y;
    all += m;
    if (c != row) off += m;
  }
  off = wave_sum(off);
  all = wave_sum(all);
  if (lane == 0) {
    atomicAdd(out, off);
    atomicAdd(out + 1, all);
  }
}

__global__ void k_pad_copy(const double2* __restrict__ S, int64_t K, int64_t Kp, double2* __restrict__ A,
                           double2* __restrict__ V) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= Kp * Kp) return;
  const int64_t r = e / Kp, c = e % Kp;
  A[e] = (r < K && c < K) ? S[r * K + c] : make_double2(0.0, 0.0);
  V[e] = make_double2(r == c ? 1.0 : 0.0, 0.0);
}

__global__ void k_eig_out(const double2* __restrict__ A, const double2* __restrict__ Vp, int64_t K, int64_t Kp,
                          double* __restrict__ lam, double2* __restrict__ V) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= K * K) return;
  const int64_t r = e / K, c = e % K;
  V[e] = Vp[r * Kp + c];
  if (r == 0) lam[c] = A[c * Kp + c].x;
}

int64_t padded(int64_t K) { return (K + BM - 1) / BM * BM; }

}  // namespace

size_t eig_ws_bytes(int64_t K) {
  const int64_t Kp = padded(K);
  return ws_round(sizeof(double2) * Kp * Kp) * 3 + 2 * ws_round(sizeof(double2) * (Kp / BM) * BM * BM) +
         ws_round(2 * sizeof(double));
}

int eig_hermitian(vmc_ctx* ctx, const double2* S, int64_t K, double tol, int max_sweeps, double* lam, double2* V,
                  void* ws) {
  hipStream_t st = ctx->stream;
  const int64_t Kp = padded(K);
  const int nb = (int)(Kp / BJ), np = nb / 2;
  char* w = (char*)ws;
  double2* A = (double2*)w;
  w += ws_round(sizeof(double2) * Kp * Kp);
  double2* A2 = (double2*)w;
  w += ws_round(sizeof(double2) * Kp * Kp);
  double2* Vp = (double2*)w;
  w += ws_round(sizeof(double2) * Kp * Kp);
  double2* Ub = (double2*)w;
  w += ws_round(sizeof(double2) * (Kp / BM) * BM * BM);
  double2* Mb = (double2*)w;
  w += ws_round(sizeof(double2) * (Kp / BM) * BM * BM);
  double* nrm = (double*)w;
  k_pad_copy<<<grid_for(Kp * Kp, 256), 256, 0, st>>>(S, K, Kp, A, Vp);
  VMC_HIP(hipGetLastError());
  double* hn = (double*)pinned_host(ctx, 2 * sizeof(double));
  int sweeps = 0;
  for (;;) {
    VMC_HIP(hipMemsetAsync(nrm, 0, 2 * sizeof(double), st));
    k_offnorm<<<(unsigned)((Kp + 3) / 4), 256, 0, st>>>(A, Kp, nrm);
    VMC_HIP(hipMemcpyAsync(hn, nrm, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    VMC_HIP(hipStreamSynchronize(st));
    if (!(hn[0] > tol * tol * hn[1]) || sweeps >= max_sweeps) break;
    for (int r = 0; r < nb - 1; ++r) {
      k_bj_solve<<<(unsigned)np, 256, 0, st>>>(A, Kp, nb, r, INNER_TOL * tol, MAX_INNER, Ub, Mb);
      k_bj_apply<<<dim3((unsigned)np, (unsigned)(np + Kp / BM)), 256, 0, st>>>(A, A2, Vp, Kp, nb, r, Ub, Mb);
      std::swap(A, A2);
    }
    VMC_HIP(hipGetLastError());
    ++sweeps;
  }
  if (!std::isfinite(hn[0]) || !std::isfinite(hn[1]))
    throw vmc_error{VMC_ERR_NONFINITE, "eigendecomposition produced non-finite values"};
  k_eig_out<<<grid_for(K * K, 256), 256, 0, st>>>(A, Vp, K, Kp, lam, V);
  VMC_HIP(hipGetLastError());
  return sweeps;
}

extern "C" int vmc_eigh(vmc_ctx* ctx, const double* A, int64_t K, double tol, int max_sweeps, double* evals,
                        double* V, int* sweeps_host) {
  return guard(ctx, [&] {
    VMC_REQUIRE(ctx && A && evals && V, "NULL argument");
    VMC_REQUIRE(K >= 1 && K <= 16384, "K must be in [1, 16384]");
    VMC_REQUIRE(std::isfinite(tol) && tol >= 0.0, "tol must be finite and non-negative");
    VMC_REQUIRE(max_sweeps >= 0, "max_sweeps < 0");
    set_device(ctx);
    phase_scope ps(ctx, "eig");
    ws_reserve(ctx, eig_ws_bytes(K));
    void* w = ws_take(ctx, eig_ws_bytes(K));
    const int s = eig_hermitian(ctx, (const double2*)A, K, tol > 0.0 ? tol : 1e-14, max_sweeps > 0 ? max_sweeps : 50,
                                evals, (double2*)V, w);
    if (sweeps_host) *sweeps_host = s;
  });
}
