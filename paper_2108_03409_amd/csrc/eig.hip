// Hermitian eigendecomposition on the device (float64), for the pseudo-inverse
// and signal-to-noise regularisations of the TDVP equation (Sec. 3.3: the
// regularised inverse needs S = V diag(lambda) V^dagger).
//
// Parallel cyclic Jacobi: a sweep is Kp - 1 rounds (Kp = K rounded up to even;
// an odd K gets one decoupled zero row and column).  Round r pairs every index
// once (circle ordering: (Kp-1, r) and ((r+i) mod (Kp-1), (r-i) mod (Kp-1))
// for i = 1 .. Kp/2-1).  For a pair (p, q) with A_pp = a, A_qq = b, A_pq =
// |z| e^{i phi}, the unitary
//     J = [[c, s], [-s e, c e]],  e = e^{-i phi},  t = s / c the smaller root of
//     t^2 + 2 tau t - 1 = 0,  tau = (b - a) / (2 |z|),
// zeroes A_pq (A <- J^H A J on rows and columns p, q; V <- V J).  The pairs of a
// round are disjoint, so the update is a set of independent 2 x 2 block
// transforms, one per thread; a round is one launch (every thread derives the
// rotations it needs from the previous round's matrix, so the matrix is
// double-buffered; V is updated in place).  Sweeps stop when the off-diagonal
// Frobenius norm is below tol times the full norm.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.h"

using namespace dev;

namespace {

struct jrot {
  int p, q;
  double c, s;
  double2 e;
  double a_new, b_new;  // diagonal after the rotation
  int active;
};

__device__ __forceinline__ void round_pair(int i, int r, int Kp, int& p, int& q) {
  const int m = Kp - 1;
  if (i == 0) {
    p = m;
    q = r;
  } else {
    p = (r + i) % m;
    q = (r - i + m) % m;
  }
}

__device__ __forceinline__ jrot make_rot(const double2* __restrict__ A, int64_t Kp, int i, int r) {
  int p, q;
  round_pair(i, r, (int)Kp, p, q);
  const double a = A[(int64_t)p * Kp + p].x, b = A[(int64_t)q * Kp + q].x;
  const double2 z = A[(int64_t)p * Kp + q];
  const double az = hypot(z.x, z.y);
  jrot R;
  R.p = p;
  R.q = q;
  // negligible coupling: no rotation (also for the decoupled padding index)
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

// One round in one launch.  Groups with blockIdx.y < ceil(half / 4) update the
// matrix: block (bi, bj) of rows {p_bi, q_bi} x columns {p_bj, q_bj} becomes
// J_bi^H M J_bj, read from Ain and written to Aout (the rotations of a round are
// derived by every thread from Ain, so Ain must not change during the round).
// The remaining groups update V <- V J in place (each thread owns two entries of
// one row).
__global__ __launch_bounds__(256) void k_jacobi_round(const double2* __restrict__ Ain, double2* __restrict__ Aout,
                                                      double2* __restrict__ V, int64_t Kp, int r, int ya) {
  const int64_t half = Kp / 2;
  if ((int)blockIdx.y < ya) {
    const int64_t bj = blockIdx.x * 64ll + (threadIdx.x & 63);
    const int64_t bi = blockIdx.y * 4ll + (threadIdx.x >> 6);
    if (bi >= half || bj >= half) return;
    const jrot Ri = make_rot(Ain, Kp, (int)bi, r), Rj = make_rot(Ain, Kp, (int)bj, r);
    const double2* r0 = Ain + (int64_t)Ri.p * Kp;
    const double2* r1 = Ain + (int64_t)Ri.q * Kp;
    double2* w0 = Aout + (int64_t)Ri.p * Kp;
    double2* w1 = Aout + (int64_t)Ri.q * Kp;
    if (bi == bj) {
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
      return;
    }
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
  } else {
    const int64_t n = blockIdx.x * 64ll + (threadIdx.x & 63);
    const int64_t bj = (blockIdx.y - ya) * 4ll + (threadIdx.x >> 6);
    if (n >= Kp || bj >= half) return;
    const jrot R = make_rot(Ain, Kp, (int)bj, r);
    if (!R.active) return;
    double2* row = V + n * Kp;
    const double2 v0 = row[R.p], v1 = row[R.q];
    const double2 ev1 = cmul(R.e, v1);
    row[R.p] = make_double2(R.c * v0.x - R.s * ev1.x, R.c * v0.y - R.s * ev1.y);
    row[R.q] = make_double2(R.s * v0.x + R.c * ev1.x, R.s * v0.y + R.c * ev1.y);
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

}  // namespace

size_t eig_ws_bytes(int64_t K) {
  const int64_t Kp = K + (K & 1);
  return ws_round(sizeof(double2) * Kp * Kp) * 3 + ws_round(2 * sizeof(double));
}

int eig_hermitian(vmc_ctx* ctx, const double2* S, int64_t K, double tol, int max_sweeps, double* lam, double2* V,
                  void* ws) {
  hipStream_t st = ctx->stream;
  const int64_t Kp = K + (K & 1);
  char* w = (char*)ws;
  double2* A = (double2*)w;
  w += ws_round(sizeof(double2) * Kp * Kp);
  double2* A2 = (double2*)w;
  w += ws_round(sizeof(double2) * Kp * Kp);
  double2* Vp = (double2*)w;
  w += ws_round(sizeof(double2) * Kp * Kp);
  double* nrm = (double*)w;
  k_pad_copy<<<grid_for(Kp * Kp, 256), 256, 0, st>>>(S, K, Kp, A, Vp);
  VMC_HIP(hipGetLastError());
  double* hn = (double*)pinned_host(ctx, 2 * sizeof(double));
  int sweeps = 0;
  if (Kp >= 2) {
    const int64_t half = Kp / 2;
    const int ya = (int)((half + 3) / 4);        // row-pair groups of the matrix update
    const int yv = (int)((half + 3) / 4);        // column-pair groups of the V update
    const unsigned gx = (unsigned)std::max<int64_t>((half + 63) / 64, (Kp + 63) / 64);
    const dim3 g(gx, (unsigned)(ya + yv));
    for (;;) {
      VMC_HIP(hipMemsetAsync(nrm, 0, 2 * sizeof(double), st));
      k_offnorm<<<(unsigned)((Kp + 3) / 4), 256, 0, st>>>(A, Kp, nrm);
      VMC_HIP(hipMemcpyAsync(hn, nrm, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
      VMC_HIP(hipStreamSynchronize(st));
      if (!(hn[0] > tol * tol * hn[1]) || sweeps >= max_sweeps) break;
      for (int r = 0; r < Kp - 1; ++r) {
        k_jacobi_round<<<g, 256, 0, st>>>(A, A2, Vp, Kp, r, ya);
        std::swap(A, A2);
      }
      VMC_HIP(hipGetLastError());
      ++sweeps;
    }
    if (!std::isfinite(hn[0]) || !std::isfinite(hn[1]))
      throw vmc_error{VMC_ERR_NONFINITE, "eigendecomposition produced non-finite values"};
  }
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
