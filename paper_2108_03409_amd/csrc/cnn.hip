// Two-layer periodic CNN (C channels, k x k kernels, log-cosh after both
// layers, sum-pool) on an Lx x Ly torus, float64 path:
//   z1[c,p] = b1_c + sum_t W1[c,t] sigma[p + t],      a1 = logcosh(z1)
//   z2[c,p] = b2_c + sum_{c',t} W2[c,c',t] a1[c',p + t],  log psi = sum logcosh(z2)
// with p + t the periodic shift of position p by tap t = (dy, dx).
//
// Kernels (one 256-thread work-group per sample, activations in LDS):
//   k_cnn_forward  log psi
//   k_cnn_grad     O_k by the chain rule with recomputation of both layers
//                  (no activations are stored between calls)
//   k_cnn_eloc     local energies of the TFIM: for a flip of site s only the
//                  k x k layer-1 positions p with p + t = s change, and only the
//                  (2k-1) x (2k-1) layer-2 positions that read them, so each
//                  connected configuration costs C*C*k^4 complex multiply-adds
//                  instead of a full evaluation (requires Lx, Ly >= 2k - 1;
//                  smaller tori re-evaluate layer 2 in full per slot).
#include <hip/hip_runtime.h>

#include "internal.h"

using namespace dev;

namespace {

struct cnn_geom {
  int Lx, Ly, N, C, k, W;
  const double2* W1;  // [C][k][k]
  const double2* b1;  // [C]
  const double2* W2;  // [C][C][k][k]
  const double2* b2;  // [C]
};

__device__ __forceinline__ int shift_pos(const cnn_geom& g, int p, int dy, int dx) {
  const int y = p / g.Lx, x = p - y * g.Lx;
  int yy = y + dy, xx = x + dx;
  yy %= g.Ly;
  xx %= g.Lx;
  if (yy < 0) yy += g.Ly;
  if (xx < 0) xx += g.Lx;
  return yy * g.Lx + xx;
}

__device__ __forceinline__ double sig_at(const uint64_t* s, int i) { return ((s[i >> 6] >> (i & 63)) & 1ull) ? 1.0 : -1.0; }

__device__ __forceinline__ double2 z1_at(const cnn_geom& g, const uint64_t* s, int c, int p) {
  double2 z = g.b1[c];
  for (int dy = 0; dy < g.k; ++dy)
    for (int dx = 0; dx < g.k; ++dx) {
      const double sg = sig_at(s, shift_pos(g, p, dy, dx));
      const double2 w = g.W1[(c * g.k + dy) * g.k + dx];
      z.x += sg * w.x;
      z.y += sg * w.y;
    }
  return z;
}

// layer 1 into a1[c][p] (LDS), layer 2 value at (c, p) from LDS a1
// sum_ci W2[c][ci][tap] DA[ci][w] for one (c, tap, w): w2 points at W2[c][0][tap],
// da at DA[0][w]; both advance by k*k per input channel.  Four independent
// partial sums keep several loads in flight.
__device__ __forceinline__ double2 window_tap(const double2* __restrict__ w2, const double2* __restrict__ da, int C,
                                              int kk) {
  double2 s0 = make_double2(0.0, 0.0), s1 = s0, s2 = s0, s3 = s0;
  int ci = 0;
  for (; ci + 4 <= C; ci += 4) {
    s0 = cadd(s0, cmul(w2[ci * kk], da[ci * kk]));
    s1 = cadd(s1, cmul(w2[(ci + 1) * kk], da[(ci + 1) * kk]));
    s2 = cadd(s2, cmul(w2[(ci + 2) * kk], da[(ci + 2) * kk]));
    s3 = cadd(s3, cmul(w2[(ci + 3) * kk], da[(ci + 3) * kk]));
  }
  for (; ci < C; ++ci) s0 = cadd(s0, cmul(w2[ci * kk], da[ci * kk]));
  return cadd(cadd(s0, s1), cadd(s2, s3));
}

__device__ __forceinline__ double2 z2_at(const cnn_geom& g, const double2* a1, int c, int p) {
  double2 z = g.b2[c];
  const int kk = g.k * g.k;
  for (int ci = 0; ci < g.C; ++ci)
    for (int dy = 0; dy < g.k; ++dy)
      for (int dx = 0; dx < g.k; ++dx) {
        const double2 w = g.W2[((c * g.C + ci) * g.k + dy) * g.k + dx];
        z = cadd(z, cmul(w, a1[ci * g.N + shift_pos(g, p, dy, dx)]));
      }
  (void)kk;
  return z;
}

__device__ double2 block_sum(double2 v, double2* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double2 t = make_double2(0.0, 0.0);
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t = cadd(t, red[q]);
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(256) void k_cnn_forward(cnn_geom g, const uint64_t* __restrict__ s, int64_t B,
                                                     double2* __restrict__ logpsi) {
  extern __shared__ double2 sm[];
  double2* a1 = sm;                 // [C][N]
  double2* red = sm + g.C * g.N;    // [4]
  const int64_t b = blockIdx.x;
  if (b >= B) return;
  const uint64_t* sb = s + b * g.W;
  const int CN = g.C * g.N;
  for (int e = threadIdx.x; e < CN; e += 256) a1[e] = clogcosh_pv(z1_at(g, sb, e / g.N, e % g.N));
  __syncthreads();
  double2 acc = make_double2(0.0, 0.0);
  for (int e = threadIdx.x; e < CN; e += 256) acc = cadd(acc, clogcosh(z2_at(g, a1, e / g.N, e % g.N)));
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) logpsi[b] = acc;
}

// O_k rows [W1 (C k k), b1 (C), W2 (C C k k), b2 (C)].  LDS: bufA [C][N] (a1, later
// d log psi / d z1), bufB [C][N] (tanh z2).  Work-group x takes samples x,
// x + gridDim.x, ...  With gv == NULL each O_k(s_b) is written to row b of O;
// otherwise (reverse-mode product) the group accumulates g_b conj(O_k(s_b))
// over its samples into row x of part, each entry by the one thread that
// forms it, so no sample's O is stored.
template <typename OutT>
__global__ __launch_bounds__(256) void k_cnn_grad(cnn_geom g, const uint64_t* __restrict__ s, int64_t B, int64_t K,
                                                  OutT* __restrict__ O, const double2* __restrict__ gv,
                                                  double2* __restrict__ part) {
  extern __shared__ double2 sm[];
  const int CN = g.C * g.N, kk = g.k * g.k;
  double2* A = sm;
  double2* G2 = sm + CN;
  for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
  const uint64_t* sb = s + b * g.W;
  OutT* row = gv ? nullptr : O + b * K;
  const bool first = b == (int64_t)blockIdx.x;
  const double2 gb = gv ? gv[b] : make_double2(0.0, 0.0);
  auto put = [&](int64_t k, double2 v) {
    if (gv) {
      const double2 t = cmul(gb, cconj(v));
      double2* q = part + (int64_t)blockIdx.x * K + k;
      *q = first ? t : cadd(*q, t);
    } else if constexpr (sizeof(OutT) == sizeof(double2)) {
      row[k] = v;
    } else {
      row[k] = make_float2((float)v.x, (float)v.y);
    }
  };
  __syncthreads();  // the previous sample's last LDS reads are done
  const int off_b1 = g.C * kk, off_W2 = off_b1 + g.C, off_b2 = off_W2 + g.C * g.C * kk;
  for (int e = threadIdx.x; e < CN; e += 256) A[e] = clogcosh_pv(z1_at(g, sb, e / g.N, e % g.N));
  __syncthreads();
  for (int e = threadIdx.x; e < CN; e += 256) G2[e] = ctanh(z2_at(g, A, e / g.N, e % g.N));
  __syncthreads();
  // dW2[c][c'][t] = sum_p g2[c][p] a1[c'][p + t];  db2[c] = sum_p g2[c][p]
  for (int e = threadIdx.x; e < g.C * g.C * kk; e += 256) {
    const int c = e / (g.C * kk), r = e % (g.C * kk), ci = r / kk, t = r % kk;
    const int dy = t / g.k, dx = t % g.k;
    double2 acc = make_double2(0.0, 0.0);
    for (int p = 0; p < g.N; ++p) acc = cadd(acc, cmul(G2[c * g.N + p], A[ci * g.N + shift_pos(g, p, dy, dx)]));
    put(off_W2 + e, acc);
  }
  for (int c = threadIdx.x; c < g.C; c += 256) {
    double2 acc = make_double2(0.0, 0.0);
    for (int p = 0; p < g.N; ++p) acc = cadd(acc, G2[c * g.N + p]);
    put(off_b2 + c, acc);
  }
  __syncthreads();
  // d log psi / d a1[c'][P] = sum_{c,t} W2[c][c'][t] g2[c][P - t], times tanh(z1) -> A
  for (int e = threadIdx.x; e < CN; e += 256) {
    const int ci = e / g.N, P = e % g.N;
    double2 acc = make_double2(0.0, 0.0);
    for (int c = 0; c < g.C; ++c)
      for (int dy = 0; dy < g.k; ++dy)
        for (int dx = 0; dx < g.k; ++dx)
          acc = cadd(acc, cmul(g.W2[((c * g.C + ci) * g.k + dy) * g.k + dx], G2[c * g.N + shift_pos(g, P, -dy, -dx)]));
    A[e] = acc;  // each thread overwrites only its own entries; a1 is no longer read
  }
  __syncthreads();
  for (int e = threadIdx.x; e < CN; e += 256) A[e] = cmul(A[e], ctanh(z1_at(g, sb, e / g.N, e % g.N)));
  __syncthreads();
  // dW1[c][t] = sum_p g1[c][p] sigma[p + t];  db1[c] = sum_p g1[c][p]
  for (int e = threadIdx.x; e < g.C * kk; e += 256) {
    const int c = e / kk, t = e % kk, dy = t / g.k, dx = t % g.k;
    double2 acc = make_double2(0.0, 0.0);
    for (int p = 0; p < g.N; ++p) acc = cadd(acc, cscale(A[c * g.N + p], sig_at(sb, shift_pos(g, p, dy, dx))));
    put(e, acc);
  }
  for (int c = threadIdx.x; c < g.C; c += 256) {
    double2 acc = make_double2(0.0, 0.0);
    for (int p = 0; p < g.N; ++p) acc = cadd(acc, A[c * g.N + p]);
    put(off_b1 + c, acc);
  }
  }
}

// TFIM local energies.  LDS: z2 [C][N], lc2 = logcosh(z2) [C][N], da1 [C][k*k]
// (the changed layer-1 values of the current flip), sigma words, reduction.
__global__ __launch_bounds__(256) void k_cnn_eloc(cnn_geom g, const uint64_t* __restrict__ s, int64_t B, double J,
                                                  double h, const int2* __restrict__ bonds, int n_bonds,
                                                  double2* __restrict__ eloc, double2* __restrict__ a1_scratch) {
  extern __shared__ double2 sm[];
  const int CN = g.C * g.N, kk = g.k * g.k;
  double2* Z2 = sm;
  double2* LC2 = sm + CN;
  double2* DA = sm + 2 * CN;         // [C][kk]
  double2* red = DA + g.C * kk;      // [4]
  const int64_t b = blockIdx.x;
  if (b >= B) return;
  const uint64_t* sb = s + b * g.W;
  double2* a1 = a1_scratch + b * CN;  // global scratch for the full layer 1 of this sample
  const int tid = threadIdx.x;
  for (int e = tid; e < CN; e += 256) a1[e] = clogcosh_pv(z1_at(g, sb, e / g.N, e % g.N));
  __syncthreads();
  for (int e = tid; e < CN; e += 256) {
    const double2 z = z2_at(g, a1, e / g.N, e % g.N);
    Z2[e] = z;
    LC2[e] = clogcosh(z);
  }
  // diagonal element
  int n_al = 0;
  for (int q = tid; q < n_bonds; q += 256) n_al += sig_at(sb, bonds[q].x) == sig_at(sb, bonds[q].y);
  __syncthreads();
  double2 tot = block_sum(make_double2((double)n_al, 0.0), red);
  const int nal = (int)tot.x;
  const double diag = -J * (double)(nal - (n_bonds - nal));
  double2 acc = make_double2(0.0, 0.0);
  const int win = 2 * g.k - 1;
  const bool incremental = g.Lx >= win && g.Ly >= win;
  if (h != 0.0) {
    for (int site = 0; site < g.N; ++site) {
      const double ds = -2.0 * sig_at(sb, site);
      const int Ys = site / g.Lx, Xs = site % g.Lx;
      // changed layer-1 values: positions p = site - (dy, dx)
      for (int e = tid; e < g.C * kk; e += 256) {
        const int c = e / kk, t = e % kk, dy = t / g.k, dx = t % g.k;
        const int p = shift_pos(g, site, -dy, -dx);
        const double2 z = z1_at(g, sb, c, p);
        const double2 w = g.W1[(c * g.k + dy) * g.k + dx];
        const double2 zn = make_double2(z.x + ds * w.x, z.y + ds * w.y);
        DA[e] = csub(clogcosh_pv(zn), clogcosh_pv(z));
      }
      __syncthreads();
      double2 part = make_double2(0.0, 0.0);
      if (incremental) {
        // affected layer-2 outputs: q = site - (ey, ex), 0 <= ey, ex < 2k - 1
        for (int e = tid; e < g.C * win * win; e += 256) {
          const int c = e / (win * win), r = e % (win * win), ey = r / win, ex = r % win;
          double2 dz = make_double2(0.0, 0.0);
          for (int dy1 = max(0, ey - g.k + 1); dy1 <= min(g.k - 1, ey); ++dy1)
            for (int dx1 = max(0, ex - g.k + 1); dx1 <= min(g.k - 1, ex); ++dx1) {
              const int dy2 = ey - dy1, dx2 = ex - dx1;  // tap from q to the changed position
              dz = cadd(dz, window_tap(g.W2 + (c * g.C * g.k + dy2) * g.k + dx2, DA + dy1 * g.k + dx1, g.C, kk));
            }
          int qy = Ys - ey, qx = Xs - ex;
          if (qy < 0) qy += g.Ly;
          if (qx < 0) qx += g.Lx;
          const int qi = c * g.N + qy * g.Lx + qx;
          part = cadd(part, csub(clogcosh(cadd(Z2[qi], dz)), LC2[qi]));
        }
      } else {
        // small torus: re-evaluate layer 2 from the updated layer 1
        for (int e = tid; e < CN; e += 256) {
          const int c = e / g.N, q = e % g.N;
          double2 dz = make_double2(0.0, 0.0);
          for (int ci = 0; ci < g.C; ++ci)
            for (int dy = 0; dy < g.k; ++dy)
              for (int dx = 0; dx < g.k; ++dx) {
                const int p = shift_pos(g, q, dy, dx);
                // the flip changes a1[ci][p] through every tap that lands on the site
                const double2 zo = z1_at(g, sb, ci, p);
                double2 zn = zo;
                for (int ty = 0; ty < g.k; ++ty)
                  for (int tx = 0; tx < g.k; ++tx)
                    if (shift_pos(g, p, ty, tx) == site) {
                      const double2 w = g.W1[(ci * g.k + ty) * g.k + tx];
                      zn.x += ds * w.x;
                      zn.y += ds * w.y;
                    }
                if (zn.x != zo.x || zn.y != zo.y)
                  dz = cadd(dz, cmul(g.W2[((c * g.C + ci) * g.k + dy) * g.k + dx], csub(clogcosh_pv(zn), a1[ci * g.N + p])));
              }
          part = cadd(part, csub(clogcosh(cadd(Z2[e], dz)), LC2[e]));
        }
      }
      const double2 dl = block_sum(part, red);
      acc = cadd(acc, cscale(cexp(dl), -h));
      __syncthreads();
    }
  }
  if (tid == 0) eloc[b] = make_double2(acc.x + diag, acc.y);
}

// Metropolis chains for the CNN (single-spin flips; the randomness of
// sampler.hip): one work-group per chain, z2 and Re log cosh(z2) of the current
// configuration in LDS, layer 1 of the chain in global scratch.  A proposal
// evaluates Re(log psi(s') - log psi(s)) on the (2k-1) x (2k-1) window only;
// on acceptance the window of z2 is updated in place.
__global__ __launch_bounds__(256) void k_cnn_metropolis(cnn_geom g, int n_chains, uint64_t* __restrict__ bits,
                                                        uint2 key, uint64_t t0, int init, int64_t therm_steps,
                                                        int64_t n_record, int sweep, uint64_t* __restrict__ s_out,
                                                        double2* __restrict__ logpsi_out,
                                                        unsigned long long* __restrict__ acc,
                                                        double2* __restrict__ a1_scratch) {
  extern __shared__ double2 sm[];
  const int CN = g.C * g.N, kk = g.k * g.k, win = 2 * g.k - 1;
  double2* Z2 = sm;                        // [C][N]
  double* RL = (double*)(sm + CN);         // [C][N] Re logcosh(z2)
  double2* DA = sm + CN + (CN + 1) / 2;    // [C][kk]
  double2* red = DA + g.C * kk;            // [4]
  uint64_t* cb = (uint64_t*)(red + 4);     // [W]
  const int c = blockIdx.x;
  if (c >= n_chains) return;
  const int tid = threadIdx.x;
  double2* a1 = a1_scratch + (int64_t)c * CN;
  if (init) {
    if (tid == 0)
      for (int w = 0; w < g.W; ++w) {
        uint4 y = philox(make_uint4((uint32_t)c, (uint32_t)(w >> 1), 0u, 2u), key);
        uint64_t word = (w & 1) ? ((uint64_t)y.z | ((uint64_t)y.w << 32)) : ((uint64_t)y.x | ((uint64_t)y.y << 32));
        const int rem = g.N - 64 * w;
        if (rem < 64) word &= (1ull << rem) - 1ull;
        cb[w] = word;
      }
  } else {
    for (int w = tid; w < g.W; w += 256) cb[w] = bits[(int64_t)c * g.W + w];
  }
  __syncthreads();
  for (int e = tid; e < CN; e += 256) a1[e] = clogcosh_pv(z1_at(g, cb, e / g.N, e % g.N));
  __syncthreads();
  for (int e = tid; e < CN; e += 256) {
    const double2 z = z2_at(g, a1, e / g.N, e % g.N);
    Z2[e] = z;
    RL[e] = clogcosh(z).x;
  }
  __syncthreads();
  unsigned long long accepted = 0;
  const int64_t total = therm_steps + n_record * sweep;
  constexpr int MAXOUT = 8;  // window outputs per thread (C (2k-1)^2 <= 2048)
  for (int64_t step = 0; step < total; ++step) {
    const uint64_t t = t0 + (uint64_t)step;
    const uint4 x = philox(make_uint4((uint32_t)c, (uint32_t)t, (uint32_t)(t >> 32), 0u), key);
    const int site = (int)to_index(x.x, (uint32_t)g.N);
    const double u = to_uniform(x.y, x.z);
    const double ds = -2.0 * sig_at(cb, site);
    const int Ys = site / g.Lx, Xs = site % g.Lx;
    for (int e = tid; e < g.C * kk; e += 256) {
      const int ch = e / kk, tp = e % kk, dy = tp / g.k, dx = tp % g.k;
      const int p = shift_pos(g, site, -dy, -dx);
      const double2 z = z1_at(g, cb, ch, p);
      const double2 w = g.W1[(ch * g.k + dy) * g.k + dx];
      DA[e] = csub(clogcosh_pv(make_double2(z.x + ds * w.x, z.y + ds * w.y)), a1[ch * g.N + p]);
    }
    __syncthreads();
    double2 dzs[MAXOUT];
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < MAXOUT; ++q) {
      const int e = tid + 256 * q;
      dzs[q] = make_double2(0.0, 0.0);
      if (e >= g.C * win * win) continue;
      const int ch = e / (win * win), r = e % (win * win), ey = r / win, ex = r % win;
      double2 dz = make_double2(0.0, 0.0);
      for (int dy1 = max(0, ey - g.k + 1); dy1 <= min(g.k - 1, ey); ++dy1)
        for (int dx1 = max(0, ex - g.k + 1); dx1 <= min(g.k - 1, ex); ++dx1)
          dz = cadd(dz, window_tap(g.W2 + (ch * g.C * g.k + ey - dy1) * g.k + ex - dx1, DA + dy1 * g.k + dx1, g.C, kk));
      dzs[q] = dz;
      int qy = Ys - ey, qx = Xs - ex;
      if (qy < 0) qy += g.Ly;
      if (qx < 0) qx += g.Lx;
      const int qi = ch * g.N + qy * g.Lx + qx;
      part += clogcosh(cadd(Z2[qi], dz)).x - RL[qi];
    }
    const double r = 2.0 * block_sum(make_double2(part, 0.0), red).x;
    const bool accept = (r >= 0.0) || (u < exp(r));
    if (accept) {
      ++accepted;
#pragma unroll
      for (int q = 0; q < MAXOUT; ++q) {
        const int e = tid + 256 * q;
        if (e >= g.C * win * win) continue;
        const int ch = e / (win * win), rr = e % (win * win), ey = rr / win, ex = rr % win;
        int qy = Ys - ey, qx = Xs - ex;
        if (qy < 0) qy += g.Ly;
        if (qx < 0) qx += g.Lx;
        const int qi = ch * g.N + qy * g.Lx + qx;
        const double2 zn = cadd(Z2[qi], dzs[q]);
        Z2[qi] = zn;
        RL[qi] = clogcosh(zn).x;
      }
      for (int e = tid; e < g.C * kk; e += 256) {
        const int ch = e / kk, tp = e % kk, dy = tp / g.k, dx = tp % g.k;
        const int p = shift_pos(g, site, -dy, -dx);
        a1[ch * g.N + p] = cadd(a1[ch * g.N + p], DA[e]);
      }
      __syncthreads();
      if (tid == 0) cb[site >> 6] ^= 1ull << (site & 63);
    }
    __syncthreads();
    if (step >= therm_steps && ((step - therm_steps + 1) % sweep) == 0) {
      const int64_t kr = (step - therm_steps + 1) / sweep - 1;
      const int64_t row = kr * n_chains + c;
      for (int w = tid; w < g.W; w += 256) s_out[row * g.W + w] = cb[w];
      double2 lp = make_double2(0.0, 0.0);
      for (int e = tid; e < CN; e += 256) lp = cadd(lp, clogcosh(Z2[e]));
      lp = block_sum(lp, red);
      if (tid == 0 && logpsi_out) logpsi_out[row] = lp;
    }
  }
  for (int w = tid; w < g.W; w += 256) bits[(int64_t)c * g.W + w] = cb[w];
  if (tid == 0) acc[c] = accepted;
}

constexpr int64_t kChunk = 1 << 14;

cnn_geom geom(const vmc_model* m) {
  cnn_geom g;
  g.Lx = m->Lx;
  g.Ly = m->Ly;
  g.N = m->N;
  g.C = m->C;
  g.k = m->k;
  g.W = m->W;
  const int kk = m->k * m->k;
  g.W1 = m->params;
  g.b1 = m->params + m->C * kk;
  g.W2 = g.b1 + m->C;
  g.b2 = g.W2 + m->C * m->C * kk;
  return g;
}

size_t lds_limit() { return 160 * 1024; }

template <typename Kern>
void allow_lds(Kern k, size_t bytes) {
  VMC_REQUIRE(bytes <= lds_limit(), "CNN too large for the per-sample LDS budget");
  if (bytes > 64 * 1024) VMC_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

}  // namespace

void cnn_log_psi(vmc_model* m, const uint64_t* s, int64_t B, double2* logpsi) {
  const cnn_geom g = geom(m);
  const size_t lds = sizeof(double2) * ((size_t)g.C * g.N + 4);
  allow_lds(k_cnn_forward, lds);
  k_cnn_forward<<<(unsigned)B, 256, lds, m->ctx->stream>>>(g, s, B, logpsi);
  VMC_HIP(hipGetLastError());
}

void cnn_grad(vmc_model* m, const uint64_t* s, int64_t B, void* O, int dtype) {
  const cnn_geom g = geom(m);
  const size_t lds = sizeof(double2) * 2 * (size_t)g.C * g.N;
  if (dtype == VMC_DT_C128) {
    allow_lds(k_cnn_grad<double2>, lds);
    k_cnn_grad<double2><<<(unsigned)B, 256, lds, m->ctx->stream>>>(g, s, B, m->K, (double2*)O, nullptr, nullptr);
  } else {
    allow_lds(k_cnn_grad<float2>, lds);
    k_cnn_grad<float2><<<(unsigned)B, 256, lds, m->ctx->stream>>>(g, s, B, m->K, (float2*)O, nullptr, nullptr);
  }
  VMC_HIP(hipGetLastError());
}

void cnn_vjp_partial(vmc_model* m, const uint64_t* s, int64_t B, const double2* gv, int groups, double2* part) {
  const cnn_geom g = geom(m);
  const size_t lds = sizeof(double2) * 2 * (size_t)g.C * g.N;
  allow_lds(k_cnn_grad<double2>, lds);
  k_cnn_grad<double2><<<(unsigned)groups, 256, lds, m->ctx->stream>>>(g, s, B, m->K, nullptr, gv, part);
  VMC_HIP(hipGetLastError());
}

void cnn_local_energy(vmc_model* m, vmc_ham* H, const uint64_t* s, int64_t B, double2* eloc) {
  VMC_REQUIRE(H->kind == HAM_TFIM, "the CNN local energy supports the transverse-field Ising model");
  VMC_REQUIRE(H->Lx == m->Lx && H->Ly == m->Ly, "lattice of the Hamiltonian differs from the CNN's");
  const cnn_geom g = geom(m);
  const int kk = g.k * g.k;
  const size_t lds = sizeof(double2) * (2 * (size_t)g.C * g.N + (size_t)g.C * kk + 4);
  allow_lds(k_cnn_eloc, lds);
  vmc_ctx* ctx = m->ctx;
  const int64_t chunk = std::min<int64_t>(B, kChunk);
  ws_reserve(ctx, ws_round(sizeof(double2) * chunk * g.C * g.N));
  double2* a1 = (double2*)ws_take(ctx, sizeof(double2) * chunk * g.C * g.N);
  for (int64_t b0 = 0; b0 < B; b0 += chunk) {
    const int64_t nb = std::min(chunk, B - b0);
    k_cnn_eloc<<<(unsigned)nb, 256, lds, ctx->stream>>>(g, s + b0 * g.W, nb, H->J, H->h, H->bonds, H->n_bonds,
                                                        eloc + b0, a1);
    VMC_HIP(hipGetLastError());
  }
}

void cnn_sampler_run(vmc_sampler* S, int64_t n_per_chain, uint64_t* s_out, double2* logpsi_out) {
  vmc_model* m = S->model;
  const cnn_geom g = geom(m);
  VMC_REQUIRE(S->opts.proposal == VMC_PROP_FLIP, "the CNN sampler uses single-spin flips");
  VMC_REQUIRE(g.Lx >= 2 * g.k - 1 && g.Ly >= 2 * g.k - 1, "the CNN sampler needs Lx, Ly >= 2 kernel - 1");
  VMC_REQUIRE(g.C * (2 * g.k - 1) * (2 * g.k - 1) <= 8 * 256, "CNN window too large for the sampler");
  const int CN = g.C * g.N, kk = g.k * g.k;
  const size_t lds = sizeof(double2) * ((size_t)CN + (CN + 1) / 2 + (size_t)g.C * kk + 4) + sizeof(uint64_t) * g.W;
  allow_lds(k_cnn_metropolis, lds);
  vmc_ctx* ctx = S->ctx;
  ws_reserve(ctx, ws_round(sizeof(double2) * (size_t)S->opts.n_chains * CN));
  double2* a1 = (double2*)ws_take(ctx, sizeof(double2) * (size_t)S->opts.n_chains * CN);
  const int64_t therm = S->thermalized ? 0 : (int64_t)S->opts.therm_sweeps * S->opts.sweep_steps;
  const uint2 key = make_uint2((uint32_t)S->opts.seed, (uint32_t)(S->opts.seed >> 32));
  k_cnn_metropolis<<<S->opts.n_chains, 256, lds, ctx->stream>>>(g, S->opts.n_chains, S->bits, key, S->t,
                                                                 !S->bits_valid, therm, n_per_chain,
                                                                 S->opts.sweep_steps, s_out, logpsi_out, S->acc, a1);
  VMC_HIP(hipGetLastError());
  S->t += (uint64_t)(therm + n_per_chain * S->opts.sweep_steps);
  S->thermalized = 1;
  S->bits_valid = 1;
}
