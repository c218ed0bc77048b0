// CNN local energies of the TFIM in float32 / bfloat16 on the matrix cores.
//
// Flipping site f changes layer 1 only at the k*k positions p = f - w
// (w in [0,k)^2), by
//   dA[ci][w] = logcosh(z1 + d) - logcosh(z1) = log(1 + (cosh d - 1) + tanh(z1) sinh d),
//   d = -2 sigma_f W1[ci][w],
// and layer 2 only at the (2k-1)^2 positions q = f - e, by
//   dZ[c][e] = sum_{ci} sum_{t + w = e} W2[c][ci][t] dA[ci][w].
// The amplitude ratio is a product over that window (no logarithms needed):
//   psi(s_f) / psi(s) = prod_{c,e} cosh(z2 + dZ) / cosh(z2)
//                     = prod_{c,e} (cosh dZ + tanh(z2) sinh dZ).
// One work-group (8 waves) takes one sample: the forward pass z2 = W2 * a1 is
// a matrix-core product (rows = positions, inner = (t, ci), columns = c), the
// flips are processed 16 at a time, and for each window offset e the dZ of 16
// flips x 16 channels is one matrix-core product with inner index (t, ci) over
// the offsets t valid for e.  Complex products run on real MFMA with two
// accumulators (re += Ar Br + (-Ai) Bi, im += Ar Bi + Ai Br).
//
// Precision: VMC_BF16 feeds bfloat16 operands (a1, W2, dA) to
// v_mfma_f32_16x16x32_bf16; VMC_F32 keeps float32 operands
// (v_mfma_f32_16x16x4_f32).  Both accumulate in float32, evaluate tanh, the
// log1p of dA and the window factors in float32, keep the running product as
// float32 mantissa + integer exponent, and sum the slots in float64.  The
// hidden-layer log cosh is on the principal branch, as in the float64 path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "internal.h"

using namespace dev;

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short ushortx8 __attribute__((ext_vector_type(8)));

constexpr int NT = 1024;  // threads per work-group (four waves per SIMD)
constexpr int NW = NT / 64;
constexpr float PI_F = 3.14159265358979324f;
constexpr float TWO_PI_F = 6.28318530717958648f;

// Geometry and LDS layout (bytes), computed on the host.
struct lp_geom {
  int Lx, Ly, N, W, C, k, kk, win;
  int Cp, Cn, Np;  // C rounded up to 8 / 16; row stride of the [C][N] float tables
  int nrb, ncb;    // row blocks of 16 flips; column blocks of 16 channels
  int sW, sA1, sDA;  // element strides of the operand planes (see the accessors)
  int Lh, nslot;     // row length of the spin halo (Lx + k - 1); tap slots per window offset
  int p1_dc, p1_dp;  // phase 1 stride of NT elements as (channels, positions)
  int p3_drow, p3_dpr;  // dA stride of NT elements as (rows, pairs) of kk * Cp pairs per row
  int o_t1, o_a1i, o_t2, o_wre, o_wim, o_cd, o_sd, o_ure, o_uim, o_pm, o_pe, o_diag, o_pyx, o_wyx, o_eh, o_opt,
      o_sp;
  int a1_plane, da_plane, lds;
};

template <int PREC>
struct lp_t;
template <>
struct lp_t<VMC_BF16> {
  typedef __bf16 T;
};
template <>
struct lp_t<VMC_F32> {
  typedef float T;
};

// Operand layouts.  bfloat16: each lane reads 8 consecutive channels ci, so ci
// is fastest, with 8-element row padding against bank conflicts.  float32:
// each lane reads one element; lanes (li, lk) map to (c or position, ci), laid
// out so that the 64 lanes of a fragment fall in distinct banks.
template <int PREC>
__device__ __forceinline__ int w2_idx(const lp_geom& g, int t, int c, int ci) {
  if constexpr (PREC == VMC_BF16)
    return (t * g.Cn + c) * g.sW + ci;
  else
    return (t * g.Cp + ci) * g.Cn + c;
}
template <int PREC>
__device__ __forceinline__ int a1_idx(const lp_geom& g, int pos, int ci) {
  if constexpr (PREC == VMC_BF16)
    return pos * g.sA1 + ci;
  else
    return ci * g.sA1 + pos;
}
__device__ __forceinline__ int da_idx(const lp_geom& g, int row, int w, int ci) { return row * g.sDA + w * g.Cp + ci; }

// site p shifted by (dy, dx) on the torus; |dy| < Ly, |dx| < Lx
// Fast float32 elementary functions of the flip loops.  Measured in a float32
// emulation (exact log2 and reciprocal assumed): about 4 ulp relative each.

// atan r for r in [0, 1] as r + r z Q(z), z = r^2: Q of degree 7, its
// coefficients fitted to the relative error of the whole polynomial (1.5e-8 in
// exact arithmetic)
__device__ __forceinline__ float atan01(float r) {
  const float z = r * r;
  float q = 2.849890618e-03f;
  q = fmaf(q, z, -1.606863365e-02f);
  q = fmaf(q, z, 4.269152507e-02f);
  q = fmaf(q, z, -7.504294813e-02f);
  q = fmaf(q, z, 1.064093411e-01f);
  q = fmaf(q, z, -1.420364380e-01f);
  q = fmaf(q, z, 1.999261975e-01f);
  q = fmaf(q, z, -3.333307207e-01f);
  return fmaf(q * z, r, r);
}

// atan2 by reduction to the first octant: r = min / max by the hardware
// reciprocal, then pi/2 - a, pi - a and the sign of y
__device__ __forceinline__ float atan2_fast(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
  const float r = mx > 0.f ? mn * __builtin_amdgcn_rcpf(mx) : 0.f;
  float a = atan01(r);
  if (ay > ax) a = 1.57079632679489662f - a;
  if (x < 0.f) a = PI_F - a;
  return copysignf(a, y);
}

// log1p v = log(w) v / (w - 1) with w = 1 + v rounded: the rounding of w
// cancels in the quotient (hardware log2 and reciprocal)
__device__ __forceinline__ float log1p_fast(float v) {
  const float w = 1.f + v, wm = w - 1.f;
  if (wm == 0.f) return v;
  return __builtin_amdgcn_logf(w) * 0.693147180559945309f * (v * __builtin_amdgcn_rcpf(wm));
}

// log(1 + u), complex u
__device__ __forceinline__ float2 fclog1p(float2 u) {
  return make_float2(0.5f * log1p_fast(fmaf(u.x, u.x + 2.f, u.y * u.y)), atan2_fast(u.y, 1.f + u.x));
}

// tanh z = (sinh 2x + i sin 2y) / (cosh 2x + cos 2y) with the hardware
// exponential, reciprocal, sine and cosine (about 2^-21 relative away from the
// poles): y is reduced modulo pi (tanh has period i pi) and x clamped to
// [-10, 10], where tanh x is +-1 to float32 precision.  For the float32 chains,
// whose tanh values feed only acceptance ratios.
__device__ __forceinline__ float2 fctanh_fast(float2 z) {
  const float x = fminf(fmaxf(z.x, -10.f), 10.f);
  const float y = fmaf(-PI_F, rintf(z.y * 0.318309886183790672f), z.y);
  const float e = __expf(2.f * x), ie = __builtin_amdgcn_rcpf(e);
  float sn, cs;
  __sincosf(2.f * y, &sn, &cs);
  const float sh = 0.5f * (e - ie), ch = 0.5f * (e + ie);
  const float inv = __builtin_amdgcn_rcpf(ch + cs);
  return make_float2(sh * inv, sn * inv);
}

// tanh z and the principal log cosh z from one exponential and one sine /
// cosine pair: with w = e^{-2 z'}, z' = +-z and Re z' >= 0,
//   tanh z' = (1 - w) / (1 + w),  log cosh z = z' - log 2 + log(1 + w)
__device__ __forceinline__ void fctanh_logcosh_pv(float2 z, float2& t, float2& a) {
  const bool neg = z.x < 0.f;
  if (neg) z = make_float2(-z.x, -z.y);
  const float e = expf(-2.f * z.x);
  float sn, cs;
  sincosf(-2.f * z.y, &sn, &cs);
  const float er = e * cs, ei = e * sn;
  const float2 r = fcdiv(make_float2(1.f - er, -ei), make_float2(1.f + er, ei));
  t = neg ? make_float2(-r.x, -r.y) : r;
  const float2 l = fclog1p(make_float2(er, ei));
  a = make_float2(z.x - 0.69314718f + l.x, remainderf(z.y + l.y, TWO_PI_F));
}

// cosh dz + tz sinh dz, with the hardware exponential, sine, cosine and
// reciprocal (measured on this chip: exp within 4 ulp on [-4, 4], sin and cos
// within 4.5 x 2^-24 absolute on [-pi, pi], the reciprocal within 1 ulp); in
// float32 Im dz is reduced to [-pi, pi] first (the float32 error bound of a
// factor allows 16 x 2^-24).
template <int PREC>
__device__ __forceinline__ float2 window_factor(float2 dz, float2 tz) {
  const float ea = __expf(dz.x);
  const float y = PREC == VMC_F32 ? fmaf(-TWO_PI_F, rintf(dz.y * 0.159154943091895336f), dz.y) : dz.y;
  // cos y as 1 - 2 sin^2(y / 2): near y = 0, where the window changes lie, the
  // hardware cosine's error is a fraction of an ulp of 1 with a consistent
  // sign, which the product over a window's factors accumulates
  const float sb = __sinf(y), sh2 = __sinf(0.5f * y);
  const float cb = fmaf(-2.f * sh2, sh2, 1.f);
  const float ia = __builtin_amdgcn_rcpf(ea);
  const float ch = 0.5f * (ea + ia), sh = 0.5f * (ea - ia);
  const float2 cz = make_float2(ch * cb, sh * sb), sz = make_float2(sh * cb, ch * sb);
  return fcadd(cz, fcmul(tz, sz));
}

// running product m 2^e; keeps max(|re|, |im|) of m in [0.5, 1)
__device__ __forceinline__ void renorm(float2& m, int& e) {
  int x;
  frexpf(fmaxf(fabsf(m.x), fabsf(m.y)), &x);
  m.x = ldexpf(m.x, -x);
  m.y = ldexpf(m.y, -x);
  e += x;
}

// float32 tables from the float64 parameters:
//   [params (K)] [cosh 2W1 - 1 (n1)] [sinh 2W1 (n1)] [tanh 2W1 (n1)]
__global__ void k_lp_tables(const double2* __restrict__ p, int64_t K, int n1, float2* __restrict__ out) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= K + 3 * (int64_t)n1) return;
  if (e < K) {
    out[e] = make_float2((float)p[e].x, (float)p[e].y);
    return;
  }
  const int j = (int)((e - K) % n1);
  const int which = (int)((e - K) / n1);
  const double a = 2.0 * p[j].x, b = 2.0 * p[j].y;
  double r, i;
  if (which == 1) {  // sinh(a + ib) = sinh a cos b + i cosh a sin b
    r = sinh(a) * cos(b);
    i = cosh(a) * sin(b);
  } else if (which == 0) {  // cosh(a + ib) - 1 = 2 sinh^2((a + ib) / 2)
    const double hr = sinh(0.5 * a) * cos(0.5 * b), hi = cosh(0.5 * a) * sin(0.5 * b);
    r = 2.0 * (hr * hr - hi * hi);
    i = 4.0 * hr * hi;
  } else {
    const double2 th = ctanh(make_double2(a, b));
    r = th.x;
    i = th.y;
  }
  out[e] = make_float2((float)r, (float)i);
}

// site p shifted by (dy, dx), |dy| < Ly, |dx| < Lx, from the (y, x) table of
// the positions (no division)
__device__ __forceinline__ int tpos_t(const lp_geom& g, const int* __restrict__ pyx, int p, int dy, int dx) {
  const int v = pyx[p];
  int y = (v >> 16) + dy, x = (v & 0xffff) + dx;
  y += y < 0 ? g.Ly : (y >= g.Ly ? -g.Ly : 0);
  x += x < 0 ? g.Lx : (x >= g.Lx ? -g.Lx : 0);
  return y * g.Lx + x;
}

// CP: the padded channel count Cp when known at compile time (0: g.Cp).
// Persistent: each work-group builds the sample-independent tables once and
// then takes samples b = blockIdx.x, blockIdx.x + gridDim.x, ...
template <int PREC, int CP>
__global__ __launch_bounds__(NT) void k_cnn_eloc_lp(lp_geom g, const float2* __restrict__ P32,
                                                    const uint64_t* __restrict__ s, int64_t B, double J, double h,
                                                    const int2* __restrict__ bonds, int n_bonds,
                                                    double2* __restrict__ eloc) {
  typedef typename lp_t<PREC>::T T;
  extern __shared__ __align__(16) char smem[];
  float2* t1 = (float2*)(smem + g.o_t1);
  float* a1i = (float*)(smem + g.o_a1i);
  float2* t2 = (float2*)(smem + g.o_t2);
  T* wre = (T*)(smem + g.o_wre);
  T* wim = (T*)(smem + g.o_wim);
  float2* cD = (float2*)(smem + g.o_cd);
  float2* sD = (float2*)(smem + g.o_sd);
  T* ure = (T*)(smem + g.o_ure);  // a1 (forward pass), then dA (flips)
  T* uim = (T*)(smem + g.o_uim);
  float2* pm = (float2*)(smem + g.o_pm);
  int* pe = (int*)(smem + g.o_pe);
  double* sdiag = (double*)(smem + g.o_diag);
  int* pyx = (int*)(smem + g.o_pyx);       // [N] (y << 16) | x
  int* wyx = (int*)(smem + g.o_wyx);       // [kk] (wy << 16) | wx of the layer-1 offsets
  int4* eh = (int4*)(smem + g.o_eh);       // [win^2] (ey, ex, matrix-core steps, taps) of the window offsets
  unsigned* opt = (unsigned*)(smem + g.o_opt);  // [win^2][nslot] (A element << 16) | B element of each tap slot
  float* sp = (float*)(smem + g.o_sp);     // [Ly + k - 1][Lh] spins +-1, periodic halo of k - 1 rows / columns

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int C = g.C, N = g.N, kk = g.kk, k = g.k, Cp = CP ? CP : g.Cp, Lh = g.Lh;
  const int nwin = g.win * g.win;
  static_assert(NW == 16, "window offset 0 is shared by sixteen waves");
  const float2* W1f = P32;
  const float2* b1f = P32 + C * kk;
  const float2* W2f = b1f + C;
  const float2* b2f = W2f + C * C * kk;
  const float2* tabs = b2f + C;

  // ---- set-up: position and offset tables, tap slots, W2 operand planes, cosh / sinh tables
  for (int p = tid; p < N; p += NT) pyx[p] = ((p / g.Lx) << 16) | (p % g.Lx);
  for (int w = tid; w < kk; w += NT) wyx[w] = ((w / k) << 16) | (w % k);
  for (int q = tid; q < nwin * g.nslot; q += NT) {
    const int e = q / g.nslot, ti = q % g.nslot, ey = e / g.win, ex = e % g.win;
    const int ty0 = max(0, ey - k + 1), ty1 = min(k - 1, ey);
    const int tx0 = max(0, ex - k + 1), tx1 = min(k - 1, ex);
    const int ntx = tx1 - tx0 + 1, nt = (ty1 - ty0 + 1) * ntx;
    // slots past the taps read the zero tap kk of the dA rows
    unsigned v = (unsigned)(kk * Cp) << 16;
    if (ti < nt) {
      const int ty = ty0 + ti / ntx, tx = tx0 + ti % ntx;
      const int w = (ey - ty) * k + (ex - tx), t = ty * k + tx;
      v = ((unsigned)(w * Cp) << 16) | (unsigned)(PREC == VMC_BF16 ? t * g.Cn * g.sW : t * Cp * g.Cn);
    }
    opt[q] = v;
    if (ti == 0) eh[e] = make_int4(ey, ex, PREC == VMC_BF16 ? (nt * Cp + 31) / 32 : nt * Cp / 4, nt);
  }
  for (int e = tid; e < kk * g.Cn * Cp; e += NT) {
    const int t = e / (g.Cn * Cp), r = e % (g.Cn * Cp), c = r / Cp, ci = r % Cp;
    const float2 v = (c < C && ci < C) ? W2f[(c * C + ci) * kk + t] : make_float2(0.f, 0.f);
    wre[w2_idx<PREC>(g, t, c, ci)] = (T)v.x;
    wim[w2_idx<PREC>(g, t, c, ci)] = (T)v.y;
  }
  for (int e = tid; e < C * kk; e += NT) {
    cD[e] = tabs[e];
    sD[e] = tabs[C * kk + e];
  }
  __syncthreads();

  const int P1 = kk * Cp;  // (layer-1 offset, channel) pairs of one dA row
  for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
    const uint64_t* sb = s + b * g.W;
    // ---- spins with their periodic halo, and the diagonal element
    for (int q = tid; q < (g.Ly + k - 1) * Lh; q += NT) {
      int y = q / Lh, x = q % Lh;
      y -= y >= g.Ly ? g.Ly : 0;
      x -= x >= g.Lx ? g.Lx : 0;
      const int p = y * g.Lx + x;
      sp[q] = ((sb[p >> 6] >> (p & 63)) & 1ull) ? 1.f : -1.f;
    }
    {
      int n_al = 0;
      for (int q = tid; q < n_bonds; q += NT) {
        const int2 bd = bonds[q];
        n_al += ((sb[bd.x >> 6] >> (bd.x & 63)) & 1ull) == ((sb[bd.y >> 6] >> (bd.y & 63)) & 1ull);
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) n_al += __shfl_xor(n_al, o, 64);
      if (lane == 0) pe[wave] = n_al;
    }
    __syncthreads();
    if (tid == 0) {
      int t = 0;
      for (int w = 0; w < NW; ++w) t += pe[w];
      sdiag[0] = -J * (double)(t - (n_bonds - t));
    }

    // ---- phase 1: layer 1 (tanh, principal log cosh) of every (channel, position)
    {
      int c = tid / N, p = tid % N;
      for (int e = tid; e < Cp * N; e += NT) {
        if (c < C) {
          const int v = pyx[p];
          const float* q = sp + (v >> 16) * Lh + (v & 0xffff);
          const float2* wc = W1f + c * kk;
          float2 z = b1f[c];
          for (int wy = 0; wy < k; ++wy)
            for (int wx = 0; wx < k; ++wx) {
              const float sg = q[wy * Lh + wx];
              const float2 wv = wc[wy * k + wx];
              z.x = fmaf(sg, wv.x, z.x);
              z.y = fmaf(sg, wv.y, z.y);
            }
          float2 tz, a;
          fctanh_logcosh_pv(z, tz, a);
          t1[c * g.Np + p] = tz;
          a1i[c * g.Np + p] = a.y;
          ure[a1_idx<PREC>(g, p, c)] = (T)a.x;
          uim[a1_idx<PREC>(g, p, c)] = (T)a.y;
        } else {
          ure[a1_idx<PREC>(g, p, c)] = (T)0.f;
          uim[a1_idx<PREC>(g, p, c)] = (T)0.f;
        }
        p += g.p1_dp;
        c += g.p1_dc;
        if (p >= N) {
          p -= N;
          ++c;
        }
      }
    }
    __syncthreads();

    // ---- phase 2: z2 = b2 + sum_{t, ci} W2[c][ci][t] a1[ci][p + t] on the matrix cores, t2 = tanh z2
    for (int job = wave; job < g.nrb * g.ncb; job += NW) {
      const int rb = job / g.ncb, cb = job % g.ncb;
      const int prow = rb * 16 + li;  // A row of this lane
      const bool prow_ok = prow < N;
      floatx4 re = {0.f, 0.f, 0.f, 0.f}, im = {0.f, 0.f, 0.f, 0.f};
      if constexpr (PREC == VMC_BF16) {
        const int ng = Cp / 8;
        floatx4 ii = {0.f, 0.f, 0.f, 0.f};  // sum Im a Im w, subtracted from re at the end
        for (int k0 = 0; k0 < kk * Cp; k0 += 32) {
          const int gi = k0 / 8 + lk, t = gi / ng, c8 = (gi % ng) * 8;
          bf16x8 ar{}, ai{}, br{}, bi{};
          if (t < kk) {
            if (prow_ok) {
              const int vw = wyx[t];
              const int pos = tpos_t(g, pyx, prow, vw >> 16, vw & 0xffff);
              ar = *(const bf16x8*)(ure + a1_idx<PREC>(g, pos, c8));
              ai = *(const bf16x8*)(uim + a1_idx<PREC>(g, pos, c8));
            }
            br = *(const bf16x8*)(wre + w2_idx<PREC>(g, t, cb * 16 + li, c8));
            bi = *(const bf16x8*)(wim + w2_idx<PREC>(g, t, cb * 16 + li, c8));
          }
          re = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar, br, re, 0, 0, 0);
          ii = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai, bi, ii, 0, 0, 0);
          im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar, bi, im, 0, 0, 0);
          im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai, br, im, 0, 0, 0);
        }
        re -= ii;
      } else {
        for (int k0 = 0; k0 < kk * Cp; k0 += 4) {
          const int kx = k0 + lk, t = kx / Cp, ci = kx % Cp;  // kk * Cp is a multiple of 8
          float ar = 0.f, ai = 0.f;
          if (prow_ok) {
            const int vw = wyx[t];
            const int pos = tpos_t(g, pyx, prow, vw >> 16, vw & 0xffff);
            ar = ure[a1_idx<PREC>(g, pos, ci)];
            ai = uim[a1_idx<PREC>(g, pos, ci)];
          }
          const float br = wre[w2_idx<PREC>(g, t, cb * 16 + li, ci)], bi = wim[w2_idx<PREC>(g, t, cb * 16 + li, ci)];
          re = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br, re, 0, 0, 0);
          re = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai, bi, re, 0, 0, 0);
          im = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, bi, im, 0, 0, 0);
          im = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, br, im, 0, 0, 0);
        }
      }
      const int c = cb * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int p = rb * 16 + 4 * lk + r;
        if (p < N && c < C) t2[c * g.Np + p] = fctanh(make_float2(re[r] + b2f[c].x, im[r] + b2f[c].y));
      }
    }
    __syncthreads();  // the a1 planes are dead from here on; the same LDS holds dA
    // bfloat16: the zero tap kk of the dA rows (read by the padded tap slots)
    if constexpr (PREC == VMC_BF16)
      for (int q = tid; q < 16 * Cp; q += NT) {
        ure[da_idx(g, q / Cp, kk, q % Cp)] = (T)0.f;
        uim[da_idx(g, q / Cp, kk, q % Cp)] = (T)0.f;
      }

    // ---- phase 3: flips, 16 at a time
    double2 esum = make_double2(0.0, 0.0);  // threads 0..15: sum of the ratios of their row
    for (int rb = 0; rb < g.nrb; ++rb) {
      // dA[row][w][ci] of flips f = rb * 16 + row; thread -> pairs pr = (w, ci), rows row, row + ...
      auto da_elem = [&](int row, int w, int ci, int vw, float2 c1, float2 s1) {
        const int f = rb * 16 + row;
        float2 d = make_float2(0.f, 0.f);
        if (f < N && ci < C) {
          // position f - w on the torus: f - (wy Lx + wx), plus N if fy < wy, plus Lx if fx < wx
          const int vf = pyx[f];
          const int fy = vf >> 16, fx = vf & 0xffff, wy = vw >> 16, wx = vw & 0xffff;
          const int p = f - __mul24(wy, g.Lx) - wx + (fy < wy ? N : 0) + (fx < wx ? g.Lx : 0);
          const float sg = sp[__mul24(fy, Lh) + fx];
          const float2 ts = fcmul(t1[ci * g.Np + p], s1);
          d = fclog1p(make_float2(c1.x - sg * ts.x, c1.y - sg * ts.y));
          // principal branch of the new activation: Im a1' = wrap(Im a1 + Im d)
          const float sum = a1i[ci * g.Np + p] + d.y;
          d.y += sum > PI_F ? -TWO_PI_F : (sum <= -PI_F ? TWO_PI_F : 0.f);
        }
        ure[da_idx(g, row, w, ci)] = (T)d.x;
        uim[da_idx(g, row, w, ci)] = (T)d.y;
      };
      if (g.p3_dpr == 0) {  // kk * Cp divides the group: the thread's pair is fixed
        const int pr = tid % P1, w = pr / Cp, ci = pr % Cp;
        if (tid < g.p3_drow * P1) {
          const int vw = wyx[w];
          const float2 c1 = ci < C ? cD[ci * kk + w] : make_float2(0.f, 0.f);
          const float2 s1 = ci < C ? sD[ci * kk + w] : make_float2(0.f, 0.f);
          for (int row = tid / P1; row < 16; row += g.p3_drow) da_elem(row, w, ci, vw, c1, s1);
        }
      } else {
        for (int q = tid; q < 16 * P1; q += NT) {
          const int row = q / P1, pr = q % P1, w = pr / Cp, ci = pr % Cp;
          const float2 c1 = ci < C ? cD[ci * kk + w] : make_float2(0.f, 0.f);
          const float2 s1 = ci < C ? sD[ci * kk + w] : make_float2(0.f, 0.f);
          da_elem(row, w, ci, wyx[w], c1, s1);
        }
      }
      __syncthreads();
      float2 P[4];
      int E[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        P[r] = make_float2(1.f, 0.f);
        E[r] = 0;
      }
      // (y, x) of this lane's four flips f = rb * 16 + 4 lk + r
      int fy[4], fx[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int v = pyx[min(rb * 16 + 4 * lk + r, N - 1)];
        fy[r] = v >> 16;
        fx[r] = v & 0xffff;
      }
      const T* a_re = ure + li * g.sDA;  // dA row of this lane's A operand (flip rb * 16 + li)
      const T* a_im = uim + li * g.sDA;
      // dZ of window offset e for 16 flips x 16 channels per column block, then the window
      // factors of the lane's rows.  The running products are renormalised after every second
      // factor (two float32 factors cannot overflow unless one exceeds 2^63 in magnitude).
      // Window offset 0 (one tap) is shared: every wave forms its dZ and takes the factors
      // of one row r = wave & 3 in the 16 lanes lk = wave >> 2; offsets 1 .. nwin - 1
      // ((2k - 1)^2 - 1 = 4 k (k - 1): 48 for k = 4) split over the waves, so that no wave
      // waits at the barrier for one extra offset.
      int nf = 0;
      auto window = [&](int e, bool shared) {
        const int4 hd = eh[e];
        const int ey = __builtin_amdgcn_readfirstlane(hd.x), ex = __builtin_amdgcn_readfirstlane(hd.y);
        const int steps = __builtin_amdgcn_readfirstlane(hd.z), nt = __builtin_amdgcn_readfirstlane(hd.w);
        const unsigned* op = opt + e * g.nslot;
        const int eoff = __mul24(ey, g.Lx) + ex;
        for (int cb = 0; cb < g.ncb; ++cb) {
          floatx4 re = {0.f, 0.f, 0.f, 0.f}, im = {0.f, 0.f, 0.f, 0.f};
          if constexpr (PREC == VMC_BF16) {
            const T* b_re = wre + (cb * 16 + li) * g.sW;
            const T* b_im = wim + (cb * 16 + li) * g.sW;
            floatx4 ii;
            // step st: operands of the lane's tap slot and channel group
            auto operands = [&](int st, bf16x8& ar, bf16x8& ai, bf16x8& br, bf16x8& bi) {
              int ti, c8;
              if constexpr (CP == 16) {
                ti = 2 * st + (lk >> 1);
                c8 = (lk & 1) * 8;
              } else {
                const int ng = Cp / 8, gi = 4 * st + lk;
                ti = gi / ng;
                c8 = (gi % ng) * 8;
              }
              const unsigned v = op[ti];
              const int ao = (int)(v >> 16) + c8, bo = (int)(v & 0xffffu) + c8;
              ar = *(const bf16x8*)(a_re + ao);
              ai = *(const bf16x8*)(a_im + ao);
              br = *(const bf16x8*)(b_re + bo);
              bi = *(const bf16x8*)(b_im + bo);
            };
            {  // first step (every window offset has one) with zero accumulators
              bf16x8 ar, ai, br, bi;
              operands(0, ar, ai, br, bi);
              const floatx4 z = {0.f, 0.f, 0.f, 0.f};
              re = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar, br, z, 0, 0, 0);
              ii = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai, bi, z, 0, 0, 0);
              im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar, bi, z, 0, 0, 0);
              im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai, br, im, 0, 0, 0);
            }
            for (int st = 1; st < steps; ++st) {
              bf16x8 ar, ai, br, bi;
              operands(st, ar, ai, br, bi);
              re = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar, br, re, 0, 0, 0);
              ii = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai, bi, ii, 0, 0, 0);
              im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar, bi, im, 0, 0, 0);
              im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai, br, im, 0, 0, 0);
            }
            re -= ii;
          } else {
            // three real products per complex term (Gauss): P = sum Ar Br, Q = sum Ai Bi,
            // R = sum (Ar + Ai)(Br + Bi); Re dZ = P - Q, Im dZ = R - P - Q (the rounding
            // bound of Im at most doubles)
            const T* b_re = wre + cb * 16 + li;
            const T* b_im = wim + cb * 16 + li;
            floatx4 pp = {0.f, 0.f, 0.f, 0.f}, qq = pp, rr = pp;
            for (int ti = 0; ti < nt; ++ti) {
              const unsigned v = op[ti];
              const int ao = (int)(v >> 16), bo = (int)(v & 0xffffu);
#pragma unroll 4
              for (int c4 = 0; c4 < Cp; c4 += 4) {
                const int ci = c4 + lk;
                const float ar = a_re[ao + ci], ai = a_im[ao + ci];
                const float br = b_re[bo + ci * g.Cn], bi = b_im[bo + ci * g.Cn];
                pp = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br, pp, 0, 0, 0);
                qq = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, bi, qq, 0, 0, 0);
                rr = __builtin_amdgcn_mfma_f32_16x16x4f32(ar + ai, br + bi, rr, 0, 0, 0);
              }
            }
            re = pp - qq;
            im = rr - pp - qq;
          }
          // the lane holds dZ of flips rb*16 + 4 lk + r, channel cb*16 + li; position
          // f - e on the torus: f - (ey Lx + ex), plus N if fy < ey, plus Lx if fx < ex
          const int c = cb * 16 + li;
          const bool mine = c < C && (!shared || lk == (wave >> 2));
          if (mine) {
            const int cbase = __mul24(c, g.Np) - eoff;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              if (shared && r != (wave & 3)) continue;
              const int f = rb * 16 + 4 * lk + r;
              if (f >= N) continue;
              const int q = cbase + f + (fy[r] < ey ? N : 0) + (fx[r] < ex ? g.Lx : 0);
              P[r] = fcmul(P[r], window_factor<PREC>(make_float2(re[r], im[r]), t2[q]));
            }
          }
          if (++nf == 2) {
            nf = 0;
#pragma unroll
            for (int r = 0; r < 4; ++r) renorm(P[r], E[r]);
          }
        }
      };
      window(0, true);
      for (int e = 1 + wave; e < nwin; e += NW) window(e, false);
#pragma unroll
      for (int r = 0; r < 4; ++r) renorm(P[r], E[r]);
      // product over the 16 channel lanes of each row: every factor has max(|re|, |im|)
      // in [0.5, 1], so the 16-fold product stays within [2^-16, 2^8] in magnitude
#pragma unroll
      for (int r = 0; r < 4; ++r) {
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
          const float2 q = make_float2(__shfl_xor(P[r].x, o, 64), __shfl_xor(P[r].y, o, 64));
          E[r] += __shfl_xor(E[r], o, 64);
          P[r] = fcmul(P[r], q);
        }
        renorm(P[r], E[r]);
      }
      if (li == 0)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          pm[wave * 16 + 4 * lk + r] = P[r];
          pe[wave * 16 + 4 * lk + r] = E[r];
        }
      __syncthreads();
      if (tid < 16 && rb * 16 + tid < N) {
        double2 m = make_double2(1.0, 0.0);
        int ex = 0;
        for (int w = 0; w < NW; ++w) {
          const float2 q = pm[w * 16 + tid];
          m = cmul(m, make_double2(q.x, q.y));
          ex += pe[w * 16 + tid];
        }
        esum.x += ldexp(m.x, ex);
        esum.y += ldexp(m.y, ex);
      }
    }
    if (wave == 0) {
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        esum.x += __shfl_xor(esum.x, o, 64);
        esum.y += __shfl_xor(esum.y, o, 64);
      }
      if (lane == 0) eloc[b] = make_double2(sdiag[0] - h * esum.x, -h * esum.y);
    }
    __syncthreads();  // pm / pe, the spins and the planes are rewritten by the next sample
  }
}

// ---------------------------------------------------------------------------
// Metropolis chains for the CNN in float32 (single-spin flips, the Philox
// stream of the float64 sampler): one work-group per chain.  The chain keeps
// z1, Im a1 (principal branch), z2 and t2 = tanh z2 of its configuration in
// LDS.  A proposal at site f costs the k*k layer-1 changes dA (as in the
// local-energy kernel, with tanh z1 evaluated on the fly), the window changes
// dZ = W2 * dA by direct sums, and the ratio
//   psi(s_f) / psi(s) = prod_window (cosh dZ + t2 sinh dZ)
// (float32 mantissa, integer exponent).  On acceptance z1 += -2 sigma_f W1 and
// z2 += dZ are updated additively and t2 is re-evaluated from z2, so rounding
// grows only additively; log psi of a recorded sample is re-summed from z2.
// Everything is rebuilt from the bits at the start of every call.
struct mh_geom {
  int Lx, Ly, N, W, C, k, kk, win, nout;
  int o_z1, o_a1i, o_z2, o_t2, o_w2, o_da, o_cd, o_sd, o_red, o_cb, lds;
};

constexpr int MH_NT = 512;
constexpr int MH_MAXOUT = 4;  // window outputs per thread: C (2k-1)^2 <= 2048

__device__ __forceinline__ int mpos(const mh_geom& g, int p, int dy, int dx) {
  int y = p / g.Lx + dy, x = p % g.Lx + dx;
  if (y >= g.Ly) y -= g.Ly;
  if (y < 0) y += g.Ly;
  if (x >= g.Lx) x -= g.Lx;
  if (x < 0) x += g.Lx;
  return y * g.Lx + x;
}

// sum over the block of a double2 (all threads get the total); red holds 2 doubles per wave
__device__ __forceinline__ double2 mh_block_sum(double2 v, double* red) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[3 * wave] = v.x;
    red[3 * wave + 1] = v.y;
  }
  __syncthreads();
  double2 t = make_double2(0.0, 0.0);
  for (int w = 0; w < MH_NT / 64; ++w) {
    t.x += red[3 * w];
    t.y += red[3 * w + 1];
  }
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(MH_NT) void k_cnn_mh_lp(mh_geom g, const float2* __restrict__ P32, int n_chains,
                                                     uint64_t* __restrict__ bits, uint2 key, uint64_t t0, int init,
                                                     int64_t therm_steps, int64_t n_record, int sweep,
                                                     uint64_t* __restrict__ s_out, double2* __restrict__ logpsi_out,
                                                     unsigned long long* __restrict__ acc,
                                                     float2* __restrict__ a1_scratch) {
  extern __shared__ __align__(16) char smem[];
  float2* z1 = (float2*)(smem + g.o_z1);
  float* a1i = (float*)(smem + g.o_a1i);
  float2* z2 = (float2*)(smem + g.o_z2);
  float2* t2 = (float2*)(smem + g.o_t2);
  float2* w2 = (float2*)(smem + g.o_w2);  // [t][ci][c]
  float2* dA = (float2*)(smem + g.o_da);  // [ci][w]
  float2* cD = (float2*)(smem + g.o_cd);
  float2* sD = (float2*)(smem + g.o_sd);
  double* red = (double*)(smem + g.o_red);  // [4 waves][3]
  uint64_t* cb = (uint64_t*)(smem + g.o_cb);
  const int ch = blockIdx.x;
  if (ch >= n_chains) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int C = g.C, N = g.N, kk = g.kk, CN = C * N;
  const float2* W1f = P32;
  const float2* b1f = P32 + C * kk;
  const float2* W2f = b1f + C;
  const float2* b2f = W2f + C * C * kk;
  const float2* tabs = b2f + C;
  float2* a1g = a1_scratch + (int64_t)ch * CN;

  if (init) {
    if (tid == 0)
      for (int w = 0; w < g.W; ++w) {
        const uint4 y = philox(make_uint4((uint32_t)ch, (uint32_t)(w >> 1), 0u, 2u), key);
        uint64_t word = (w & 1) ? ((uint64_t)y.z | ((uint64_t)y.w << 32)) : ((uint64_t)y.x | ((uint64_t)y.y << 32));
        const int rem = N - 64 * w;
        if (rem < 64) word &= (1ull << rem) - 1ull;
        cb[w] = word;
      }
  } else {
    for (int w = tid; w < g.W; w += MH_NT) cb[w] = bits[(int64_t)ch * g.W + w];
  }
  for (int e = tid; e < kk * C * C; e += MH_NT) {
    const int tt = e / (C * C), r = e % (C * C), ci = r / C, c = r % C;
    w2[e] = W2f[(c * C + ci) * kk + tt];
  }
  for (int e = tid; e < C * kk; e += MH_NT) {
    cD[e] = tabs[e];
    sD[e] = tabs[C * kk + e];
  }
  __syncthreads();
  auto sig = [&](int q) { return ((cb[q >> 6] >> (q & 63)) & 1ull) ? 1.f : -1.f; };
  // layer 1 from the bits; a1 goes to global scratch for the layer-2 sums
  for (int e = tid; e < CN; e += MH_NT) {
    const int c = e / N, p = e % N;
    float2 z = b1f[c];
    for (int w = 0; w < kk; ++w) {
      const float s = sig(mpos(g, p, w / g.k, w % g.k));
      const float2 wv = W1f[c * kk + w];
      z.x += s * wv.x;
      z.y += s * wv.y;
    }
    z1[e] = z;
    const float2 a = fclogcosh_pv(z);
    a1i[e] = a.y;
    a1g[e] = a;
  }
  __syncthreads();
  for (int e = tid; e < CN; e += MH_NT) {
    const int c = e / N, p = e % N;
    float2 z = b2f[c];
    for (int ci = 0; ci < C; ++ci)
      for (int w = 0; w < kk; ++w)
        z = fcadd(z, fcmul(w2[(w * C + ci) * C + c], a1g[ci * N + mpos(g, p, w / g.k, w % g.k)]));
    z2[e] = z;
    t2[e] = fctanh(z);
  }
  __syncthreads();

  unsigned long long accepted = 0;
  const int64_t total = therm_steps + n_record * sweep;
  for (int64_t step = 0; step < total; ++step) {
    const uint64_t t = t0 + (uint64_t)step;
    const uint4 x = philox(make_uint4((uint32_t)ch, (uint32_t)t, (uint32_t)(t >> 32), 0u), key);
    const int site = (int)to_index(x.x, (uint32_t)N);
    const double u = to_uniform(x.y, x.z);
    const float sg = sig(site);
    // layer-1 changes at p = site - w
    for (int e = tid; e < C * kk; e += MH_NT) {
      const int ci = e / kk, w = e % kk;
      const int p = mpos(g, site, -(w / g.k), -(w % g.k));
      const float2 ts = fcmul(fctanh(z1[ci * N + p]), sD[e]);
      float2 d = fclog1p(make_float2(cD[e].x - sg * ts.x, cD[e].y - sg * ts.y));
      const float sum = a1i[ci * N + p] + d.y;
      if (sum > PI_F)
        d.y -= TWO_PI_F;
      else if (sum <= -PI_F)
        d.y += TWO_PI_F;
      dA[e] = d;
    }
    __syncthreads();
    // window: dZ, factors, running product
    float2 dzs[MH_MAXOUT];
    float2 P = make_float2(1.f, 0.f);
    int E = 0;
#pragma unroll
    for (int q = 0; q < MH_MAXOUT; ++q) {
      const int o = tid + MH_NT * q;
      dzs[q] = make_float2(0.f, 0.f);
      if (o >= g.nout) continue;
      const int c = o % C, e = o / C, ey = e / g.win, ex = e % g.win;
      float2 dz = make_float2(0.f, 0.f);
      for (int ty = max(0, ey - g.k + 1); ty <= min(g.k - 1, ey); ++ty)
        for (int tx = max(0, ex - g.k + 1); tx <= min(g.k - 1, ex); ++tx) {
          const int tt = ty * g.k + tx, w = (ey - ty) * g.k + (ex - tx);
          const float2* wr = w2 + tt * C * C + c;
          const float2* ar = dA + w;
          int ci = 0;
          // four independent products per round keep several LDS loads in flight
          float2 d1 = make_float2(0.f, 0.f), d2 = d1, d3 = d1;
          for (; ci + 4 <= C; ci += 4) {
            const float2 wa = wr[ci * C], wb = wr[(ci + 1) * C], wc = wr[(ci + 2) * C], wd = wr[(ci + 3) * C];
            const float2 aa = ar[ci * kk], ab = ar[(ci + 1) * kk], ac = ar[(ci + 2) * kk], ad = ar[(ci + 3) * kk];
            dz = fcadd(dz, fcmul(wa, aa));
            d1 = fcadd(d1, fcmul(wb, ab));
            d2 = fcadd(d2, fcmul(wc, ac));
            d3 = fcadd(d3, fcmul(wd, ad));
          }
          for (; ci < C; ++ci) dz = fcadd(dz, fcmul(wr[ci * C], ar[ci * kk]));
          dz = fcadd(fcadd(dz, d1), fcadd(d2, d3));
        }
      dzs[q] = dz;
      P = fcmul(P, window_factor<VMC_F32>(dz, t2[c * N + mpos(g, site, -ey, -ex)]));
      renorm(P, E);
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const float2 pq = make_float2(__shfl_xor(P.x, o, 64), __shfl_xor(P.y, o, 64));
      const int eq = __shfl_xor(E, o, 64);
      P = fcmul(P, pq);
      E += eq;
      renorm(P, E);
    }
    if (lane == 0) {
      red[3 * wave] = P.x;
      red[3 * wave + 1] = P.y;
      red[3 * wave + 2] = (double)E;
    }
    __syncthreads();
    double2 m = make_double2(1.0, 0.0);
    double ex2 = 0.0;
    for (int w = 0; w < MH_NT / 64; ++w) {
      m = cmul(m, make_double2(red[3 * w], red[3 * w + 1]));
      ex2 += red[3 * w + 2];
    }
    const double r = log(m.x * m.x + m.y * m.y) + 2.0 * ex2 * 0.69314718055994530942;
    const bool accept = (r >= 0.0) || (u < exp(r));
    if (accept) {
      ++accepted;
#pragma unroll
      for (int q = 0; q < MH_MAXOUT; ++q) {
        const int o = tid + MH_NT * q;
        if (o >= g.nout) continue;
        const int c = o % C, e = o / C, ey = e / g.win, ex = e % g.win;
        const int qi = c * N + mpos(g, site, -ey, -ex);
        const float2 zn = fcadd(z2[qi], dzs[q]);
        z2[qi] = zn;
        t2[qi] = fctanh(zn);
      }
      for (int e = tid; e < C * kk; e += MH_NT) {
        const int ci = e / kk, w = e % kk;
        const int p = mpos(g, site, -(w / g.k), -(w % g.k));
        const float2 wv = W1f[e];
        z1[ci * N + p] = make_float2(z1[ci * N + p].x - 2.f * sg * wv.x, z1[ci * N + p].y - 2.f * sg * wv.y);
        a1i[ci * N + p] += dA[e].y;
      }
      if (tid == 0) cb[site >> 6] ^= 1ull << (site & 63);
    }
    __syncthreads();
    if (step >= therm_steps && ((step - therm_steps + 1) % sweep) == 0) {
      const int64_t kr = (step - therm_steps + 1) / sweep - 1;
      const int64_t row = kr * n_chains + ch;
      for (int w = tid; w < g.W; w += MH_NT) s_out[row * g.W + w] = cb[w];
      if (logpsi_out) {
        double2 lp = make_double2(0.0, 0.0);
        for (int e = tid; e < CN; e += MH_NT) {
          const float2 l = fclogcosh(z2[e]);
          lp.x += l.x;
          lp.y += l.y;
        }
        lp = mh_block_sum(lp, red);
        if (tid == 0) logpsi_out[row] = lp;
      }
    }
  }
  for (int w = tid; w < g.W; w += MH_NT) bits[(int64_t)ch * g.W + w] = cb[w];
  if (tid == 0) acc[ch] = accepted;
}

mh_geom make_mh_geom(const vmc_model* m) {
  mh_geom g{};
  g.Lx = m->Lx;
  g.Ly = m->Ly;
  g.N = m->N;
  g.W = m->W;
  g.C = m->C;
  g.k = m->k;
  g.kk = m->k * m->k;
  g.win = 2 * m->k - 1;
  g.nout = m->C * g.win * g.win;
  const int CN = g.C * g.N;
  int o = 0;
  auto take = [&](int bytes) {
    const int r = o;
    o = (o + bytes + 15) & ~15;
    return r;
  };
  g.o_z1 = take(8 * CN);
  g.o_a1i = take(4 * CN);
  g.o_z2 = take(8 * CN);
  g.o_t2 = take(8 * CN);
  g.o_w2 = take(8 * g.kk * g.C * g.C);
  g.o_da = take(8 * g.C * g.kk);
  g.o_cd = take(8 * g.C * g.kk);
  g.o_sd = take(8 * g.C * g.kk);
  g.o_red = take(8 * 3 * (MH_NT / 64));
  g.o_cb = take(8 * g.W);
  g.lds = o;
  return g;
}

// ---------------------------------------------------------------------------
// Metropolis chains for the CNN in float32, 16 chains per work-group (the
// Philox stream of the float64 sampler: chain ch proposes the same sites and
// draws the same uniforms).  The chains are the rows of the matrix-core
// products: per step each chain proposes a flip at its own site, the layer-1
// changes dA of the 16 chains form the A operand (rows), W2 the B operand, and
// for every window offset e one float32 product gives dZ of 16 chains x 16
// channels, as in the local-energy kernel.  The per-chain state (z1, Im a1 on
// the principal branch, z2; position-major, channel fastest) lives in global
// memory: 16 chains do not fit in LDS.  tanh z1 and tanh z2 are evaluated where
// they are used; an accepted move stores z1 - 2 sigma W1 and z2 + dZ (float32,
// additive), so rounding grows only additively; log psi of a recorded sample is
// re-summed from z2.  The state is rebuilt from the bits at the start of every
// call.  Used for C <= 16 and k <= 4.
constexpr int MB_NT = 512;  // two waves per SIMD: the window offsets' new z2 stay in registers until the decision
constexpr int MB_NW = MB_NT / 64;
constexpr int MB_CH = 16;    // chains per work-group
constexpr int MB_MAXE = 6;   // window offsets per wave besides the shared offset 0: (2k - 1)^2 - 1 <= 48
constexpr int MB_DA = MB_CH * 256 / MB_NT;  // layer-1 changes per thread: k^2 Cp <= 256

struct mb_geom {
  int Lx, Ly, N, W, C, k, kk, win;
  int Cp, Cn, sDA;  // channels rounded up to 8 / 16; dA row stride (floats)
  int o_wre, o_wim, o_wsum, o_are, o_aim, o_asum, o_cd, o_sd, o_pyx, o_wyx, o_eh, o_opt, o_bits, o_site, o_u, o_sg,
      o_acc, o_pm, o_pe, o_l1, lds;
  // window offsets 1 .. (2k - 1)^2 - 1 of each wave (-1: none), balanced by their taps
  short eslot[MB_NW][MB_MAXE];
};

// KS = Cp / 4: the matrix-core k steps per tap; lane lk takes channels KS lk .. KS lk + KS - 1
template <int KS>
__global__ __launch_bounds__(MB_NT) void k_cnn_mh_batch(mb_geom g, const float2* __restrict__ P32, int n_chains,
                                                        uint64_t* __restrict__ bits, uint2 key, uint64_t t0, int init,
                                                        int64_t therm_steps, int64_t n_record, int sweep,
                                                        uint64_t* __restrict__ s_out, double2* __restrict__ logpsi_out,
                                                        unsigned long long* __restrict__ acc, float2* __restrict__ z1g,
                                                        float* __restrict__ a1ig, float2* __restrict__ z2g,
                                                        float2* __restrict__ a1t) {
  extern __shared__ __align__(16) char smem[];
  float* wre = (float*)(smem + g.o_wre);  // W2 operand planes [t][c][ci]: Re, Im, Re + Im
  float* wim = (float*)(smem + g.o_wim);
  float* wsum = (float*)(smem + g.o_wsum);
  float* are = (float*)(smem + g.o_are);  // dA operand planes [chain][w][ci]: Re, Im, Re + Im
  float* aim = (float*)(smem + g.o_aim);
  float* asum = (float*)(smem + g.o_asum);
  float2* cD = (float2*)(smem + g.o_cd);
  float2* sD = (float2*)(smem + g.o_sd);
  int* pyx = (int*)(smem + g.o_pyx);
  int* wyx = (int*)(smem + g.o_wyx);
  int4* eh = (int4*)(smem + g.o_eh);
  unsigned* opt = (unsigned*)(smem + g.o_opt);
  uint64_t* cb = (uint64_t*)(smem + g.o_bits);  // [MB_CH][W]
  int* site_s = (int*)(smem + g.o_site);
  double* u_s = (double*)(smem + g.o_u);
  float* sg_s = (float*)(smem + g.o_sg);
  int* acc_s = (int*)(smem + g.o_acc);
  float2* pm = (float2*)(smem + g.o_pm);  // [MB_NW][16]
  int* pe = (int*)(smem + g.o_pe);
  int* l1tab = (int*)(smem + g.o_l1);     // [MB_DA][MB_NT]

  static_assert(MB_NW == 8, "window offset 0 is shared by eight waves");
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int C = g.C, N = g.N, kk = g.kk, k = g.k, Cp = g.Cp, Cn = g.Cn, W = g.W;
  const int64_t CN = (int64_t)C * N;
  const int nwin = g.win * g.win;
  const int ch0 = blockIdx.x * MB_CH;
  const int nch = min(MB_CH, n_chains - ch0);
  const float2* W1f = P32;
  const float2* b1f = P32 + C * kk;
  const float2* W2f = b1f + C;
  const float2* b2f = W2f + C * C * kk;
  const float2* tabs = b2f + C;

  // ---- set-up: tables, W2 operand planes, cosh / sinh tables, the bits of the chains
  for (int p = tid; p < N; p += MB_NT) pyx[p] = ((p / g.Lx) << 16) | (p % g.Lx);
  for (int w = tid; w < kk; w += MB_NT) wyx[w] = ((w / k) << 16) | (w % k);
  for (int q = tid; q < nwin * kk; q += MB_NT) {
    const int e = q / kk, ti = q % kk, ey = e / g.win, ex = e % g.win;
    const int ty0 = max(0, ey - k + 1), ty1 = min(k - 1, ey);
    const int tx0 = max(0, ex - k + 1), tx1 = min(k - 1, ex);
    const int ntx = tx1 - tx0 + 1, nt = (ty1 - ty0 + 1) * ntx;
    unsigned v = 0;
    if (ti < nt) {
      const int ty = ty0 + ti / ntx, tx = tx0 + ti % ntx;
      v = ((unsigned)(((ey - ty) * k + (ex - tx)) * Cp) << 16) | (unsigned)((ty * k + tx) * Cn * Cp);
    }
    opt[q] = v;
    if (ti == 0) eh[e] = make_int4(ey, ex, __mul24(ey, g.Lx) + ex, nt);
  }
  for (int e = tid; e < kk * Cn * Cp; e += MB_NT) {
    const int t = e / (Cn * Cp), r = e % (Cn * Cp), c = r / Cp, ci = r % Cp;
    const float2 v = (c < C && ci < C) ? W2f[(c * C + ci) * kk + t] : make_float2(0.f, 0.f);
    wre[e] = v.x;
    wim[e] = v.y;
    wsum[e] = v.x + v.y;
  }
  for (int e = tid; e < C * kk; e += MB_NT) {
    cD[e] = tabs[e];
    sD[e] = tabs[C * kk + e];
  }
  // (chain row, w, ci) of the layer-1 change q = tid + j MB_NT; row 255: none
  for (int q = tid; q < MB_DA * MB_NT; q += MB_NT) {
    const int P1 = kk * Cp, r = q / P1, pr = q % P1;
    l1tab[q] = q < MB_CH * P1 ? (r << 16) | ((pr / Cp) << 8) | (pr % Cp) : (255 << 16);
  }
  for (int q = tid; q < MB_CH * W; q += MB_NT) {
    const int r = q / W, w = q % W;
    uint64_t word = 0;
    if (r < nch) {
      if (init) {
        const uint4 y = philox(make_uint4((uint32_t)(ch0 + r), (uint32_t)(w >> 1), 0u, 2u), key);
        word = (w & 1) ? ((uint64_t)y.z | ((uint64_t)y.w << 32)) : ((uint64_t)y.x | ((uint64_t)y.y << 32));
        const int rem = N - 64 * w;
        if (rem < 64) word &= (1ull << rem) - 1ull;
      } else {
        word = bits[(int64_t)(ch0 + r) * W + w];
      }
    }
    cb[q] = word;
  }
  __syncthreads();

  // ---- the state of the chains from their bits (a1 itself is kept in a1t while z2 is formed)
  for (int r = 0; r < nch; ++r) {
    const int64_t base = (int64_t)(ch0 + r) * CN;
    const uint64_t* br = cb + r * W;
    for (int e = tid; e < (int)CN; e += MB_NT) {
      const int p = e / C, c = e % C;
      const int v = pyx[p], y = v >> 16, x = v & 0xffff;
      float2 z = b1f[c];
      for (int wy = 0; wy < k; ++wy) {
        const int yy = y + wy - (y + wy >= g.Ly ? g.Ly : 0);
        for (int wx = 0; wx < k; ++wx) {
          const int xx = x + wx - (x + wx >= g.Lx ? g.Lx : 0);
          const int q = __mul24(yy, g.Lx) + xx;
          const float sg = ((br[q >> 6] >> (q & 63)) & 1ull) ? 1.f : -1.f;
          const float2 wv = W1f[c * kk + wy * k + wx];
          z.x = fmaf(sg, wv.x, z.x);
          z.y = fmaf(sg, wv.y, z.y);
        }
      }
      float2 tz, a;
      fctanh_logcosh_pv(z, tz, a);
      z1g[base + e] = z;
      a1ig[base + e] = a.y;
      a1t[base + e] = a;
    }
    __syncthreads();
    for (int e = tid; e < (int)CN; e += MB_NT) {
      const int p = e / C, c = e % C;
      const int v = pyx[p], y = v >> 16, x = v & 0xffff;
      float2 z = b2f[c];
      for (int t = 0; t < kk; ++t) {
        const int vw = wyx[t];
        const int yy = y + (vw >> 16) - (y + (vw >> 16) >= g.Ly ? g.Ly : 0);
        const int xx = x + (vw & 0xffff) - (x + (vw & 0xffff) >= g.Lx ? g.Lx : 0);
        const float2* a1p = a1t + base + (int64_t)(__mul24(yy, g.Lx) + xx) * C;
        for (int ci = 0; ci < C; ++ci) z = fcadd(z, fcmul(W2f[(c * C + ci) * kk + t], a1p[ci]));
      }
      z2g[base + e] = z;
    }
    __syncthreads();
  }

  unsigned long long n_acc = 0;  // thread r < nch: accepted moves of chain ch0 + r
  const int64_t total = therm_steps + n_record * sweep;
  // Global-memory phases issue all their loads before any store: loads and
  // stores share one in-order counter, so a load issued after a store would wait
  // for it.
  // element q = tid + j MB_NT of the [chain][w][ci] layer-1 changes: its state index (-1: none)
  auto l1_index = [&](int j, int& r, int& w, int& ci) {
    const int v = l1tab[j * MB_NT + tid];
    r = v >> 16;
    w = (v >> 8) & 0xff;
    ci = v & 0xff;
    if (r >= nch || ci >= C) return -1;
    const int site = site_s[r], vs = pyx[site], vw = wyx[w];
    const int sy = vs >> 16, sx = vs & 0xffff, wy = vw >> 16, wx = vw & 0xffff;
    const int p = site - __mul24(wy, g.Lx) - wx + (sy < wy ? N : 0) + (sx < wx ? g.Lx : 0);
    return (ch0 + r) * (int)CN + p * C + ci;
  };
  // three real products per complex term: with A = sum Re Re', B = sum Im Im',
  // S = sum (Re + Im)(Re' + Im'):  Re dZ = A - B,  Im dZ = S - A - B
  typedef float vks __attribute__((ext_vector_type(KS)));
  const int ak = li * g.sDA + KS * lk, bk = li * Cp + KS * lk;
  auto product = [&](int e, floatx4& re, floatx4& im) {
    const int nt = __builtin_amdgcn_readfirstlane(eh[e].w);
    const unsigned* op = opt + e * kk;
    floatx4 A = {0.f, 0.f, 0.f, 0.f}, Bq = A, S = A;
    for (int ti = 0; ti < nt; ++ti) {
      const unsigned v = op[ti];
      const int ao = ak + (int)(v >> 16), bo = bk + (int)(v & 0xffffu);
      const vks xr = *(const vks*)(are + ao), xi = *(const vks*)(aim + ao), xs = *(const vks*)(asum + ao);
      const vks yr = *(const vks*)(wre + bo), yi = *(const vks*)(wim + bo), ys = *(const vks*)(wsum + bo);
#pragma unroll
      for (int q = 0; q < KS; ++q) {
        A = __builtin_amdgcn_mfma_f32_16x16x4f32(xr[q], yr[q], A, 0, 0, 0);
        Bq = __builtin_amdgcn_mfma_f32_16x16x4f32(xi[q], yi[q], Bq, 0, 0, 0);
        S = __builtin_amdgcn_mfma_f32_16x16x4f32(xs[q], ys[q], S, 0, 0, 0);
      }
    }
    re = A - Bq;
    im = S - A - Bq;
  };
  for (int64_t step = 0; step < total; ++step) {
    const uint64_t t = t0 + (uint64_t)step;
    if (tid < nch) {
      const uint4 x = philox(make_uint4((uint32_t)(ch0 + tid), (uint32_t)t, (uint32_t)(t >> 32), 0u), key);
      const int site = (int)to_index(x.x, (uint32_t)N);
      site_s[tid] = site;
      u_s[tid] = to_uniform(x.y, x.z);
      sg_s[tid] = ((cb[tid * W + (site >> 6)] >> (site & 63)) & 1ull) ? 1.f : -1.f;
    }
    __syncthreads();
    // ---- dA[chain][w][ci] at the layer-1 positions site - w
    {
      float2 zv[MB_DA];
      float av[MB_DA];
#pragma unroll
      for (int j = 0; j < MB_DA; ++j) {
        int r, w, ci;
        const int idx = l1_index(j, r, w, ci);
        zv[j] = idx >= 0 ? z1g[idx] : make_float2(0.f, 0.f);
        av[j] = idx >= 0 ? a1ig[idx] : 0.f;
      }
#pragma unroll
      for (int j = 0; j < MB_DA; ++j) {
        int r, w, ci;
        const int idx = l1_index(j, r, w, ci);
        if (r >= MB_CH) continue;
        float2 d = make_float2(0.f, 0.f);
        if (idx >= 0) {
          const float2 ts = fcmul(fctanh_fast(zv[j]), sD[ci * kk + w]);
          const float2 c1 = cD[ci * kk + w];
          const float sg = sg_s[r];
          d = fclog1p(make_float2(c1.x - sg * ts.x, c1.y - sg * ts.y));
          const float sum = av[j] + d.y;
          d.y += sum > PI_F ? -TWO_PI_F : (sum <= -PI_F ? TWO_PI_F : 0.f);
        }
        are[r * g.sDA + w * Cp + ci] = d.x;
        aim[r * g.sDA + w * Cp + ci] = d.y;
        asum[r * g.sDA + w * Cp + ci] = d.x + d.y;
      }
    }
    __syncthreads();

    // ---- window offsets: dZ of 16 chains x 16 channels, the factors of the lane's chains
    // rows 4 lk + i of the product are chains; the lane's channel is li.  State element of
    // chain row i, channel li, at position site - e (fewer than 2^31 elements per array):
    //   rb[i] - (ey Lx + ex) C + (N C if sy < ey) + (Lx C if sx < ex),  rb[i] = chain CN + site C + li
    // Rows past the group's chains (a partial last group) and padded channels take no part.
    int rb[4], rsy[4], rsx[4];
    unsigned rok = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int site = site_s[4 * lk + i], v = pyx[site];
      rsy[i] = v >> 16;
      rsx[i] = v & 0xffff;
      rb[i] = (ch0 + 4 * lk + i) * (int)CN + __mul24(site, C) + li;
      if (li < C && 4 * lk + i < nch) rok |= 1u << i;
    }
    // offset 0 is shared: this wave takes row i = wave & 3 in the lanes lk >> 1 == wave >> 2
    const unsigned rok0 = (lk >> 1) == (wave >> 2) ? rok & (1u << (wave & 3)) : 0u;
    auto widx = [&](int e, int i) {
      const int4 hd = eh[e];
      const int ey = __builtin_amdgcn_readfirstlane(hd.x), ex = __builtin_amdgcn_readfirstlane(hd.y);
      const int eo = __builtin_amdgcn_readfirstlane(hd.z) * C;
      return rb[i] - eo + (rsy[i] < ey ? N * C : 0) + (rsx[i] < ex ? g.Lx * C : 0);
    };
    auto slot_e = [&](int j) { return j == 0 ? 0 : (int)g.eslot[wave][j - 1]; };
    float2 P[4];
    int E[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      P[i] = make_float2(1.f, 0.f);
      E[i] = 0;
    }
    float2 zn[MB_MAXE + 1][4];  // z2 + dZ of the window positions, stored if the move is accepted
    int nf = 0;
    // slot j: z2 loaded before the product so that the loads overlap it; tanh z2 and the
    // factors use the hardware exponential, sine and reciprocal (they feed only the ratio)
#pragma unroll
    for (int j = 0; j <= MB_MAXE; ++j) {
      const int e = slot_e(j);
      const unsigned ok = e < 0 ? 0u : (j == 0 ? rok0 : rok);
      if (e < 0) continue;
      float2 z2v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) z2v[i] = (ok >> i) & 1u ? z2g[widx(e, i)] : make_float2(0.f, 0.f);
      floatx4 re, im;
      product(e, re, im);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        zn[j][i] = make_float2(z2v[i].x + re[i], z2v[i].y + im[i]);
        const float2 f = window_factor<VMC_BF16>(make_float2(re[i], im[i]), fctanh_fast(z2v[i]));
        P[i] = (ok >> i) & 1u ? fcmul(P[i], f) : P[i];
      }
      if (++nf == 2) {
        nf = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) renorm(P[i], E[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      renorm(P[i], E[i]);
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        const float2 q = make_float2(__shfl_xor(P[i].x, o, 64), __shfl_xor(P[i].y, o, 64));
        E[i] += __shfl_xor(E[i], o, 64);
        P[i] = fcmul(P[i], q);
      }
      renorm(P[i], E[i]);
    }
    if (li == 0)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        pm[wave * 16 + 4 * lk + i] = P[i];
        pe[wave * 16 + 4 * lk + i] = E[i];
      }
    __syncthreads();
    // ---- accept or reject (float64 log ratio)
    if (tid < MB_CH) {
      int a = 0;
      if (tid < nch) {
        double2 m = make_double2(1.0, 0.0);
        int ex = 0;
        for (int w = 0; w < MB_NW; ++w) {
          const float2 q = pm[w * 16 + tid];
          m = cmul(m, make_double2(q.x, q.y));
          ex += pe[w * 16 + tid];
        }
        const double lr = log(m.x * m.x + m.y * m.y) + 2.0 * ex * 0.69314718055994530942;
        a = (lr >= 0.0) || (u_s[tid] < exp(lr));
        if (a) {
          ++n_acc;
          const int site = site_s[tid];
          cb[tid * W + (site >> 6)] ^= 1ull << (site & 63);
        }
      }
      acc_s[tid] = a;
    }
    __syncthreads();
    // ---- accepted moves: z1 -= 2 sigma W1 and Im a1 += Im dA at the layer-1 positions
    // (loads first), z2 + dZ at the window positions (each wave its offsets)
    {
      float2 z1v[MB_DA];
      float av[MB_DA];
#pragma unroll
      for (int j = 0; j < MB_DA; ++j) {
        int r, w, ci;
        int idx = l1_index(j, r, w, ci);
        if (idx >= 0 && !acc_s[r]) idx = -1;
        z1v[j] = idx >= 0 ? z1g[idx] : make_float2(0.f, 0.f);
        av[j] = idx >= 0 ? a1ig[idx] : 0.f;
      }
      unsigned racc = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) racc |= acc_s[4 * lk + i] ? 1u << i : 0u;
#pragma unroll
      for (int j = 0; j <= MB_MAXE; ++j) {
        const int e = slot_e(j);
        if (e < 0) continue;
        const unsigned ok = (j == 0 ? rok0 : rok) & racc;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if ((ok >> i) & 1u) z2g[widx(e, i)] = zn[j][i];
      }
#pragma unroll
      for (int j = 0; j < MB_DA; ++j) {
        int r, w, ci;
        const int idx = l1_index(j, r, w, ci);
        if (idx < 0 || !acc_s[r]) continue;
        const float2 wv = W1f[ci * kk + w];
        const float sg = sg_s[r];
        z1g[idx] = make_float2(z1v[j].x - 2.f * sg * wv.x, z1v[j].y - 2.f * sg * wv.y);
        a1ig[idx] = av[j] + aim[r * g.sDA + w * Cp + ci];
      }
    }
    __syncthreads();
    // ---- record
    if (step >= therm_steps && ((step - therm_steps + 1) % sweep) == 0) {
      const int64_t kr = (step - therm_steps + 1) / sweep - 1;
      for (int q = tid; q < nch * W; q += MB_NT) {
        const int r = q / W, w = q % W;
        s_out[(kr * n_chains + ch0 + r) * W + w] = cb[q];
      }
      if (logpsi_out)
        for (int r = wave; r < nch; r += MB_NW) {
          const int64_t base = (int64_t)(ch0 + r) * CN;
          double2 lp = make_double2(0.0, 0.0);
          for (int64_t e = lane; e < CN; e += 64) {
            const float2 l = fclogcosh(z2g[base + e]);
            lp.x += l.x;
            lp.y += l.y;
          }
          lp = wave_sum(lp);
          if (lane == 0) logpsi_out[kr * n_chains + ch0 + r] = lp;
        }
    }
  }
  for (int q = tid; q < nch * W; q += MB_NT) bits[(int64_t)ch0 * W + q] = cb[q];
  if (tid < nch) acc[ch0 + tid] = n_acc;
}

mb_geom make_mb_geom(const vmc_model* m) {
  mb_geom g{};
  g.Lx = m->Lx;
  g.Ly = m->Ly;
  g.N = m->N;
  g.W = m->W;
  g.C = m->C;
  g.k = m->k;
  g.kk = m->k * m->k;
  g.win = 2 * m->k - 1;
  g.Cp = (m->C + 7) / 8 * 8;
  g.Cn = 16;
  g.sDA = g.kk * g.Cp + 4;
  int o = 0;
  auto take = [&](int bytes) {
    const int r = o;
    o = (o + bytes + 15) & ~15;
    return r;
  };
  g.o_wre = take(4 * g.kk * g.Cp * g.Cn);
  g.o_wim = take(4 * g.kk * g.Cp * g.Cn);
  g.o_wsum = take(4 * g.kk * g.Cp * g.Cn);
  g.o_are = take(4 * MB_CH * g.sDA);
  g.o_aim = take(4 * MB_CH * g.sDA);
  g.o_asum = take(4 * MB_CH * g.sDA);
  g.o_cd = take(8 * g.C * g.kk);
  g.o_sd = take(8 * g.C * g.kk);
  g.o_pyx = take(4 * g.N);
  g.o_wyx = take(4 * g.kk);
  g.o_eh = take(16 * g.win * g.win);
  g.o_opt = take(4 * g.win * g.win * g.kk);
  g.o_bits = take(8 * MB_CH * g.W);
  g.o_site = take(4 * MB_CH);
  g.o_u = take(8 * MB_CH);
  g.o_sg = take(4 * MB_CH);
  g.o_acc = take(4 * MB_CH);
  g.o_pm = take(8 * MB_NW * 16);
  g.o_pe = take(4 * MB_NW * 16);
  g.o_l1 = take(4 * MB_DA * MB_NT);
  g.lds = o;
  // window offsets 1 .. nwin - 1 to the waves, MB_MAXE at most each, by longest
  // processing time on their tap counts (the matrix-core work of an offset)
  for (int w = 0; w < MB_NW; ++w)
    for (int j = 0; j < MB_MAXE; ++j) g.eslot[w][j] = -1;
  std::vector<int> es;
  for (int e = 1; e < g.win * g.win; ++e) es.push_back(e);
  auto taps = [&](int e) {
    const int ey = e / g.win, ex = e % g.win;
    return (std::min(g.k - 1, ey) - std::max(0, ey - g.k + 1) + 1) * (std::min(g.k - 1, ex) - std::max(0, ex - g.k + 1) + 1);
  };
  std::stable_sort(es.begin(), es.end(), [&](int a, int b) { return taps(a) > taps(b); });
  int load[MB_NW] = {}, cnt[MB_NW] = {};
  for (int e : es) {
    int best = -1;
    for (int w = 0; w < MB_NW; ++w)
      if (cnt[w] < MB_MAXE && (best < 0 || load[w] < load[best])) best = w;
    if (best < 0) throw vmc_error{VMC_ERR_UNSUPPORTED, "CNN window too large for the batched sampler"};
    g.eslot[best][cnt[best]++] = (short)e;
    load[best] += taps(e);
  }
  return g;
}

int align16(int x) { return (x + 15) & ~15; }

lp_geom make_geom(const vmc_model* m, int prec) {
  lp_geom g{};
  g.Lx = m->Lx;
  g.Ly = m->Ly;
  g.N = m->N;
  g.W = m->W;
  g.C = m->C;
  g.k = m->k;
  g.kk = m->k * m->k;
  g.win = 2 * m->k - 1;
  g.Cp = (m->C + 7) / 8 * 8;
  g.Cn = (m->C + 15) / 16 * 16;
  g.Np = m->N + 1;
  g.nrb = (m->N + 15) / 16;
  g.ncb = g.Cn / 16;
  g.Lh = m->Lx + m->k - 1;
  const bool bf = prec == VMC_BF16;
  // tap slots per window offset: bfloat16 steps take 32 / Cp taps at a time and
  // may run past the last tap (those slots read the zero tap); float32 does not
  g.nslot = g.kk;
  if (bf) {
    const int ng = g.Cp / 8;
    for (int nt = 1; nt <= g.kk; ++nt) g.nslot = std::max(g.nslot, (4 * ((nt * ng + 3) / 4) - 1) / ng + 1);
  }
  g.p1_dc = NT / g.N;
  g.p1_dp = NT % g.N;
  g.p3_drow = NT / (g.kk * g.Cp);
  g.p3_dpr = NT % (g.kk * g.Cp);
  const int es = bf ? 2 : 4;
  g.sW = bf ? g.Cp + 8 : 0;
  g.sA1 = bf ? g.Cp + 8 : g.N + 16;
  g.sDA = bf ? (g.kk + 1) * g.Cp + 8 : g.kk * g.Cp + 4;  // bfloat16: kk taps and the zero tap
  const int wplane = bf ? g.kk * g.Cn * g.sW : g.kk * g.Cp * g.Cn;
  g.a1_plane = bf ? g.N * g.sA1 : g.Cp * g.sA1;
  g.da_plane = 16 * g.sDA;
  int o = 0;
  auto take = [&](int bytes) {
    const int r = o;
    o = align16(o + bytes);
    return r;
  };
  g.o_t1 = take(8 * g.C * g.Np);
  g.o_a1i = take(4 * g.C * g.Np);
  g.o_t2 = take(8 * g.C * g.Np);
  g.o_wre = take(es * wplane);
  g.o_wim = take(es * wplane);
  g.o_cd = take(8 * g.C * g.kk);
  g.o_sd = take(8 * g.C * g.kk);
  const int uplane = es * std::max(g.a1_plane, g.da_plane);
  g.o_ure = take(uplane);
  g.o_uim = take(uplane);
  g.o_pm = take(8 * NW * 16);
  g.o_pe = take(4 * NW * 16);
  g.o_diag = take(8);
  g.o_pyx = take(4 * g.N);
  g.o_wyx = take(4 * g.kk);
  g.o_eh = take(16 * g.win * g.win);
  g.o_opt = take(4 * g.win * g.win * g.nslot);
  g.o_sp = take(4 * (g.Ly + g.k - 1) * g.Lh);
  g.lds = o;
  // tap slots hold element offsets in 16 bits
  if (g.kk * g.Cp + g.Cp > 65535 || wplane > 65535) g.lds = 1 << 30;
  return g;
}

}  // namespace

void cnn_lowp_local_energy(vmc_model* m, vmc_ham* H, const uint64_t* s, int64_t B, double2* eloc) {
  VMC_REQUIRE(H->kind == HAM_TFIM, "the CNN local energy supports the transverse-field Ising model");
  VMC_REQUIRE(H->Lx == m->Lx && H->Ly == m->Ly, "lattice of the Hamiltonian differs from the CNN's");
  VMC_REQUIRE(m->Lx >= 2 * m->k - 1 && m->Ly >= 2 * m->k - 1,
              "low-precision CNN local energies need Lx, Ly >= 2 kernel - 1");
  const lp_geom g = make_geom(m, m->prec);
  if (g.lds > 160 * 1024)
    throw vmc_error{VMC_ERR_UNSUPPORTED, "CNN too large for the low-precision local-energy kernel (LDS)"};
  vmc_ctx* ctx = m->ctx;
  hipStream_t st = ctx->stream;
  const int n1 = m->C * m->k * m->k;
  const size_t tb = sizeof(float2) * (size_t)(m->K + 3 * n1);
  ws_reserve(ctx, ws_round(tb));
  float2* P32 = (float2*)ws_take(ctx, tb);
  k_lp_tables<<<grid_for(m->K + 3 * n1, 256), 256, 0, st>>>(m->params, m->K, n1, P32);
  auto launch = [&](auto kern) {
    VMC_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, g.lds));
    // persistent work-groups: as many as are resident at once
    int per_cu = 0;
    VMC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, NT, g.lds));
    const int64_t grid = std::min<int64_t>(B, (int64_t)std::max(1, per_cu) * cu_count(ctx));
    if (grid > 0) kern<<<(unsigned)grid, NT, g.lds, st>>>(g, P32, s, B, H->J, H->h, H->bonds, H->n_bonds, eloc);
  };
  if (m->prec == VMC_BF16)
    g.Cp == 16 ? launch(k_cnn_eloc_lp<VMC_BF16, 16>) : launch(k_cnn_eloc_lp<VMC_BF16, 0>);
  else
    g.Cp == 16 ? launch(k_cnn_eloc_lp<VMC_F32, 16>) : launch(k_cnn_eloc_lp<VMC_F32, 0>);
  VMC_HIP(hipGetLastError());
}

void cnn_lowp_sampler_run(vmc_sampler* S, int64_t n_per_chain, uint64_t* s_out, double2* logpsi_out) {
  vmc_model* m = S->model;
  VMC_REQUIRE(S->opts.proposal == VMC_PROP_FLIP, "the CNN sampler uses single-spin flips");
  VMC_REQUIRE(m->Lx >= 2 * m->k - 1 && m->Ly >= 2 * m->k - 1, "the CNN sampler needs Lx, Ly >= 2 kernel - 1");
  vmc_ctx* ctx = m->ctx;
  hipStream_t st = ctx->stream;
  const int n1 = m->C * m->k * m->k;
  const size_t tb = sizeof(float2) * (size_t)(m->K + 3 * n1);
  const int64_t therm = S->thermalized ? 0 : (int64_t)S->opts.therm_sweeps * S->opts.sweep_steps;
  const uint2 key = make_uint2((uint32_t)S->opts.seed, (uint32_t)(S->opts.seed >> 32));
  const int nc = S->opts.n_chains;
  const mb_geom gb = make_mb_geom(m);
  if (m->C <= 16 && m->k <= 4 && gb.lds <= 160 * 1024 && (int64_t)nc * m->C * m->N < ((int64_t)1 << 31)) {
    // 16 chains per work-group, state in global memory
    const size_t cn = (size_t)nc * m->C * m->N;
    const size_t b2 = ws_round(sizeof(float2) * cn), b1 = ws_round(sizeof(float) * cn);
    ws_reserve(ctx, ws_round(tb) + 3 * b2 + b1);
    float2* P32 = (float2*)ws_take(ctx, tb);
    float2* z1 = (float2*)ws_take(ctx, b2);
    float2* z2 = (float2*)ws_take(ctx, b2);
    float2* a1t = (float2*)ws_take(ctx, b2);
    float* a1i = (float*)ws_take(ctx, b1);
    k_lp_tables<<<grid_for(m->K + 3 * n1, 256), 256, 0, st>>>(m->params, m->K, n1, P32);
    auto launch = [&](auto kern) {
      VMC_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, gb.lds));
      kern<<<(nc + MB_CH - 1) / MB_CH, MB_NT, gb.lds, st>>>(gb, P32, nc, S->bits, key, S->t, !S->bits_valid, therm,
                                                            n_per_chain, S->opts.sweep_steps, s_out, logpsi_out, S->acc,
                                                            z1, a1i, z2, a1t);
    };
    gb.Cp == 16 ? launch(k_cnn_mh_batch<4>) : launch(k_cnn_mh_batch<2>);
  } else {
    const mh_geom g = make_mh_geom(m);
    VMC_REQUIRE(g.nout <= MH_MAXOUT * MH_NT, "CNN window too large for the sampler");
    if (g.lds > 160 * 1024)
      throw vmc_error{VMC_ERR_UNSUPPORTED, "CNN too large for the float32 sampler (LDS)"};
    const size_t ab = sizeof(float2) * (size_t)nc * m->C * m->N;
    ws_reserve(ctx, ws_round(tb) + ws_round(ab));
    float2* P32 = (float2*)ws_take(ctx, tb);
    float2* a1 = (float2*)ws_take(ctx, ab);
    k_lp_tables<<<grid_for(m->K + 3 * n1, 256), 256, 0, st>>>(m->params, m->K, n1, P32);
    VMC_HIP(hipFuncSetAttribute((const void*)k_cnn_mh_lp, hipFuncAttributeMaxDynamicSharedMemorySize, g.lds));
    k_cnn_mh_lp<<<nc, MH_NT, g.lds, st>>>(g, P32, nc, S->bits, key, S->t, !S->bits_valid, therm, n_per_chain,
                                          S->opts.sweep_steps, s_out, logpsi_out, S->acc, a1);
  }
  VMC_HIP(hipGetLastError());
  S->t += (uint64_t)(therm + n_per_chain * S->opts.sweep_steps);
  S->thermalized = 1;
  S->bits_valid = 1;
}

