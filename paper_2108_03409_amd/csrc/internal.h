// Internal declarations of libnqsvmc: handle structs, error plumbing, device
// math helpers (complex float64, Philox4x32-10) and kernel launch wrappers.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstring>
#include <exception>
#include <new>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "nqsvmc.h"

// ---------------------------------------------------------------- errors --
struct vmc_error {
  int code;
  std::string msg;
};

// Error string of the calling thread for calls made without a context.
std::string& thread_error();

// Runs f, turning exceptions into status codes and the context's (or the
// thread's) error string; no exception crosses the C ABI.
template <class F>
int guard(vmc_ctx* ctx, F&& f);

#define VMC_HIP(call)                                                           \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess)                                                       \
      throw vmc_error{VMC_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define VMC_REQUIRE(cond, msg)                                                  \
  do {                                                                          \
    if (!(cond)) throw vmc_error{VMC_ERR_INVALID_ARG, msg};                     \
  } while (0)

// ------------------------------------------------------------- workspace --
// Grow-only device arena owned by a context.  Buffers carved from it are
// valid until the next call on the same context.
struct vmc_arena {
  void* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
};

struct vmc_ctx {
  // references: the handle itself plus every model, Hamiltonian, sampler and
  // MADE created from it; the context is freed when the last one is released
  std::atomic<int> refs{1};
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  size_t ws_limit = 0;
  vmc_arena ws;
  // pinned host staging for small readbacks
  void* pinned = nullptr;
  size_t pinned_cap = 0;
  // per-phase event timing
  int timing = 0;
  struct pending_t {
    std::string name;
    hipEvent_t a, b;
  };
  std::vector<pending_t> pending;
  std::map<std::string, std::pair<double, int64_t>> phases;
  std::vector<hipEvent_t> event_pool;
  // second stream (default priority) and two events for work that overlaps
  // the context's stream inside one call; created on first use
  hipStream_t aux = nullptr;
  hipEvent_t ev_main = nullptr, ev_aux = nullptr;
  int n_cu = 0;  // compute units of the device (queried on first use)
};

// The context's auxiliary stream and events (created on first use).
hipStream_t aux_stream(vmc_ctx* ctx);
// Compute units of the context's device.
int cu_count(vmc_ctx* ctx);

template <class F>
int guard(vmc_ctx* ctx, F&& f) {
  try {
    f();
    if (ctx) ctx->err.clear();
    return VMC_OK;
  } catch (vmc_error& e) {
    (ctx ? ctx->err : thread_error()) = e.msg;
    return e.code;
  } catch (std::bad_alloc&) {
    (ctx ? ctx->err : thread_error()) = "host allocation failed";
    return VMC_ERR_OOM;
  } catch (std::exception& e) {
    (ctx ? ctx->err : thread_error()) = e.what();
    return VMC_ERR_INVALID_ARG;
  } catch (...) {
    (ctx ? ctx->err : thread_error()) = "unknown failure";
    return VMC_ERR_INVALID_ARG;
  }
}

void set_device(vmc_ctx* ctx);

// RAII bracket of one timed phase (no-op unless timing is enabled).
struct phase_scope {
  vmc_ctx* ctx;
  size_t idx;
  phase_scope(vmc_ctx* c, const char* name);
  ~phase_scope();
  phase_scope(const phase_scope&) = delete;
  phase_scope& operator=(const phase_scope&) = delete;
};

// Carving: call ws_begin, then ws_take for each buffer (256-byte aligned).
void ctx_retain(vmc_ctx* ctx);
void ctx_release(vmc_ctx* ctx);
void ws_reserve(vmc_ctx* ctx, size_t bytes);
void* ws_take(vmc_ctx* ctx, size_t bytes);
inline size_t ws_round(size_t b) { return (b + 255) & ~size_t(255); }
void* pinned_host(vmc_ctx* ctx, size_t bytes);

// ---------------------------------------------------------------- models --
enum { MODEL_RBM = 0, MODEL_CNN = 1, MODEL_AR = 2, MODEL_TABLE = 3, MODEL_SYMELU = 4 };

struct vmc_ham;
struct vmc_made;

// Per (model, move set) tables of the RBM ratio identity (see rbm.hip).
struct rbm_move_tables {
  int move_kind = -1;  // 0 = site flips, 1 = bond exchanges
  int n_moves = 0;
  uint64_t param_version = 0;
  uint64_t ham_uid = 0;     // Hamiltonian the exchange tables were built for
  double2* T = nullptr;    // [N_h][n_moves] tanh(2 D_jm)
  double2* D = nullptr;    // [N_h][n_moves] D_jm
  double2* LC = nullptr;   // [n_moves] sum_j logcosh(2 D_jm)
  double2* alpha = nullptr;  // [n_moves] visible-bias difference
  double2* Tt = nullptr;     // [n_moves][N_h] T transposed (sampler: lanes over hidden units)
  double2* Dt = nullptr;     // [n_moves][N_h] D transposed
};

struct vmc_model {
  vmc_ctx* ctx = nullptr;
  int kind = MODEL_RBM;
  int N = 0;          // sites
  int W = 1;          // words per configuration
  int Nh = 0;         // RBM hidden units
  int is_complex = 1;
  int Lx = 0, Ly = 0, C = 0, k = 0;  // CNN geometry
  int64_t K = 0;
  int prec = VMC_F64;
  uint64_t version = 1;     // bumped on every set_params
  double2* params = nullptr;  // K complex float64 master copy (device)
  double2* Wt = nullptr;      // RBM: W transposed [N][N_h]
  rbm_move_tables tab[2];     // flip / exchange tables
  // float32 / bfloat16 evaluation (RBM): parameters rounded to the precision,
  // stored as float32; rebuilt when the parameters or the precision change
  uint64_t lowp_version = 0;
  int lowp_prec = -1;
  float2* Wt32 = nullptr;   // [N][N_h]
  float2* ab32 = nullptr;   // [N + N_h]: a then b
  struct lowp_tables {
    uint64_t version = 0;
    int prec = -1, n_moves = 0;
    uint64_t ham_uid = 0;
    float2 *T = nullptr, *LC = nullptr, *alpha = nullptr;
  } tab32[2];
  // autoregressive state (psi = sqrt(q) of a masked network with Nh hidden units):
  // the network's dense masked parameters, the compact-to-dense index pairs and
  // W2 * M2 transposed (Nh x N)
  vmc_made* made = nullptr;
  int2* ar_idx = nullptr;
  double* ar_w2t = nullptr;
  int64_t ar_r1 = 0, ar_r2 = 0, ar_r3 = 0;  // ends of the W1, b1 and W2 blocks of the compact vector
};

// ----------------------------------------------------------- Hamiltonians --
enum { HAM_TFIM = 0, HAM_HEIS = 1 };

struct vmc_ham {
  vmc_ctx* ctx = nullptr;
  uint64_t uid = 0;  // unique per Hamiltonian created in this process (table cache key)
  int kind = HAM_TFIM;
  int Lx = 0, Ly = 1, periodic = 1;
  int N = 0, W = 1;
  double J = 0.0, h = 0.0;
  int n_bonds = 0;
  std::vector<int2> bonds_host;
  int2* bonds = nullptr;  // device copy
  int M_max = 1;
};

struct vmc_made;

struct vmc_sampler {
  vmc_ctx* ctx = nullptr;
  vmc_model* model = nullptr;
  vmc_ham* ham = nullptr;
  vmc_sampler_opts opts{};
  int N = 0, W = 1;
  uint64_t t = 0;            // proposals made per chain so far
  int thermalized = 0;
  int bits_valid = 0;         // chain configurations drawn or restored
  uint64_t* bits = nullptr;  // [n_chains][W] chain configurations (device)
  // [3][n_chains]: accepted proposals, accepted global proposals, global proposals (last call)
  unsigned long long* acc = nullptr;
  double last_accept = 0.0, last_global_accept = 0.0;
  int64_t last_n_global = 0;
  // frozen MADE proposal (VMC_PROP_MADE_MIX): [W1m^T (N x H) | W2m (N x H) | b1 (H) | b2 (N)]
  int made_H = 0;
  double* made_buf = nullptr;
  int* mix_perm = nullptr;            // [H] units sorted by degree, then [N + 1] first position per degree
  uint64_t g = 0;                     // global proposals per chain so far
  // The proposals of a global step do not depend on the chains: those of step
  // g + 1 are formed on a second stream while the main stream runs the sweep
  // after step g.  Two buffers b = g & 1 of proposals, their log q and theta.
  uint64_t* mix_prop = nullptr;       // [2][n_chains][W] proposals
  double* mix_lq = nullptr;           // [3][n_chains] log q of the chain states, then of the proposals of buffers 0, 1
  double2* mix_theta = nullptr;       // [n_chains][N_h] theta of the chain states between launches
  double2* mix_theta_prop = nullptr;  // [2][n_chains][N_h] theta of the proposals
  double* mix_tf = nullptr;           // teacher forcing of the chain states: A [n_chains][H], L [n_chains][N]
  hipStream_t mix_side = nullptr;     // the proposals' stream (default priority)
  hipEvent_t mix_ev_main = nullptr;   // main stream past the last acceptance
  hipEvent_t mix_ev_prop[2] = {nullptr, nullptr};  // proposals of buffer b formed
  uint64_t mix_pg[2] = {~0ull, ~0ull};             // global step whose proposals buffer b holds (~0: none)
  uint64_t mix_pver[2] = {0, 0};                   // RBM parameter version of buffer b's theta
  int mix_side_buf = -1;                           // buffer last formed on the proposals' stream (-1: none pending)
};

struct vmc_made {
  vmc_ctx* ctx = nullptr;
  int N = 0, H = 0, W = 1;
  int64_t P = 0;
  double* params = nullptr;  // device float64 master
  double* adam_m = nullptr;
  double* adam_v = nullptr;
  int64_t adam_t = 0;
  double* W1m = nullptr;   // masked W1 (H x N)
  double* W1mT = nullptr;  // its transpose (N x H)
  double* W2m = nullptr;   // masked W2 (N x H)
};

// ------------------------------------------------------- device helpers --
namespace dev {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  // Smith's algorithm
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, d = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  } else {
    double r = b.x / b.y, d = b.x * r + b.y;
    return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
  }
}
__device__ __forceinline__ double2 cexp(double2 z) {
  double e = exp(z.x), s, c;
  sincos(z.y, &s, &c);
  return make_double2(e * c, e * s);
}
__device__ __forceinline__ double2 clog(double2 z) {
  return make_double2(log(hypot(z.x, z.y)), atan2(z.y, z.x));
}

// log cosh z without overflow: with z~ = +-z such that Re z~ >= 0,
//   log cosh z = z~ - ln 2 + log(1 + e^{-2 z~})   (mod 2 pi i).
__device__ __forceinline__ double2 clogcosh(double2 z) {
  if (z.x < 0.0) z = make_double2(-z.x, -z.y);
  double e = exp(-2.0 * z.x), s, c;
  sincos(-2.0 * z.y, &s, &c);
  double er = e * c, ei = e * s;  // e^{-2 z~}
  // log|1 + w| = 0.5 log1p(2 Re w + |w|^2)
  double lr = 0.5 * log1p(2.0 * er + er * er + ei * ei);
  double li = atan2(ei, 1.0 + er);
  return make_double2(z.x - 0.69314718055994530942 + lr, z.y + li);
}

// log cosh z on the principal branch of the logarithm (imaginary part in
// [-pi, pi]); a hidden layer's activation feeds a further linear layer, where
// a shift by 2 pi i would change the result.
__device__ __forceinline__ double2 clogcosh_pv(double2 z) {
  double2 r = clogcosh(z);
  r.y = remainder(r.y, 6.283185307179586477);
  return r;
}

// tanh z = (1 - e^{-2z})/(1 + e^{-2z}) for Re z >= 0; odd in z.
__device__ __forceinline__ double2 ctanh(double2 z) {
  bool neg = z.x < 0.0;
  if (neg) z = make_double2(-z.x, -z.y);
  double e = exp(-2.0 * z.x), s, c;
  sincos(-2.0 * z.y, &s, &c);
  double2 w = make_double2(e * c, e * s);
  double2 r = cdiv(make_double2(1.0 - w.x, -w.y), make_double2(1.0 + w.x, w.y));
  return neg ? make_double2(-r.x, -r.y) : r;
}

// float32 complex helpers (low-precision network evaluation)
__device__ __forceinline__ float2 fcadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 fcmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 fcdiv(float2 a, float2 b) {
  if (fabsf(b.x) >= fabsf(b.y)) {
    float r = b.y / b.x, d = b.x + b.y * r;
    return make_float2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  } else {
    float r = b.x / b.y, d = b.x * r + b.y;
    return make_float2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
  }
}
__device__ __forceinline__ float2 fclog(float2 z) { return make_float2(logf(hypotf(z.x, z.y)), atan2f(z.y, z.x)); }
__device__ __forceinline__ float2 fcexp(float2 z) {
  float e = expf(z.x), s, c;
  sincosf(z.y, &s, &c);
  return make_float2(e * c, e * s);
}
__device__ __forceinline__ float2 fclogcosh(float2 z) {
  if (z.x < 0.f) z = make_float2(-z.x, -z.y);
  float e = expf(-2.f * z.x), s, c;
  sincosf(-2.f * z.y, &s, &c);
  float er = e * c, ei = e * s;
  float lr = 0.5f * log1pf(2.f * er + er * er + ei * ei);
  float li = atan2f(ei, 1.f + er);
  return make_float2(z.x - 0.69314718f + lr, z.y + li);
}
__device__ __forceinline__ float2 fclogcosh_pv(float2 z) {
  float2 r = fclogcosh(z);
  r.y = remainderf(r.y, 6.28318530717958648f);
  return r;
}
__device__ __forceinline__ float2 fctanh(float2 z) {
  bool neg = z.x < 0.f;
  if (neg) z = make_float2(-z.x, -z.y);
  float e = expf(-2.f * z.x), s, c;
  sincosf(-2.f * z.y, &s, &c);
  float2 w = make_float2(e * c, e * s);
  float2 r = fcdiv(make_float2(1.f - w.x, -w.y), make_float2(1.f + w.x, w.y));
  return neg ? make_float2(-r.x, -r.y) : r;
}
// round-to-nearest-even float32 -> bfloat16 -> float32
__device__ __forceinline__ float bf16_round(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return x;
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
__device__ __forceinline__ uint4 philox(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k.x += 0x9E3779B9u;
      k.y += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k.x, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k.y,
                   (uint32_t)p0);
  }
  return c;
}
__device__ __forceinline__ uint32_t to_index(uint32_t x, uint32_t n) {
  return (uint32_t)(((uint64_t)x * n) >> 32);
}
__device__ __forceinline__ double to_uniform(uint32_t x1, uint32_t x2) {
  uint64_t m = ((uint64_t)x1 << 21) | (x2 >> 11);
  return (double)m * 0x1.0p-53;
}

__device__ __forceinline__ int get_bit(const uint64_t* w, int i) { return (int)((w[i >> 6] >> (i & 63)) & 1ull); }

// Wave-wide (64-lane) reductions.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double2 wave_sum(double2 v) {
  v.x = wave_sum(v.x);
  v.y = wave_sum(v.y);
  return v;
}

// Cross-lane sums without an LDS round trip, for reductions on the dependent
// path of a sequential loop: DPP moves inside each row of 16 lanes, then
// v_readlane across the four rows.  Every lane of the wavefront must be active.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xf, 0xf, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// Sum over each row of 16 lanes (lanes 16 r .. 16 r + 15), the same bits in
// all 16: partner lanes add the same two values, and addition commutes.
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]: lane ^ 1
  v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]: lane ^ 2
  v += dpp_f64<0x141>(v);  // row_half_mirror: the two quads of each half row
  v += dpp_f64<0x140>(v);  // row_mirror: the two halves of the row
  return v;
}
// Sum over the wavefront, returned wave-uniform to every lane.
__device__ __forceinline__ double wave_sum_uniform(double v) {
  v = row16_sum(v);
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}
// Product over the wavefront, wave-uniform (multiplication commutes as well).
__device__ __forceinline__ double wave_prod_uniform(double v) {
  v *= dpp_f64<0xB1>(v);
  v *= dpp_f64<0x4E>(v);
  v *= dpp_f64<0x141>(v);
  v *= dpp_f64<0x140>(v);
  return (readlane_f64(v, 0) * readlane_f64(v, 16)) * (readlane_f64(v, 32) * readlane_f64(v, 48));
}
__device__ __forceinline__ int wave_isum_uniform(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xf, 0xf, false);
  return (__builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16)) +
         (__builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48));
}

}  // namespace dev

// -------------------------------------------------- cross-file launchers --
// rbm.hip
void rbm_theta(vmc_model* m, const uint64_t* s, int64_t B, double2* theta, hipStream_t st = nullptr);
void rbm_ensure_tables(vmc_model* m, const vmc_ham* H, int move_kind);
void rbm_log_psi(vmc_model* m, const uint64_t* s, int64_t B, double2* logpsi);
void rbm_local_energy(vmc_model* m, vmc_ham* H, const uint64_t* s, int64_t B, double2* eloc);
void rbm_grad(vmc_model* m, const uint64_t* s, int64_t B, void* O, int dtype);
// cnn.hip
void cnn_log_psi(vmc_model* m, const uint64_t* s, int64_t B, double2* logpsi);
void cnn_grad(vmc_model* m, const uint64_t* s, int64_t B, void* O, int dtype);
void cnn_vjp_partial(vmc_model* m, const uint64_t* s, int64_t B, const double2* gv, int groups, double2* part);
void cnn_local_energy(vmc_model* m, vmc_ham* H, const uint64_t* s, int64_t B, double2* eloc);
void cnn_lowp_local_energy(vmc_model* m, vmc_ham* H, const uint64_t* s, int64_t B, double2* eloc);
void cnn_sampler_run(vmc_sampler* S, int64_t n_per_chain, uint64_t* s_out, double2* logpsi_out);
void cnn_lowp_sampler_run(vmc_sampler* S, int64_t n_per_chain, uint64_t* s_out, double2* logpsi_out);
// symelu.hip (translation-symmetric ELU network; C holds alpha)
void symelu_check(const vmc_model* m);
void symelu_log_psi(vmc_model* m, const uint64_t* s, int64_t B, double2* out);
void symelu_local_energy(vmc_model* m, vmc_ham* H, const uint64_t* s, int64_t B, double2* eloc);
void symelu_grad(vmc_model* m, const uint64_t* s, int64_t B, void* O, int dtype);
void symelu_sampler_run(vmc_sampler* S, int64_t n_per_chain, uint64_t* s_out, double2* logpsi_out);
// table.hip (tabulated log-amplitudes, test model)
void table_log_psi(vmc_model* m, const uint64_t* s, int64_t B, double2* out);
void table_local_energy(vmc_model* m, vmc_ham* H, const uint64_t* s, int64_t B, double2* eloc);
void table_grad(vmc_model* m, const uint64_t* s, int64_t B, void* O, int dtype);
void table_sampler_run(vmc_sampler* S, int64_t n_per_chain, uint64_t* s_out, double2* logpsi_out);
// arnqs.hip (autoregressive state)
void ar_init(vmc_model* m);
void ar_free(vmc_model* m);
void ar_set_params(vmc_model* m);
void ar_log_psi(vmc_model* m, const uint64_t* s, int64_t B, double2* out);
void ar_local_energy(vmc_model* m, vmc_ham* H, const uint64_t* s, int64_t B, double2* eloc);
void ar_grad(vmc_model* m, const uint64_t* s, int64_t B, void* O, int dtype);
void ar_sample(vmc_sampler* S, int64_t B, uint64_t* s_out, double2* logpsi_out);
// made.hip
void made_refresh(vmc_made* md);
void made_sample_impl(vmc_made* md, int64_t B, uint64_t seed, uint64_t counter, uint64_t* s_out, double* logq);
// vjp.hip
void log_psi_vjp_impl(vmc_model* m, const uint64_t* s, int64_t B, const double2* g, double2* out);
void log_psi_vjp_noalloc_impl(vmc_model* m, const uint64_t* s, int64_t B, const double2* g, double2* out);
// rbm_lowp.hip
void rbm_lowp_log_psi(vmc_model* m, const uint64_t* s, int64_t B, double2* logpsi);
void rbm_lowp_local_energy(vmc_model* m, vmc_ham* H, const uint64_t* s, int64_t B, double2* eloc);
void rbm_lowp_free(vmc_model* m);
// sampler.hip
void sampler_run(vmc_sampler* S, int64_t n_per_chain, uint64_t* s_out, double2* logpsi_out);
void mix_ensure(vmc_sampler* S);
// mixsampler.hip
void mix_made_layout(int N, int H, std::vector<int>& perm, std::vector<int>& mstart);
bool mix_made_fits(int H, int W);
void mix_global_step(vmc_sampler* S, uint64_t g);
void mix_release(vmc_sampler* S);
void mix_wait_side(vmc_sampler* S);  // orders later main-stream work after the proposals formed ahead  // waits for the proposals' stream, frees the global-step buffers
// gemm64.hip: C = beta C + op(A) op(B) in float64 with arbitrary strides
struct dgemm_args {
  const double* A;
  int64_t sam, sak;
  const double* B;
  int64_t sbk, sbn;
  double* C;
  int64_t ldc;
  int64_t M, N, K;
  double beta;
  int64_t kchunk = 0;  // split-K: grid z takes rows [z kchunk, (z + 1) kchunk) of the reduction (0: all)
  int64_t cz = 0;      // ... and writes C + z cz
};
void dgemm(vmc_ctx* ctx, const dgemm_args& g, int nsplit = 1);
// herk.hip
size_t herk_ws_bytes(int64_t N, int64_t K, int mode);
void herk_mfma_f32(vmc_ctx* ctx, const float2* X, int64_t N, int64_t K, int mode, double nu, double eps, double2* S,
                   double2* diag, void* ws);
// chol.hip
size_t chol_linv_bytes(int64_t K);
int chol_block();
void chol_factor(vmc_ctx* ctx, double2* S, int64_t K, double2* Linv, long long* fail, double* pivmin);
size_t chol_sync_bytes(int64_t K);
int chol_sync_err_index(int64_t K);
void chol_solve(vmc_ctx* ctx, const double2* S, int64_t K, const double2* Linv, const double2* rhs, double2* y,
                double2* x, int* sync);
// herk16.hip
size_t herk16_ws_bytes(int64_t N, int64_t K);
void herk_split16(vmc_ctx* ctx, const float2* X, int64_t N, int64_t K, int mode, double nu, double eps, double2* S,
                  double2* diag, void* ws);
// sr.hip
void sr_solve_impl(vmc_ctx* ctx, const void* O, int dtype, const double2* eloc, const double* w, int64_t N,
                   int64_t K, const vmc_sr_opts* o, double2* x, vmc_sr_info* info, const vmc_eig_opts* eo,
                   double* evals, double* snr, int* sweeps, double2* S_out = nullptr, double2* F_out = nullptr);
double fisher_quad_impl(vmc_ctx* ctx, const void* O, int dtype, const double* w, int64_t N, int64_t K,
                        const double2* v);
// eig.hip
size_t eig_ws_bytes(int64_t K);
int eig_hermitian(vmc_ctx* ctx, const double2* S, int64_t K, double tol, int max_sweeps, double* lam, double2* V,
                  void* ws);
void sr_solve_cg_impl(vmc_ctx* ctx, const void* O, int dtype, const double2* eloc, const double* w, int64_t N,
                      int64_t K, const vmc_sr_opts* o, double tol, int max_iter, double2* x, vmc_sr_info* info,
                      int* iters);
// ham
void ham_connected_impl(vmc_ham* H, const uint64_t* s, int64_t B, uint64_t* sp, double* mel, int32_t* cnt);

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }
