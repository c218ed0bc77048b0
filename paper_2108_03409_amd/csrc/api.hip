// Host side of the C ABI: contexts, models, Hamiltonians, argument checks and
// dispatch to the kernels in rbm.hip, sampler.hip, sr.hip and made.hip.
#include <cmath>
#include <exception>
#include <new>

#include "internal.h"

std::string& thread_error() {
  static thread_local std::string e;
  return e;
}

void set_device(vmc_ctx* ctx) { VMC_HIP(hipSetDevice(ctx->device)); }

namespace {
void* dmalloc(size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) bytes = 256;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    throw vmc_error{VMC_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
  }
  return p;
}

}  // namespace

// ------------------------------------------------------------- workspace --
void ws_reserve(vmc_ctx* ctx, size_t bytes) {
  if (ctx->ws_limit && bytes > ctx->ws_limit)
    throw vmc_error{VMC_ERR_WORKSPACE, "workspace of " + std::to_string(bytes) + " bytes exceeds the limit of " +
                                           std::to_string(ctx->ws_limit)};
  if (bytes > ctx->ws.cap) {
    VMC_HIP(hipStreamSynchronize(ctx->stream));
    if (ctx->ws.base) VMC_HIP(hipFree(ctx->ws.base));
    ctx->ws.base = nullptr;
    ctx->ws.cap = 0;
    ctx->ws.base = dmalloc(bytes);
    ctx->ws.cap = bytes;
  }
  ctx->ws.used = 0;
}

void* ws_take(vmc_ctx* ctx, size_t bytes) {
  size_t b = ws_round(bytes);
  if (ctx->ws.used + b > ctx->ws.cap) throw vmc_error{VMC_ERR_WORKSPACE, "internal: workspace under-reserved"};
  void* p = (char*)ctx->ws.base + ctx->ws.used;
  ctx->ws.used += b;
  return p;
}

void* pinned_host(vmc_ctx* ctx, size_t bytes) {
  if (bytes > ctx->pinned_cap) {
    VMC_HIP(hipStreamSynchronize(ctx->stream));
    if (ctx->pinned) VMC_HIP(hipHostFree(ctx->pinned));
    ctx->pinned = nullptr;
    ctx->pinned_cap = 0;
    VMC_HIP(hipHostMalloc(&ctx->pinned, bytes, hipHostMallocDefault));
    ctx->pinned_cap = bytes;
  }
  return ctx->pinned;
}

// ----------------------------------------------------------------- timing --
namespace {
hipEvent_t pool_event(vmc_ctx* ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  VMC_HIP(hipEventCreate(&e));
  return e;
}

void resolve_timing(vmc_ctx* ctx) {
  VMC_HIP(hipStreamSynchronize(ctx->stream));
  for (auto& p : ctx->pending) {
    float ms = 0.f;
    if (p.b) VMC_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    auto& acc = ctx->phases[p.name];
    acc.first += ms;
    acc.second += 1;
    ctx->event_pool.push_back(p.a);
    if (p.b) ctx->event_pool.push_back(p.b);
  }
  ctx->pending.clear();
}
}  // namespace

phase_scope::phase_scope(vmc_ctx* c, const char* name) : ctx(c), idx((size_t)-1) {
  if (!ctx || !ctx->timing) return;
  hipEvent_t a = pool_event(ctx);
  VMC_HIP(hipEventRecord(a, ctx->stream));
  ctx->pending.push_back({name, a, nullptr});
  idx = ctx->pending.size() - 1;
}

phase_scope::~phase_scope() {
  if (idx == (size_t)-1) return;
  hipEvent_t b = nullptr;
  if (!ctx->event_pool.empty()) {
    b = ctx->event_pool.back();
    ctx->event_pool.pop_back();
  } else if (hipEventCreate(&b) != hipSuccess) {
    b = nullptr;
  }
  if (b && hipEventRecord(b, ctx->stream) == hipSuccess) ctx->pending[idx].b = b;
}

extern "C" int vmc_ctx_set_timing(vmc_ctx* ctx, int enable) {
  return guard(ctx, [&] {
    VMC_REQUIRE(ctx, "ctx is NULL");
    set_device(ctx);
    resolve_timing(ctx);
    ctx->phases.clear();
    ctx->timing = enable ? 1 : 0;
  });
}

extern "C" int vmc_ctx_get_timing(vmc_ctx* ctx, const char* phase, double* total_ms, int64_t* count) {
  return guard(ctx, [&] {
    VMC_REQUIRE(ctx && phase && total_ms && count, "NULL argument");
    set_device(ctx);
    resolve_timing(ctx);
    auto it = ctx->phases.find(phase);
    *total_ms = it == ctx->phases.end() ? 0.0 : it->second.first;
    *count = it == ctx->phases.end() ? 0 : it->second.second;
  });
}

// ---------------------------------------------------------------- context --
extern "C" const char* vmc_version(void) { return "nqsvmc 0.1 (gfx950)"; }

extern "C" int vmc_ctx_create(int hip_device, void* hip_stream, vmc_ctx** out) {
  return guard(nullptr, [&] {
    VMC_REQUIRE(out != nullptr, "out is NULL");
    int n = 0;
    VMC_HIP(hipGetDeviceCount(&n));
    VMC_REQUIRE(hip_device >= 0 && hip_device < n, "no such HIP device");
    VMC_HIP(hipSetDevice(hip_device));
    hipDeviceProp_t prop;
    VMC_HIP(hipGetDeviceProperties(&prop, hip_device));
    if (std::string(prop.gcnArchName).rfind("gfx950", 0) != 0)
      throw vmc_error{VMC_ERR_UNSUPPORTED, std::string("library is built for gfx950, device is ") + prop.gcnArchName};
    auto* c = new vmc_ctx;
    c->device = hip_device;
    c->stream = (hipStream_t)hip_stream;
    *out = c;
  });
}

void ctx_retain(vmc_ctx* ctx) { ctx->refs.fetch_add(1); }

void ctx_release(vmc_ctx* ctx) {
  if (ctx->refs.fetch_sub(1) != 1) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->ws.base) (void)hipFree(ctx->ws.base);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  for (auto& p : ctx->pending) {
    (void)hipEventDestroy(p.a);
    if (p.b) (void)hipEventDestroy(p.b);
  }
  for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
  if (ctx->aux) {
    (void)hipStreamSynchronize(ctx->aux);
    (void)hipStreamDestroy(ctx->aux);
  }
  if (ctx->ev_main) (void)hipEventDestroy(ctx->ev_main);
  if (ctx->ev_aux) (void)hipEventDestroy(ctx->ev_aux);
  delete ctx;
}

int cu_count(vmc_ctx* ctx) {
  if (ctx->n_cu <= 0) VMC_HIP(hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device));
  return ctx->n_cu;
}

hipStream_t aux_stream(vmc_ctx* ctx) {
  if (!ctx->aux) {
    VMC_HIP(hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
    VMC_HIP(hipEventCreateWithFlags(&ctx->ev_main, hipEventDisableTiming));
    VMC_HIP(hipEventCreateWithFlags(&ctx->ev_aux, hipEventDisableTiming));
  }
  return ctx->aux;
}

extern "C" int vmc_ctx_destroy(vmc_ctx* ctx) {
  if (!ctx) return VMC_ERR_INVALID_ARG;
  ctx_release(ctx);
  return VMC_OK;
}

extern "C" int vmc_ctx_sync(vmc_ctx* ctx) {
  return guard(ctx, [&] {
    VMC_REQUIRE(ctx, "ctx is NULL");
    VMC_HIP(hipStreamSynchronize(ctx->stream));
  });
}

extern "C" const char* vmc_last_error(vmc_ctx* ctx) { return ctx ? ctx->err.c_str() : thread_error().c_str(); }

extern "C" int vmc_ctx_set_workspace_limit(vmc_ctx* ctx, size_t bytes) {
  return guard(ctx, [&] {
    VMC_REQUIRE(ctx, "ctx is NULL");
    ctx->ws_limit = bytes;
  });
}

// ----------------------------------------------------------------- models --
extern "C" int vmc_model_create_rbm(vmc_ctx* ctx, int n_visible, int n_hidden, int is_complex, vmc_model** out) {
  return guard(ctx, [&] {
    VMC_REQUIRE(ctx && out, "NULL argument");
    VMC_REQUIRE(n_visible >= 1 && n_visible <= 4096, "n_visible must be in [1, 4096]");
    VMC_REQUIRE(n_hidden >= 1 && n_hidden <= 1024, "n_hidden must be in [1, 1024]");
    set_device(ctx);
    auto* m = new vmc_model;
    m->ctx = ctx;
    m->kind = MODEL_RBM;
    m->N = n_visible;
    m->W = (n_visible + 63) / 64;
    m->Nh = n_hidden;
    m->is_complex = is_complex ? 1 : 0;
    m->K = (int64_t)n_visible + n_hidden + (int64_t)n_visible * n_hidden;
    try {
      m->params = (double2*)dmalloc(sizeof(double2) * m->K);
      m->Wt = (double2*)dmalloc(sizeof(double2) * (size_t)n_visible * n_hidden);
      VMC_HIP(hipMemsetAsync(m->params, 0, sizeof(double2) * m->K, ctx->stream));
      VMC_HIP(hipMemsetAsync(m->Wt, 0, sizeof(double2) * (size_t)n_visible * n_hidden, ctx->stream));
    } catch (...) {
      if (m->params) (void)hipFree(m->params);
      if (m->Wt) (void)hipFree(m->Wt);
      delete m;
      throw;
    }
    ctx_retain(ctx);
    *out = m;
  });
}

extern "C" int vmc_model_create_cnn(vmc_ctx* ctx, int Lx, int Ly, int channels, int kernel, vmc_model** out) {
  return guard(ctx, [&] {
    VMC_REQUIRE(ctx && out, "NULL argument");
    VMC_REQUIRE(Lx >= 1 && Ly >= 1 && (int64_t)Lx * Ly <= 4096, "lattice must have 1..4096 sites");
    VMC_REQUIRE(channels >= 1 && channels <= 64, "channels must be in [1, 64]");
    VMC_REQUIRE(kernel >= 1 && kernel <= Lx && kernel <= Ly && kernel <= 8, "kernel must be in [1, min(Lx, Ly, 8)]");
    VMC_REQUIRE(2ull * channels * Lx * Ly * sizeof(double2) + 4096 <= 160 * 1024,
                "channels * sites too large for the per-sample LDS budget");
    set_device(ctx);
    auto* m = new vmc_model;
    m->ctx = ctx;
    m->kind = MODEL_CNN;
    m->Lx = Lx;
    m->Ly = Ly;
    m->N = Lx * Ly;
    m->W = (m->N + 63) / 64;
    m->C = channels;
    m->k = kernel;
    m->is_complex = 1;
    const int64_t kk = (int64_t)kernel * kernel;
    m->K = channels * kk + channels + (int64_t)channels * channels * kk + channels;
    try {
      m->params = (double2*)dmalloc(sizeof(double2) * m->K);
      VMC_HIP(hipMemsetAsync(m->params, 0, sizeof(double2) * m->K, ctx->stream));
    } catch (...) {
      if (m->params) (void)hipFree(m->params);
      delete m;
      throw;
    }
    ctx_retain(ctx);
    *out = m;
  });
}

extern "C" int vmc_model_create_autoregressive(vmc_ctx* ctx, int n_sites, int n_hidden, vmc_model** out) {
  return guard(ctx, [&] {
    VMC_REQUIRE(ctx && out, "NULL argument");
    VMC_REQUIRE(n_sites >= 2 && n_sites <= 1024, "n_sites must be in [2, 1024]");
    VMC_REQUIRE(n_hidden >= 1 && n_hidden <= 1024, "n_hidden must be in [1, 1024]");
    set_device(ctx);
    auto* m = new vmc_model;
    m->ctx = ctx;
    m->kind = MODEL_AR;
    m->N = n_sites;
    m->W = (n_sites + 63) / 64;
    m->Nh = n_hidden;
    m->is_complex = 0;
    m->K = (int64_t)n_sites * n_hidden + n_hidden + n_sites;
    try {
      m->params = (double2*)dmalloc(sizeof(double2) * m->K);
      VMC_HIP(hipMemsetAsync(m->params, 0, sizeof(double2) * m->K, ctx->stream));
      ar_init(m);
    } catch (...) {
      ar_free(m);
      if (m->params) (void)hipFree(m->params);
      delete m;
      throw;
    }
    ctx_retain(ctx);
    *out = m;
  });
}

extern "C" int vmc_model_create_symelu(vmc_ctx* ctx, int L, int alpha, vmc_model** out) {
  return guard(ctx, [&] {
    VMC_REQUIRE(ctx && out, "NULL argument");
    VMC_REQUIRE(L >= 2 && L <= 1024, "L must be in [2, 1024]");
    VMC_REQUIRE(alpha >= 1 && alpha <= 64, "alpha must be in [1, 64]");
    set_device(ctx);
    auto* m = new vmc_model;
    m->ctx = ctx;
    m->kind = MODEL_SYMELU;
    m->N = L;
    m->Lx = L;
    m->Ly = 1;
    m->W = (L + 63) / 64;
    m->C = alpha;
    m->is_complex = 0;
    m->K = (int64_t)alpha * (L + 1);
    try {
      symelu_check(m);
      m->params = (double2*)dmalloc(sizeof(double2) * m->K);
      VMC_HIP(hipMemsetAsync(m->params, 0, sizeof(double2) * m->K, ctx->stream));
    } catch (...) {
      if (m->params) (void)hipFree(m->params);
      delete m;
      throw;
    }
    ctx_retain(ctx);
    *out = m;
  });
}

extern "C" int vmc_model_create_table(vmc_ctx* ctx, int n_sites, const void* logpsi_table_c128, vmc_model** out) {
  vmc_model* m = nullptr;
  int rc = guard(ctx, [&] {
    VMC_REQUIRE(ctx && out, "NULL argument");
    VMC_REQUIRE(n_sites >= 1 && n_sites <= 24, "n_sites must be in [1, 24]");
    set_device(ctx);
    m = new vmc_model;
    m->ctx = ctx;
    m->kind = MODEL_TABLE;
    m->N = n_sites;
    m->W = 1;
    m->is_complex = 1;
    m->K = (int64_t)1 << n_sites;
    try {
      m->params = (double2*)dmalloc(sizeof(double2) * m->K);
      VMC_HIP(hipMemsetAsync(m->params, 0, sizeof(double2) * m->K, ctx->stream));
    } catch (...) {
      if (m->params) (void)hipFree(m->params);
      delete m;
      m = nullptr;
      throw;
    }
    ctx_retain(ctx);
  });
  if (rc != VMC_OK) return rc;
  if (logpsi_table_c128) {
    rc = vmc_model_set_params(m, logpsi_table_c128, VMC_DT_C128);
    if (rc != VMC_OK) {
      std::string msg = vmc_last_error(ctx);
      (void)vmc_model_destroy(m);
      guard(ctx, [&] { throw vmc_error{rc, msg}; });
      return rc;
    }
  }
  *out = m;
  return VMC_OK;
}

extern "C" int vmc_model_num_params(const vmc_model* m, int64_t* K) {
  if (!m || !K) return VMC_ERR_INVALID_ARG;
  *K = m->K;
  return VMC_OK;
}

extern "C" int vmc_model_num_sites(const vmc_model* m, int* N) {
  if (!m || !N) return VMC_ERR_INVALID_ARG;
  *N = m->N;
  return VMC_OK;
}

// conversion + finiteness check kernel
namespace {
__global__ void k_import_params(const void* src, int dtype, int64_t K, int force_real, double2* dst,
                                int* nonfinite) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= K) return;
  double2 v;
  if (dtype == VMC_DT_C128) {
    v = ((const double2*)src)[i];
  } else if (dtype == VMC_DT_C64) {
    float2 f = ((const float2*)src)[i];
    v = make_double2(f.x, f.y);
  } else {  // VMC_DT_F64
    v = make_double2(((const double*)src)[i], 0.0);
  }
  if (force_real) v.y = 0.0;
  if (!isfinite(v.x) || !isfinite(v.y)) atomicOr(nonfinite, 1);
  dst[i] = v;
}

__global__ void k_export_params(const double2* src, int dtype, int64_t K, void* dst) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= K) return;
  if (dtype == VMC_DT_C128)
    ((double2*)dst)[i] = src[i];
  else
    ((float2*)dst)[i] = make_float2((float)src[i].x, (float)src[i].y);
}

// Wt[i][j] = W[j][i] for the RBM weight block of the flat parameters.
__global__ void k_rbm_transpose(const double2* params, int N, int Nh, double2* Wt) {
  int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)N * Nh) return;
  int j = (int)(idx / N), i = (int)(idx % N);
  Wt[(int64_t)i * Nh + j] = params[N + Nh + idx];
}
}  // namespace

extern "C" int vmc_model_set_params(vmc_model* m, const void* params_dev, int dtype) {
  return guard(m ? m->ctx : nullptr, [&] {
    VMC_REQUIRE(m && params_dev, "NULL argument");
    VMC_REQUIRE(dtype == VMC_DT_C128 || dtype == VMC_DT_C64 || (dtype == VMC_DT_F64 && !m->is_complex),
                "dtype must be C128, C64, or F64 for a real model");
    vmc_ctx* ctx = m->ctx;
    set_device(ctx);
    ws_reserve(ctx, ws_round(sizeof(double2) * m->K) + 256);
    double2* tmp = (double2*)ws_take(ctx, sizeof(double2) * m->K);
    int* flag = (int*)ws_take(ctx, sizeof(int));
    VMC_HIP(hipMemsetAsync(flag, 0, sizeof(int), ctx->stream));
    k_import_params<<<grid_for(m->K, 256), 256, 0, ctx->stream>>>(params_dev, dtype, m->K, !m->is_complex, tmp, flag);
    VMC_HIP(hipGetLastError());
    int* hflag = (int*)pinned_host(ctx, sizeof(int));
    VMC_HIP(hipMemcpyAsync(hflag, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    VMC_HIP(hipStreamSynchronize(ctx->stream));
    if (*hflag) throw vmc_error{VMC_ERR_NONFINITE, "parameters contain NaN or Inf"};
    VMC_HIP(hipMemcpyAsync(m->params, tmp, sizeof(double2) * m->K, hipMemcpyDeviceToDevice, ctx->stream));
    if (m->kind == MODEL_RBM) {
      int64_t n = (int64_t)m->N * m->Nh;
      k_rbm_transpose<<<grid_for(n, 256), 256, 0, ctx->stream>>>(m->params, m->N, m->Nh, m->Wt);
      VMC_HIP(hipGetLastError());
    } else if (m->kind == MODEL_AR) {
      ar_set_params(m);
    }
    m->version++;
  });
}

extern "C" int vmc_model_get_params(const vmc_model* m, void* params_dev, int dtype) {
  return guard(m ? m->ctx : nullptr, [&] {
    VMC_REQUIRE(m && params_dev, "NULL argument");
    VMC_REQUIRE(dtype == VMC_DT_C128 || dtype == VMC_DT_C64, "dtype must be C128 or C64");
    set_device(m->ctx);
    k_export_params<<<grid_for(m->K, 256), 256, 0, m->ctx->stream>>>(m->params, dtype, m->K, params_dev);
    VMC_HIP(hipGetLastError());
  });
}

extern "C" int vmc_model_set_precision(vmc_model* m, int prec) {
  return guard(m ? m->ctx : nullptr, [&] {
    VMC_REQUIRE(m, "NULL model");
    VMC_REQUIRE(prec == VMC_F64 || prec == VMC_F32 || prec == VMC_BF16, "unknown precision");
    if (prec != VMC_F64 && m->kind == MODEL_AR)
      throw vmc_error{VMC_ERR_UNSUPPORTED, "the autoregressive state is evaluated in float64 only"};
    if (prec != VMC_F64 && (m->kind == MODEL_TABLE || m->kind == MODEL_SYMELU))
      throw vmc_error{VMC_ERR_UNSUPPORTED, "this model kind is evaluated in float64 only"};
    if (prec != VMC_F64 && m->kind == MODEL_CNN && (m->Lx < 2 * m->k - 1 || m->Ly < 2 * m->k - 1))
      throw vmc_error{VMC_ERR_UNSUPPORTED, "float32 / bfloat16 CNN local energies need Lx, Ly >= 2 kernel - 1"};
    m->prec = prec;
  });
}

extern "C" int vmc_model_destroy(vmc_model* m) {
  if (!m) return VMC_ERR_INVALID_ARG;
  (void)hipSetDevice(m->ctx->device);
  (void)hipStreamSynchronize(m->ctx->stream);
  if (m->params) (void)hipFree(m->params);
  if (m->Wt) (void)hipFree(m->Wt);
  rbm_lowp_free(m);
  ar_free(m);
  for (auto& t : m->tab) {
    if (t.T) (void)hipFree(t.T);
    if (t.D) (void)hipFree(t.D);
    if (t.LC) (void)hipFree(t.LC);
    if (t.alpha) (void)hipFree(t.alpha);
    if (t.Tt) (void)hipFree(t.Tt);
    if (t.Dt) (void)hipFree(t.Dt);
  }
  vmc_ctx* ctx = m->ctx;
  delete m;
  ctx_release(ctx);
  return VMC_OK;
}

// ----------------------------------------------------------- Hamiltonians --
static int make_ham(vmc_ctx* ctx, int kind, int Lx, int Ly, int periodic, double J, double h, vmc_ham** out) {
  return guard(ctx, [&] {
    VMC_REQUIRE(ctx && out, "NULL argument");
    VMC_REQUIRE(Lx >= 1 && Ly >= 1 && (int64_t)Lx * Ly <= 4096, "lattice must have 1..4096 sites");
    VMC_REQUIRE(std::isfinite(J) && std::isfinite(h), "couplings must be finite");
    if (periodic) VMC_REQUIRE(Lx >= 3 && (Ly == 1 || Ly >= 3), "a periodic direction needs length >= 3");
    set_device(ctx);
    static std::atomic<uint64_t> next_uid{1};
    auto* H = new vmc_ham;
    H->ctx = ctx;
    H->uid = next_uid.fetch_add(1);
    H->kind = kind;
    H->Lx = Lx;
    H->Ly = Ly;
    H->periodic = periodic ? 1 : 0;
    H->N = Lx * Ly;
    H->W = (H->N + 63) / 64;
    H->J = J;
    H->h = h;
    for (int y = 0; y < Ly; ++y)
      for (int x = 0; x < Lx; ++x) {
        int i = y * Lx + x;
        if (x + 1 < Lx || (periodic && Lx > 1)) H->bonds_host.push_back(make_int2(i, y * Lx + (x + 1) % Lx));
        if (Ly > 1 && (y + 1 < Ly || periodic)) H->bonds_host.push_back(make_int2(i, ((y + 1) % Ly) * Lx + x));
      }
    H->n_bonds = (int)H->bonds_host.size();
    H->M_max = 1 + (kind == HAM_TFIM ? H->N : H->n_bonds);
    try {
      H->bonds = (int2*)dmalloc(sizeof(int2) * std::max(1, H->n_bonds));
      if (H->n_bonds)
        VMC_HIP(hipMemcpy(H->bonds, H->bonds_host.data(), sizeof(int2) * H->n_bonds, hipMemcpyHostToDevice));
    } catch (...) {
      if (H->bonds) (void)hipFree(H->bonds);
      delete H;
      throw;
    }
    ctx_retain(ctx);
    *out = H;
  });
}

extern "C" int vmc_ham_create_tfim(vmc_ctx* ctx, int Lx, int Ly, int periodic, double J, double h, vmc_ham** out) {
  return make_ham(ctx, HAM_TFIM, Lx, Ly, periodic, J, h, out);
}

extern "C" int vmc_ham_create_heisenberg(vmc_ctx* ctx, int Lx, int Ly, int periodic, double J, vmc_ham** out) {
  return make_ham(ctx, HAM_HEIS, Lx, Ly, periodic, J, 0.0, out);
}

extern "C" int vmc_ham_max_connected(const vmc_ham* H, int* M_max) {
  if (!H || !M_max) return VMC_ERR_INVALID_ARG;
  *M_max = H->M_max;
  return VMC_OK;
}

extern "C" int vmc_ham_num_bonds(const vmc_ham* H, int* n_bonds) {
  if (!H || !n_bonds) return VMC_ERR_INVALID_ARG;
  *n_bonds = H->n_bonds;
  return VMC_OK;
}

extern "C" int vmc_ham_connected(vmc_ham* H, const uint64_t* s, int64_t B, uint64_t* sp, double* mel, int32_t* count) {
  return guard(H ? H->ctx : nullptr, [&] {
    VMC_REQUIRE(H, "NULL Hamiltonian");
    VMC_REQUIRE(B >= 0, "B < 0");
    if (B == 0) return;
    VMC_REQUIRE(s && sp && mel && count, "NULL buffer");
    set_device(H->ctx);
    ham_connected_impl(H, s, B, sp, mel, count);
  });
}

extern "C" int vmc_ham_destroy(vmc_ham* H) {
  if (!H) return VMC_ERR_INVALID_ARG;
  (void)hipSetDevice(H->ctx->device);
  (void)hipStreamSynchronize(H->ctx->stream);
  if (H->bonds) (void)hipFree(H->bonds);
  vmc_ctx* ctx = H->ctx;
  delete H;
  ctx_release(ctx);
  return VMC_OK;
}

// --------------------------------------------------------------- hot path --
extern "C" int vmc_log_psi(vmc_model* m, const uint64_t* s, int64_t B, double* logpsi) {
  return guard(m ? m->ctx : nullptr, [&] {
    VMC_REQUIRE(m, "NULL model");
    VMC_REQUIRE(B >= 0, "B < 0");
    if (B == 0) return;
    VMC_REQUIRE(s && logpsi, "NULL buffer");
    set_device(m->ctx);
    phase_scope ps(m->ctx, "log_psi");
    if (m->kind == MODEL_RBM && m->prec != VMC_F64)
      rbm_lowp_log_psi(m, s, B, (double2*)logpsi);
    else if (m->kind == MODEL_RBM)
      rbm_log_psi(m, s, B, (double2*)logpsi);
    else if (m->kind == MODEL_AR)
      ar_log_psi(m, s, B, (double2*)logpsi);
    else if (m->kind == MODEL_TABLE)
      table_log_psi(m, s, B, (double2*)logpsi);
    else if (m->kind == MODEL_SYMELU)
      symelu_log_psi(m, s, B, (double2*)logpsi);
    else
      cnn_log_psi(m, s, B, (double2*)logpsi);
  });
}

extern "C" int vmc_local_energy(vmc_model* m, vmc_ham* H, const uint64_t* s, int64_t B, const double* logpsi_s,
                                double* eloc) {
  (void)logpsi_s;
  return guard(m ? m->ctx : nullptr, [&] {
    VMC_REQUIRE(m && H, "NULL handle");
    VMC_REQUIRE(m->ctx == H->ctx, "model and Hamiltonian belong to different contexts");
    VMC_REQUIRE(m->N == H->N, "model and Hamiltonian have different site counts");
    VMC_REQUIRE(B >= 0, "B < 0");
    if (B == 0) return;
    VMC_REQUIRE(s && eloc, "NULL buffer");
    set_device(m->ctx);
    phase_scope ps(m->ctx, "eloc");
    if (m->kind == MODEL_RBM && m->prec != VMC_F64)
      rbm_lowp_local_energy(m, H, s, B, (double2*)eloc);
    else if (m->kind == MODEL_RBM)
      rbm_local_energy(m, H, s, B, (double2*)eloc);
    else if (m->kind == MODEL_AR)
      ar_local_energy(m, H, s, B, (double2*)eloc);
    else if (m->kind == MODEL_TABLE)
      table_local_energy(m, H, s, B, (double2*)eloc);
    else if (m->kind == MODEL_SYMELU)
      symelu_local_energy(m, H, s, B, (double2*)eloc);
    else if (m->prec != VMC_F64)
      cnn_lowp_local_energy(m, H, s, B, (double2*)eloc);
    else
      cnn_local_energy(m, H, s, B, (double2*)eloc);
  });
}

extern "C" int vmc_grad_log_psi(vmc_model* m, const uint64_t* s, int64_t B, void* O, int dtype) {
  return guard(m ? m->ctx : nullptr, [&] {
    VMC_REQUIRE(m, "NULL model");
    VMC_REQUIRE(dtype == VMC_DT_C128 || dtype == VMC_DT_C64 || dtype == VMC_DT_F32 || dtype == VMC_DT_F64,
                "dtype must be C128, C64, F32 or F64");
    if (dtype == VMC_DT_F32 || dtype == VMC_DT_F64)
      VMC_REQUIRE(m->kind == MODEL_AR || m->kind == MODEL_SYMELU,
                  "real O_k (F32 / F64) are written for the real-parameter networks (autoregressive, symmetric ELU)");
    VMC_REQUIRE(B >= 0, "B < 0");
    if (B == 0) return;
    VMC_REQUIRE(s && O, "NULL buffer");
    set_device(m->ctx);
    phase_scope ps(m->ctx, "grad");
    if (m->kind == MODEL_RBM)
      rbm_grad(m, s, B, O, dtype);
    else if (m->kind == MODEL_AR)
      ar_grad(m, s, B, O, dtype);
    else if (m->kind == MODEL_TABLE)
      table_grad(m, s, B, O, dtype);
    else if (m->kind == MODEL_SYMELU)
      symelu_grad(m, s, B, O, dtype);
    else
      cnn_grad(m, s, B, O, dtype);
  });
}

extern "C" int vmc_log_psi_vjp(vmc_model* m, const uint64_t* s, int64_t B, const double* g, double* out) {
  return guard(m ? m->ctx : nullptr, [&] {
    VMC_REQUIRE(m, "NULL model");
    VMC_REQUIRE(B >= 0, "B < 0");
    VMC_REQUIRE(out, "NULL out");
    if (m->kind == MODEL_AR || m->kind == MODEL_TABLE || m->kind == MODEL_SYMELU)
      throw vmc_error{VMC_ERR_UNSUPPORTED, "no vector-Jacobian product for this model kind"};
    VMC_REQUIRE(B == 0 || (s && g), "NULL buffer");
    set_device(m->ctx);
    phase_scope ps(m->ctx, "vjp");
    log_psi_vjp_impl(m, s, B, (const double2*)g, (double2*)out);
  });
}

extern "C" int vmc_log_psi_vjp_noalloc(vmc_model* m, const uint64_t* s, int64_t B, const double* g, double* out) {
  return guard(m ? m->ctx : nullptr, [&] {
    VMC_REQUIRE(m, "NULL model");
    VMC_REQUIRE(B >= 0, "B < 0");
    VMC_REQUIRE(out, "NULL out");
    if (m->kind != MODEL_RBM && m->kind != MODEL_CNN)
      throw vmc_error{VMC_ERR_UNSUPPORTED, "no vector-Jacobian product for this model kind"};
    VMC_REQUIRE(B == 0 || (s && g), "NULL buffer");
    set_device(m->ctx);
    log_psi_vjp_noalloc_impl(m, s, B, (const double2*)g, (double2*)out);
  });
}

// ---------------------------------------------------------------- sampler --
extern "C" int vmc_sampler_create(vmc_ctx* ctx, vmc_model* m, vmc_ham* H, const vmc_sampler_opts* o,
                                  vmc_sampler** out) {
  return guard(ctx, [&] {
    VMC_REQUIRE(ctx && m && H && o && out, "NULL argument");
    VMC_REQUIRE(m->ctx == ctx && H->ctx == ctx, "handles belong to another context");
    VMC_REQUIRE(m->N == H->N, "model and Hamiltonian have different site counts");
    VMC_REQUIRE(o->n_chains > 0 && o->n_chains <= (1 << 22), "n_chains must be in [1, 2^22]");
    VMC_REQUIRE(o->sweep_steps >= 0 && o->therm_sweeps >= 0, "negative sweep settings");
    VMC_REQUIRE(o->proposal == VMC_PROP_FLIP || o->proposal == VMC_PROP_EXCHANGE || o->proposal == VMC_PROP_MADE_MIX,
                "unknown proposal");
    if (o->proposal == VMC_PROP_EXCHANGE) {
      VMC_REQUIRE(H->n_bonds > 0, "exchange moves need bonds");
      VMC_REQUIRE(m->N % 2 == 0, "exchange sampling starts in Sz = 0 and needs an even site count");
    }
    if (o->proposal == VMC_PROP_MADE_MIX)
      VMC_REQUIRE(o->global_steps >= 0 && o->global_steps <= 1024, "global_steps must be in [0, 1024]");
    VMC_REQUIRE(m->kind == MODEL_RBM || o->proposal == VMC_PROP_FLIP ||
                    (m->kind == MODEL_TABLE && o->proposal == VMC_PROP_EXCHANGE),
                "CNN models are sampled with single flips; autoregressive states take VMC_PROP_FLIP (direct "
                "sampling); tabulated models take flips or exchanges");
    set_device(ctx);
    auto* S = new vmc_sampler;
    S->ctx = ctx;
    S->model = m;
    S->ham = H;
    S->opts = *o;
    if (S->opts.sweep_steps == 0) S->opts.sweep_steps = m->N;
    S->N = m->N;
    S->W = m->W;
    try {
      S->bits = (uint64_t*)dmalloc(sizeof(uint64_t) * (size_t)o->n_chains * S->W);
      S->acc = (unsigned long long*)dmalloc(sizeof(unsigned long long) * 3 * (size_t)o->n_chains);
    } catch (...) {
      if (S->bits) (void)hipFree(S->bits);
      delete S;
      throw;
    }
    S->t = 0;
    S->thermalized = 0;
    // initial states are drawn lazily by the first vmc_sample (t == 0)
    ctx_retain(ctx);
    *out = S;
  });
}

extern "C" int vmc_sample(vmc_sampler* S, int64_t n_samples, uint64_t* s_out, double* logpsi_out, int64_t* n_written,
                          double* accept_rate_host) {
  return guard(S ? S->ctx : nullptr, [&] {
    VMC_REQUIRE(S, "NULL sampler");
    VMC_REQUIRE(n_samples >= 0, "n_samples < 0");
    int64_t per_chain = (n_samples + S->opts.n_chains - 1) / S->opts.n_chains;
    if (n_written) *n_written = per_chain * S->opts.n_chains;
    if (per_chain == 0) {
      if (accept_rate_host) *accept_rate_host = 0.0;
      return;
    }
    VMC_REQUIRE(s_out, "NULL s_out");
    if (S->opts.proposal == VMC_PROP_MADE_MIX)
      VMC_REQUIRE(S->made_buf, "VMC_PROP_MADE_MIX needs vmc_sampler_set_proposal_made first");
    set_device(S->ctx);
    if (S->model->kind == MODEL_AR) {  // direct sampling: independent draws, nothing rejected
      phase_scope ps(S->ctx, "sample");
      ar_sample(S, per_chain * S->opts.n_chains, s_out, (double2*)logpsi_out);
      S->bits_valid = 1;
      S->thermalized = 1;
      S->last_accept = 1.0;
      S->last_global_accept = 0.0;
      S->last_n_global = 0;
      if (accept_rate_host) *accept_rate_host = 1.0;
      return;
    }
    uint64_t t0 = S->t;
    {
      phase_scope ps(S->ctx, "sample");
      if (S->model->kind == MODEL_TABLE)
        table_sampler_run(S, per_chain, s_out, (double2*)logpsi_out);
      else if (S->model->kind == MODEL_SYMELU)
        symelu_sampler_run(S, per_chain, s_out, (double2*)logpsi_out);
      else if (S->model->kind == MODEL_CNN && S->model->prec != VMC_F64)
        cnn_lowp_sampler_run(S, per_chain, s_out, (double2*)logpsi_out);
      else if (S->model->kind == MODEL_CNN)
        cnn_sampler_run(S, per_chain, s_out, (double2*)logpsi_out);
      else
        sampler_run(S, per_chain, s_out, (double2*)logpsi_out);
    }
    const int nc = S->opts.n_chains;
    const int nrows = S->opts.proposal == VMC_PROP_MADE_MIX ? 3 : 1;
    auto* h = (unsigned long long*)pinned_host(S->ctx, sizeof(unsigned long long) * nrows * (size_t)nc);
    VMC_HIP(hipMemcpyAsync(h, S->acc, sizeof(unsigned long long) * nrows * (size_t)nc, hipMemcpyDeviceToHost,
                           S->ctx->stream));
    VMC_HIP(hipStreamSynchronize(S->ctx->stream));
    double tot = 0, tg = 0, ng = 0;
    for (int c = 0; c < nc; ++c) tot += (double)h[c];
    if (nrows == 3)
      for (int c = 0; c < nc; ++c) {
        tg += (double)h[nc + c];
        ng += (double)h[2 * nc + c];
      }
    const double steps = (double)(S->t - t0) * nc + ng;  // flips and global proposals
    S->last_accept = steps > 0 ? tot / steps : 0.0;
    S->last_global_accept = ng > 0 ? tg / ng : 0.0;
    S->last_n_global = (int64_t)ng;
    if (accept_rate_host) *accept_rate_host = S->last_accept;
  });
}

namespace {
struct state_header {
  uint64_t magic, N, W, n_chains, t, thermalized, seed, proposal, g;
};
const uint64_t kStateMagic = 0x4e51535653414d32ull;  // "NQSVSAM2"
}  // namespace

extern "C" int vmc_sampler_get_state(vmc_sampler* S, void* buf_host, size_t* bytes) {
  return guard(S ? S->ctx : nullptr, [&] {
    VMC_REQUIRE(S && bytes, "NULL argument");
    VMC_REQUIRE(S->bits_valid, "the sampler has no chain state yet (call vmc_sample first)");
    size_t need = sizeof(state_header) + sizeof(uint64_t) * (size_t)S->opts.n_chains * S->W;
    if (!buf_host) {
      *bytes = need;
      return;
    }
    VMC_REQUIRE(*bytes >= need, "state buffer too small");
    set_device(S->ctx);
    state_header h{kStateMagic, (uint64_t)S->N, (uint64_t)S->W, (uint64_t)S->opts.n_chains, S->t,
                   (uint64_t)S->thermalized, S->opts.seed, (uint64_t)S->opts.proposal, S->g};
    std::memcpy(buf_host, &h, sizeof(h));
    VMC_HIP(hipStreamSynchronize(S->ctx->stream));
    VMC_HIP(hipMemcpy((char*)buf_host + sizeof(h), S->bits, need - sizeof(h), hipMemcpyDeviceToHost));
    *bytes = need;
  });
}

extern "C" int vmc_sampler_set_state(vmc_sampler* S, const void* buf_host, size_t bytes) {
  return guard(S ? S->ctx : nullptr, [&] {
    VMC_REQUIRE(S && buf_host, "NULL argument");
    state_header h;
    VMC_REQUIRE(bytes >= sizeof(h), "state blob too short");
    std::memcpy(&h, buf_host, sizeof(h));
    size_t need = sizeof(state_header) + sizeof(uint64_t) * (size_t)S->opts.n_chains * S->W;
    VMC_REQUIRE(h.magic == kStateMagic, "not a sampler state blob");
    VMC_REQUIRE(h.N == (uint64_t)S->N && h.W == (uint64_t)S->W && h.n_chains == (uint64_t)S->opts.n_chains &&
                    h.proposal == (uint64_t)S->opts.proposal,
                "state blob belongs to a sampler of another shape");
    VMC_REQUIRE(bytes >= need, "state blob too short");
    set_device(S->ctx);
    VMC_HIP(hipStreamSynchronize(S->ctx->stream));
    VMC_HIP(hipMemcpy(S->bits, (const char*)buf_host + sizeof(h), need - sizeof(h), hipMemcpyHostToDevice));
    S->t = h.t;
    S->g = h.g;
    S->thermalized = (int)h.thermalized;
    S->opts.seed = h.seed;
    S->mix_pg[0] = S->mix_pg[1] = ~0ull;  // proposals formed ahead belong to the replaced state
    S->bits_valid = 1;
  });
}

extern "C" int vmc_sampler_get_stats(vmc_sampler* S, double* accept_rate_host, double* global_accept_rate_host,
                                     int64_t* n_global_host) {
  return guard(S ? S->ctx : nullptr, [&] {
    VMC_REQUIRE(S, "NULL sampler");
    if (accept_rate_host) *accept_rate_host = S->last_accept;
    if (global_accept_rate_host) *global_accept_rate_host = S->last_global_accept;
    if (n_global_host) *n_global_host = S->last_n_global;
  });
}

extern "C" int vmc_sampler_destroy(vmc_sampler* S) {
  if (!S) return VMC_ERR_INVALID_ARG;
  (void)hipSetDevice(S->ctx->device);
  (void)hipStreamSynchronize(S->ctx->stream);
  mix_release(S);
  if (S->bits) (void)hipFree(S->bits);
  if (S->acc) (void)hipFree(S->acc);
  for (void* p : {(void*)S->made_buf, (void*)S->mix_perm})
    if (p) (void)hipFree(p);
  vmc_ctx* ctx = S->ctx;
  delete S;
  ctx_release(ctx);
  return VMC_OK;
}

// --------------------------------------------------------------------- SR --
extern "C" int vmc_sr_solve(vmc_ctx* ctx, const void* O, int O_dtype, const double* eloc, const double* weights,
                            int64_t N, int64_t K, const vmc_sr_opts* opts, double* x, vmc_sr_info* info_host) {
  vmc_sr_info info{};
  info.fail_index = -1;
  int rc = guard(ctx, [&] {
    VMC_REQUIRE(ctx && opts, "NULL argument");
    VMC_REQUIRE(O_dtype == VMC_DT_C64 || O_dtype == VMC_DT_C128 || O_dtype == VMC_DT_F32 || O_dtype == VMC_DT_F64,
                "O dtype must be C64, C128, F32 or F64");
    VMC_REQUIRE(N >= 1 && K >= 1, "N and K must be positive");
    VMC_REQUIRE(K <= 65536, "K above 65536 is not supported by the dense solve");
    VMC_REQUIRE(O && eloc && x, "NULL buffer");
    VMC_REQUIRE(std::isfinite(opts->nu_rel) && opts->nu_rel >= 0 && std::isfinite(opts->eps_abs) &&
                    opts->eps_abs >= 0,
                "shifts must be finite and non-negative");
    VMC_REQUIRE(opts->mode == VMC_SR_COMPLEX || opts->mode == VMC_SR_REAL || opts->mode == VMC_SR_IMAG,
                "unknown mode");
    if (opts->mode == VMC_SR_IMAG)
      throw vmc_error{VMC_ERR_UNSUPPORTED, "Im S is antisymmetric; the Cholesky solve needs COMPLEX or REAL"};
    VMC_REQUIRE(opts->gram == 0 || opts->gram == 1, "gram must be 0 or 1");
    VMC_REQUIRE(opts->gram == 0 || O_dtype == VMC_DT_C64 || O_dtype == VMC_DT_F32,
                "the split-float16 product needs float32 O (C64 or F32)");
    set_device(ctx);
    sr_solve_impl(ctx, O, O_dtype, (const double2*)eloc, weights, N, K, opts, (double2*)x, &info, nullptr, nullptr,
                  nullptr, nullptr);
    if (info.fail_index >= 0)
      throw vmc_error{VMC_ERR_NOT_PD, "shifted S is not positive definite at column " +
                                          std::to_string(info.fail_index)};
    if (!std::isfinite(info.residual)) throw vmc_error{VMC_ERR_NONFINITE, "solution is not finite"};
  });
  if (info_host) *info_host = info;
  return rc;
}

extern "C" int vmc_sr_solve_eig(vmc_ctx* ctx, const void* O, int O_dtype, const double* eloc, const double* weights,
                                int64_t N, int64_t K, const vmc_sr_opts* opts, const vmc_eig_opts* eo, double* x,
                                vmc_sr_info* info_host, double* evals, double* snr, int* sweeps_host) {
  vmc_sr_info info{};
  info.fail_index = -1;
  info.residual = NAN;
  int sw = 0;
  int rc = guard(ctx, [&] {
    VMC_REQUIRE(ctx && opts && eo, "NULL argument");
    VMC_REQUIRE(O_dtype == VMC_DT_C64 || O_dtype == VMC_DT_C128 || O_dtype == VMC_DT_F32 || O_dtype == VMC_DT_F64,
                "O dtype must be C64, C128, F32 or F64");
    VMC_REQUIRE(N >= 1 && K >= 1, "N and K must be positive");
    VMC_REQUIRE(K <= 16384, "K above 16384 is not supported by the eigendecomposition");
    VMC_REQUIRE(O && eloc && x, "NULL buffer");
    VMC_REQUIRE(std::isfinite(opts->nu_rel) && opts->nu_rel >= 0 && std::isfinite(opts->eps_abs) &&
                    opts->eps_abs >= 0,
                "shifts must be finite and non-negative");
    VMC_REQUIRE(opts->mode == VMC_SR_COMPLEX || opts->mode == VMC_SR_REAL || opts->mode == VMC_SR_IMAG,
                "unknown mode");
    if (opts->mode == VMC_SR_IMAG) {
      VMC_REQUIRE(O_dtype == VMC_DT_C64 || O_dtype == VMC_DT_C128,
                  "the Im projection needs complex O (C64 or C128): Im S of real log-derivatives is zero");
      VMC_REQUIRE(opts->eps_abs == 0.0, "an additive shift breaks the antisymmetry of Im S (eps_abs must be 0)");
    }
    VMC_REQUIRE(opts->gram == 0 || opts->gram == 1, "gram must be 0 or 1");
    VMC_REQUIRE(opts->gram == 0 || O_dtype == VMC_DT_C64 || O_dtype == VMC_DT_F32,
                "the split-float16 product needs float32 O (C64 or F32)");
    VMC_REQUIRE(std::isfinite(eo->eps_pinv) && eo->eps_pinv >= 0 && std::isfinite(eo->eps_snr) && eo->eps_snr >= 0,
                "cutoffs must be finite and non-negative");
    VMC_REQUIRE(eo->soft == 0 || eo->soft == 1, "soft must be 0 or 1");
    VMC_REQUIRE(std::isfinite(eo->tol) && eo->tol >= 0 && eo->max_sweeps >= 0, "bad Jacobi settings");
    set_device(ctx);
    sr_solve_impl(ctx, O, O_dtype, (const double2*)eloc, weights, N, K, opts, (double2*)x, &info, eo, evals, snr,
                  &sw);
    if (!std::isfinite(info.residual)) throw vmc_error{VMC_ERR_NONFINITE, "solution is not finite"};
  });
  if (info_host) *info_host = info;
  if (sweeps_host) *sweeps_host = sw;
  return rc;
}

extern "C" int vmc_sr_fisher(vmc_ctx* ctx, const void* O, int O_dtype, const double* eloc, const double* weights,
                             int64_t N, int64_t K, const vmc_sr_opts* opts, double* S_out, double* F_out,
                             vmc_sr_info* info_host) {
  vmc_sr_info info{};
  info.fail_index = -1;
  info.residual = NAN;
  info.min_pivot = NAN;
  int rc = guard(ctx, [&] {
    VMC_REQUIRE(ctx && opts, "NULL argument");
    VMC_REQUIRE(O_dtype == VMC_DT_C64 || O_dtype == VMC_DT_C128 || O_dtype == VMC_DT_F32 || O_dtype == VMC_DT_F64,
                "O dtype must be C64, C128, F32 or F64");
    VMC_REQUIRE(N >= 1 && K >= 1, "N and K must be positive");
    VMC_REQUIRE(K <= 65536, "K above 65536 is not supported by the dense solve");
    VMC_REQUIRE(O && eloc && S_out && F_out, "NULL buffer");
    VMC_REQUIRE(std::isfinite(opts->nu_rel) && opts->nu_rel >= 0 && std::isfinite(opts->eps_abs) &&
                    opts->eps_abs >= 0,
                "shifts must be finite and non-negative");
    VMC_REQUIRE(opts->mode == VMC_SR_COMPLEX || opts->mode == VMC_SR_REAL || opts->mode == VMC_SR_IMAG,
                "unknown mode");
    VMC_REQUIRE(opts->gram == 0 || opts->gram == 1, "gram must be 0 or 1");
    VMC_REQUIRE(opts->gram == 0 || O_dtype == VMC_DT_C64 || O_dtype == VMC_DT_F32,
                "the split-float16 product needs float32 O (C64 or F32)");
    set_device(ctx);
    sr_solve_impl(ctx, O, O_dtype, (const double2*)eloc, weights, N, K, opts, nullptr, &info, nullptr, nullptr,
                  nullptr, nullptr, (double2*)S_out, (double2*)F_out);
  });
  if (info_host) *info_host = info;
  return rc;
}

extern "C" int vmc_fisher_quad(vmc_ctx* ctx, const void* O, int O_dtype, const double* weights, int64_t N, int64_t K,
                               const double* v, double* out_host) {
  return guard(ctx, [&] {
    VMC_REQUIRE(ctx && O && v && out_host, "NULL argument");
    VMC_REQUIRE(O_dtype == VMC_DT_C64 || O_dtype == VMC_DT_C128 || O_dtype == VMC_DT_F32 || O_dtype == VMC_DT_F64,
                "O dtype must be C64, C128, F32 or F64");
    VMC_REQUIRE(N >= 1 && K >= 1, "N and K must be positive");
    set_device(ctx);
    phase_scope ps(ctx, "fisher");
    *out_host = fisher_quad_impl(ctx, O, O_dtype, weights, N, K, (const double2*)v);
  });
}

extern "C" int vmc_sr_solve_cg(vmc_ctx* ctx, const void* O, int O_dtype, const double* eloc, const double* weights,
                               int64_t N, int64_t K, const vmc_sr_opts* opts, const vmc_cg_opts* cg, double* x,
                               vmc_sr_info* info_host, int* iterations_host) {
  vmc_sr_info info{};
  info.fail_index = -1;
  info.residual = NAN;
  info.min_pivot = NAN;
  int iters = 0;
  int rc = guard(ctx, [&] {
    VMC_REQUIRE(ctx && opts && cg, "NULL argument");
    VMC_REQUIRE(O_dtype == VMC_DT_C64 || O_dtype == VMC_DT_C128, "O dtype must be C64 or C128");
    VMC_REQUIRE(N >= 1 && K >= 1, "N and K must be positive");
    VMC_REQUIRE(O && eloc && x, "NULL buffer");
    VMC_REQUIRE(std::isfinite(opts->nu_rel) && opts->nu_rel >= 0 && std::isfinite(opts->eps_abs) &&
                    opts->eps_abs >= 0,
                "shifts must be finite and non-negative");
    VMC_REQUIRE(opts->mode == VMC_SR_COMPLEX || opts->mode == VMC_SR_REAL || opts->mode == VMC_SR_IMAG,
                "unknown mode");
    if (opts->mode == VMC_SR_IMAG)
      throw vmc_error{VMC_ERR_UNSUPPORTED, "Im S is antisymmetric; conjugate gradient needs COMPLEX or REAL"};
    VMC_REQUIRE(std::isfinite(cg->tol) && cg->tol > 0 && cg->max_iter >= 1, "tol > 0 and max_iter >= 1 required");
    set_device(ctx);
    sr_solve_cg_impl(ctx, O, O_dtype, (const double2*)eloc, weights, N, K, opts, cg->tol, cg->max_iter, (double2*)x,
                     &info, &iters);
    if (!std::isfinite(info.residual)) throw vmc_error{VMC_ERR_NONFINITE, "solution is not finite"};
  });
  if (info_host) *info_host = info;
  if (iterations_host) *iterations_host = iters;
  return rc;
}
