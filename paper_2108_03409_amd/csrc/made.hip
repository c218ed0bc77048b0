// Masked autoregressive proposal network (MADE): entry points.
#include "internal.h"

namespace {
thread_local std::string g_made_err;
int unsupported(vmc_ctx* ctx) {
  if (ctx) ctx->err = "MADE proposal is not built yet";
  return VMC_ERR_UNSUPPORTED;
}
}  // namespace

extern "C" int vmc_made_create(vmc_ctx* ctx, int, int, vmc_made** out) {
  if (!ctx || !out) return VMC_ERR_INVALID_ARG;
  return unsupported(ctx);
}
extern "C" int vmc_made_num_params(const vmc_made* md, int64_t* P) {
  if (!md || !P) return VMC_ERR_INVALID_ARG;
  *P = md->P;
  return VMC_OK;
}
extern "C" int vmc_made_set_params(vmc_made* md, const double*) { return md ? unsupported(md->ctx) : VMC_ERR_INVALID_ARG; }
extern "C" int vmc_made_get_params(const vmc_made* md, double*) { return md ? unsupported(md->ctx) : VMC_ERR_INVALID_ARG; }
extern "C" int vmc_made_log_q(vmc_made* md, const uint64_t*, int64_t, double*) {
  return md ? unsupported(md->ctx) : VMC_ERR_INVALID_ARG;
}
extern "C" int vmc_made_nll_grad(vmc_made* md, const uint64_t*, int64_t, double*, double*) {
  return md ? unsupported(md->ctx) : VMC_ERR_INVALID_ARG;
}
extern "C" int vmc_made_train(vmc_made* md, const uint64_t*, int64_t, int, int, double, double*) {
  return md ? unsupported(md->ctx) : VMC_ERR_INVALID_ARG;
}
extern "C" int vmc_made_sample(vmc_made* md, int64_t, uint64_t, uint64_t, uint64_t*, double*) {
  return md ? unsupported(md->ctx) : VMC_ERR_INVALID_ARG;
}
extern "C" int vmc_made_destroy(vmc_made* md) {
  if (!md) return VMC_ERR_INVALID_ARG;
  delete md;
  return VMC_OK;
}
extern "C" int vmc_sampler_set_proposal_made(vmc_sampler* S, const vmc_made* md) {
  if (!S || !md) return VMC_ERR_INVALID_ARG;
  return unsupported(S->ctx);
}
