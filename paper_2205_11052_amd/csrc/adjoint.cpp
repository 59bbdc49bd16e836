// Discrete adjoint (placeholder until the adjoint kernels land).
#include "../../include/dgw.h"
#include "dgw_ctx.h"

struct dgw_ctx::Adjoint {};

void dgw_ctx::free_adjoint() {
  delete adj;
  adj = nullptr;
}

extern "C" {
int dgw_forward_checkpointed(dgw_ctx *c, int64_t, int64_t, const double *, double *) {
  if (!c) return DGW_EINVAL;
  return c->fail(DGW_ESTATE, "adjoint not available in this build");
}
int dgw_adjoint(dgw_ctx *c, double *, double *, double *) {
  if (!c) return DGW_EINVAL;
  return c->fail(DGW_ESTATE, "adjoint not available in this build");
}
int dgw_autotune(dgw_ctx *c, const char *, int *) {
  if (!c) return DGW_EINVAL;
  return c->fail(DGW_ESTATE, "autotuner not available in this build");
}
}
