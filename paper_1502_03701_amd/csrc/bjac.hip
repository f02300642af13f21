// Block-Jacobi preconditioner (placeholder until the batched kernels land).
#include "sa_runtime.h"

namespace sa {
template <typename R>
hipError_t precond_apply(Ctx* c, int ishift, int nrhs, const R* r, R* z, const int* active) {
  (void)c; (void)ishift; (void)nrhs; (void)r; (void)z; (void)active;
  return hipErrorNotSupported;
}
template hipError_t precond_apply<double>(Ctx*, int, int, const double*, double*, const int*);
template hipError_t precond_apply<float>(Ctx*, int, int, const float*, float*, const int*);
}  // namespace sa

extern "C" {
int sa_precond_setup(sa_ctx* c, const sa_precond_opts*, int, const double*) {
  return c ? c->fail(SA_ESTATE, "sa_precond_setup: not available") : SA_EINVAL;
}
int sa_precond_apply(sa_ctx* c, sa_prec, int, int, const void*, void*) {
  return c ? c->fail(SA_ESTATE, "sa_precond_apply: not available") : SA_EINVAL;
}
int sa_arnoldi_eigs(sa_ctx* const* ctxs, int, const sa_eig_opts*, const double* const*, sa_eig_result*) {
  (void)ctxs;
  return SA_ESTATE;
}
}
