// Adjoint (implicit-function-theorem) kernels of the coupling solve.
#include "nmc_internal.h"

extern "C" int nmc_solve_batch_adjoint(const nmc_model*, int64_t, double, const nmc_batch_in*, const nmc_batch_out*,
                                       const double*, double*, double*, void*, size_t, void*) {
  return NMC_E_UNSUPPORTED;
}
