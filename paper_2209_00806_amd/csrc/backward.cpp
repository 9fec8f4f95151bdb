// placeholder, replaced by the adjoint implementation
#include "tbpm_engine.h"
namespace tbpm {
tbpm_status backward_impl(tbpm_hamiltonian *, const double *, int32_t, int32_t, double, double, double, const double *,
                          int32_t, const double *, double *, double *, hipStream_t) {
    return fail(TBPM_E_ARG, "tbpm_backward: not built yet");
}
}  // namespace tbpm
