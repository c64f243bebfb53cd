// Entry points still under construction: mixed-precision refinement, the
// adjoint and the autotuner.
#include "handle.h"

namespace jac {
jac_status solve_refine(Handle&, double, int32_t, int, int32_t*, double*)
{
    fail(JAC_E_INVALID, "JAC_FP32_REFINE is not available in this build");
}
}  // namespace jac

extern "C" {
jac_status jac_adjoint(jac_handle, int32_t, int32_t, const double*, double*, double*)
{
    jac::set_last_error("jac_adjoint is not available in this build");
    return JAC_E_INVALID;
}
jac_status jac_autotune(jac_handle, int32_t)
{
    jac::set_last_error("jac_autotune is not available in this build");
    return JAC_E_INVALID;
}
}
