// Entry points still under construction: the autotuner.
#include "handle.h"


extern "C" {
jac_status jac_autotune(jac_handle, int32_t)
{
    jac::set_last_error("jac_autotune is not available in this build");
    return JAC_E_INVALID;
}
}
