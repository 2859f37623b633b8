// Differentiation form: discrete adjoint of one implicit step.
#include "common.h"

isc_status isc_adjoint_impl(isc_ctx* ctx, const double*, const double*, double, const double*, double, double*,
                            double*, double*, isc_solve_info*) {
    ctx->err = "adjoint not available in this build";
    return ISC_ERR_ARG;
}
