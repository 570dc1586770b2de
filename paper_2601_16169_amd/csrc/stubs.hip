// Entry points of subsystems that are not built yet.
#include "sqd_internal.h"
int sqd_sigma_ab_kh(sqd_ctx* ctx, sqd_space*, const void*, void*, int, const int*) {
    return sqd_fail(ctx, SQD_E_STATE, "KH path not available");
}
int sqd_rdm_impl(sqd_ctx* ctx, sqd_space*, const double*, double*, double*) {
    return sqd_fail(ctx, SQD_E_STATE, "not available");
}
int sqd_davidson_batched_impl(sqd_ctx* ctx, int, sqd_space* const*, const sqd_davidson_opts*, double*, double* const*,
                              sqd_report*) {
    return sqd_fail(ctx, SQD_E_STATE, "not available");
}
