// mmoc_mlp.cpp -- learned flow-map surrogate (placeholder until its kernels land).
#include <hip/hip_runtime.h>

#include "../../include/mmoc.h"
#include "mmoc_internal.h"

void mmoc_mlp_free_state(mmoc_ctx*) {}

extern "C" {
int64_t mmoc_mlp_nparams(void) { return 4 * 64 + 64 + 2 * (64 * 64 + 64) + 64 * 3 + 3; }
mmoc_status mmoc_mlp_configure(mmoc_ctx*, const double*, const double*, double) { return MMOC_E_UNSUPPORTED; }
mmoc_status mmoc_mlp_record(mmoc_ctx*, double, double, const double*, int64_t) { return MMOC_E_UNSUPPORTED; }
mmoc_status mmoc_mlp_train(mmoc_ctx*, int64_t, int, int, float, unsigned long long, double*) { return MMOC_E_UNSUPPORTED; }
mmoc_status mmoc_mlp_get_weights(mmoc_ctx*, float*, int64_t) { return MMOC_E_UNSUPPORTED; }
mmoc_status mmoc_mlp_set_weights(mmoc_ctx*, const float*, int64_t) { return MMOC_E_UNSUPPORTED; }
mmoc_status mmoc_mlp_infer(mmoc_ctx*, double, double, double*) { return MMOC_E_UNSUPPORTED; }
mmoc_status mmoc_trace_step_surrogate(mmoc_ctx*, double, double, int, float, double, int64_t, void*, double*)
{
    return MMOC_E_UNSUPPORTED;
}
}
