// Batched launches (not yet implemented in this build).
#include "swc_internal.h"

extern "C" {

struct swc_batch_plan {
    int dummy;
};

swc_status swc_batch_plan_create(int32_t n, const swc_problem* p, const void* const* x,
                                 const void* const* y, float* const* c, uint8_t* const* flags,
                                 const swc_launch_params* lp, swc_batch_plan** out)
{
    (void)n; (void)p; (void)x; (void)y; (void)c; (void)flags; (void)lp;
    if (!out) return SWC_ERR_NULL;
    *out = nullptr;
    return SWC_ERR_UNSUPPORTED;
}

swc_status swc_batch_launch(const swc_batch_plan* plan, void* stream)
{
    (void)stream;
    return plan ? SWC_ERR_UNSUPPORTED : SWC_ERR_NULL;
}

int64_t swc_batch_plan_items(const swc_batch_plan* plan) { (void)plan; return 0; }

void swc_batch_plan_destroy(swc_batch_plan* plan) { (void)plan; }

}
