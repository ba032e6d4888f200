// net.hip -- learned PCG warm start (placeholder entry points until the kernels land).
#include "bsc_internal.h"

using namespace bsc;

extern "C" {

bsc_status bsc_warmstart_load(bsc_ctx *c, const float *, int32_t) { return fail(c, BSC_E_INVAL, "warm start not available"); }
bsc_status bsc_net_forward(bsc_ctx *c, int32_t, const float *, const float *, float *, float *) { return fail(c, BSC_E_INVAL, "not available"); }
bsc_status bsc_net_backward(bsc_ctx *c, int32_t, const float *, const float *, const float *, const float *, float *, float *, void *) { return fail(c, BSC_E_INVAL, "not available"); }
bsc_status bsc_net_scratch_size(const bsc_ctx *, int32_t, size_t *b) { if (b) *b = 0; return BSC_E_INVAL; }
bsc_status bsc_adam_step(bsc_ctx *c, int32_t, float *, const float *, float *, float *, float, float, float, float, int32_t) { return fail(c, BSC_E_INVAL, "not available"); }
bsc_status bsc_net_loss(bsc_ctx *c, int32_t, const float *, const float *, float *, float *) { return fail(c, BSC_E_INVAL, "not available"); }

}
