// Batched instances: placeholder until the batched kernel lands.
#include <hip/hip_runtime.h>
#include "../../include/ep.h"

extern "C" {
ep_status ep_batch_bind(ep_ctx*) { return EP_ERR_ORDER; }
ep_status ep_batch_add_instance(ep_ctx*, int64_t, const double*, int64_t, const int32_t*, ep_model, const double*, int,
                                double, int64_t, const int32_t*, int64_t, const int32_t*, const double*, int64_t,
                                const double*, const double*, int32_t*) { return EP_ERR_ORDER; }
ep_status ep_batch_set_state(ep_ctx*, int32_t, double, const double*, const double*) { return EP_ERR_ORDER; }
ep_status ep_batch_step(ep_ctx*, double, int64_t) { return EP_ERR_ORDER; }
ep_status ep_batch_get_state(ep_ctx*, int32_t, double*, double*, double*) { return EP_ERR_ORDER; }
ep_status ep_batch_get_stats(ep_ctx*, int32_t, int64_t*, int*, int*, double*) { return EP_ERR_ORDER; }
}
