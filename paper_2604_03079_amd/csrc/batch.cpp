// Batches of circuits and the adjoint entry points.
#include "colorstamp.h"
#include "internal.hpp"

using namespace cs;

extern "C" {

cs_status cs_vjp(cs_circuit *, const double *, double, const double *, const double *,
                 const double *, double *, double *, double *, void *) {
    set_error("cs_vjp: not built yet");
    return CS_ENOTSUP;
}

cs_status cs_batch_create(int32_t, cs_circuit *const *, cs_batch **out) {
    if (out) *out = nullptr;
    set_error("batches: not built yet");
    return CS_ENOTSUP;
}
void cs_batch_destroy(cs_batch *b) { delete b; }
cs_status cs_batch_layout(const cs_batch *, int64_t *, int64_t *, int64_t *) { return CS_ENOTSUP; }
cs_status cs_batch_set_params(cs_batch *, const double *, const double *, const double *, void *) {
    return CS_ENOTSUP;
}
cs_status cs_batch_set_launch(cs_batch *, int32_t, int32_t, int32_t) { return CS_ENOTSUP; }
cs_status cs_batch_get_info(const cs_batch *, int64_t *, int64_t *, int64_t *, int32_t *, int32_t *,
                            int32_t *, int32_t *, int32_t *) {
    return CS_ENOTSUP;
}
cs_status cs_batch_eval_stamp(cs_batch *, const double *, double, const double *, double *, double *,
                              void *) {
    return CS_ENOTSUP;
}
cs_status cs_batch_vjp(cs_batch *, const double *, double, const double *, const double *,
                       const double *, double *, double *, double *, void *) {
    return CS_ENOTSUP;
}
cs_status cs_batch_check(cs_batch *, void *) { return CS_ENOTSUP; }

}  // extern "C"
