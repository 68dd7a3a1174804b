// Temporary: entry points whose kernels are not in this build yet.
#include "cqk_internal.h"
namespace cqk {
cqk_status run_simplex_f32(cqk_ctx*, int64_t, const float*, double, float*, bool, const cqk_opts&, cqk_info*) { return CQK_DEVICE_ERROR; }
cqk_status run_simplex_f64(cqk_ctx*, int64_t, const double*, double, double*, bool, const cqk_opts&, cqk_info*) { return CQK_DEVICE_ERROR; }
cqk_status run_batched_f32(cqk_ctx*, int32_t, const int64_t*, const float*, const double*, double, float*, double*, int32_t*, const cqk_opts&, cqk_info*) { return CQK_DEVICE_ERROR; }
cqk_status run_batched_backward_f32(cqk_ctx*, int32_t, const int64_t*, const float*, const float*, float*, double*, const cqk_opts&) { return CQK_DEVICE_ERROR; }
}
