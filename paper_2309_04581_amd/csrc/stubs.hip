// Entry points whose kernels are not built yet.
#include "mr_field_kernels.h"
#include "mr_render.h"

using namespace mr;

mr_status mr_field_query_bf16(const mr_field*, int64_t, const float*, const float*, float*, float*, float*, float*,
                              void*) {
  return fail(MR_ERR_UNSUPPORTED, "bf16 MLP path not built");
}

namespace mr {
mr_status dispatch_march_proposal(const mr_field*, const mr_field*, RayQueue, const int*, int*, const MarchParams&, int,
                                  int, unsigned long long*, int, hipStream_t) {
  return fail(MR_ERR_UNSUPPORTED, "proposal sampler not built");
}
}  // namespace mr
