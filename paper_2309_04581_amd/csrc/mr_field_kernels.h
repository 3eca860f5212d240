// Declarations shared by the field, march and proposal modules.
#pragma once
#include "mr_device.h"

namespace mr {
// matrix-core field query and march, and their weight fragments (march_mfma.hip)
std::vector<uint32_t> build_fragments(const mr_field_desc& d, const float* mlp, bool bf);
mr_status query_mfma(const mr_field* f, int64_t n, const float* x, const float* dirs, float* sigma, float* rgb,
                     float* feat, float* raw, hipStream_t st);
}  // namespace mr
