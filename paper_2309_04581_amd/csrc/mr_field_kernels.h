// Field point-query kernel (FP32 MLP path) shared by the field module.
#pragma once
#include "mr_device.h"

namespace mr {

// One point per thread; the block stages all MLP weights in LDS once.
template <int NL, int SH, int CL, typename TabT>
__global__ __launch_bounds__(256) void k_field_query(FieldView F, const TabT* __restrict__ table, int64_t n,
                                                     const float* __restrict__ x, const float* __restrict__ dirs,
                                                     float* __restrict__ sigma, float* __restrict__ rgb,
                                                     float* __restrict__ feat_out, float* __restrict__ raw_out) {
  __shared__ __align__(16) float sW[MlpLayout<CL>::TOTAL];
  for (int i = threadIdx.x; i < MlpLayout<CL>::TOTAL; i += blockDim.x) sW[i] = F.mlp[i];
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float px = x[3 * i], py = x[3 * i + 1], pz = x[3 * i + 2];
    float feat[32], raw[16];
    hash_encode<NL, TabT>(F, table, px, py, pz, feat);
    if (feat_out)
      for (int k = 0; k < 2 * NL; ++k) feat_out[i * 2 * NL + k] = feat[k];
    density_mlp<NL>(sW, feat, raw);
    sigma[i] = softplusf(raw[0] + F.density_offset);
    if (raw_out)
      for (int k = 0; k < 16; ++k) raw_out[i * 16 + k] = raw[k];
    if (rgb) {
      float c[3];
      color_mlp<SH, CL>(sW, raw, dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2], c);
      rgb[3 * i] = c[0];
      rgb[3 * i + 1] = c[1];
      rgb[3 * i + 2] = c[2];
    }
  }
}

}  // namespace mr

namespace mr {
// matrix-core field query and march, and their weight fragments (march_mfma.hip)
std::vector<uint32_t> build_fragments(const mr_field_desc& d, const float* mlp, bool bf);
mr_status query_mfma(const mr_field* f, int64_t n, const float* x, const float* dirs, float* sigma, float* rgb,
                     float* feat, float* raw, hipStream_t st);
}  // namespace mr
