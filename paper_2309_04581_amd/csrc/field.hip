// Radiance field: creation, point queries and the occupancy grid.
//
// The field is the hash grid + small MLP radiance field the paper embeds its
// meshes in (Sec. 3.3, an Instant-NGP model; colour emitted as linear HDR
// radiance per Sec. 3.1 "Unifying color space").
#include <cmath>
#include <cstring>
#include <vector>

#include "mr_device.h"
#include "mr_field_kernels.h"

using namespace mr;

namespace {

__global__ void k_f32_to_f16(const float* __restrict__ src, __half* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = __float2half_rn(src[i]);
}

uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// occupancy: one thread per cell, 8 density probes at the sub-cell centres
template <int NL, typename TabT>
__global__ __launch_bounds__(256) void k_occupancy(FieldView F, const TabT* __restrict__ table, int res,
                                                   float thresh, uint32_t* __restrict__ words,
                                                   uint8_t* __restrict__ bytes) {
  __shared__ __align__(16) float sW[2048 + 1024];
  for (int i = threadIdx.x; i < 2048 + 1024; i += blockDim.x) sW[i] = F.mlp[i];
  __syncthreads();
  const int64_t n = (int64_t)res * res * res;
  const int64_t nwave_cells = ((n + 63) / 64) * 64;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nwave_cells;
       c += (int64_t)gridDim.x * blockDim.x) {
    bool occ = false;
    if (c < n) {
      const int cx = (int)(c % res), cy = (int)((c / res) % res), cz = (int)(c / ((int64_t)res * res));
      float best = -INFINITY;
      for (int s = 0; s < 8; ++s) {
        const float xh = (cx + 0.25f + 0.5f * (s & 1)) / res;
        const float yh = (cy + 0.25f + 0.5f * ((s >> 1) & 1)) / res;
        const float zh = (cz + 0.25f + 0.5f * ((s >> 2) & 1)) / res;
        const float px = F.amin[0] + xh * (F.amax[0] - F.amin[0]);
        const float py = F.amin[1] + yh * (F.amax[1] - F.amin[1]);
        const float pz = F.amin[2] + zh * (F.amax[2] - F.amin[2]);
        float feat[32], raw[16];
        hash_encode<NL, TabT>(F, table, px, py, pz, feat);
        density_mlp<NL>(sW, feat, raw);
        best = fmaxf(best, softplusf(raw[0] + F.density_offset));
      }
      occ = best >= thresh;
      if (bytes) bytes[c] = occ ? 1 : 0;
    }
    // a wave covers 64 consecutive cells = two whole words
    const uint64_t m = __ballot(occ);
    const int lane = threadIdx.x & 63;
    const int64_t w0 = (c - lane) >> 5;
    if (lane == 0 && w0 * 32 < n) words[w0] = (uint32_t)m;
    if (lane == 1 && (w0 + 1) * 32 < n) words[w0 + 1] = (uint32_t)(m >> 32);
  }
}

template <int NL, typename TabT>
mr_status launch_occ(mr_field* f, int res, float thresh, uint8_t* bytes, hipStream_t st) {
  const int64_t n = (int64_t)res * res * res;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 16384);
  hipLaunchKernelGGL((k_occupancy<NL, TabT>), dim3(blocks), dim3(256), 0, st, f->view,
                     reinterpret_cast<const TabT*>(f->table_dev), res, thresh, f->occ_dev, bytes);
  MR_HIP(hipGetLastError());
  return MR_OK;
}

}  // namespace

namespace mr {

bool field_supported(const mr_field_desc& d, std::string& why) {
  if (d.color_hidden_layers == 0) {
    const int nin = d.n_levels * d.feats_per_level;
    if (d.density_out != 1 || d.density_hidden != 16 || d.density_in != nin || nin > 16 || d.n_levels != 5) {
      why = "proposal fields must be 5 levels x 2 features -> 16 -> 1";
      return false;
    }
    return true;
  }
  if (d.density_in != 32 || d.density_hidden != 64 || d.density_out != 16 || d.color_in != 32 ||
      d.color_hidden != 64) {
    why = "supported radiance fields: density 32->64->16, colour 32->64(->64)->3";
    return false;
  }
  if (!(d.n_levels == 8 || d.n_levels == 16)) {
    why = "supported level counts: 8 and 16";
    return false;
  }
  if (!march_layout(d.n_levels, d.sh_components, d.color_hidden_layers)) {
    why = "supported layouts (levels, SH components, colour hidden layers): (8, 4, 1), (16, 16, 2), (16, 4, 1), "
          "(8, 16, 2)";
    return false;
  }
  if (16 + d.sh_components > d.color_in) {
    why = "16 density outputs + SH components must fit color_in";
    return false;
  }
  return true;
}

}  // namespace mr

extern "C" mr_status mr_mlp_fragments(const mr_field_desc* desc, const float* host_mlp, int32_t bf16,
                                      uint32_t* out, int64_t capacity_words, int64_t* words) {
  if (!desc || !host_mlp || !words) return fail(MR_ERR_INVALID_ARG, "null argument");
  const mr_field_desc& d = *desc;
  if (d.color_hidden_layers < 1) return fail(MR_ERR_INVALID_ARG, "a radiance field (colour layers >= 1) has fragments");
  if (d.feats_per_level != 2) return fail(MR_ERR_UNSUPPORTED, "feats_per_level must be 2");
  std::string why;
  if (!field_supported(d, why)) return fail(MR_ERR_UNSUPPORTED, why);
  const std::vector<uint32_t> fr = build_fragments(d, host_mlp, bf16 != 0);
  *words = (int64_t)fr.size();
  if (!out) return MR_OK;
  if (capacity_words < (int64_t)fr.size()) return fail(MR_ERR_INVALID_ARG, "capacity below the fragment size");
  std::memcpy(out, fr.data(), fr.size() * sizeof(uint32_t));
  return MR_OK;
}

extern "C" mr_status mr_field_create(const mr_field_desc* desc, const float* host_table,
                                     const float* host_mlp, void* stream, mr_field** out) {
  if (!desc || !host_table || !host_mlp || !out) return fail(MR_ERR_INVALID_ARG, "null argument");
  const mr_field_desc& d = *desc;
  if (d.n_levels < 1 || d.n_levels > kMaxLevels) return fail(MR_ERR_INVALID_ARG, "n_levels must be in 1..16");
  if (d.feats_per_level != 2) return fail(MR_ERR_UNSUPPORTED, "feats_per_level must be 2");
  if (d.log2_table_size < 10 || d.log2_table_size > 24)
    return fail(MR_ERR_INVALID_ARG, "log2_table_size must be in 10..24");
  if (!d.host_resolutions) return fail(MR_ERR_INVALID_ARG, "null host_resolutions");
  for (int l = 0; l < d.n_levels; ++l)
    if (d.host_resolutions[l] < 1 || d.host_resolutions[l] > (1 << 20))
      return fail(MR_ERR_INVALID_ARG, "resolutions must be in 1..2^20");
  if (d.table_dtype != MR_F32 && d.table_dtype != MR_F16)
    return fail(MR_ERR_INVALID_ARG, "table_dtype must be MR_F32 or MR_F16");
  if (d.mlp_dtype != MR_F32 && d.mlp_dtype != MR_BF16)
    return fail(MR_ERR_INVALID_ARG, "mlp_dtype must be MR_F32 or MR_BF16");
  for (int k = 0; k < 3; ++k)
    if (!(d.aabb_max[k] > d.aabb_min[k]) || !std::isfinite(d.aabb_min[k]) || !std::isfinite(d.aabb_max[k]))
      return fail(MR_ERR_INVALID_ARG, "aabb_max must exceed aabb_min (finite)");
  if (!std::isfinite(d.density_offset)) return fail(MR_ERR_INVALID_ARG, "density_offset not finite");
  std::string why;
  if (!field_supported(d, why)) return fail(MR_ERR_UNSUPPORTED, why);

  const int64_t T = (int64_t)1 << d.log2_table_size;
  const int64_t n_table = (int64_t)d.n_levels * T * d.feats_per_level;
  int64_t n_mlp = (int64_t)d.density_hidden * d.density_in + (int64_t)d.density_out * d.density_hidden;
  if (d.color_hidden_layers > 0) {
    n_mlp += (int64_t)d.color_hidden * d.color_in;
    n_mlp += (int64_t)(d.color_hidden_layers - 1) * d.color_hidden * d.color_hidden;
    n_mlp += 3LL * d.color_hidden;
  }
  for (int64_t i = 0; i < n_mlp; ++i)
    if (!std::isfinite(host_mlp[i])) return fail(MR_ERR_INVALID_ARG, "non-finite MLP weight");
  for (int64_t i = 0; i < n_table; ++i)
    if (!std::isfinite(host_table[i])) return fail(MR_ERR_INVALID_ARG, "non-finite table entry");

  hipStream_t st = (hipStream_t)stream;
  mr_field* f = new mr_field();
  f->desc = d;
  f->n_table = n_table;
  f->n_mlp = n_mlp;
  for (int l = 0; l < d.n_levels; ++l) f->resolutions[l] = d.host_resolutions[l];
  f->desc.host_resolutions = nullptr;
  auto cleanup = [&](mr_status s, const std::string& m) {
    mr_field_destroy(f);
    return fail(s, m);
  };
  // FP32 MLP weights (padded to whole float4 rows) and their bf16 rounding
  const int64_t n_mlp_alloc = ((n_mlp + 3) / 4) * 4 + 4;
  if (hipMalloc(&f->mlp_dev, n_mlp_alloc * sizeof(float)) != hipSuccess) return cleanup(MR_ERR_OOM, "mlp alloc");
  if (hipMemsetAsync(f->mlp_dev, 0, n_mlp_alloc * sizeof(float), st) != hipSuccess)
    return cleanup(MR_ERR_DEVICE, "mlp memset");
  if (hipMemcpyAsync(f->mlp_dev, host_mlp, n_mlp * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess)
    return cleanup(MR_ERR_DEVICE, "mlp upload");
  std::vector<uint16_t> wb(n_mlp_alloc, 0);
  for (int64_t i = 0; i < n_mlp; ++i) wb[i] = bf16_rne(host_mlp[i]);
  if (hipMalloc(&f->mlp_bf16_dev, n_mlp_alloc * sizeof(uint16_t)) != hipSuccess)
    return cleanup(MR_ERR_OOM, "bf16 mlp alloc");
  if (hipMemcpyAsync(f->mlp_bf16_dev, wb.data(), n_mlp_alloc * sizeof(uint16_t), hipMemcpyHostToDevice, st) !=
      hipSuccess)
    return cleanup(MR_ERR_DEVICE, "bf16 upload");
  // table
  if (d.table_dtype == MR_F32) {
    if (hipMalloc(&f->table_dev, n_table * sizeof(float)) != hipSuccess) return cleanup(MR_ERR_OOM, "table alloc");
    if (hipMemcpyAsync(f->table_dev, host_table, n_table * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess)
      return cleanup(MR_ERR_DEVICE, "table upload");
  } else {
    float* tmp = nullptr;
    if (hipMalloc(&f->table_dev, n_table * sizeof(__half)) != hipSuccess) return cleanup(MR_ERR_OOM, "table alloc");
    if (hipMalloc(&tmp, n_table * sizeof(float)) != hipSuccess) return cleanup(MR_ERR_OOM, "staging alloc");
    bool ok = hipMemcpyAsync(tmp, host_table, n_table * sizeof(float), hipMemcpyHostToDevice, st) == hipSuccess;
    if (ok) {
      hipLaunchKernelGGL(k_f32_to_f16, dim3(1024), dim3(256), 0, st, tmp, (__half*)f->table_dev, n_table);
      ok = hipGetLastError() == hipSuccess && hipStreamSynchronize(st) == hipSuccess;
    }
    (void)hipFree(tmp);
    if (!ok) return cleanup(MR_ERR_DEVICE, "fp16 conversion");
  }
  if (d.color_hidden_layers == 0) {
    if (hipMalloc(&f->master_dev, n_table * sizeof(float)) != hipSuccess) return cleanup(MR_ERR_OOM, "master alloc");
    if (hipMemcpyAsync(f->master_dev, host_table, n_table * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return cleanup(MR_ERR_DEVICE, "master upload");
  }
  if (d.color_hidden_layers > 0) {
    for (int k = 0; k < 2; ++k) {
      const std::vector<uint32_t> fr = build_fragments(d, host_mlp, k == 1);
      uint32_t** dst = k == 0 ? &f->frag_f32_dev : &f->frag_bf16_dev;
      if (hipMalloc(dst, fr.size() * sizeof(uint32_t)) != hipSuccess) return cleanup(MR_ERR_OOM, "fragment alloc");
      if (hipMemcpyAsync(*dst, fr.data(), fr.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return cleanup(MR_ERR_DEVICE, "fragment upload");
    }
  }
  if (hipStreamSynchronize(st) != hipSuccess) return cleanup(MR_ERR_DEVICE, "upload sync");

  FieldView& v = f->view;
  std::memset(&v, 0, sizeof(v));
  v.n_levels = d.n_levels;
  v.feats = d.feats_per_level;
  v.log2_table = d.log2_table_size;
  v.table_mask = (uint32_t)(T - 1);
  v.dense_mask = 0;
  for (int l = 0; l < d.n_levels; ++l) {
    v.res[l] = d.host_resolutions[l];
    const int64_t n1 = (int64_t)v.res[l] + 1;
    if (n1 * n1 * n1 <= T) v.dense_mask |= 1u << l;
  }
  v.table = d.table_dtype == MR_F32 ? (const float*)f->table_dev : nullptr;
  v.table_h = d.table_dtype == MR_F16 ? (const __half*)f->table_dev : nullptr;
  v.mlp = f->mlp_dev;
  v.mlp_bf16 = f->mlp_bf16_dev;
  v.d_in = d.density_in;
  v.d_hidden = d.density_hidden;
  v.d_out = d.density_out;
  v.c_in = d.color_in;
  v.c_hidden = d.color_hidden;
  v.c_layers = d.color_hidden_layers;
  v.sh = d.sh_components;
  v.n_mlp = (int)n_mlp;
  v.density_offset = d.density_offset;
  for (int k = 0; k < 3; ++k) {
    v.amin[k] = d.aabb_min[k];
    v.amax[k] = d.aabb_max[k];
    v.inv_ext[k] = 1.0f / (d.aabb_max[k] - d.aabb_min[k]);
  }
  v.occ = nullptr;
  v.occ_res = 0;
  v.table_dtype = d.table_dtype;
  v.mlp_dtype = d.mlp_dtype;
  *out = f;
  return MR_OK;
}

extern "C" mr_status mr_field_destroy(mr_field* f) {
  if (!f) return MR_OK;
  if (f->table_dev) (void)hipFree(f->table_dev);
  if (f->mlp_dev) (void)hipFree(f->mlp_dev);
  if (f->mlp_bf16_dev) (void)hipFree(f->mlp_bf16_dev);
  if (f->occ_dev) (void)hipFree(f->occ_dev);
  if (f->frag_f32_dev) (void)hipFree(f->frag_f32_dev);
  if (f->frag_bf16_dev) (void)hipFree(f->frag_bf16_dev);
  if (f->master_dev) (void)hipFree(f->master_dev);
  if (f->opt_dev) (void)hipFree(f->opt_dev);
  delete f;
  return MR_OK;
}

extern "C" mr_status mr_field_params(mr_field* f, void** table, float** mlp, int64_t* n_table, int64_t* n_mlp) {
  if (!f) return fail(MR_ERR_INVALID_ARG, "null field");
  if (table) *table = f->table_dev;
  if (mlp) *mlp = f->mlp_dev;
  if (n_table) *n_table = f->n_table;
  if (n_mlp) *n_mlp = f->n_mlp;
  return MR_OK;
}

extern "C" mr_status mr_field_set_pose(mr_field* f, const float* host_pose) {
  if (!f) return fail(MR_ERR_INVALID_ARG, "null field");
  if (!host_pose) {
    f->view.has_pose = 0;
    return MR_OK;
  }
  double R[3][3];
  for (int i = 0; i < 3; ++i) {
    for (int k = 0; k < 3; ++k) R[i][k] = host_pose[4 * i + k];
    if (!std::isfinite(host_pose[4 * i + 3])) return fail(MR_ERR_INVALID_ARG, "pose translation not finite");
  }
  // R^T R = I within FP32 rounding, det R = +1
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double s = 0.0;
      for (int i = 0; i < 3; ++i) s += R[i][a] * R[i][b];
      if (!(std::fabs(s - (a == b ? 1.0 : 0.0)) <= 1e-5)) return fail(MR_ERR_INVALID_ARG, "pose rotation not orthonormal");
    }
  const double det = R[0][0] * (R[1][1] * R[2][2] - R[1][2] * R[2][1]) -
                     R[0][1] * (R[1][0] * R[2][2] - R[1][2] * R[2][0]) +
                     R[0][2] * (R[1][0] * R[2][1] - R[1][1] * R[2][0]);
  if (!(det > 0.0)) return fail(MR_ERR_INVALID_ARG, "pose rotation has determinant -1");
  for (int k = 0; k < 12; ++k) f->view.pose[k] = host_pose[k];
  f->view.has_pose = 1;
  return MR_OK;
}

extern "C" mr_status mr_field_query(const mr_field* f, int64_t n, const float* x, const float* dirs,
                                    float* sigma, float* rgb, float* feat, float* raw, void* stream) {
  if (!f) return fail(MR_ERR_INVALID_ARG, "null field");
  if (n < 0) return fail(MR_ERR_INVALID_ARG, "n < 0");
  if (n == 0) return MR_OK;
  if (!x || !sigma) return fail(MR_ERR_INVALID_ARG, "x and sigma are required");
  if (rgb && !dirs) return fail(MR_ERR_INVALID_ARG, "rgb needs dirs");
  if (f->view.c_layers == 0) return fail(MR_ERR_UNSUPPORTED, "use the proposal entry points for proposal fields");
  return query_mfma(f, n, x, dirs, sigma, rgb, feat, raw, (hipStream_t)stream);
}

extern "C" mr_status mr_field_build_occupancy(mr_field* f, int32_t res, float thresh, uint8_t* bits_out,
                                              void* stream) {
  if (!f) return fail(MR_ERR_INVALID_ARG, "null field");
  if (res < 1 || res > 512) return fail(MR_ERR_INVALID_ARG, "res must be in 1..512");
  if (!std::isfinite(thresh)) return fail(MR_ERR_INVALID_ARG, "thresh not finite");
  if (f->view.c_layers == 0) return fail(MR_ERR_UNSUPPORTED, "occupancy of a proposal field");
  const int64_t cells = (int64_t)res * res * res;
  const int64_t words = (cells + 31) / 32 + 2;
  if (f->occ_dev && f->occ_res != res) {
    (void)hipFree(f->occ_dev);
    f->occ_dev = nullptr;
  }
  if (!f->occ_dev) {
    if (hipMalloc(&f->occ_dev, words * sizeof(uint32_t)) != hipSuccess) return fail(MR_ERR_OOM, "occupancy alloc");
  }
  f->occ_res = res;
  hipStream_t st = (hipStream_t)stream;
  mr_status s;
  const bool h = f->view.table_dtype == MR_F16;
  if (f->view.n_levels == 8)
    s = h ? launch_occ<8, __half>(f, res, thresh, bits_out, st) : launch_occ<8, float>(f, res, thresh, bits_out, st);
  else
    s = h ? launch_occ<16, __half>(f, res, thresh, bits_out, st) : launch_occ<16, float>(f, res, thresh, bits_out, st);
  if (s != MR_OK) return s;
  f->view.occ = f->occ_dev;
  f->view.occ_res = res;
  return MR_OK;
}
