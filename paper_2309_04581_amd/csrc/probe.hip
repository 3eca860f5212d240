// Random-gather ceiling of the memory level that holds a field's hash table:
// every lane loads table entries at pseudo-random positions, eight
// independent loads per round (as the eight corners of a level), so nothing
// coalesces and every load is a cache-line lookup.  The rate it reaches is the
// ceiling that the march's gather phase is compared against.
#include <algorithm>

#include "mr_common.h"
#include "mr_render.h"

using namespace mr;

namespace {

template <typename EntryT>
__global__ __launch_bounds__(256) void k_probe_gather(const EntryT* __restrict__ table, uint32_t mask, int rounds,
                                                      uint32_t seed, int per_die, uint32_t* __restrict__ sink) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  // per-lane linear congruential stream (Numerical Recipes constants), seeded by a mix of the lane id
  uint32_t x = (tid ^ seed) * 2654435761u + 0x9E3779B9u;
  // per_die: block b reads region b % 8 of size mask + 1 (workgroups go to the
  // eight dies in turn, so each die then reads a region of its own)
  const uint32_t base = per_die ? (blockIdx.x & 7u) * (mask + 1u) : 0u;
  uint32_t acc = 0;
  for (int i = 0; i < rounds; ++i) {
    uint32_t idx[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      x = x * 1664525u + 1013904223u;
      idx[c] = base + ((x >> 7) & mask);
    }
    EntryT v[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] = table[idx[c]];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc += reinterpret_cast<const uint32_t*>(&v[c])[0];
  }
  if (acc == 0x7FFFFFFFu) sink[0] = acc;   // keeps the loads; practically never taken
}

mr_status probe(const mr_field* f, int log2_region, bool per_die, int64_t n_loads, uint32_t seed, uint32_t* sink,
                float* ms_out, int64_t* loads_out, void* stream) {
  const uint32_t mask = (uint32_t)((1ull << log2_region) - 1u);
  hipStream_t st = (hipStream_t)stream;
  const int blocks = mr::device_cus() * 8;
  const int64_t lanes = (int64_t)blocks * 256;
  const int rounds = (int)std::max<int64_t>(1, n_loads / (lanes * 8));
  hipEvent_t a, b;
  MR_HIP(hipEventCreate(&a));
  MR_HIP(hipEventCreate(&b));
  MR_HIP(hipEventRecord(a, st));
  if (f->view.table_dtype == MR_F16)
    hipLaunchKernelGGL(k_probe_gather<uint32_t>, dim3(blocks), dim3(256), 0, st,
                       reinterpret_cast<const uint32_t*>(f->table_dev), mask, rounds, seed, per_die ? 1 : 0, sink);
  else
    hipLaunchKernelGGL(k_probe_gather<uint2>, dim3(blocks), dim3(256), 0, st,
                       reinterpret_cast<const uint2*>(f->table_dev), mask, rounds, seed, per_die ? 1 : 0, sink);
  MR_HIP(hipGetLastError());
  MR_HIP(hipEventRecord(b, st));
  MR_HIP(hipEventSynchronize(b));
  float ms = 0.0f;
  MR_HIP(hipEventElapsedTime(&ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *ms_out = ms;
  *loads_out = lanes * 8 * (int64_t)rounds;
  return MR_OK;
}

// log2 of the largest power of two of entries in the field's [L][T] table
int table_log2(const mr_field* f) {
  const int64_t entries = (int64_t)f->view.n_levels << f->view.log2_table;
  int lg = 0;
  while ((int64_t)2 << lg <= entries && lg < 31) ++lg;
  return lg;
}

}  // namespace

extern "C" mr_status mr_probe_gather(const mr_field* f, int64_t n_loads, uint32_t seed, uint32_t* sink,
                                     float* ms_out, int64_t* loads_out, void* stream) {
  if (!f || !sink || !ms_out || !loads_out) return mr::fail(MR_ERR_INVALID_ARG, "null field, sink or outputs");
  if (n_loads < 8) return mr::fail(MR_ERR_INVALID_ARG, "n_loads must be >= 8");
  if (f->view.feats != 2) return mr::fail(MR_ERR_UNSUPPORTED, "probe expects 2 features per level");
  // a power-of-two prefix of the table (all of it when n_levels is a power of two)
  return probe(f, table_log2(f), false, n_loads, seed, sink, ms_out, loads_out, stream);
}

extern "C" mr_status mr_probe_gather_region(const mr_field* f, int32_t log2_region, int32_t per_die, int64_t n_loads,
                                            uint32_t seed, uint32_t* sink, float* ms_out, int64_t* loads_out,
                                            void* stream) {
  if (!f || !sink || !ms_out || !loads_out) return mr::fail(MR_ERR_INVALID_ARG, "null field, sink or outputs");
  if (n_loads < 8) return mr::fail(MR_ERR_INVALID_ARG, "n_loads must be >= 8");
  if (f->view.feats != 2) return mr::fail(MR_ERR_UNSUPPORTED, "probe expects 2 features per level");
  const int lg = table_log2(f);
  if (log2_region < 8 || log2_region + (per_die ? 3 : 0) > lg)
    return mr::fail(MR_ERR_INVALID_ARG, "region outside the table (2^log2_region entries, 8 of them with per_die)");
  return probe(f, log2_region, per_die != 0, n_loads, seed, sink, ms_out, loads_out, stream);
}
