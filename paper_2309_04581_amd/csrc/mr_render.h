// Ray queues and launch parameters of the render path.
#pragma once
#include "mr_common.h"

namespace mr {

constexpr int kQueueArrays = 16;       // 4-byte arrays per queue slot
constexpr size_t kHeaderBytes = 4096;  // counters at the start of the workspace
constexpr int kMaxBounces = 60;
constexpr int kMaxCamsPerLaunch = 16;

// Structure-of-arrays ray queue: one slot per live ray.
struct RayQueue {
  float *ox, *oy, *oz, *dx, *dy, *dz;  // origin, unit direction
  float *tr, *tg, *tb;                 // path throughput T
  float *lr, *lg, *lb;                 // accumulated radiance L
  int* rid;                            // caller's ray index
  int* depth;                          // segment index (= scatter count) | max bounces << 16
  float* hit_t;                        // closest hit distance of the current segment
  int* hit_p;                          // hit primitive (leaf order), -1 = miss
};

struct MarchParams {
  float t_near, span, delta;
  int n_samples;
  int use_occupancy;
};

struct ShadeParams {
  int n_lights;
  float lights[kMaxLights][6];
  uint32_t seed;
  int rr_after;
  float t_min;
};

struct RenderOut {
  float* radiance;
  float* throughput;
  int32_t* bounces;
};

size_t queue_bytes(int64_t cap);
RayQueue queue_at(void* base, int64_t cap);
int device_cus();

// matrix-core march (march_mfma.hip)
mr_status dispatch_march_mfma(const mr_field* f, RayQueue q, const int* count, int* work, const MarchParams& P,
                              unsigned long long* stats, int blocks, hipStream_t st);

// proposal-sampled march (defined with the proposal kernels)
mr_status dispatch_march_proposal(const mr_field* f, const mr_field* prop, RayQueue q, const int* count, int* work,
                                  const MarchParams& P, int n_prop, int n_fine, unsigned long long* stats, int blocks,
                                  hipStream_t st);

}  // namespace mr
