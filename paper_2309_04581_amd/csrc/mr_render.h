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
  int chunk;          // rays per die chunk of the march queue (0 = one global queue)
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

constexpr int kXcds = 8;               // accelerator complex dies; workgroups go round-robin over them

// Next ray for a wave.  chunk == 0: one queue for the whole device.  chunk > 0:
// the queue [0, cnt) is cut into chunks of `chunk` rays dealt round-robin to
// the kXcds dies; the waves of workgroups on die x = blockIdx.x % kXcds take
// the rays of die x's chunks in order (neighbouring rays then share that die's
// L2), then help the other dies.  ctr: kXcds counters, zero at launch.
// Returns -1 when every ray has been taken.
__device__ __forceinline__ int next_ray(int* __restrict__ ctr, int cnt, int chunk, int lane) {
  int r = -1;
  if (lane == 0) {
    if (chunk <= 0) {
      const int i = atomicAdd(ctr, 1);
      r = i < cnt ? i : -1;
    } else {
      const int home = blockIdx.x % kXcds;
      for (int k = 0; k < kXcds && r < 0; ++k) {
        const int x = (home + k) % kXcds;
        const int c0 = __hip_atomic_load(ctr + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (((int64_t)(c0 / chunk) * kXcds + x) * chunk + c0 % chunk >= cnt) continue;
        const int i = atomicAdd(ctr + x, 1);
        const int64_t ray = ((int64_t)(i / chunk) * kXcds + x) * chunk + i % chunk;
        if (ray < cnt) r = (int)ray;
      }
    }
  }
  return __shfl(r, 0, 64);
}

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
