// Ray queues and launch parameters of the render path.
#pragma once
#include "mr_common.h"
#include "mr_device.h"

namespace mr {

constexpr int kQueueArrays = 16;       // 4-byte arrays per queue slot
constexpr size_t kHeaderBytes = 4096;  // counters at the start of the workspace
constexpr int kMaxBounces = 60;
constexpr int kMaxCamsPerLaunch = 16;
constexpr int kMaxFields = 8;          // fields marched together by mr_render_fields

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
  int batch;          // queue positions a wave takes per atomic
  // shadow mask per field sample: each light a mesh hides from the sample
  // multiplies its emitted radiance by shadow_mask
  int shadows;
  float shadow_mask;
  int n_lights;
  float light_pos[kMaxLights][3];
  // producer/consumer packet march: polls each wait takes at most, and the
  // device word that counts the waves whose wait gave up (their packets'
  // rays are then left without this segment's medium)
  int wait_polls;
  int* gave_up;
};

// Shadow mask of the sample of column j (Sec. 3.1 "Shadow rays"): a lane of
// group 0 sends a ray from the sample's world position to every light, and
// each light a mesh hides multiplies the mask by P.shadow_mask; every lane
// returns its column's mask.  stack: that lane's LDS stack, stride 16.
// This form takes the sample's world position; sample_shadow below takes a
// point in the frame of field F.
__device__ __forceinline__ float sample_shadow_world(const BvhView& B, const MarchParams& P, bool valid, float px,
                                                     float py, float pz, int lane, int* stack) {
  float m = 1.0f;
  if (lane < 16 && valid) {
    for (int li = 0; li < P.n_lights; ++li) {
      const float sx = P.light_pos[li][0] - px, sy = P.light_pos[li][1] - py, sz = P.light_pos[li][2] - pz;
      const float dist = sqrtf(sx * sx + sy * sy + sz * sz);
      const RayPre sr = ray_pre(v3(px, py, pz), v3(sx / dist, sy / dist, sz / dist));
      float th;
      if (bvh_trace<true>(B, sr, dist, th, stack, nullptr, 16) >= 0) m *= P.shadow_mask;
    }
  }
  return __shfl(m, lane & 15, 64);
}

__device__ __forceinline__ float sample_shadow(const FieldView& F, const BvhView& B, const MarchParams& P,
                                               bool valid, float px, float py, float pz, int lane, int* stack) {
  if (lane < 16 && valid) field_to_world(F, px, py, pz);
  return sample_shadow_world(B, P, valid, px, py, pz, lane, stack);
}

struct ShadeParams {
  int n_lights;
  float lights[kMaxLights][6];
  uint32_t seed;
  int rr_after;
  float t_min;
  int sample_emitters;   // light sampling toward the mesh's emitting triangles
};

// The medium a light sample's shadow segment crosses (light sampling toward
// emitters): the fields of the render and the spacing of the march's grid.
struct ShadowMedium {
  int n;                        // fields (0: the light sample sees no medium)
  float delta;                  // grid spacing (t_far - t_near) / n_samples
  int use_occupancy;
  FieldView f[kMaxFields];
};

// Ray queue depth word: bits 0-15 segment index (= scatter count so far),
// bits 16-23 the ray's bounce limit, bit 24 set when the last scatter was
// diffuse.
constexpr int kDepthAfterDiffuse = 1 << 24;

struct RenderOut {
  float* radiance;
  float* throughput;
  int32_t* bounces;
};

constexpr int kXcds = 8;               // accelerator complex dies; workgroups go round-robin over them

// Ray work queue of the persistent march kernels.  chunk == 0: one queue for
// the whole device.  chunk > 0: the rays [0, cnt) are cut into chunks of
// `chunk` rays dealt round-robin to the kXcds dies; the waves of workgroups on
// die x = blockIdx.x % kXcds take the rays of die x's chunks in order
// (neighbouring rays then share that die's L2), then help the other dies.
// A wave takes `batch` queue positions per atomic, when it needs them: taking
// them any earlier widens the window of rays in flight, and the march is
// fastest when neighbouring rays are marched at the same time (they share
// cache lines of the hash table).  ctr: kXcds counters, zero at launch.
struct WorkQueue {
  int* ctr;
  int cnt, chunk, batch, die, tries;
  __device__ __forceinline__ WorkQueue(int* c, int n, int ch, int b)
      : ctr(c), cnt(n), chunk(ch), batch(b > 0 ? b : 1), die(ch > 0 ? (int)(blockIdx.x % kXcds) : 0), tries(0) {}
  __device__ __forceinline__ int map(int i) const {
    if (chunk <= 0) return i;
    const int64_t r = ((int64_t)(i / chunk) * kXcds + die) * chunk + i % chunk;
    return r < cnt ? (int)r : cnt;
  }
  // Start of the wave's next batch in queue positions of `die`, or -1 when
  // every ray has been taken.
  __device__ __forceinline__ int next(int lane) {
    while (true) {
      int v = 0;
      if (lane == 0) v = atomicAdd(ctr + die, batch);
      const int base = __shfl(v, 0, 64);
      if (map(base) < cnt) return base;
      if (chunk <= 0 || ++tries >= kXcds) return -1;
      die = (die + 1) % kXcds;
    }
  }
};

size_t queue_bytes(int64_t cap);
RayQueue queue_at(void* base, int64_t cap);
int device_cus();

// Blocks of a persistent grid of `kernel` (blocks of `threads`): `per_cu`
// per compute unit, or, for per_cu = 0, as many as are resident at once by
// the occupancy calculator (queried once per kernel); at least kXcds and at
// most `cap`.
int persistent_blocks(const void* kernel, int threads, int per_cu, int64_t cap);

// matrix-core march (march_mfma.hip)
// packets: 16 consecutive queue rays per wave in step (else one ray per wave);
// blocks_per_cu: 0 = as many as fit; n: rays in the queue at most
mr_status dispatch_march_mfma(const mr_field* f, RayQueue q, const int* count, int* work, const MarchParams& P,
                              const BvhView& B, bool packets, unsigned long long* stats, int blocks_per_cu, int64_t n,
                              hipStream_t st);

// march of several fields, overlapping or not, over their summed medium
// (march_fields.hip) on the uniform grid; the fields share one layout
// (levels, SH components, colour layers, table and MLP types).  packets: 16
// consecutive queue rays per wave in step (else one ray per wave)
mr_status dispatch_march_fields(const mr_field* const* fields, int n_fields, RayQueue q, const int* count, int* work,
                                const MarchParams& P, const BvhView& B, bool packets, unsigned long long* stats,
                                int blocks_per_cu, int64_t n, hipStream_t st);

// proposal-sampled march (defined with the proposal kernels)
// packets: 16 consecutive queue rays per wave when n_prop = 32 and n_fine <= 32
mr_status dispatch_march_proposal(const mr_field* f, const mr_field* prop, RayQueue q, const int* count, int* work,
                                  const MarchParams& P, const BvhView& B, int n_prop, int n_fine, bool packets,
                                  unsigned long long* stats, int blocks_per_cu, int64_t n, hipStream_t st);

}  // namespace mr
