// Segment march and point queries with the field MLPs on the matrix cores.
//
// Quadrature of Eq. 10-11 (alpha compositing of midpoint samples on the
// fixed interval grid, Eq. 8-9).  Each lane gathers the hash features of one
// level group for one sample (mr_mfma.h) and the density and colour MLPs run
// as 16x16 MFMA tiles (FP32 as exact BF16 splits, or BF16; FP32 accumulation) whose 16 columns
// are 16 samples.  Two ways to fill the columns:
//   packets  - a wave takes 16 consecutive queue rays and steps them through
//              the same sample index together (column j = ray j); neighbouring
//              camera pixels then read the same cache lines of the table at
//              every level, and compositing is a running product per column;
//   per ray  - a wave takes one ray and 16 consecutive samples of it per tile
//              (column j = sample j), composited by a 16-lane prefix product
//              carried from tile to tile; better for incoherent bounce rays
//              and for short queues, where one ray's samples would otherwise
//              be walked one at a time.
#include <cstring>
#include <vector>

#include "mr_field_kernels.h"
#include "mr_mfma.h"
#include "mr_render.h"

using namespace mr;

namespace {

// A ray's segment in the field: origin and direction in the field frame,
// the range [lo, hi] it marches and the sample indices k0 .. k1 that cover it.
struct RaySeg {
  float ox, oy, oz, dx, dy, dz, t_a, lo, hi;
  int k0, k1;
};

__device__ __forceinline__ bool ray_seg(const RayQueue& q, int r, const FieldView& F, const MarchParams& P,
                                        RaySeg& S) {
  S.ox = q.ox[r]; S.oy = q.oy[r]; S.oz = q.oz[r];
  S.dx = q.dx[r]; S.dy = q.dy[r]; S.dz = q.dz[r];
  to_field_frame(F, S.ox, S.oy, S.oz, S.dx, S.dy, S.dz);
  S.t_a = (q.depth[r] & 0xFFFF) == 0 ? P.t_near : 0.0f;
  float box0, box1;
  if (!slab_box(F, S.ox, S.oy, S.oz, S.dx, S.dy, S.dz, box0, box1)) return false;
  S.lo = fmaxf(S.t_a, box0);
  S.hi = fminf(fminf(S.t_a + P.span, q.hit_t[r]), box1);
  if (!(S.hi > S.lo)) return false;
  S.k0 = max(0, (int)floorf((S.lo - S.t_a) / P.delta) - 1);
  S.k1 = min(P.n_samples, (int)ceilf((S.hi - S.t_a) / P.delta) + 1);
  return true;
}

// Samples kb0 .. kb1 - 1 of the segment, one wave: lane j takes sample kb + j
// of each 16-sample tile, and transmittance is a 16-lane prefix product
// carried from tile to tile in Tseg (radiance in acc, both per wave).
template <int NL, int SH, int CL, typename TabT, bool BF, bool SHADOW>
__device__ __forceinline__ void march_tiles(const RaySeg& S, int kb0, int kb1, const FieldView& F,
                                            const TabT* __restrict__ table, const uint32_t* __restrict__ sW,
                                            const MarchParams& P, const BvhView& B, int* sstack, bool use_occ,
                                            int lane, const float (&u)[4][4], float& Tseg, float& acc0, float& acc1,
                                            float& acc2, unsigned long long& nsamp) {
  using LY = FragLayout<NL, SH, CL, BF>;
  const int g = lane >> 4, j = lane & 15;
  const float delta = P.delta;
  for (int kb = kb0; kb < kb1; kb += 16) {
    const int k = kb + j;
    const float a = fmaxf(S.t_a + (float)k * delta, S.lo);
    const float b = fminf(S.t_a + (float)(k + 1) * delta, S.hi);
    bool valid = k < kb1 && b > a;
    const float tm = 0.5f * (a + b), D = b - a;
    const float px = S.ox + tm * S.dx, py = S.oy + tm * S.dy, pz = S.oz + tm * S.dz;
    if (valid && use_occ) valid = occ_lookup(F, px, py, pz);
    if (__ballot(valid) == 0ull) continue;
    float fe[LY::NF];
    encode_group<NL, TabT>(F, table, px, py, pz, g, fe);
    float sigma, rgb[3];
    f4v raw;
    mlp_tile<NL, SH, CL, BF>(sW, fe, u, F.density_offset, lane, sigma, rgb, raw);
    const float alpha = valid ? -expm1f(-sigma * D) : 0.0f;
    const float incl = scan16_mul(1.0f - alpha, j);
    float excl = __shfl_up(incl, 1, 16);
    if (j == 0) excl = 1.0f;
    float msk = 1.0f;
    if constexpr (SHADOW) msk = sample_shadow(F, B, P, valid, px, py, pz, lane, sstack);
    const float w = Tseg * excl * alpha * msk;
    acc0 += w * rgb[0];
    acc1 += w * rgb[1];
    acc2 += w * rgb[2];
    Tseg *= __shfl(incl, 15, 16);
    if (g == 0 && valid) ++nsamp;
  }
}

__device__ __forceinline__ void ray_update(const RayQueue& q, int r, float T, float l0, float l1, float l2) {
  const float tr = q.tr[r], tg = q.tg[r], tb = q.tb[r];
  q.lr[r] += tr * l0;
  q.lg[r] += tg * l1;
  q.lb[r] += tb * l2;
  q.tr[r] = tr * T;
  q.tg[r] = tg * T;
  q.tb[r] = tb * T;
}

// One ray per wave, all of its tiles in order.
template <int NL, int SH, int CL, typename TabT, bool BF, bool SHADOW>
__device__ __forceinline__ void march_ray(const RayQueue& q, int r, const FieldView& F, const TabT* __restrict__ table,
                                          const uint32_t* __restrict__ sW, const MarchParams& P, const BvhView& B,
                                          int* sstack, bool use_occ, int lane, unsigned long long& nsamp) {
  RaySeg S;
  if (!ray_seg(q, r, F, P, S)) return;
  float u[4][4];
  sh_rows<NL, SH, CL, BF>(sW, S.dx, S.dy, S.dz, lane, u);
  float Tseg = 1.0f, acc0 = 0.0f, acc1 = 0.0f, acc2 = 0.0f;
  march_tiles<NL, SH, CL, TabT, BF, SHADOW>(S, S.k0, S.k1, F, table, sW, P, B, sstack, use_occ, lane, u, Tseg, acc0,
                                            acc1, acc2, nsamp);
  acc0 = sum16(acc0);
  acc1 = sum16(acc1);
  acc2 = sum16(acc2);
  if (lane == 0) ray_update(q, r, Tseg, acc0, acc1, acc2);
}

// Short queues: one ray per block of four waves, each wave marching a
// contiguous quarter of the ray's tiles from transmittance 1; the quarters are
// chained in order at the end (L = L0 + T0 L1 + T0 T1 L2 + ..., T = T0 T1 T2
// T3).  Then the longest ray no longer sets the launch's duration alone.  The
// same samples and arithmetic up to the association of the transmittance
// products (a few ulp).
template <int NL, int SH, int CL, typename TabT, bool BF>
__device__ __forceinline__ void march_ray_split(const RayQueue& q, int r, const FieldView& F,
                                                const TabT* __restrict__ table, const uint32_t* __restrict__ sW,
                                                const MarchParams& P, const BvhView& B, bool use_occ, int lane,
                                                int wave, float (*part)[4], unsigned long long& nsamp) {
  RaySeg S;
  const bool live = ray_seg(q, r, F, P, S);   // the same for the whole block
  float Tseg = 1.0f, acc0 = 0.0f, acc1 = 0.0f, acc2 = 0.0f;
  if (live) {
    float u[4][4];
    sh_rows<NL, SH, CL, BF>(sW, S.dx, S.dy, S.dz, lane, u);
    const int ntiles = (S.k1 - S.k0 + 15) / 16, per = (ntiles + 3) / 4;
    const int kb0 = S.k0 + 16 * per * wave, kb1 = min(S.k1, S.k0 + 16 * per * (wave + 1));
    march_tiles<NL, SH, CL, TabT, BF, false>(S, kb0, kb1, F, table, sW, P, B, nullptr, use_occ, lane, u, Tseg, acc0,
                                             acc1, acc2, nsamp);
  }
  acc0 = sum16(acc0);
  acc1 = sum16(acc1);
  acc2 = sum16(acc2);
  if (lane == 0) {
    part[wave][0] = Tseg;
    part[wave][1] = acc0;
    part[wave][2] = acc1;
    part[wave][3] = acc2;
  }
  __syncthreads();
  if (live && threadIdx.x == 0) {
    float T = 1.0f, l0 = 0.0f, l1 = 0.0f, l2 = 0.0f;
    for (int w = 0; w < 4; ++w) {
      l0 += T * part[w][1];
      l1 += T * part[w][2];
      l2 += T * part[w][3];
      T *= part[w][0];
    }
    ray_update(q, r, T, l0, l1, l2);
  }
  __syncthreads();
}

// Column j's ray of a 16-ray packet (every lane group holds the same 16).
struct PacketRay {
  float ox, oy, oz, dx, dy, dz;
  int r;
  bool live;   // a ray in the queue
};

__device__ __forceinline__ PacketRay packet_ray(const RayQueue& q, int r, int cnt, const FieldView& F) {
  PacketRay R;
  R.r = r;
  R.live = r < cnt;
  R.ox = R.oy = R.oz = R.dx = R.dy = 0.0f;
  R.dz = 1.0f;
  if (R.live) {
    R.ox = q.ox[r]; R.oy = q.oy[r]; R.oz = q.oz[r];
    R.dx = q.dx[r]; R.dy = q.dy[r]; R.dz = q.dz[r];
    to_field_frame(F, R.ox, R.oy, R.oz, R.dx, R.dy, R.dz);
  }
  return R;
}

// A packet of 16 rays stepped through the same sample index together:
// column j of every tile is ray j at sample k, composited by a running
// product per column.
template <int NL, int SH, int CL, typename TabT, bool BF, bool SHADOW>
__device__ __forceinline__ void march_packet(const RayQueue& q, const PacketRay& R, const FieldView& F,
                                             const TabT* __restrict__ table, const uint32_t* __restrict__ sW,
                                             const MarchParams& P, const BvhView& B, int* sstack, bool use_occ,
                                             int lane, unsigned long long& nsamp) {
  using LY = FragLayout<NL, SH, CL, BF>;
  const int g = lane >> 4;
  const float delta = P.delta;
  const float ox = R.ox, oy = R.oy, oz = R.oz, dx = R.dx, dy = R.dy, dz = R.dz;
  const int r = R.r;
  bool live = R.live;
  float t_a = 0.0f, lo = 0.0f, hi = 0.0f;
  int k0 = P.n_samples, k1 = 0;
  if (live) {
    t_a = (q.depth[r] & 0xFFFF) == 0 ? P.t_near : 0.0f;
    float box0, box1;
    live = slab_box(F, ox, oy, oz, dx, dy, dz, box0, box1);
    if (live) {
      lo = fmaxf(t_a, box0);
      hi = fminf(fminf(t_a + P.span, q.hit_t[r]), box1);
      live = hi > lo;
    }
    if (live) {
      k0 = max(0, (int)floorf((lo - t_a) / delta) - 1);
      k1 = min(P.n_samples, (int)ceilf((hi - t_a) / delta) + 1);
    }
  }
  int kmin = k0, kmax = k1;
#pragma unroll
  for (int off = 1; off < 16; off <<= 1) {
    kmin = min(kmin, __shfl_xor(kmin, off, 16));
    kmax = max(kmax, __shfl_xor(kmax, off, 16));
  }
  if (kmin >= kmax) return;
  float u[4][4];
  sh_rows<NL, SH, CL, BF>(sW, dx, dy, dz, lane, u);
  float T = 1.0f, acc0 = 0.0f, acc1 = 0.0f, acc2 = 0.0f;
  for (int k = kmin; k < kmax; ++k) {
    const float a = fmaxf(t_a + (float)k * delta, lo);
    const float b = fminf(t_a + (float)(k + 1) * delta, hi);
    bool valid = live && k >= k0 && k < k1 && b > a;
    const float tm = 0.5f * (a + b), D = b - a;
    const float px = ox + tm * dx, py = oy + tm * dy, pz = oz + tm * dz;
    if (valid && use_occ) valid = occ_lookup(F, px, py, pz);
    if (__ballot(valid) == 0ull) continue;
    float fe[LY::NF];
    encode_group<NL, TabT>(F, table, px, py, pz, g, fe);
    float sigma, rgb[3];
    f4v raw;
    mlp_tile<NL, SH, CL, BF>(sW, fe, u, F.density_offset, lane, sigma, rgb, raw);
    const float alpha = valid ? -expm1f(-sigma * D) : 0.0f;
    float msk = 1.0f;
    if constexpr (SHADOW) msk = sample_shadow(F, B, P, valid, px, py, pz, lane, sstack);
    const float w = T * alpha * msk;
    acc0 += w * rgb[0];
    acc1 += w * rgb[1];
    acc2 += w * rgb[2];
    T *= 1.0f - alpha;
    if (g == 0 && valid) ++nsamp;
  }
  if (live && g == 0) {
    const float tr = q.tr[r], tg = q.tg[r], tb = q.tb[r];
    q.lr[r] += tr * acc0;
    q.lg[r] += tg * acc1;
    q.lb[r] += tb * acc2;
    q.tr[r] = tr * T;
    q.tg[r] = tg * T;
    q.tb[r] = tb * T;
  }
}

// PK: 16-ray packets (march_packet), else one ray per wave (march_ray).
// SHADOW: the shadow mask per field sample (instances without it carry none
// of its code or registers).
// At most this many rays per block: the per-ray march splits each ray over
// the four waves of a block instead of taking one ray per wave.
constexpr int kSplitRaysPerBlock = 8;

template <int NL, int SH, int CL, typename TabT, bool BF, bool PK, bool SHADOW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_march_mfma(
    RayQueue q, const int* __restrict__ count, int* __restrict__ work, FieldView F, const TabT* __restrict__ table,
    const uint32_t* __restrict__ frags, MarchParams P, BvhView B, unsigned long long* __restrict__ stats) {
  using LY = FragLayout<NL, SH, CL, BF>;
  __shared__ __align__(16) uint32_t sW[LY::TOTAL];
  __shared__ int sstack[4 * 16 * kStack];   // shadow-ray stacks: 16 lanes per wave
  for (int i = threadIdx.x; i < LY::TOTAL; i += blockDim.x) sW[i] = frags[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, j = lane & 15;
  const int cnt = *count;
  const bool use_occ = P.use_occupancy && F.occ;
  int* stack = sstack + (threadIdx.x >> 6) * 16 * kStack + j;
  unsigned long long nsamp = 0;
  bool cnt_done = false;   // the short-queue path marched every ray
  if constexpr (!PK && !SHADOW) {
    if (cnt <= kSplitRaysPerBlock * (int)gridDim.x) {
      __shared__ float part[4][4];
      for (int r = blockIdx.x; r < cnt; r += gridDim.x)
        march_ray_split<NL, SH, CL, TabT, BF>(q, r, F, table, sW, P, B, use_occ, lane, threadIdx.x >> 6, part, nsamp);
      cnt_done = true;
    }
  }
  if constexpr (!PK) {
    if (!cnt_done) {
      WorkQueue wq(work, cnt, P.chunk, P.batch);
      for (int base = wq.next(lane); base >= 0; base = wq.next(lane))
        for (int bi = 0; bi < wq.batch; ++bi) {
          const int r = wq.map(base + bi);
          if (r >= cnt) break;
          march_ray<NL, SH, CL, TabT, BF, SHADOW>(q, r, F, table, sW, P, B, stack, use_occ, lane, nsamp);
        }
    }
  } else {
    WorkQueue wq(work, cnt, P.chunk, 16);
    for (int base = wq.next(lane); base >= 0; base = wq.next(lane)) {
      const PacketRay R = packet_ray(q, wq.map(base + j), cnt, F);
      march_packet<NL, SH, CL, TabT, BF, SHADOW>(q, R, F, table, sW, P, B, stack, use_occ, lane, nsamp);
    }
  }
  if (stats) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) nsamp += __shfl_xor(nsamp, off, 64);
    if (lane == 0 && nsamp) atomicAdd(stats + 0, nsamp);
  }
}

// ---------------------------------------------------------------------------
// Packets with specialised waves: producer waves take the 16-ray packets,
// place the samples and gather their hash features (vector units and memory);
// consumer waves, one per producer, run the MLP tiles on the matrix cores and
// composite.  A pair hands tiles over through two LDS slots, so that while a
// consumer's MFMAs run, the producer on the same SIMD gathers the next tile:
// the two kinds of work overlap by construction instead of by the scheduler's
// chance.  Same samples, same arithmetic and the same results as
// march_packet.
// ---------------------------------------------------------------------------
constexpr int kPcPairs = 4;                 // producer/consumer pairs per block
constexpr int kPcThreads = 128 * kPcPairs;  // waves 0..3 produce, 4..7 consume
constexpr int kPcSpin = 1 << 26;            // default polls before a wait gives up (seconds)
enum { kSlotEmpty = 0, kSlotStart = 1, kSlotTile = 2, kSlotEnd = 3, kSlotDone = 4 };

template <int NF>
struct PcSlot {
  float feat[NF][64];   // lane (g, j)'s features of column j, as the MFMA B operand takes them
  float D[16];          // interval length of column j (0: no sample there)
  float dir[16][3];     // START: column j's ray direction in the field frame
  int r[16];            // START: column j's queue index (-1: no ray)
  int state;
};

__device__ __forceinline__ int pc_load(const int* st) {
  return __hip_atomic_load(st, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void pc_store(int* st, int v) {
  __hip_atomic_store(st, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Wait until the slot is empty (producer) or holds a message (consumer);
// false if the wait gave up (then the wave stops: a bound, not a protocol).
__device__ __forceinline__ bool pc_wait(const int* st, bool want_empty, int polls) {
  for (int i = 0; i < polls; ++i) {
    const int v = pc_load(st);
    if ((v == kSlotEmpty) == want_empty) return true;
    __builtin_amdgcn_s_sleep(1);
  }
  return false;
}

template <int NL, int SH, int CL, typename TabT, bool BF>
__global__ __launch_bounds__(kPcThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_march_pc(RayQueue q, const int* __restrict__ count,
                                                         int* __restrict__ work, FieldView F,
                                                         const TabT* __restrict__ table,
                                                         const uint32_t* __restrict__ frags, MarchParams P,
                                                         unsigned long long* __restrict__ stats) {
  using LY = FragLayout<NL, SH, CL, BF>;
  constexpr int NF = LY::NF;
  __shared__ __align__(16) uint32_t sW[LY::TOTAL];
  __shared__ PcSlot<NF> slots[kPcPairs][2];
  for (int i = threadIdx.x; i < LY::TOTAL; i += blockDim.x) sW[i] = frags[i];
  if (threadIdx.x < kPcPairs * 2) slots[threadIdx.x >> 1][threadIdx.x & 1].state = kSlotEmpty;
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
  const int wave = threadIdx.x >> 6, pair = wave % kPcPairs;
  const bool producer = wave < kPcPairs;
  PcSlot<NF>* sl = slots[pair];
  int s = 0;
  unsigned long long nsamp = 0;
  bool ok = true;
  if (producer) {
    const int cnt = *count;
    const bool use_occ = P.use_occupancy && F.occ;
    const float delta = P.delta;
    WorkQueue wq(work, cnt, P.chunk, 16);
    for (int base = wq.next(lane); base >= 0 && ok; base = wq.next(lane)) {
      const PacketRay R = packet_ray(q, wq.map(base + j), cnt, F);
      bool live = R.live;
      float t_a = 0.0f, lo = 0.0f, hi = 0.0f;
      int k0 = P.n_samples, k1 = 0;
      if (live) {
        t_a = (q.depth[R.r] & 0xFFFF) == 0 ? P.t_near : 0.0f;
        float box0, box1;
        live = slab_box(F, R.ox, R.oy, R.oz, R.dx, R.dy, R.dz, box0, box1);
        if (live) {
          lo = fmaxf(t_a, box0);
          hi = fminf(fminf(t_a + P.span, q.hit_t[R.r]), box1);
          live = hi > lo;
        }
        if (live) {
          k0 = max(0, (int)floorf((lo - t_a) / delta) - 1);
          k1 = min(P.n_samples, (int)ceilf((hi - t_a) / delta) + 1);
        }
      }
      int kmin = k0, kmax = k1;
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) {
        kmin = min(kmin, __shfl_xor(kmin, off, 16));
        kmax = max(kmax, __shfl_xor(kmax, off, 16));
      }
      if (kmin >= kmax) continue;
      // START: the packet's rays
      if (!(ok = pc_wait(&sl[s].state, true, P.wait_polls))) break;
      if (g == 0) {
        sl[s].r[j] = live ? R.r : -1;
        sl[s].dir[j][0] = R.dx;
        sl[s].dir[j][1] = R.dy;
        sl[s].dir[j][2] = R.dz;
      }
      if (lane == 0) pc_store(&sl[s].state, kSlotStart);
      s ^= 1;
      for (int k = kmin; k < kmax; ++k) {
        const float a = fmaxf(t_a + (float)k * delta, lo);
        const float b = fminf(t_a + (float)(k + 1) * delta, hi);
        bool valid = live && k >= k0 && k < k1 && b > a;
        const float tm = 0.5f * (a + b);
        const float px = R.ox + tm * R.dx, py = R.oy + tm * R.dy, pz = R.oz + tm * R.dz;
        if (valid && use_occ) valid = occ_lookup(F, px, py, pz);
        if (__ballot(valid) == 0ull) continue;
        if (!(ok = pc_wait(&sl[s].state, true, P.wait_polls))) break;
        // the lane's levels in two halves straight into the slot (16 corner
        // loads in flight instead of 32 keeps the producer within its registers)
        float xh, yh, zh;
        to_unit(F, px, py, pz, xh, yh, zh);
        constexpr int LPG = NL / 4, HL = LPG / 2;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          float f2[HL][2];
#pragma unroll
          for (int i = 0; i < HL; ++i) encode_level<TabT>(F, table, xh, yh, zh, (h * HL + i) * 4 + g, f2[i][0], f2[i][1]);
#pragma unroll
          for (int i = 0; i < HL; ++i) {
            sl[s].feat[2 * (h * HL + i)][lane] = f2[i][0];
            sl[s].feat[2 * (h * HL + i) + 1][lane] = f2[i][1];
          }
          __builtin_amdgcn_sched_barrier(0);   // the second half's loads start here
        }
        if (g == 0) sl[s].D[j] = valid ? b - a : 0.0f;
        if (lane == 0) pc_store(&sl[s].state, kSlotTile);
        s ^= 1;
        if (g == 0 && valid) ++nsamp;
      }
      if (!ok) break;
      if (!(ok = pc_wait(&sl[s].state, true, P.wait_polls))) break;
      if (lane == 0) pc_store(&sl[s].state, kSlotEnd);
      s ^= 1;
    }
    if (ok && (ok = pc_wait(&sl[s].state, true, P.wait_polls)))
      if (lane == 0) pc_store(&sl[s].state, kSlotDone);
  } else {
    float u[4][4];
    float T = 1.0f, acc0 = 0.0f, acc1 = 0.0f, acc2 = 0.0f;
    int r = -1;
    while (true) {
      if (!(ok = pc_wait(&sl[s].state, false, P.wait_polls))) break;
      const int kind = pc_load(&sl[s].state);
      if (kind == kSlotDone) break;
      if (kind == kSlotStart) {
        r = sl[s].r[j];
        const float dx = sl[s].dir[j][0], dy = sl[s].dir[j][1], dz = sl[s].dir[j][2];
        T = 1.0f;
        acc0 = acc1 = acc2 = 0.0f;
        if (lane == 0) pc_store(&sl[s].state, kSlotEmpty);
        sh_rows<NL, SH, CL, BF>(sW, dx, dy, dz, lane, u);
      } else if (kind == kSlotTile) {
        float fe[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) fe[f] = sl[s].feat[f][lane];
        const float D = sl[s].D[j];
        if (lane == 0) pc_store(&sl[s].state, kSlotEmpty);
        float sigma, rgb[3];
        f4v raw;
        mlp_tile<NL, SH, CL, BF>(sW, fe, u, F.density_offset, lane, sigma, rgb, raw);
        const float alpha = D > 0.0f ? -expm1f(-sigma * D) : 0.0f;
        const float w = T * alpha;
        acc0 += w * rgb[0];
        acc1 += w * rgb[1];
        acc2 += w * rgb[2];
        T *= 1.0f - alpha;
      } else {   // kSlotEnd
        if (lane == 0) pc_store(&sl[s].state, kSlotEmpty);
        if (r >= 0 && g == 0) {
          const float tr = q.tr[r], tg = q.tg[r], tb = q.tb[r];
          q.lr[r] += tr * acc0;
          q.lg[r] += tg * acc1;
          q.lb[r] += tb * acc2;
          q.tr[r] = tr * T;
          q.tg[r] = tg * T;
          q.tb[r] = tb * T;
        }
      }
      s ^= 1;
    }
  }
  if (!ok && lane == 0 && P.gave_up) atomicAdd(P.gave_up, 1);
  if (stats) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) nsamp += __shfl_xor(nsamp, off, 64);
    if (lane == 0 && nsamp) atomicAdd(stats + 0, nsamp);
  }
}

template <int NL, int SH, int CL, typename TabT, bool BF>
__global__ __launch_bounds__(256) void k_query_mfma(FieldView F, const TabT* __restrict__ table,
                                                    const uint32_t* __restrict__ frags, int64_t n,
                                                    const float* __restrict__ x, const float* __restrict__ dirs,
                                                    float* __restrict__ sigma_out, float* __restrict__ rgb_out,
                                                    float* __restrict__ feat_out, float* __restrict__ raw_out) {
  using LY = FragLayout<NL, SH, CL, BF>;
  __shared__ __align__(16) uint32_t sW[LY::TOTAL];
  for (int i = threadIdx.x; i < LY::TOTAL; i += blockDim.x) sW[i] = frags[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  for (int64_t t = wave; t * 16 < n; t += waves) {
    const int64_t p = t * 16 + j;
    const bool valid = p < n;
    const int64_t pc = valid ? p : n - 1;
    float px = x[3 * pc], py = x[3 * pc + 1], pz = x[3 * pc + 2];
    float dx = 0.0f, dy = 0.0f, dz = 1.0f;
    if (dirs) { dx = dirs[3 * pc]; dy = dirs[3 * pc + 1]; dz = dirs[3 * pc + 2]; }
    to_field_frame(F, px, py, pz, dx, dy, dz);
    float u[4][4];
    sh_rows<NL, SH, CL, BF>(sW, dx, dy, dz, lane, u);
    float fe[LY::NF];
    encode_group<NL, TabT>(F, table, px, py, pz, g, fe);
    float sigma, rgb[3];
    f4v raw;
    mlp_tile<NL, SH, CL, BF>(sW, fe, u, F.density_offset, lane, sigma, rgb, raw);
    if (!valid) continue;
    if (g == 0) {
      sigma_out[p] = sigma;
      if (rgb_out) {
        rgb_out[3 * p] = rgb[0];
        rgb_out[3 * p + 1] = rgb[1];
        rgb_out[3 * p + 2] = rgb[2];
      }
    }
    if (feat_out)
#pragma unroll
      for (int k = 0; k < LY::NF; ++k) feat_out[p * 2 * NL + frag_k(0, LY::NF, 0, g, k)] = fe[k];
    if (raw_out)
#pragma unroll
      for (int v = 0; v < 4; ++v) raw_out[p * 16 + 4 * g + v] = raw[v];
  }
}

template <int NL, int SH, int CL, typename TabT, bool BF, bool PK, bool SHADOW>
mr_status launch_march_mode(const mr_field* f, RayQueue q, const int* count, int* work, const MarchParams& P,
                            const BvhView& B, unsigned long long* stats, int blocks_per_cu, int64_t n, hipStream_t st) {
  const uint32_t* fr = BF ? f->frag_bf16_dev : f->frag_f32_dev;
  const TabT* tab = reinterpret_cast<const TabT*>(f->table_dev);
  // producer and consumer waves pay for the 16-level layout; with 8 levels a
  // producer's gather is too short to hide behind a consumer's tile (the cloth
  // workload ran 6.24 ms per frame with them against 5.56 ms without)
  if constexpr (PK && !SHADOW && NL == 16) {
    auto* kp = k_march_pc<NL, SH, CL, TabT, BF>;
    const int blocks = persistent_blocks(reinterpret_cast<const void*>(kp), kPcThreads, blocks_per_cu,
                                         (n + 16 * kPcPairs - 1) / (16 * kPcPairs));
    MarchParams Pw = P;
    if (Pw.wait_polls <= 0) Pw.wait_polls = kPcSpin;
    hipLaunchKernelGGL(kp, dim3(blocks), dim3(kPcThreads), 0, st, q, count, work, f->view, tab, fr, Pw, stats);
    MR_HIP(hipGetLastError());
    return MR_OK;
  }
  auto* k = k_march_mfma<NL, SH, CL, TabT, BF, PK, SHADOW>;
  const int64_t cap = PK ? (n + 63) / 64 : (n + 3) / 4;
  const int blocks = persistent_blocks(reinterpret_cast<const void*>(k), 256, blocks_per_cu, cap);
  hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, st, q, count, work, f->view, tab, fr, P, B, stats);
  MR_HIP(hipGetLastError());
  return MR_OK;
}

template <int NL, int SH, int CL, typename TabT, bool BF>
mr_status launch_march_mfma(const mr_field* f, RayQueue q, const int* count, int* work, const MarchParams& P,
                            const BvhView& B, bool packets, unsigned long long* stats, int blocks_per_cu, int64_t n,
                            hipStream_t st) {
  if (P.shadows) {
    if (packets)
      return launch_march_mode<NL, SH, CL, TabT, BF, true, true>(f, q, count, work, P, B, stats, blocks_per_cu, n, st);
    return launch_march_mode<NL, SH, CL, TabT, BF, false, true>(f, q, count, work, P, B, stats, blocks_per_cu, n, st);
  }
  if (packets)
    return launch_march_mode<NL, SH, CL, TabT, BF, true, false>(f, q, count, work, P, B, stats, blocks_per_cu, n, st);
  return launch_march_mode<NL, SH, CL, TabT, BF, false, false>(f, q, count, work, P, B, stats, blocks_per_cu, n, st);
}

template <int NL, int SH, int CL, typename TabT, bool BF>
mr_status launch_query_mfma(const mr_field* f, int64_t n, const float* x, const float* dirs, float* sigma, float* rgb,
                            float* feat, float* raw, hipStream_t st) {
  const uint32_t* fr = BF ? f->frag_bf16_dev : f->frag_f32_dev;
  const int blocks = (int)std::min<int64_t>((n + 63) / 64, 4096);
  hipLaunchKernelGGL((k_query_mfma<NL, SH, CL, TabT, BF>), dim3(blocks), dim3(256), 0, st, f->view,
                     reinterpret_cast<const TabT*>(f->table_dev), fr, n, x, dirs, sigma, rgb, feat, raw);
  MR_HIP(hipGetLastError());
  return MR_OK;
}

}  // namespace

namespace mr {

// Weight fragments in the order mlp_tile reads them (see mr_mfma.h).
std::vector<uint32_t> build_fragments(const mr_field_desc& d, const float* mlp, bool bf) {
  const int NL = d.n_levels, SH = d.sh_components, CL = d.color_hidden_layers;
  const int NF = NL / 2;
  // FragLayout: BF16 fragment shape; BF16 weights one piece, FP32 weights three
  const int NP = bf ? 1 : 3;
  const int KP1 = bf_kpl(0, NF), KP2 = bf_kpl(1, NF), KPC = bf_kpl(2, NF);
  const int KS1 = NF / KP1, KS2 = 16 / KP2, KSC = 4 / KPC;
  const int WL1 = KP1 / 2, WL2 = KP2 / 2, WLC = KPC / 2;
  const int P1 = 4 * KS1 * 64 * WL1, P2 = KS2 * 64 * WL2, PC = 4 * KSC * 64 * WLC, PC2 = 4 * KS2 * 64 * WL2;
  const int L1 = 0, L2 = L1 + NP * P1, C1 = L2 + NP * P2, C2 = C1 + NP * PC;
  const int OUT = C2 + (CL == 2 ? NP * PC2 : 0), SHW = OUT + 192, TOTAL = SHW + 64 * SH;
  std::vector<uint32_t> w(TOTAL, 0u);
  const float* W1 = mlp;
  const float* W2 = W1 + 64 * d.density_in;
  const float* Wc1 = W2 + 16 * 64;
  const float* Wc2 = Wc1 + 64 * d.color_in;
  const float* Wout = Wc2 + (CL == 2 ? 64 * 64 : 0);
  auto bits = [](float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return u;
  };
  auto from_bits = [](uint32_t u) {
    float f;
    std::memcpy(&f, &u, 4);
    return f;
  };
  auto bf16 = [&](float f) {
    const uint32_t u = bits(f);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
  };
  // piece q of a weight: BF16 of the residual left by the pieces before it
  auto piece = [&](float v, int q) {
    uint32_t b = bf16(v);
    for (int i = 0; i < q; ++i) {
      v -= from_bits(b << 16);
      b = bf16(v);
    }
    return b;
  };
  // one fragment of every piece: kp bf16 values per lane, kp / 2 words,
  // element 0 in the low half; piece q at base + q * psize
  auto put = [&](int base, int psize, int mt, int ks, int nks, const float* M, int in_dim, int rows, int kind) {
    const int kp = bf_kpl(kind, NF);
    for (int q = 0; q < NP; ++q)
      for (int lane = 0; lane < 64; ++lane) {
        const int g = lane / 16, row = mt * 16 + lane % 16;
        const int slot = (mt * nks + ks) * 64 + lane;
        for (int e = 0; e < kp; ++e) {
          const int k = frag_k(kind, NF, ks, g, e);
          const uint32_t v = row < rows ? piece(M[row * in_dim + k], q) : 0u;
          w[base + q * psize + (kp / 2) * slot + e / 2] |= v << (16 * (e % 2));
        }
      }
  };
  for (int mt = 0; mt < 4; ++mt)
    for (int ks = 0; ks < KS1; ++ks) put(L1, P1, mt, ks, KS1, W1, d.density_in, 64, 0);
  for (int ks = 0; ks < KS2; ++ks) put(L2, P2, 0, ks, KS2, W2, 64, 16, 1);
  for (int mt = 0; mt < 4; ++mt)
    for (int ks = 0; ks < KSC; ++ks) put(C1, PC, mt, ks, KSC, Wc1, d.color_in, 64, 2);
  if (CL == 2)
    for (int mt = 0; mt < 4; ++mt)
      for (int ks = 0; ks < KS2; ++ks) put(C2, PC2, mt, ks, KS2, Wc2, 64, 64, 1);
  for (int i = 0; i < 192; ++i) w[OUT + i] = bits(Wout[i]);
  // SH columns of colour layer 1 as FP32 fragments [4 mt][SH/4][64]: lane
  // (g, j) of step ks holds row mt*16 + j, SH component 4 ks + g
  for (int mt = 0; mt < 4; ++mt)
    for (int ks = 0; ks < SH / 4; ++ks)
      for (int lane = 0; lane < 64; ++lane)
        w[SHW + (mt * (SH / 4) + ks) * 64 + lane] =
            bits(Wc1[(mt * 16 + lane % 16) * d.color_in + 16 + 4 * ks + lane / 16]);
  return w;
}

mr_status dispatch_march_mfma(const mr_field* f, RayQueue q, const int* count, int* work, const MarchParams& P,
                              const BvhView& B, bool packets, unsigned long long* stats, int blocks_per_cu, int64_t n,
                              hipStream_t st) {
  const auto& v = f->view;
  const bool h = v.table_dtype == MR_F16, bf = v.mlp_dtype == MR_BF16;
#define M(NL, SH, CL)                                                                                              \
  if (v.n_levels == NL && v.sh == SH && v.c_layers == CL) {                                                         \
    if (bf) return h ? launch_march_mfma<NL, SH, CL, __half, true>(f, q, count, work, P, B, packets, stats, blocks_per_cu, n, st)         \
                     : launch_march_mfma<NL, SH, CL, float, true>(f, q, count, work, P, B, packets, stats, blocks_per_cu, n, st);         \
    return h ? launch_march_mfma<NL, SH, CL, __half, false>(f, q, count, work, P, B, packets, stats, blocks_per_cu, n, st)                \
             : launch_march_mfma<NL, SH, CL, float, false>(f, q, count, work, P, B, packets, stats, blocks_per_cu, n, st);                \
  }
  M(8, 4, 1)
  M(16, 16, 2)
  M(16, 4, 1)
  M(8, 16, 2)
#undef M
  return fail(MR_ERR_UNSUPPORTED, "field shape not instantiated");
}

mr_status query_mfma(const mr_field* f, int64_t n, const float* x, const float* dirs, float* sigma, float* rgb,
                     float* feat, float* raw, hipStream_t st) {
  const auto& v = f->view;
  const bool h = v.table_dtype == MR_F16, bf = v.mlp_dtype == MR_BF16;
#define Q(NL, SH, CL)                                                                                          \
  if (v.n_levels == NL && v.sh == SH && v.c_layers == CL) {                                                     \
    if (bf) return h ? launch_query_mfma<NL, SH, CL, __half, true>(f, n, x, dirs, sigma, rgb, feat, raw, st)    \
                     : launch_query_mfma<NL, SH, CL, float, true>(f, n, x, dirs, sigma, rgb, feat, raw, st);    \
    return h ? launch_query_mfma<NL, SH, CL, __half, false>(f, n, x, dirs, sigma, rgb, feat, raw, st)           \
             : launch_query_mfma<NL, SH, CL, float, false>(f, n, x, dirs, sigma, rgb, feat, raw, st);           \
  }
  Q(8, 4, 1)
  Q(16, 16, 2)
  Q(16, 4, 1)
  Q(8, 16, 2)
#undef Q
  return fail(MR_ERR_UNSUPPORTED, "field shape not instantiated");
}

}  // namespace mr
