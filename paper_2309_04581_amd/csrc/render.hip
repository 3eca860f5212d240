// The hybrid rendering path (Algorithm 1 of "Dynamic Mesh-Aware Radiance
// Fields"): per bounce, (1) cast every live ray to its closest surface
// (Eq. 3), (2) march the radiance field along the segment up to that surface
// and integrate throughput and radiance (Eq. 10-11, quadrature of Eq. 8-9),
// (3) at the surface sample the BSDF, add the shadow-ray contribution of the
// point lights at diffuse hits, update the throughput (Eq. 12-13) and apply
// the termination rules (escape, low throughput, bounce limit), compacting
// the survivors into the next ray queue.
//
// Rays live in structure-of-arrays queues in HBM; each stage is one kernel
// reading the live count from device memory, so the host never waits and the
// whole sequence can be captured into a HIP graph.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "mr_device.h"
#include "mr_mfma.h"
#include "mr_render.h"

using namespace mr;

namespace mr {

// ---------------------------------------------------------------------------
// stage timing (event pairs on the launching stream)
// ---------------------------------------------------------------------------
struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
static Profiler g_prof;

struct StageTimer {
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  StageTimer(int s, hipStream_t stream, bool allowed = true) : stage(s), st(stream) {
    if (!allowed || !g_prof.on) return;
    a = g_prof.get();
    b = g_prof.get();
    if (a && b) (void)hipEventRecord(a, st);
  }
  ~StageTimer() {
    if (!a || !b) return;
    (void)hipEventRecord(b, st);
    g_prof.pending.push_back({stage, {a, b}});
  }
};

size_t queue_bytes(int64_t cap) { return (size_t)kQueueArrays * 4 * (size_t)cap; }

RayQueue queue_at(void* base, int64_t cap) {
  RayQueue q;
  float* f = reinterpret_cast<float*>(base);
  q.ox = f + 0 * cap; q.oy = f + 1 * cap; q.oz = f + 2 * cap;
  q.dx = f + 3 * cap; q.dy = f + 4 * cap; q.dz = f + 5 * cap;
  q.tr = f + 6 * cap; q.tg = f + 7 * cap; q.tb = f + 8 * cap;
  q.lr = f + 9 * cap; q.lg = f + 10 * cap; q.lb = f + 11 * cap;
  q.rid = reinterpret_cast<int*>(f + 12 * cap);
  q.depth = reinterpret_cast<int*>(f + 13 * cap);
  q.hit_t = f + 14 * cap;
  q.hit_p = reinterpret_cast<int*>(f + 15 * cap);
  return q;
}

}  // namespace mr

namespace {

// a*b - c*d as the difference of the exact products, rounded: Kahan's method
// (the rounding error of c*d recovered by an FMA) is within 1.5 ulp, so its
// sign is the exact one, and two equal nonzero products give +0.  When c*d is
// zero the plain difference is that value already, with the signed zero that
// IEEE arithmetic gives.
__device__ __forceinline__ float diff_prod(float a, float b, float c, float d) {
  const float w = c * d;
  if (w == 0.0f) return a * b - w;
  const float e = __fmaf_rn(-c, d, w);   // w - c d, exactly
  const float f = __fmaf_rn(a, b, -w);   // a b - w, rounded once
  return f + e;
}

// Unnormalised face normal e1 x e2 with every component the rounded
// difference of exact products.  The cosine-sampling basis switches on the
// sign of the normal's z: for a triangle parallel to z (two vertices with
// equal x and y) a plain FMA-contracted product difference returns the
// rounding error of one product, of either sign, instead of zero.
__device__ __forceinline__ V3 face_normal(V3 a, V3 b) {
  return v3(diff_prod(a.y, b.z, a.z, b.y), diff_prod(a.z, b.x, a.x, b.z), diff_prod(a.x, b.y, a.y, b.x));
}

// ---------------------------------------------------------------------------
// queue initialisation from caller rays
// ---------------------------------------------------------------------------
__global__ void k_init(int64_t n, const float* __restrict__ o, const float* __restrict__ d,
                       const int32_t* __restrict__ per_ray_mb, int max_bounces, RayQueue q, int* __restrict__ counts,
                       int n_counts, int32_t* __restrict__ hit_ids, int hit_stride, unsigned long long* __restrict__ stats) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid == 0) {
    for (int k = 0; k < n_counts; ++k) counts[k] = 0;
    counts[0] = (int)n;
    if (stats)
      for (int k = 0; k < 4; ++k) stats[k] = 0ull;
  }
  for (int64_t i = tid; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    q.ox[i] = o[3 * i]; q.oy[i] = o[3 * i + 1]; q.oz[i] = o[3 * i + 2];
    q.dx[i] = d[3 * i]; q.dy[i] = d[3 * i + 1]; q.dz[i] = d[3 * i + 2];
    q.tr[i] = 1.0f; q.tg[i] = 1.0f; q.tb[i] = 1.0f;
    q.lr[i] = 0.0f; q.lg[i] = 0.0f; q.lb[i] = 0.0f;
    q.rid[i] = (int)i;
    const int mb = per_ray_mb ? min(max(per_ray_mb[i], 0), max_bounces) : max_bounces;
    q.depth[i] = mb << 16;
    if (hit_ids)
      for (int s = 0; s < hit_stride; ++s) hit_ids[i * hit_stride + s] = -1;
  }
}

// ---------------------------------------------------------------------------
// closest hit of every live ray
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kTraceBlock) void k_trace(RayQueue q, const int* __restrict__ count, int* __restrict__ work,
                                                       int tile, BvhView B, float t_far, float span,
                                                       int32_t* __restrict__ hit_ids, int hit_stride) {
  __shared__ int stack[kStack * kTraceBlock];
  __shared__ float tstack[kStack * kTraceBlock];
  __shared__ int s_base;
  const int cnt = *count;
  while (true) {
    if (threadIdx.x == 0) s_base = atomicAdd(work, tile);
    __syncthreads();
    const int base = s_base;
    __syncthreads();
    if (base >= cnt) break;
    const int end = min(base + tile, cnt);
    for (int i = base + threadIdx.x; i < end; i += blockDim.x) {
      const int seg = q.depth[i] & 0xFFFF;
      const RayPre r = ray_pre(v3(q.ox[i], q.oy[i], q.oz[i]), v3(q.dx[i], q.dy[i], q.dz[i]));
      float t = INFINITY;
      const int p = B.n_prims ? bvh_trace<false>(B, r, seg == 0 ? t_far : span, t, stack + threadIdx.x,
                                                            tstack + threadIdx.x, kTraceBlock) : -1;
      q.hit_t[i] = p >= 0 ? t : INFINITY;
      q.hit_p[i] = p;
      if (hit_ids && seg < hit_stride)
        hit_ids[(int64_t)q.rid[i] * hit_stride + seg] = p >= 0 ? __float_as_int(B.tris[3 * p].w) : -1;
    }
  }
}

// Queues of at most kTailRays rays have their closest hits traced by
// k_trace_wide (one wave per ray) after the shade pass, not by it.
constexpr int kTailRays = 2048;   // queues this short are traced a wave per ray
constexpr int kWideFront = 512;   // frontier nodes per wave and level
constexpr int kWideWaves = 4;     // waves per block

// ---------------------------------------------------------------------------
// surface interaction, shadow rays, roulette, termination and compaction
// ---------------------------------------------------------------------------
__device__ __forceinline__ void finalize(const RenderOut& out, int rid, float tr, float tg, float tb, float lr, float lg,
                                         float lb, int bounces) {
  out.radiance[3 * (int64_t)rid] = lr;
  out.radiance[3 * (int64_t)rid + 1] = lg;
  out.radiance[3 * (int64_t)rid + 2] = lb;
  out.throughput[3 * (int64_t)rid] = tr;
  out.throughput[3 * (int64_t)rid + 1] = tg;
  out.throughput[3 * (int64_t)rid + 2] = tb;
  out.bounces[rid] = bounces;
}

// Optical depth of one field along [0, len] of the world ray so + t sd: the
// density at the midpoints of the march's grid intervals (spacing delta from
// t = 0), each clipped to the segment and the field's box, times their
// lengths; samples in empty occupancy cells count zero.  The density MLP's
// first layer is accumulated level by level (64 hidden sums, the weights read
// at uniform addresses), so one thread holds about a hundred registers.
template <int NL, typename TabT>
__device__ float field_depth(const FieldView& F, const TabT* __restrict__ tab, V3 so, V3 sd, float len, float delta,
                             bool occ) {
  float ox = so.x, oy = so.y, oz = so.z, dx = sd.x, dy = sd.y, dz = sd.z;
  to_field_frame(F, ox, oy, oz, dx, dy, dz);
  float b0, b1;
  if (!slab_box(F, ox, oy, oz, dx, dy, dz, b0, b1)) return 0.0f;
  const float lo = fmaxf(0.0f, b0), hi = fminf(len, b1);
  if (!(hi > lo)) return 0.0f;
  const size_t T = (size_t)F.table_mask + 1u;
  // the weights are constant for the kernel and read at wave-uniform
  // addresses: through the constant address space they are scalar loads
  typedef const __attribute__((address_space(4))) float* ConstF;
  const ConstF W0 = (ConstF)F.mlp;               // [64][32]
  const ConstF W1 = (ConstF)(F.mlp + 2048);      // row 0 of [16][64]
  float tau = 0.0f;
  // the intervals that meet [lo, hi], started one early so that FP32 rounding
  // of k delta cannot skip the first; at most 2^20 per field (a box 2^20 grid
  // intervals across), so the loop is bounded (indices clamped below 2^40)
  const float kf0 = fminf(fmaxf(0.0f, floorf(lo / delta) - 1.0f), 1.0995e12f);
  const float kf1 = fminf(ceilf(hi / delta) + 1.0f, kf0 + (float)(1 << 20));
  const int64_t k0 = (int64_t)kf0, k1 = (int64_t)kf1;
#pragma unroll 1
  for (int64_t k = k0; k <= k1; ++k) {
    float a = (float)k * delta, b = (float)(k + 1) * delta;
    if (b <= lo) continue;
    if (a >= hi) break;
    a = fmaxf(a, lo);
    b = fminf(b, hi);
    const float tm = 0.5f * (a + b);
    const float px = ox + tm * dx, py = oy + tm * dy, pz = oz + tm * dz;
    if (occ && !occ_lookup(F, px, py, pz)) continue;
    float xh, yh, zh;
    to_unit(F, px, py, pz, xh, yh, zh);
    float h[64];
#pragma unroll
    for (int j = 0; j < 64; ++j) h[j] = 0.0f;
#pragma unroll 1
    for (int l = 0; l < NL; ++l) {
      uint32_t idx[8];
      float w[8];
      level_corners(F, l, xh, yh, zh, idx, w);
      const TabT* t = tab + (size_t)l * T * 2;
      float f0 = 0.0f, f1 = 0.0f;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const float2 e = load_entry<TabT>(t, idx[c]);
        f0 += w[c] * e.x;
        f1 += w[c] * e.y;
      }
#pragma unroll
      for (int j = 0; j < 64; ++j) h[j] += W0[j * 32 + 2 * l] * f0 + W0[j * 32 + 2 * l + 1] * f1;
    }
    float r = 0.0f;
#pragma unroll
    for (int j = 0; j < 64; ++j) r += W1[j] * fmaxf(h[j], 0.0f);
    tau += softplusf(r + F.density_offset) * (b - a);
  }
  return tau;
}

// Transmittance of the medium along a light sample's shadow segment (the sum
// of the fields' optical depths): the light the sample carries crosses it, as
// a bounce that reaches the emitter is attenuated by its own march.
__device__ float shadow_transmittance(const ShadowMedium& SM, V3 so, V3 sd, float len) {
  float tau = 0.0f;
  for (int k = 0; k < SM.n; ++k) {
    const FieldView& F = SM.f[k];
    const bool occ = SM.use_occupancy && F.occ;
    if (F.n_levels == 16)
      tau += F.table_h ? field_depth<16, __half>(F, F.table_h, so, sd, len, SM.delta, occ)
                       : field_depth<16, float>(F, F.table, so, sd, len, SM.delta, occ);
    else
      tau += F.table_h ? field_depth<8, __half>(F, F.table_h, so, sd, len, SM.delta, occ)
                       : field_depth<8, float>(F, F.table, so, sd, len, SM.delta, occ);
  }
  return expf(-tau);
}

// MEDIUM: light samples toward emitters are attenuated by the fields in SM
// (only launched with light sampling and a medium; the other instance
// carries none of that code).
template <bool MEDIUM>
__global__ __launch_bounds__(kTraceBlock) void k_shade(RayQueue qi, const int* __restrict__ count_in,
                                                       int* __restrict__ work, int tile, RayQueue qo,
                                                       int* __restrict__ count_out, MeshView M, ShadeParams S,
                                                       RenderOut out, float span, int32_t* __restrict__ hit_ids,
                                                       int hit_stride, unsigned long long* __restrict__ stats,
                                                       ShadowMedium SM) {
  __shared__ int stack[kStack * kTraceBlock];
  __shared__ float tstack[kStack * kTraceBlock];
  __shared__ int s_base;
  const int cnt = *count_in;
  const int lane = threadIdx.x & 63;
  unsigned long long n_seg = 0, n_shadow = 0, n_scat = 0;
  while (true) {
  if (threadIdx.x == 0) s_base = atomicAdd(work, tile);
  __syncthreads();
  const int tbase = s_base;
  __syncthreads();
  if (tbase >= cnt) break;
  const int tend = min(tbase + tile, cnt);
  for (int i0 = tbase; i0 < tend; i0 += blockDim.x) {
    const int i = i0 + threadIdx.x;
    bool keep = false;
    float nox = 0, noy = 0, noz = 0, ndx = 0, ndy = 0, ndz = 0, tr = 0, tg = 0, tb = 0, lr = 0, lg = 0, lb = 0;
    int rid = 0, ndepth = 0;
    if (i < tend) {
      ++n_seg;
      rid = qi.rid[i];
      const int depth = qi.depth[i];
      const int seg = depth & 0xFFFF, mb = (depth >> 16) & 0xFF;
      const int p = qi.hit_p[i];
      tr = qi.tr[i]; tg = qi.tg[i]; tb = qi.tb[i];
      lr = qi.lr[i]; lg = qi.lg[i]; lb = qi.lb[i];
      // with light sampling, the emission a diffuse bounce reaches was estimated at that bounce
      if (p >= 0 && M.emissive && !(S.sample_emitters && (depth & kDepthAfterDiffuse))) {
        // Eq. 12: emitted radiance at the hit, attenuated by the marched segment
        const Material& em = M.mat[__float_as_int(M.bvh.tris[3 * p + 1].w)];
        lr += tr * em.emission[0];
        lg += tg * em.emission[1];
        lb += tb * em.emission[2];
      }
      if (p < 0 || seg >= mb) {
        finalize(out, rid, tr, tg, tb, lr, lg, lb, seg);
      } else {
        const V3 o = v3(qi.ox[i], qi.oy[i], qi.oz[i]), d = v3(qi.dx[i], qi.dy[i], qi.dz[i]);
        const float t = qi.hit_t[i];
        const float4 q0 = M.bvh.tris[3 * p], q1 = M.bvh.tris[3 * p + 1], q2 = M.bvh.tris[3 * p + 2];
        const V3 v0 = v3(q0.x, q0.y, q0.z), v1 = v3(q1.x, q1.y, q1.z), v2 = v3(q2.x, q2.y, q2.z);
        V3 n = face_normal(v1 - v0, v2 - v0);
        const float nl = sqrtf(dot(n, n));
        n = v3(n.x / nl, n.y / nl, n.z / nl);
        const V3 P = o + t * d;
        const float dn = dot(d, n);
        const V3 nf = dn < 0.0f ? n : v3(-n.x, -n.y, -n.z);
        const Material mat = M.mat[__float_as_int(q1.w)];
        V3 nd, side;
        float wr = 1.0f, wg = 1.0f, wb = 1.0f;
        if (mat.kind == MR_DIFFUSE) {
          for (int li = 0; li < S.n_lights; ++li) {
            const V3 lp = v3(S.lights[li][0], S.lights[li][1], S.lights[li][2]);
            const V3 wi = lp - P;
            const float d2 = dot(wi, wi), dist = sqrtf(d2);
            const float cosl = dot(nf, wi) / dist;
            if (!(cosl > 0.0f)) continue;
            const V3 so = P + 1e-4f * nf;
            V3 sd = lp - so;
            const float sdist = sqrtf(dot(sd, sd));
            sd = v3(sd.x / sdist, sd.y / sdist, sd.z / sdist);
            const RayPre sr = ray_pre(so, sd);
            float th;
            ++n_shadow;
            if (bvh_trace<true>(M.bvh, sr, sdist, th, stack + threadIdx.x, nullptr, kTraceBlock) >= 0) continue;
            const float g = cosl / d2 * (1.0f / 3.14159265358979323846f);
            lr += tr * mat.albedo[0] * S.lights[li][3] * g;
            lg += tg * mat.albedo[1] * S.lights[li][4] * g;
            lb += tb * mat.albedo[2] * S.lights[li][5] * g;
          }
          if (S.sample_emitters && M.n_emit > 0) {
            // one point on one emitting triangle: the triangle by the cumulative
            // probabilities, the point uniform by area (s = sqrt(u1))
            const float4 ue = draw4(S.seed, (uint32_t)rid, (uint32_t)seg, kRngEmitter);
            int lo = 0, hi = M.n_emit - 1;
            while (lo < hi) {
              const int mid = (lo + hi) >> 1;
              if (ue.x < M.emit[mid].x) hi = mid;
              else lo = mid + 1;
            }
            const float4 e = M.emit[lo];
            const int ep = __float_as_int(e.z);
            const float4 a0 = M.bvh.tris[3 * ep], a1 = M.bvh.tris[3 * ep + 1], a2 = M.bvh.tris[3 * ep + 2];
            const V3 w0 = v3(a0.x, a0.y, a0.z), w1 = v3(a1.x, a1.y, a1.z), w2 = v3(a2.x, a2.y, a2.z);
            const float sq = sqrtf(ue.y);
            const V3 x = (1.0f - sq) * w0 + (sq * (1.0f - ue.z)) * w1 + (sq * ue.z) * w2;
            const V3 en = cross(w1 - w0, w2 - w0);
            const float a2x = sqrtf(dot(en, en));          // twice the area
            const V3 wi = x - P;
            const float d2 = dot(wi, wi), dist = sqrtf(d2);
            const V3 l = v3(wi.x / dist, wi.y / dist, wi.z / dist);
            const float cos_p = dot(nf, l), cos_x = fabsf(dot(en, l)) / a2x;
            if (cos_p > 0.0f && cos_x > 0.0f) {
              const V3 so = P + 1e-4f * nf;
              V3 sd = x - so;
              const float sdist = sqrtf(dot(sd, sd));
              sd = v3(sd.x / sdist, sd.y / sdist, sd.z / sdist);
              const RayPre sr = ray_pre(so, sd);
              float th;
              ++n_shadow;
              if (bvh_trace<true>(M.bvh, sr, (1.0f - 1e-3f) * sdist, th, stack + threadIdx.x, nullptr, kTraceBlock) < 0) {
                const Material& em = M.mat[__float_as_int(a1.w)];
                float g = cos_p * cos_x / d2 * (0.5f * a2x) / e.y * (1.0f / 3.14159265358979323846f);
                if constexpr (MEDIUM) g *= shadow_transmittance(SM, so, sd, sdist);
                lr += tr * mat.albedo[0] * em.emission[0] * g;
                lg += tg * mat.albedo[1] * em.emission[1] * g;
                lb += tb * mat.albedo[2] * em.emission[2] * g;
              }
            }
          }
        }
        const float4 u = draw4(S.seed, (uint32_t)rid, (uint32_t)seg, mat.kind == MR_GLASS ? kRngGlass : kRngDiffuse);
        if (mat.kind == MR_MIRROR) {
          nd = d - (2.0f * dn) * n;
          side = nf;
        } else if (mat.kind == MR_GLASS) {
          const bool entering = dn < 0.0f;
          const float eta_i = entering ? 1.0f : mat.ior, eta_t = entering ? mat.ior : 1.0f;
          const float ci = fabsf(dn);
          const float eta = eta_i / eta_t;
          const float sin2t = eta * eta * (1.0f - ci * ci);
          float R = 1.0f, ct = 0.0f;
          if (sin2t < 1.0f) {
            ct = sqrtf(1.0f - sin2t);
            const float rs = (eta_i * ci - eta_t * ct) / (eta_i * ci + eta_t * ct);
            const float rp = (eta_i * ct - eta_t * ci) / (eta_i * ct + eta_t * ci);
            R = 0.5f * (rs * rs + rp * rp);
          }
          if (u.x < R) {
            nd = d - (2.0f * dn) * n;
            side = nf;
          } else {
            nd = eta * d + (eta * ci - ct) * nf;
            const float nn = sqrtf(dot(nd, nd));
            nd = v3(nd.x / nn, nd.y / nn, nd.z / nn);
            side = v3(-nf.x, -nf.y, -nf.z);
          }
        } else {
          // cosine-weighted hemisphere about nf, basis of Duff et al. 2017
          const float rr = sqrtf(u.x), phi = 6.283185307179586f * u.y;
          const float lx = rr * cosf(phi), ly = rr * sinf(phi), lz = sqrtf(fmaxf(0.0f, 1.0f - u.x));
          const float sgn = copysignf(1.0f, nf.z);
          const float a = -1.0f / (sgn + nf.z);
          const float bb = nf.x * nf.y * a;
          const V3 b1 = v3(1.0f + sgn * nf.x * nf.x * a, sgn * bb, -sgn * nf.x);
          const V3 b2 = v3(bb, sgn + nf.y * nf.y * a, -nf.y);
          nd = lx * b1 + ly * b2 + lz * nf;
          side = nf;
          wr = mat.albedo[0]; wg = mat.albedo[1]; wb = mat.albedo[2];
        }
        tr *= wr; tg *= wg; tb *= wb;
        const int nscat = seg + 1;
        ++n_scat;
        bool alive = true;
        if (S.rr_after >= 0 && nscat >= S.rr_after) {
          const float qv = fminf(1.0f, fmaxf(tr, fmaxf(tg, tb)));
          const float4 ur = draw4(S.seed, (uint32_t)rid, (uint32_t)seg, kRngRoulette);
          if (!(ur.x < qv)) {
            alive = false;
            finalize(out, rid, 0.0f, 0.0f, 0.0f, lr, lg, lb, nscat);
          } else {
            tr /= qv; tg /= qv; tb /= qv;
          }
        }
        if (alive && fmaxf(tr, fmaxf(tg, tb)) < S.t_min) {
          alive = false;
          finalize(out, rid, tr, tg, tb, lr, lg, lb, nscat);
        }
        if (alive) {
          keep = true;
          const V3 no = P + 1e-4f * side;
          nox = no.x; noy = no.y; noz = no.z;
          ndx = nd.x; ndy = nd.y; ndz = nd.z;
          ndepth = (mb << 16) | nscat | (mat.kind == MR_DIFFUSE ? kDepthAfterDiffuse : 0);
        }
      }
    }
    const unsigned long long m = __ballot(keep);
    const int nk = __popcll(m);
    int base = 0;
    if (lane == 0 && nk) base = atomicAdd(count_out, nk);
    base = __shfl(base, 0, 64);
    if (keep) {
      const int slot = base + __popcll(m & ((1ull << lane) - 1ull));
      qo.ox[slot] = nox; qo.oy[slot] = noy; qo.oz[slot] = noz;
      qo.dx[slot] = ndx; qo.dy[slot] = ndy; qo.dz[slot] = ndz;
      qo.tr[slot] = tr; qo.tg[slot] = tg; qo.tb[slot] = tb;
      qo.lr[slot] = lr; qo.lg[slot] = lg; qo.lb[slot] = lb;
      qo.rid[slot] = rid;
      qo.depth[slot] = ndepth;
      // closest hit of the new segment, whose range starts at the spawn point
      // (for short queues k_trace_wide traces it, a wave per ray)
      if (cnt > kTailRays) {
        const RayPre nr = ray_pre(v3(nox, noy, noz), v3(ndx, ndy, ndz));
        float th = INFINITY;
        const int hp = bvh_trace<false>(M.bvh, nr, span, th, stack + threadIdx.x, tstack + threadIdx.x, kTraceBlock);
        qo.hit_t[slot] = hp >= 0 ? th : INFINITY;
        qo.hit_p[slot] = hp;
        const int nseg = ndepth & 0xFFFF;
        if (hit_ids && nseg < hit_stride)
          hit_ids[(int64_t)rid * hit_stride + nseg] = hp >= 0 ? __float_as_int(M.bvh.tris[3 * hp].w) : -1;
      }
    }
  }
  }
  if (stats) {
    // per-wave sums, one atomic each
    unsigned long long a = n_seg, b = n_shadow, c = n_scat;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      a += __shfl_xor(a, off, 64);
      b += __shfl_xor(b, off, 64);
      c += __shfl_xor(c, off, 64);
    }
    if (lane == 0) {
      if (a) atomicAdd(stats + 1, a);
      if (b) atomicAdd(stats + 2, b);
      if (c) atomicAdd(stats + 3, c);
    }
  }
}

// ---------------------------------------------------------------------------
// Closest hit of a short queue: one wave per ray, breadth first.  The nodes
// the ray enters at one depth are expanded together, one per lane, so a deep
// traversal (a ray leaving a closed, finely tessellated surface enters
// hundreds of nested boxes) costs one dependent load per level instead of one
// per node.  Each level's frontier is pruned by the best hit over the whole
// wave, and the result is the same lexicographic minimum of (t, id) as the
// per-thread traversal (the same box and triangle tests, limits that are
// never tighter).  A frontier that outgrows its LDS area hands the ray to the
// per-thread traversal on lane 0.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__global__ __launch_bounds__(64 * kWideWaves) void k_trace_wide(RayQueue q, const int* __restrict__ gate_count,
                                                               const int* __restrict__ count, int* __restrict__ work,
                                                               BvhView B, float tmax, int32_t* __restrict__ hit_ids,
                                                               int hit_stride) {
  __shared__ int s_node[kWideWaves][2][kWideFront];
  __shared__ float s_tin[kWideWaves][2][kWideFront];
  __shared__ int s_stack[kWideWaves][kStack];
  __shared__ float s_tstack[kWideWaves][kStack];
  if (*gate_count > kTailRays) return;   // the shade pass traced this queue itself
  const int cnt = *count;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned long long below = (1ull << lane) - 1ull;
  while (true) {
    int r = 0;
    if (lane == 0) r = atomicAdd(work, 1);
    r = __shfl(r, 0, 64);
    if (r >= cnt) break;
    const RayPre R = ray_pre(v3(q.ox[r], q.oy[r], q.oz[r]), v3(q.dx[r], q.dy[r], q.dz[r]));
    float tb = tmax;                     // best hit of the wave: (tb, idb) at triangle pb
    int pb = -1, idb = 0x7fffffff;
    int n = B.n_prims > 0 ? 1 : 0, cur = 0;
    bool overflow = false;
    if (lane == 0) {
      s_node[w][0][0] = 0;
      s_tin[w][0][0] = 0.0f;
    }
    wave_lds_sync();
    while (n > 0) {
      float lt = tb;
      int lp = pb, lid = idb;
      int nn = 0;
      const float reach = tb * 1.0000003576f;
      for (int base = 0; base < n; base += 64) {
        const int i = base + lane;
        int ch0 = -1, ch1 = -1;
        float tc0 = 0.0f, tc1 = 0.0f;
        if (i < n && s_tin[w][cur][i] <= reach) {
          const BvhNode nd = B.nodes[s_node[w][cur][i]];
          const float t0 = nd.d.x < 0 ? INFINITY : box_hit(R, nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x, nd.b.y, tb);
          const float t1 = nd.d.y < 0 ? INFINITY : box_hit(R, nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w, tb);
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const float tc = c == 0 ? t0 : t1;
            if (tc == INFINITY) continue;
            const int child = c == 0 ? nd.d.x : nd.d.y, cn = c == 0 ? nd.d.z : nd.d.w;
            if (cn > 0) {
              for (int pp = child; pp < child + cn; ++pp) {
                const float4 q0 = B.tris[3 * pp], q1 = B.tris[3 * pp + 1], q2 = B.tris[3 * pp + 2];
                const float t = tri_hit(R, q0, q1, q2);
                const int id = __float_as_int(q0.w);
                if (t <= tmax && (t < lt || (t == lt && id < lid))) {
                  lt = t;
                  lp = pp;
                  lid = id;
                }
              }
            } else if (c == 0) {
              ch0 = child;
              tc0 = tc;
            } else {
              ch1 = child;
              tc1 = tc;
            }
          }
        }
        // inner children enter the next level's frontier in lane order
        const unsigned long long m0 = __ballot(ch0 >= 0), m1 = __ballot(ch1 >= 0);
        const int p0 = nn + __popcll(m0 & below);
        const int p1 = nn + __popcll(m0) + __popcll(m1 & below);
        if (ch0 >= 0 && p0 < kWideFront) {
          s_node[w][cur ^ 1][p0] = ch0;
          s_tin[w][cur ^ 1][p0] = tc0;
        }
        if (ch1 >= 0 && p1 < kWideFront) {
          s_node[w][cur ^ 1][p1] = ch1;
          s_tin[w][cur ^ 1][p1] = tc1;
        }
        nn += __popcll(m0) + __popcll(m1);
      }
      // best over the wave, lexicographic in (t, id)
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const float ot = __shfl_xor(lt, off, 64);
        const int oid = __shfl_xor(lid, off, 64), op = __shfl_xor(lp, off, 64);
        if (ot < lt || (ot == lt && oid < lid)) {
          lt = ot;
          lid = oid;
          lp = op;
        }
      }
      tb = lt;
      pb = lp;
      idb = lid;
      if (nn > kWideFront) {
        overflow = true;
        break;
      }
      n = nn;
      cur ^= 1;
      wave_lds_sync();
    }
    if (overflow) {
      if (lane == 0) {
        float th = tmax;
        pb = bvh_trace<false>(B, R, tmax, th, &s_stack[w][0], &s_tstack[w][0], 1);
        tb = th;
      }
      pb = __shfl(pb, 0, 64);
      tb = __shfl(tb, 0, 64);
    }
    if (lane == 0) {
      q.hit_t[r] = pb >= 0 ? tb : INFINITY;
      q.hit_p[r] = pb;
      const int seg = q.depth[r] & 0xFFFF;
      if (hit_ids && seg < hit_stride)
        hit_ids[(int64_t)q.rid[r] * hit_stride + seg] = pb >= 0 ? __float_as_int(B.tris[3 * pb].w) : -1;
    }
    wave_lds_sync();
  }
}

// ---------------------------------------------------------------------------
// several fields: each is marched in a pass of its own into a scratch copy of
// the segment's throughput and radiance (starting at T = 1, L = 0); the
// passes are then composited in the order the ray enters the fields' boxes.
// With boxes that do not overlap, every sample lies in at most one field, so
// this is the march of the summed medium.  It serves the proposal sampler and
// fields of different layouts; fields of one layout under the uniform sampler,
// overlapping or not, are marched together in one pass (march_fields.hip).
// ---------------------------------------------------------------------------
struct FieldBoxes {
  int n;
  int has_pose[kMaxFields];
  float pose[kMaxFields][12];
  float amin[kMaxFields][3], amax[kMaxFields][3];
};

// scratch: per field six arrays of cap floats, T r g b then L r g b
__global__ void k_fields_prep(const int* __restrict__ count, float* __restrict__ scratch, int n_fields, int64_t cap,
                              int* __restrict__ ctr, int n_ctr) {
  const int cnt = *count;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid < n_ctr) ctr[tid] = 0;
  for (int64_t i = tid; i < cnt; i += (int64_t)gridDim.x * blockDim.x)
    for (int k = 0; k < n_fields; ++k) {
      float* f = scratch + (int64_t)6 * k * cap;
      f[i] = 1.0f; f[cap + i] = 1.0f; f[2 * cap + i] = 1.0f;
      f[3 * cap + i] = 0.0f; f[4 * cap + i] = 0.0f; f[5 * cap + i] = 0.0f;
    }
}

__global__ void k_fields_combine(RayQueue q, const int* __restrict__ count, const float* __restrict__ scratch,
                                 int64_t cap, FieldBoxes fb) {
  const int cnt = *count;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x) {
    const float ox = q.ox[i], oy = q.oy[i], oz = q.oz[i], dx = q.dx[i], dy = q.dy[i], dz = q.dz[i];
    float tin[kMaxFields];
    int ord[kMaxFields];
    for (int k = 0; k < fb.n; ++k) {
      float p[3] = {ox, oy, oz}, d[3] = {dx, dy, dz};
      if (fb.has_pose[k]) {
        const float* P = fb.pose[k];
        const float qx = ox - P[3], qy = oy - P[7], qz = oz - P[11];
        for (int a = 0; a < 3; ++a) {
          p[a] = P[a] * qx + P[4 + a] * qy + P[8 + a] * qz;
          d[a] = P[a] * dx + P[4 + a] * dy + P[8 + a] * dz;
        }
      }
      float lo = -INFINITY;
      for (int a = 0; a < 3; ++a) {
        const float inv = 1.0f / d[a];
        const float t0 = (fb.amin[k][a] - p[a]) * inv, t1 = (fb.amax[k][a] - p[a]) * inv;
        lo = fmaxf(lo, fminf(t0, t1));
      }
      // a field the ray misses carries T = 1, L = 0: its place in the order is immaterial
      tin[k] = lo;
      int j = k;
      while (j > 0 && tin[ord[j - 1]] > lo) {
        ord[j] = ord[j - 1];
        --j;
      }
      ord[j] = k;
    }
    float tr = 1.0f, tg = 1.0f, tb = 1.0f, lr = 0.0f, lg = 0.0f, lb = 0.0f;
    for (int j = 0; j < fb.n; ++j) {
      const float* f = scratch + (int64_t)6 * ord[j] * cap;
      lr += tr * f[3 * cap + i];
      lg += tg * f[4 * cap + i];
      lb += tb * f[5 * cap + i];
      tr *= f[i];
      tg *= f[cap + i];
      tb *= f[2 * cap + i];
    }
    const float qr = q.tr[i], qg = q.tg[i], qb = q.tb[i];
    q.lr[i] += qr * lr;
    q.lg[i] += qg * lg;
    q.lb[i] += qb * lb;
    q.tr[i] = qr * tr;
    q.tg[i] = qg * tg;
    q.tb[i] = qb * tb;
  }
}

// ---------------------------------------------------------------------------
// pinhole cameras
// ---------------------------------------------------------------------------
struct CamBatch {
  int n;
  int64_t offset[kMaxCamsPerLaunch + 1];
  float pos[kMaxCamsPerLaunch][3], f[kMaxCamsPerLaunch][3], r[kMaxCamsPerLaunch][3], u[kMaxCamsPerLaunch][3];
  float th[kMaxCamsPerLaunch];
  int w[kMaxCamsPerLaunch], h[kMaxCamsPerLaunch];
  int cam_base;
};

__global__ void k_raygen(CamBatch C, int64_t total, float* __restrict__ o, float* __restrict__ d,
                         int32_t* __restrict__ cam_index, int64_t out_base) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    int c = 0;
    while (c + 1 < C.n && i >= C.offset[c + 1]) ++c;
    const int64_t pix = i - C.offset[c];
    const int W = C.w[c], H = C.h[c];
    const int px = (int)(pix % W), py = (int)(pix / W);
    const float su = (2.0f * ((float)px + 0.5f) / (float)W - 1.0f) * C.th[c] * ((float)W / (float)H);
    const float sv = (1.0f - 2.0f * ((float)py + 0.5f) / (float)H) * C.th[c];
    float v[3];
    for (int k = 0; k < 3; ++k) v[k] = C.f[c][k] + su * C.r[c][k] + sv * C.u[c][k];
    const float nv = sqrtf(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    const int64_t j = out_base + i;
    for (int k = 0; k < 3; ++k) {
      d[3 * j + k] = v[k] / nv;
      o[3 * j + k] = C.pos[c][k];
    }
    if (cam_index) cam_index[j] = C.cam_base + c;
  }
}

}  // namespace

namespace mr {

int device_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
  }
  return cus;
}

int persistent_blocks(const void* kernel, int threads, int per_cu, int64_t cap) {
  if (per_cu <= 0) {
    static std::mutex mu;
    static std::unordered_map<const void*, int> fit;
    std::lock_guard<std::mutex> lock(mu);
    auto it = fit.find(kernel);
    if (it == fit.end()) {
      int b = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kernel, threads, 0) != hipSuccess || b <= 0) b = 2;
      it = fit.emplace(kernel, b).first;
    }
    per_cu = it->second;
  }
  return (int)std::max<int64_t>(kXcds, std::min<int64_t>(cap, (int64_t)device_cus() * per_cu));
}

mr_status validate_render(const mr_field* field, const mr_mesh* mesh, int64_t n, const float* origins,
                          const float* dirs, int32_t max_bounces, const mr_light* lights, int32_t n_lights,
                          const mr_render_opts* opts, const mr_render_out* out) {
  (void)mesh;
  if (n < 0) return fail(MR_ERR_INVALID_ARG, "n < 0");
  if (n > 0x3FFFFFFF) return fail(MR_ERR_INVALID_ARG, "at most 2^30 rays per call");
  if (!opts || !out) return fail(MR_ERR_INVALID_ARG, "null opts or out");
  if (n > 0 && (!origins || !dirs)) return fail(MR_ERR_INVALID_ARG, "null rays");
  if (n > 0 && (!out->radiance || !out->throughput || !out->bounces)) return fail(MR_ERR_INVALID_ARG, "null outputs");
  if (max_bounces < 0 || max_bounces > kMaxBounces) return fail(MR_ERR_INVALID_ARG, "max_bounces must be in 0..60");
  if (out->hit_ids && out->hit_stride < max_bounces + 1)
    return fail(MR_ERR_INVALID_ARG, "hit_stride must be >= max_bounces + 1");
  if (n_lights < 0 || n_lights > kMaxLights) return fail(MR_ERR_INVALID_ARG, "n_lights must be in 0..8");
  if (n_lights > 0 && !lights) return fail(MR_ERR_INVALID_ARG, "null lights");
  for (int i = 0; i < n_lights; ++i)
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(lights[i].pos[k]) || !(lights[i].intensity[k] >= 0.0f) || !std::isfinite(lights[i].intensity[k]))
        return fail(MR_ERR_INVALID_ARG, "light position must be finite and intensity finite >= 0");
  if (!(opts->t_far > opts->t_near) || !(opts->t_near >= 0.0f) || !std::isfinite(opts->t_far))
    return fail(MR_ERR_INVALID_ARG, "need 0 <= t_near < t_far < inf");
  if (opts->n_samples < 1 || opts->n_samples > 4096) return fail(MR_ERR_INVALID_ARG, "n_samples must be in 1..4096");
  if (!(opts->t_min_throughput >= 0.0f)) return fail(MR_ERR_INVALID_ARG, "t_min_throughput must be >= 0");
  if (opts->sampler != MR_SAMPLER_UNIFORM && opts->sampler != MR_SAMPLER_PROPOSAL)
    return fail(MR_ERR_INVALID_ARG, "unknown sampler");
  if (opts->sampler == MR_SAMPLER_PROPOSAL) {
    if (!opts->proposal || opts->proposal->view.c_layers != 0)
      return fail(MR_ERR_INVALID_ARG, "proposal sampler needs a proposal field");
    if (opts->n_proposal < 1 || opts->n_proposal > 64 || opts->n_fine < 1 || opts->n_fine > 64)
      return fail(MR_ERR_INVALID_ARG, "n_proposal and n_fine must be in 1..64");
    if (field && !proposal_march_layout(field->view.n_levels, field->view.sh, field->view.c_layers))
      return fail(MR_ERR_UNSUPPORTED, "proposal sampling supports the 8-level/SH4/1-layer and 16-level/SH16/2-layer "
                                      "fields");
  }
  if (field && field->view.c_layers == 0) return fail(MR_ERR_INVALID_ARG, "field is a proposal field");
  if (opts->march_blocks_per_cu < 0 || opts->march_blocks_per_cu > 64 || opts->stage_blocks_per_cu < 0 ||
      opts->stage_blocks_per_cu > 64)
    return fail(MR_ERR_INVALID_ARG, "blocks per compute unit must be in 0..64");
  if (opts->stage_tile < 0 || opts->stage_tile % kTraceBlock != 0 || opts->stage_tile > (1 << 20))
    return fail(MR_ERR_INVALID_ARG, "stage_tile must be a multiple of 128 (or 0)");
  if (opts->march_chunk < 0) return fail(MR_ERR_INVALID_ARG, "march_chunk must be >= 0");
  if (opts->march_batch < 0 || opts->march_batch > 64) return fail(MR_ERR_INVALID_ARG, "march_batch must be in 0..64");
  if (opts->march_packets < -1) return fail(MR_ERR_INVALID_ARG, "march_packets must be >= -1");
  if (opts->wait_polls < 0) return fail(MR_ERR_INVALID_ARG, "wait_polls must be >= 0");
  if (opts->light_depth_samples < 0 || opts->light_depth_samples > 4096)
    return fail(MR_ERR_INVALID_ARG, "light_depth_samples must be in 0..4096");
  if (opts->sample_shadows && !(opts->shadow_mask >= 0.0f && opts->shadow_mask <= 1.0f))
    return fail(MR_ERR_INVALID_ARG, "shadow_mask must be in [0, 1]");
  if (opts->use_occupancy && field && !field->occ_dev)
    return fail(MR_ERR_STATE, "use_occupancy set but the field has no occupancy grid");
  return MR_OK;
}

}  // namespace mr

extern "C" size_t mr_render_workspace_size(int64_t n) {
  const int64_t cap = ((std::max<int64_t>(n, 1) + 63) / 64) * 64;
  return kHeaderBytes + 2 * queue_bytes(cap);
}

// several fields: after the single-field workspace, 256 bytes of march
// counters (kXcds per field) and the per-field scratch T and L arrays
static constexpr size_t kFieldCtrBytes = 256;
static_assert(kMaxFields * kXcds * sizeof(int) <= kFieldCtrBytes, "field counters");
static_assert(((3 + kXcds) * (kMaxBounces + 2) + 1) * sizeof(int) <= kHeaderBytes, "workspace header");

extern "C" size_t mr_render_fields_workspace_size(int64_t n, int32_t n_fields) {
  const int64_t cap = ((std::max<int64_t>(n, 1) + 63) / 64) * 64;
  if (n_fields <= 1) return mr_render_workspace_size(n);
  return mr_render_workspace_size(n) + kFieldCtrBytes + (size_t)n_fields * 6 * sizeof(float) * (size_t)cap;
}

namespace {

// Separating-axis test of two oriented boxes (centre, half extents, unit
// axes as the columns of R): they overlap unless some face normal or edge
// cross product separates their projections.  Touching boxes do not overlap.
bool boxes_overlap(const double c1[3], const double h1[3], const double R1[3][3], const double c2[3],
                   const double h2[3], const double R2[3][3]) {
  double axes[15][3];
  int na = 0;
  for (int i = 0; i < 3; ++i) {
    for (int k = 0; k < 3; ++k) axes[na][k] = R1[k][i];
    ++na;
    for (int k = 0; k < 3; ++k) axes[na][k] = R2[k][i];
    ++na;
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const double a[3] = {R1[0][i], R1[1][i], R1[2][i]}, b[3] = {R2[0][j], R2[1][j], R2[2][j]};
      axes[na][0] = a[1] * b[2] - a[2] * b[1];
      axes[na][1] = a[2] * b[0] - a[0] * b[2];
      axes[na][2] = a[0] * b[1] - a[1] * b[0];
      ++na;
    }
  const double dc[3] = {c2[0] - c1[0], c2[1] - c1[1], c2[2] - c1[2]};
  for (int a = 0; a < na; ++a) {
    const double* L = axes[a];
    const double l2 = L[0] * L[0] + L[1] * L[1] + L[2] * L[2];
    if (l2 < 1e-12) continue;   // parallel edges: covered by the face normals
    double r1 = 0.0, r2 = 0.0;
    for (int i = 0; i < 3; ++i) {
      r1 += h1[i] * std::fabs(R1[0][i] * L[0] + R1[1][i] * L[1] + R1[2][i] * L[2]);
      r2 += h2[i] * std::fabs(R2[0][i] * L[0] + R2[1][i] * L[1] + R2[2][i] * L[2]);
    }
    const double dist = std::fabs(dc[0] * L[0] + dc[1] * L[1] + dc[2] * L[2]);
    if (dist >= (r1 + r2) * (1.0 - 1e-9)) return false;
  }
  return true;
}

void field_box(const mr_field* f, double c[3], double h[3], double R[3][3]) {
  const FieldView& v = f->view;
  double cf[3];
  for (int k = 0; k < 3; ++k) {
    cf[k] = 0.5 * ((double)v.amin[k] + (double)v.amax[k]);
    h[k] = 0.5 * ((double)v.amax[k] - (double)v.amin[k]);
  }
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) R[i][k] = v.has_pose ? (double)v.pose[4 * i + k] : (i == k ? 1.0 : 0.0);
  for (int i = 0; i < 3; ++i)
    c[i] = R[i][0] * cf[0] + R[i][1] * cf[1] + R[i][2] * cf[2] + (v.has_pose ? (double)v.pose[4 * i + 3] : 0.0);
}

mr_status render_impl(const mr_field* const* fields, const mr_field* const* proposals, int n_fields, const mr_mesh* mesh,
                      int64_t n,
                      const float* origins, const float* dirs, int32_t max_bounces,
                      const int32_t* per_ray_max_bounces, const mr_light* host_lights, int32_t n_lights,
                      const mr_render_opts* opts, mr_render_out* out, void* workspace, size_t workspace_bytes,
                      void* stream, bool joint = false, bool timed = true) {
  mr_status s = MR_OK;
  const mr_field* field = n_fields == 1 ? fields[0] : nullptr;
  if (n == 0) return MR_OK;
  if (!workspace || workspace_bytes < mr_render_fields_workspace_size(n, n_fields))
    return fail(MR_ERR_INVALID_ARG, n_fields > 1 ? "workspace smaller than mr_render_fields_workspace_size(n, n_fields)"
                                                 : "workspace smaller than mr_render_workspace_size(n)");
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(MR_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  const int64_t cap = ((n + 63) / 64) * 64;
  char* ws = reinterpret_cast<char*>(workspace);
  int* counts = reinterpret_cast<int*>(ws);                 // [kMaxBounces + 2]
  int* twork = counts + (kMaxBounces + 2);                  // closest-hit tile queue heads
  int* swork = twork + (kMaxBounces + 2);                   // shade tile queue heads
  int* work = swork + (kMaxBounces + 2);                    // march: kXcds ray queue heads per segment
  int* gave_up = work + kXcds * (kMaxBounces + 2);          // march waits that gave up (mr_render_status)
  RayQueue Q[2] = {queue_at(ws + kHeaderBytes, cap), queue_at(ws + kHeaderBytes + queue_bytes(cap), cap)};
  int* fctr = reinterpret_cast<int*>(ws + mr_render_workspace_size(n));     // several fields only
  float* fscratch = reinterpret_cast<float*>(ws + mr_render_workspace_size(n) + kFieldCtrBytes);
  FieldBoxes FB;
  std::memset(&FB, 0, sizeof(FB));
  FB.n = n_fields > 1 ? n_fields : 0;
  for (int k = 0; k < FB.n; ++k) {
    const FieldView& v = fields[k]->view;
    FB.has_pose[k] = v.has_pose;
    for (int j = 0; j < 12; ++j) FB.pose[k][j] = v.pose[j];
    for (int j = 0; j < 3; ++j) {
      FB.amin[k][j] = v.amin[j];
      FB.amax[k][j] = v.amax[j];
    }
  }
  unsigned long long* stats = reinterpret_cast<unsigned long long*>(out->counters);

  const int init_blocks = (int)std::min<int64_t>((n + 255) / 256, 65535);
  hipLaunchKernelGGL(k_init, dim3(init_blocks), dim3(256), 0, st, n, origins, dirs, per_ray_max_bounces, max_bounces,
                     Q[0], counts, (3 + kXcds) * (kMaxBounces + 2) + 1, out->hit_ids, out->hit_ids ? out->hit_stride : 0,
                     stats);
  MR_HIP(hipGetLastError());

  MeshView mv;
  std::memset(&mv, 0, sizeof(mv));
  static const BvhNode* null_nodes = nullptr;
  if (mesh) mv = mesh->view;
  else mv.bvh.nodes = null_nodes;

  MarchParams P;
  P.t_near = opts->t_near;
  P.span = opts->t_far - opts->t_near;
  P.n_samples = opts->n_samples;
  P.delta = P.span / (float)opts->n_samples;
  P.use_occupancy = opts->use_occupancy;
  P.chunk = opts->march_chunk;
  P.batch = opts->march_batch > 0 ? opts->march_batch : 1;
  P.shadows = opts->sample_shadows && mesh && n_lights > 0;
  P.shadow_mask = opts->shadow_mask;
  P.n_lights = n_lights;
  for (int i = 0; i < n_lights; ++i)
    for (int k = 0; k < 3; ++k) P.light_pos[i][k] = host_lights[i].pos[k];
  P.wait_polls = opts->wait_polls;
  P.gave_up = gave_up;

  ShadeParams S;
  std::memset(&S, 0, sizeof(S));
  S.n_lights = n_lights;
  for (int i = 0; i < n_lights; ++i)
    for (int k = 0; k < 3; ++k) {
      S.lights[i][k] = host_lights[i].pos[k];
      S.lights[i][3 + k] = host_lights[i].intensity[k];
    }
  S.seed = opts->seed;
  S.rr_after = opts->rr_after;
  S.t_min = opts->t_min_throughput;
  S.sample_emitters = opts->sample_emitters ? 1 : 0;

  // light samples toward emitters cross the render's fields
  ShadowMedium SM;
  std::memset(&SM, 0, sizeof(SM));
  if (S.sample_emitters && mesh && mv.n_emit > 0) {
    SM.delta = opts->light_depth_samples > 0 ? P.span / (float)opts->light_depth_samples : P.delta;
    SM.use_occupancy = opts->use_occupancy;
    for (int k = 0; k < n_fields; ++k)
      if (fields[k]) SM.f[SM.n++] = fields[k]->view;
  }

  RenderOut ro;
  ro.radiance = out->radiance;
  ro.throughput = out->throughput;
  ro.bounces = out->bounces;

  const int tile = opts->stage_tile > 0 ? opts->stage_tile : 128;
  const int64_t tiles = (n + tile - 1) / tile;
  const int trace_blocks =
      persistent_blocks(reinterpret_cast<const void*>(k_trace), kTraceBlock, opts->stage_blocks_per_cu, tiles);
  const int shade_blocks =
      persistent_blocks(reinterpret_cast<const void*>(k_shade<false>), kTraceBlock, opts->stage_blocks_per_cu, tiles);
  const int packet_segments = opts->march_packets == 0 ? 1 : std::max(0, opts->march_packets);
  const int wide_blocks = (int)std::max<int64_t>(
      1, std::min<int64_t>((std::min<int64_t>(n, kTailRays) + kWideWaves - 1) / kWideWaves, (int64_t)device_cus() * 4));
  for (int b = 0; b <= max_bounces; ++b) {
    RayQueue& qi = Q[b & 1];
    RayQueue& qo = Q[(b + 1) & 1];
    if (b == 0) {
      // later segments are traced by the shade pass that spawns them
      StageTimer tm(0, st, timed);
      hipLaunchKernelGGL(k_trace, dim3(trace_blocks), dim3(kTraceBlock), 0, st, qi, counts + b, twork + b, tile, mv.bvh,
                         opts->t_far, P.span, out->hit_ids, out->hit_ids ? out->hit_stride : 0);
      MR_HIP(hipGetLastError());
    }
    if (n_fields > 1 && joint) {
      // one march over the summed medium
      StageTimer tm(b == 0 ? 3 : 1, st, timed);
      s = dispatch_march_fields(fields, n_fields, qi, counts + b, work + kXcds * b, P, mv.bvh, b < packet_segments,
                                stats, opts->march_blocks_per_cu, n, st);
      if (s != MR_OK) return s;
    } else if (n_fields > 1) {
      StageTimer tm(b == 0 ? 3 : 1, st, timed);
      const int fblocks = (int)std::min<int64_t>((n + 255) / 256, 65535);
      hipLaunchKernelGGL(k_fields_prep, dim3(fblocks), dim3(256), 0, st, counts + b, fscratch, n_fields, cap, fctr,
                         n_fields * kXcds);
      MR_HIP(hipGetLastError());
      for (int k = 0; k < n_fields; ++k) {
        RayQueue qk = qi;
        float* f = fscratch + (int64_t)6 * k * cap;
        qk.tr = f; qk.tg = f + cap; qk.tb = f + 2 * cap;
        qk.lr = f + 3 * cap; qk.lg = f + 4 * cap; qk.lb = f + 5 * cap;
        if (opts->sampler == MR_SAMPLER_PROPOSAL)
          s = dispatch_march_proposal(fields[k], proposals[k], qk, counts + b, fctr + kXcds * k, P, mv.bvh,
                                      opts->n_proposal, opts->n_fine, b < packet_segments, stats,
                                      opts->march_blocks_per_cu, n, st);
        else
          s = dispatch_march_mfma(fields[k], qk, counts + b, fctr + kXcds * k, P, mv.bvh, b < packet_segments, stats,
                                  opts->march_blocks_per_cu, n, st);
        if (s != MR_OK) return s;
      }
      hipLaunchKernelGGL(k_fields_combine, dim3(fblocks), dim3(256), 0, st, qi, counts + b, fscratch, cap, FB);
      MR_HIP(hipGetLastError());
    } else if (field) {
      StageTimer tm(b == 0 ? 3 : 1, st, timed);
      if (opts->sampler == MR_SAMPLER_PROPOSAL)
        s = dispatch_march_proposal(field, opts->proposal, qi, counts + b, work + kXcds * b, P, mv.bvh, opts->n_proposal,
                                    opts->n_fine, b < packet_segments, stats, opts->march_blocks_per_cu, n, st);
      else
        s = dispatch_march_mfma(field, qi, counts + b, work + kXcds * b, P, mv.bvh, b < packet_segments, stats,
                                opts->march_blocks_per_cu, n, st);
      if (s != MR_OK) return s;
    }
    {
      StageTimer tm(2, st, timed);
      if (SM.n > 0)
        hipLaunchKernelGGL(k_shade<true>, dim3(shade_blocks), dim3(kTraceBlock), 0, st, qi, counts + b, swork + b, tile,
                           qo, counts + b + 1, mv, S, ro, P.span, out->hit_ids, out->hit_ids ? out->hit_stride : 0, stats,
                           SM);
      else
        hipLaunchKernelGGL(k_shade<false>, dim3(shade_blocks), dim3(kTraceBlock), 0, st, qi, counts + b, swork + b, tile,
                           qo, counts + b + 1, mv, S, ro, P.span, out->hit_ids, out->hit_ids ? out->hit_stride : 0, stats,
                           SM);
      MR_HIP(hipGetLastError());
    }
    if (b < max_bounces) {
      // closest hits of the next segment when this queue is short (the kernel
      // returns at once otherwise)
      StageTimer tm(0, st, timed);
      hipLaunchKernelGGL(k_trace_wide, dim3(wide_blocks), dim3(64 * kWideWaves), 0, st, qo, counts + b, counts + b + 1,
                         twork + b + 1, mv.bvh, P.span, out->hit_ids, out->hit_ids ? out->hit_stride : 0);
      MR_HIP(hipGetLastError());
    }
  }
  return MR_OK;
}

}  // namespace

extern "C" mr_status mr_render(const mr_field* field, const mr_mesh* mesh, int64_t n, const float* origins,
                               const float* dirs, int32_t max_bounces, const int32_t* per_ray_max_bounces,
                               const mr_light* host_lights, int32_t n_lights, const mr_render_opts* opts,
                               mr_render_out* out, void* workspace, size_t workspace_bytes, void* stream) {
  mr_status s = validate_render(field, mesh, n, origins, dirs, max_bounces, host_lights, n_lights, opts, out);
  if (s != MR_OK) return s;
  return render_impl(&field, nullptr, field ? 1 : 0, mesh, n, origins, dirs, max_bounces, per_ray_max_bounces,
                     host_lights, n_lights, opts, out, workspace, workspace_bytes, stream);
}

extern "C" mr_status mr_render_status(const void* workspace, int64_t* gave_up, void* stream) {
  if (!workspace) return fail(MR_ERR_INVALID_ARG, "null workspace");
  const int* w = reinterpret_cast<const int*>(workspace) + (3 + kXcds) * (kMaxBounces + 2);
  int v = 0;
  MR_HIP(hipMemcpyAsync(&v, w, sizeof(int), hipMemcpyDeviceToHost, (hipStream_t)stream));
  MR_HIP(hipStreamSynchronize((hipStream_t)stream));
  if (gave_up) *gave_up = v;
  if (v != 0)
    return fail(MR_ERR_DEVICE, std::to_string(v) + " wave(s) of the packet march gave up a bounded wait: the "
                                                    "radiance and throughput of their packets' rays are incomplete");
  return MR_OK;
}

// ---------------------------------------------------------------------------
// render without allocation: the ray queues and counters live in a fixed
// array of the library's code object, one per device, instead of a caller
// workspace
// ---------------------------------------------------------------------------
namespace {

constexpr int64_t kNoAllocMaxRays = MR_NOALLOC_MAX_RAYS;
constexpr size_t kScratchBytes = kHeaderBytes + 2 * (size_t)kQueueArrays * 4 * (size_t)kNoAllocMaxRays;
static_assert(kNoAllocMaxRays % 64 == 0, "queue capacity is a multiple of 64");

// Host code must not pass this name to a kernel or a copy: it stands for the
// device array only in device code.  scratch_on_device() gives its address.
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's copy of scratch, looked up once per device.
mr_status scratch_on_device(void** ptr) {
  int dev = 0;
  MR_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(MR_ERR_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(MR_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return MR_OK;
}

__global__ void k_copy_gave_up(const int* src, int32_t* dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

}  // namespace

extern "C" mr_status mr_render_noalloc(const mr_field* field, const mr_mesh* mesh, int64_t n, const float* origins,
                                       const float* dirs, int32_t max_bounces, const int32_t* per_ray_max_bounces,
                                       const mr_light* host_lights, int32_t n_lights, const mr_render_opts* opts,
                                       mr_render_out* out, int32_t* gave_up, void* stream) {
  if (n > kNoAllocMaxRays)
    return fail(MR_ERR_INVALID_ARG, "n = " + std::to_string(n) + " exceeds the " + std::to_string(kNoAllocMaxRays) +
                                        " rays mr_render_noalloc holds; use mr_render with a workspace");
  mr_status s = validate_render(field, mesh, n, origins, dirs, max_bounces, host_lights, n_lights, opts, out);
  if (s != MR_OK) return s;
  if (n == 0) return MR_OK;
  void* ws = nullptr;
  s = scratch_on_device(&ws);
  if (s != MR_OK) return s;
  s = render_impl(&field, nullptr, field ? 1 : 0, mesh, n, origins, dirs, max_bounces, per_ray_max_bounces,
                  host_lights, n_lights, opts, out, ws, kScratchBytes, stream, false, /*timed=*/false);
  if (s != MR_OK) return s;
  if (gave_up) {
    const int* src = reinterpret_cast<const int*>(ws) + (3 + kXcds) * (kMaxBounces + 2);
    hipLaunchKernelGGL(k_copy_gave_up, dim3(1), dim3(64), 0, (hipStream_t)stream, src, gave_up);
    MR_HIP(hipGetLastError());
  }
  return MR_OK;
}

extern "C" mr_status mr_render_fields(const mr_field* const* fields, const mr_field* const* proposals,
                                      int32_t n_fields, const mr_mesh* mesh, int64_t n, const float* origins,
                                      const float* dirs, int32_t max_bounces, const int32_t* per_ray_max_bounces,
                                      const mr_light* host_lights, int32_t n_lights, const mr_render_opts* opts,
                                      mr_render_out* out, void* workspace, size_t workspace_bytes, void* stream) {
  if (n_fields < 1 || n_fields > kMaxFields) return fail(MR_ERR_INVALID_ARG, "n_fields must be in 1..8");
  if (!fields) return fail(MR_ERR_INVALID_ARG, "null field list");
  if (!opts) return fail(MR_ERR_INVALID_ARG, "null opts");
  for (int k = 0; k < n_fields; ++k)
    if (!fields[k]) return fail(MR_ERR_INVALID_ARG, "null field in the list");
  const bool prop = opts->sampler == MR_SAMPLER_PROPOSAL;
  if (prop && !proposals) return fail(MR_ERR_INVALID_ARG, "the proposal sampler needs one proposal per field");
  for (int k = 0; k < n_fields; ++k) {
    mr_render_opts ok = *opts;   // each field is validated with its own proposal
    if (prop) ok.proposal = proposals[k];
    mr_status s = validate_render(fields[k], mesh, n, origins, dirs, max_bounces, host_lights, n_lights, &ok, out);
    if (s != MR_OK) return s;
  }
  bool overlapping = false;
  for (int a = 0; a < n_fields; ++a)
    for (int b = a + 1; b < n_fields; ++b) {
      double c1[3], h1[3], R1[3][3], c2[3], h2[3], R2[3][3];
      field_box(fields[a], c1, h1, R1);
      field_box(fields[b], c2, h2, R2);
      if (!boxes_overlap(c1, h1, R1, c2, h2, R2)) continue;
      if (prop)
        return fail(MR_ERR_UNSUPPORTED, "the boxes of fields " + std::to_string(a) + " and " + std::to_string(b) +
                                            " overlap in the world: overlapping fields take the uniform sampler");
      overlapping = true;
    }
  bool one_layout = true;
  int other = 0;
  for (int k = 1; k < n_fields; ++k) {
    const FieldView &v0 = fields[0]->view, &vk = fields[k]->view;
    if (vk.n_levels != v0.n_levels || vk.sh != v0.sh || vk.c_layers != v0.c_layers ||
        vk.table_dtype != v0.table_dtype || vk.mlp_dtype != v0.mlp_dtype) {
      one_layout = false;
      other = k;
      break;
    }
  }
  if (overlapping && !one_layout)   // one kernel marches them all: one layout
    return fail(MR_ERR_UNSUPPORTED, "fields 0 and " + std::to_string(other) +
                                        " differ in layout (levels, SH components, colour layers, table or MLP "
                                        "type); fields whose boxes overlap must share one");
  // fields of one layout under the uniform sampler are marched together
  // whether or not their boxes overlap: one pass instead of one per field
  const bool joint = !prop && one_layout;
  if (n_fields == 1) {   // one field: the ordinary render, with its proposal
    mr_render_opts o1 = *opts;
    if (prop) o1.proposal = proposals[0];
    return render_impl(fields, nullptr, 1, mesh, n, origins, dirs, max_bounces, per_ray_max_bounces, host_lights,
                       n_lights, &o1, out, workspace, workspace_bytes, stream);
  }
  return render_impl(fields, prop ? proposals : nullptr, n_fields, mesh, n, origins, dirs, max_bounces,
                     per_ray_max_bounces, host_lights, n_lights, opts, out, workspace, workspace_bytes, stream,
                     joint);
}

extern "C" mr_status mr_profile_enable(int32_t on) {
  g_prof.on = on != 0;
  return MR_OK;
}

extern "C" mr_status mr_profile_read(double* ms, int64_t* launches) {
  if (!ms || !launches) return fail(MR_ERR_INVALID_ARG, "null output");
  for (int k = 0; k < 4; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  mr_status s = MR_OK;
  for (auto& p : g_prof.pending) {
    float t = 0.0f;
    if (hipEventSynchronize(p.second.second) != hipSuccess ||
        hipEventElapsedTime(&t, p.second.first, p.second.second) != hipSuccess)
      s = fail(MR_ERR_DEVICE, "event timing failed");
    const int k = p.first < 0 || p.first > 3 ? 3 : p.first;
    ms[k] += t;
    launches[k] += 1;
    g_prof.pool.push_back(p.second.first);
    g_prof.pool.push_back(p.second.second);
  }
  g_prof.pending.clear();
  return s;
}

extern "C" mr_status mr_rays_from_cameras(const float* host_cams, int32_t n_cams, float* origins, float* dirs,
                                          int32_t* cam_index, int64_t capacity, void* stream) {
  if (!host_cams || n_cams < 1) return fail(MR_ERR_INVALID_ARG, "need at least one camera");
  if (!origins || !dirs) return fail(MR_ERR_INVALID_ARG, "null outputs");
  int64_t total = 0;
  for (int c = 0; c < n_cams; ++c) {
    const float* cam = host_cams + 12 * c;
    for (int k = 0; k < 10; ++k)
      if (!std::isfinite(cam[k])) return fail(MR_ERR_INVALID_ARG, "non-finite camera");
    const int W = (int)cam[10], H = (int)cam[11];
    if (W < 1 || H < 1 || (float)W != cam[10] || (float)H != cam[11]) return fail(MR_ERR_INVALID_ARG, "bad camera size");
    if (!(cam[9] > 0.0f && cam[9] < 180.0f)) return fail(MR_ERR_INVALID_ARG, "fov must be in (0, 180)");
    total += (int64_t)W * H;
  }
  if (total > capacity) return fail(MR_ERR_INVALID_ARG, "capacity smaller than the pixel count");
  hipStream_t st = (hipStream_t)stream;
  int64_t base = 0;
  for (int c0 = 0; c0 < n_cams; c0 += kMaxCamsPerLaunch) {
    CamBatch B;
    std::memset(&B, 0, sizeof(B));
    B.n = std::min(kMaxCamsPerLaunch, n_cams - c0);
    B.cam_base = c0;
    int64_t off = 0;
    for (int c = 0; c < B.n; ++c) {
      const float* cam = host_cams + 12 * (c0 + c);
      double pos[3] = {cam[0], cam[1], cam[2]}, at[3] = {cam[3], cam[4], cam[5]}, up[3] = {cam[6], cam[7], cam[8]};
      double f[3] = {at[0] - pos[0], at[1] - pos[1], at[2] - pos[2]};
      double nf = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
      if (!(nf > 0.0)) return fail(MR_ERR_INVALID_ARG, "camera looks at its own position");
      for (double& x : f) x /= nf;
      double r[3] = {up[1] * f[2] - up[2] * f[1], up[2] * f[0] - up[0] * f[2], up[0] * f[1] - up[1] * f[0]};
      double nr = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
      if (!(nr > 0.0)) return fail(MR_ERR_INVALID_ARG, "camera up is parallel to the view direction");
      for (double& x : r) x /= nr;
      double u[3] = {f[1] * r[2] - f[2] * r[1], f[2] * r[0] - f[0] * r[2], f[0] * r[1] - f[1] * r[0]};
      for (int k = 0; k < 3; ++k) {
        B.pos[c][k] = (float)pos[k];
        B.f[c][k] = (float)f[k];
        B.r[c][k] = (float)r[k];
        B.u[c][k] = (float)u[k];
      }
      B.th[c] = (float)std::tan(0.5 * (double)cam[9] * 3.14159265358979323846 / 180.0);
      B.w[c] = (int)cam[10];
      B.h[c] = (int)cam[11];
      B.offset[c] = off;
      off += (int64_t)B.w[c] * B.h[c];
    }
    B.offset[B.n] = off;
    const int blocks = (int)std::min<int64_t>((off + 255) / 256, 65535);
    hipLaunchKernelGGL(k_raygen, dim3(blocks), dim3(256), 0, st, B, off, origins, dirs, cam_index, base);
    MR_HIP(hipGetLastError());
    base += off;
  }
  return MR_OK;
}


struct mr_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" mr_status mr_render_graph_create(const mr_field* field, const mr_mesh* mesh, int64_t n, const float* origins,
                                            const float* dirs, int32_t max_bounces, const int32_t* per_ray_max_bounces,
                                            const mr_light* host_lights, int32_t n_lights, const mr_render_opts* opts,
                                            mr_render_out* out, void* workspace, size_t workspace_bytes,
                                            mr_graph** graph) {
  if (!graph) return fail(MR_ERR_INVALID_ARG, "null graph");
  if (g_prof.on) return fail(MR_ERR_STATE, "kernel timing is on; disable it before capturing");
  mr_status s = validate_render(field, mesh, n, origins, dirs, max_bounces, host_lights, n_lights, opts, out);
  if (s != MR_OK) return s;
  if (!workspace || workspace_bytes < mr_render_workspace_size(n))
    return fail(MR_ERR_INVALID_ARG, "workspace smaller than mr_render_workspace_size(n)");
  hipStream_t st = nullptr;
  MR_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  mr_graph* g = new mr_graph();
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipStreamDestroy(st);
    delete g;
    return fail(MR_ERR_DEVICE, "hipStreamBeginCapture failed");
  }
  s = mr_render(field, mesh, n, origins, dirs, max_bounces, per_ray_max_bounces, host_lights, n_lights, opts, out,
                workspace, workspace_bytes, st);
  const hipError_t e = hipStreamEndCapture(st, &g->graph);
  (void)hipStreamDestroy(st);
  if (s != MR_OK || e != hipSuccess) {
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return s != MR_OK ? s : fail(MR_ERR_DEVICE, "hipStreamEndCapture failed");
  }
  if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g->graph);
    delete g;
    return fail(MR_ERR_DEVICE, "hipGraphInstantiate failed");
  }
  *graph = g;
  return MR_OK;
}

extern "C" mr_status mr_graph_launch(mr_graph* graph, void* stream) {
  if (!graph || !graph->exec) return fail(MR_ERR_INVALID_ARG, "null graph");
  MR_HIP(hipGraphLaunch(graph->exec, (hipStream_t)stream));
  return MR_OK;
}

extern "C" mr_status mr_graph_destroy(mr_graph* graph) {
  if (!graph) return MR_OK;
  if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
  if (graph->graph) (void)hipGraphDestroy(graph->graph);
  delete graph;
  return MR_OK;
}

extern "C" mr_status mr_autotune_render(const mr_field* field, const mr_mesh* mesh, int64_t n, const float* origins,
                                        const float* dirs, int32_t max_bounces, const int32_t* per_ray_max_bounces,
                                        const mr_light* host_lights, int32_t n_lights, const mr_render_opts* opts,
                                        mr_render_out* out, void* workspace, size_t workspace_bytes,
                                        const mr_launch_cfg* host_cands, int32_t n_cands, int32_t reps,
                                        int32_t* best_index, float* best_ms, void* stream) {
  if (!opts || !best_index || !best_ms || !host_cands) return fail(MR_ERR_INVALID_ARG, "null argument");
  if (n_cands < 1) return fail(MR_ERR_INVALID_ARG, "need at least one candidate");
  if (reps < 1 || reps > 100) return fail(MR_ERR_INVALID_ARG, "reps must be in 1..100");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t a = nullptr, b = nullptr;
  MR_HIP(hipEventCreate(&a));
  MR_HIP(hipEventCreate(&b));
  float best_t = INFINITY;
  mr_status s = MR_OK;
  for (int c = 0; c < n_cands && s == MR_OK; ++c) {
    mr_render_opts o = *opts;
    o.march_blocks_per_cu = host_cands[c].march_blocks_per_cu;
    o.stage_blocks_per_cu = host_cands[c].stage_blocks_per_cu;
    o.stage_tile = host_cands[c].stage_tile;
    o.march_chunk = host_cands[c].march_chunk;
    o.march_batch = host_cands[c].march_batch;
    o.march_packets = host_cands[c].march_packets;
    s = mr_render(field, mesh, n, origins, dirs, max_bounces, per_ray_max_bounces, host_lights, n_lights, &o, out,
                  workspace, workspace_bytes, stream);
    if (s != MR_OK) break;
    if (hipEventRecord(a, st) != hipSuccess) { s = fail(MR_ERR_DEVICE, "event record"); break; }
    for (int r = 0; r < reps && s == MR_OK; ++r)
      s = mr_render(field, mesh, n, origins, dirs, max_bounces, per_ray_max_bounces, host_lights, n_lights, &o, out,
                    workspace, workspace_bytes, stream);
    if (s != MR_OK) break;
    float ms = 0.0f;
    if (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
        hipEventElapsedTime(&ms, a, b) != hipSuccess) {
      s = fail(MR_ERR_DEVICE, "event timing");
      break;
    }
    ms /= reps;
    if (ms < best_t) {
      best_t = ms;
      *best_index = c;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (s == MR_OK) *best_ms = best_t;
  return s;
}

namespace {

// Candidate values of each launch parameter, generated from the device's
// compute units and the queue length.  Axis order: march blocks per CU, stage
// blocks per CU, stage tile, march chunk, march batch, packet segments.
constexpr int kAxes = 6;
constexpr int kAxisMax = 6;
struct TuneAxis {
  int n;
  int v[kAxisMax];
};

void add_value(TuneAxis& a, int v) {
  for (int i = 0; i < a.n; ++i)
    if (a.v[i] == v) return;
  if (a.n < kAxisMax) a.v[a.n++] = v;
}

void tune_axes(int64_t n, int cus, TuneAxis ax[kAxes]) {
  for (int k = 0; k < kAxes; ++k) ax[k].n = 0;
  // march: as many 256-thread blocks as are resident (0), or 1, 2, 4 per CU
  for (int v : {0, 1, 2, 4}) add_value(ax[0], v);
  // closest hit and shade: resident maximum (0), or 2, 4, 8 blocks of 128 per CU
  for (int v : {0, 2, 4, 8}) add_value(ax[1], v);
  // stage tile: 128 rays per grab, and the tiles that give every block of a
  // grid of 8 blocks per CU about 16 and about 4 grabs over the queue
  add_value(ax[2], 128);
  for (int grabs : {16, 4}) {
    int64_t t = n / ((int64_t)cus * 8 * grabs);
    t = std::min<int64_t>(4096, std::max<int64_t>(128, (t / 128) * 128));
    add_value(ax[2], (int)t);
  }
  // march queue: one for the device, or chunks dealt round-robin to the dies
  // (a chunk a few times a die's share of one grab round)
  add_value(ax[3], 0);
  add_value(ax[3], 1024);
  add_value(ax[3], 4096);
  add_value(ax[3], 8192);
  // rays per march queue grab
  for (int v : {1, 2, 4, 8}) add_value(ax[4], v);
  // packets on the camera segment (0), on no segment (-1), or on the first two
  for (int v : {0, -1, 2}) add_value(ax[5], v);
}

int& axis_field(mr_launch_cfg& c, int k) {
  switch (k) {
    case 0: return c.march_blocks_per_cu;
    case 1: return c.stage_blocks_per_cu;
    case 2: return c.stage_tile;
    case 3: return c.march_chunk;
    case 4: return c.march_batch;
    default: return c.march_packets;
  }
}

void apply_cfg(mr_render_opts& o, const mr_launch_cfg& c) {
  o.march_blocks_per_cu = c.march_blocks_per_cu;
  o.stage_blocks_per_cu = c.stage_blocks_per_cu;
  o.stage_tile = c.stage_tile;
  o.march_chunk = c.march_chunk;
  o.march_batch = c.march_batch;
  o.march_packets = c.march_packets;
}

}  // namespace

extern "C" mr_status mr_autotune_candidates(int64_t n, int32_t* counts, int32_t* values) {
  if (n < 0 || !counts || !values) return fail(MR_ERR_INVALID_ARG, "null argument or n < 0");
  TuneAxis ax[kAxes];
  tune_axes(n, device_cus(), ax);
  for (int k = 0; k < kAxes; ++k) {
    counts[k] = ax[k].n;
    for (int i = 0; i < kAxisMax; ++i) values[k * kAxisMax + i] = i < ax[k].n ? ax[k].v[i] : 0;
  }
  return MR_OK;
}

extern "C" mr_status mr_autotune_search(const mr_field* field, const mr_mesh* mesh, int64_t n, const float* origins,
                                        const float* dirs, int32_t max_bounces, const int32_t* per_ray_max_bounces,
                                        const mr_light* host_lights, int32_t n_lights, const mr_render_opts* opts,
                                        mr_render_out* out, void* workspace, size_t workspace_bytes, int32_t reps,
                                        int32_t passes, mr_launch_cfg* best, float* best_ms, float* start_ms,
                                        int32_t* n_timed, void* stream) {
  if (!opts || !best || !best_ms) return fail(MR_ERR_INVALID_ARG, "null argument");
  if (reps < 1 || reps > 100) return fail(MR_ERR_INVALID_ARG, "reps must be in 1..100");
  if (passes < 1 || passes > 4) return fail(MR_ERR_INVALID_ARG, "passes must be in 1..4");
  mr_status s = validate_render(field, mesh, n, origins, dirs, max_bounces, host_lights, n_lights, opts, out);
  if (s != MR_OK) return s;
  if (!workspace || workspace_bytes < mr_render_workspace_size(n))
    return fail(MR_ERR_INVALID_ARG, "workspace smaller than mr_render_workspace_size(n)");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t a = nullptr, b = nullptr;
  MR_HIP(hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return fail(MR_ERR_DEVICE, "event create");
  }
  // mean time of reps renders with launch shape c, after one warm-up render
  auto time_cfg = [&](const mr_launch_cfg& c, float& ms) -> mr_status {
    mr_render_opts o = *opts;
    apply_cfg(o, c);
    mr_status r = mr_render(field, mesh, n, origins, dirs, max_bounces, per_ray_max_bounces, host_lights, n_lights,
                            &o, out, workspace, workspace_bytes, stream);
    if (r != MR_OK) return r;
    if (hipEventRecord(a, st) != hipSuccess) return fail(MR_ERR_DEVICE, "event record");
    for (int i = 0; i < reps && r == MR_OK; ++i)
      r = mr_render(field, mesh, n, origins, dirs, max_bounces, per_ray_max_bounces, host_lights, n_lights, &o, out,
                    workspace, workspace_bytes, stream);
    if (r != MR_OK) return r;
    if (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
        hipEventElapsedTime(&ms, a, b) != hipSuccess)
      return fail(MR_ERR_DEVICE, "event timing");
    ms /= reps;
    return MR_OK;
  };
  // coordinate descent from the caller's launch shape: one axis at a time,
  // every candidate value of it with the others held, keeping the fastest
  TuneAxis ax[kAxes];
  tune_axes(n, device_cus(), ax);
  mr_launch_cfg cur = {opts->march_blocks_per_cu, opts->stage_blocks_per_cu, opts->stage_tile, opts->march_chunk,
                       opts->march_batch, opts->march_packets};
  float cur_ms = 0.0f;
  int timed = 0;
  s = time_cfg(cur, cur_ms);
  ++timed;
  const float first_ms = cur_ms;
  for (int p = 0; p < passes && s == MR_OK; ++p) {
    bool moved = false;
    for (int k = 0; k < kAxes && s == MR_OK; ++k)
      for (int i = 0; i < ax[k].n && s == MR_OK; ++i) {
        if (ax[k].v[i] == axis_field(cur, k)) continue;
        mr_launch_cfg c = cur;
        axis_field(c, k) = ax[k].v[i];
        float ms = 0.0f;
        s = time_cfg(c, ms);
        ++timed;
        if (s == MR_OK && ms < cur_ms) {
          cur = c;
          cur_ms = ms;
          moved = true;
        }
      }
    if (!moved) break;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (s != MR_OK) return s;
  *best = cur;
  *best_ms = cur_ms;
  if (start_ms) *start_ms = first_ms;
  if (n_timed) *n_timed = timed;
  // leave the outputs holding the render of the chosen shape
  mr_render_opts o = *opts;
  apply_cfg(o, cur);
  return mr_render(field, mesh, n, origins, dirs, max_bounces, per_ray_max_bounces, host_lights, n_lights, &o, out,
                   workspace, workspace_bytes, stream);
}

namespace {
struct CamLimits {
  int n;
  int lim[64];
};
__global__ void k_cam_limits(const int32_t* __restrict__ ci, int64_t n, CamLimits L, int32_t* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int c = ci[i];
    out[i] = (c >= 0 && c < L.n) ? L.lim[c] : 0;
  }
}
}  // namespace

extern "C" mr_status mr_camera_bounce_limits(const int32_t* cam_index, int64_t n, const int32_t* host_cam_limits,
                                             int32_t n_cams, int32_t* out, void* stream) {
  if (n < 0) return fail(MR_ERR_INVALID_ARG, "n < 0");
  if (n == 0) return MR_OK;
  if (!cam_index || !out || !host_cam_limits) return fail(MR_ERR_INVALID_ARG, "null array");
  if (n_cams < 1 || n_cams > 64) return fail(MR_ERR_INVALID_ARG, "n_cams must be in 1..64");
  CamLimits L;
  L.n = n_cams;
  for (int c = 0; c < n_cams; ++c) {
    if (host_cam_limits[c] < 0 || host_cam_limits[c] > kMaxBounces) return fail(MR_ERR_INVALID_ARG, "limit out of range");
    L.lim[c] = host_cam_limits[c];
  }
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 65535);
  hipLaunchKernelGGL(k_cam_limits, dim3(blocks), dim3(256), 0, (hipStream_t)stream, cam_index, n, L, out);
  MR_HIP(hipGetLastError());
  return MR_OK;
}
