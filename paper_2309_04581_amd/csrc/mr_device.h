// Device building blocks of the marcher: Philox, hash-grid encoding, SH, the
// per-thread density MLP of the occupancy grid, the watertight ray-triangle
// test and BVH traversal with a per-thread stack in LDS.
#pragma once
#include "mr_common.h"

namespace mr {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11), keyed by (seed, 0), counter
// (ray id, segment, purpose, 0); u = (x >> 8) * 2^-24 is exact in FP32.
// ---------------------------------------------------------------------------
enum { kRngGlass = 0, kRngDiffuse = 1, kRngRoulette = 2, kRngEmitter = 3 };

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

__device__ __forceinline__ float u01(uint32_t x) { return (float)(x >> 8) * (1.0f / 16777216.0f); }

__device__ __forceinline__ float4 draw4(uint32_t seed, uint32_t ray, uint32_t seg, uint32_t purpose) {
  uint4 o = philox4x32_10(make_uint4(ray, seg, purpose, 0u), seed, 0u);
  return make_float4(u01(o.x), u01(o.y), u01(o.z), u01(o.w));
}

// ---------------------------------------------------------------------------
// small vector helpers
// ---------------------------------------------------------------------------
struct V3 { float x, y, z; };
__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return V3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator*(float s, V3 a) { return V3{s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return V3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ float comp(V3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }

// ---------------------------------------------------------------------------
// hash-grid encoding: NL levels x 2 features, FP32 interpolation of an FP32
// or FP16 table.  Vertex indices: dense when (N+1)^3 <= T, else the spatial
// hash with primes (1, 2654435761, 805459861), uint32 wrap-around.
// ---------------------------------------------------------------------------
template <typename TabT>
__device__ __forceinline__ float2 load_entry(const TabT* tab, uint32_t idx);
template <>
__device__ __forceinline__ float2 load_entry<float>(const float* tab, uint32_t idx) {
  return reinterpret_cast<const float2*>(tab)[idx];
}
template <>
__device__ __forceinline__ float2 load_entry<__half>(const __half* tab, uint32_t idx) {
  const __half2 h = reinterpret_cast<const __half2*>(tab)[idx];
  return __half22float2(h);
}

__device__ __forceinline__ void to_unit(const FieldView& F, float px, float py, float pz,
                                        float& xh, float& yh, float& zh) {
  xh = fminf(fmaxf((px - F.amin[0]) * F.inv_ext[0], 0.0f), 1.0f);
  yh = fminf(fmaxf((py - F.amin[1]) * F.inv_ext[1], 0.0f), 1.0f);
  zh = fminf(fmaxf((pz - F.amin[2]) * F.inv_ext[2], 0.0f), 1.0f);
}

// A world-space point and direction in the field's own frame (rigid, so a
// ray keeps its parameter t): p -> R^T (p - c), d -> R^T d.
__device__ __forceinline__ void to_field_frame(const FieldView& F, float& px, float& py, float& pz, float& dx,
                                               float& dy, float& dz) {
  if (!F.has_pose) return;
  const float* P = F.pose;
  const float qx = px - P[3], qy = py - P[7], qz = pz - P[11];
  px = P[0] * qx + P[4] * qy + P[8] * qz;
  py = P[1] * qx + P[5] * qy + P[9] * qz;
  pz = P[2] * qx + P[6] * qy + P[10] * qz;
  const float ex = dx, ey = dy, ez = dz;
  dx = P[0] * ex + P[4] * ey + P[8] * ez;
  dy = P[1] * ex + P[5] * ey + P[9] * ez;
  dz = P[2] * ex + P[6] * ey + P[10] * ez;
}

// The inverse map for points: field frame -> world, p -> R p + c.
__device__ __forceinline__ void field_to_world(const FieldView& F, float& px, float& py, float& pz) {
  if (!F.has_pose) return;
  const float* P = F.pose;
  const float x = px, y = py, z = pz;
  px = P[0] * x + P[1] * y + P[2] * z + P[3];
  py = P[4] * x + P[5] * y + P[6] * z + P[7];
  pz = P[8] * x + P[9] * y + P[10] * z + P[11];
}

// Corner indices and trilinear weights of one level.
__device__ __forceinline__ void level_corners(const FieldView& F, int l, float xh, float yh, float zh,
                                              uint32_t idx[8], float w[8]) {
  const int N = F.res[l];
  const float fN = (float)N;
  const float fx = xh * fN, fy = yh * fN, fz = zh * fN;
  const float flx = fminf(floorf(fx), fN - 1.0f), fly = fminf(floorf(fy), fN - 1.0f),
              flz = fminf(floorf(fz), fN - 1.0f);
  const uint32_t vx = (uint32_t)flx, vy = (uint32_t)fly, vz = (uint32_t)flz;
  const float wx = fx - flx, wy = fy - fly, wz = fz - flz;
  if ((F.dense_mask >> l) & 1u) {
    const uint32_t n1 = (uint32_t)N + 1u, n2 = n1 * n1;
    const uint32_t base = vx + vy * n1 + vz * n2;
#pragma unroll
    for (int c = 0; c < 8; ++c)
      idx[c] = base + (c & 1) + ((c >> 1) & 1) * n1 + ((c >> 2) & 1) * n2;
  } else {
    const uint32_t hy0 = vy * 2654435761u, hy1 = (vy + 1u) * 2654435761u;
    const uint32_t hz0 = vz * 805459861u, hz1 = (vz + 1u) * 805459861u;
#pragma unroll
    for (int c = 0; c < 8; ++c)
      idx[c] = ((vx + (c & 1)) ^ ((c & 2) ? hy1 : hy0) ^ ((c & 4) ? hz1 : hz0)) & F.table_mask;
  }
#pragma unroll
  for (int c = 0; c < 8; ++c)
    w[c] = ((c & 1) ? wx : 1.0f - wx) * ((c & 2) ? wy : 1.0f - wy) * ((c & 4) ? wz : 1.0f - wz);
}

template <int NL, typename TabT>
__device__ __forceinline__ void hash_encode(const FieldView& F, const TabT* __restrict__ table,
                                            float px, float py, float pz, float* feat) {
  float xh, yh, zh;
  to_unit(F, px, py, pz, xh, yh, zh);
  const size_t T = (size_t)F.table_mask + 1u;
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    uint32_t idx[8];
    float w[8];
    level_corners(F, l, xh, yh, zh, idx, w);
    const TabT* tab = table + (size_t)l * T * 2;
    float2 e[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) e[c] = load_entry<TabT>(tab, idx[c]);
    float f0 = 0.0f, f1 = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      f0 += w[c] * e[c].x;
      f1 += w[c] * e[c].y;
    }
    feat[2 * l] = f0;
    feat[2 * l + 1] = f1;
  }
}

// Real orthonormal SH (Sloan's ordering, Condon-Shortley phase), n = 4 or 16.
template <int SH>
__device__ __forceinline__ void sh_eval(float x, float y, float z, float* o) {
  o[0] = 0.28209479177387814f;
  o[1] = -0.48860251190291987f * y;
  o[2] = 0.48860251190291987f * z;
  o[3] = -0.48860251190291987f * x;
  if constexpr (SH > 4) {
    const float xx = x * x, yy = y * y, zz = z * z;
    o[4] = 1.0925484305920792f * x * y;
    o[5] = -1.0925484305920792f * y * z;
    o[6] = 0.31539156525252005f * (3.0f * zz - 1.0f);
    o[7] = -1.0925484305920792f * x * z;
    o[8] = 0.54627421529603959f * (xx - yy);
    o[9] = -0.59004358992664352f * y * (3.0f * xx - yy);
    o[10] = 2.8906114426405538f * x * y * z;
    o[11] = -0.45704579946446572f * y * (5.0f * zz - 1.0f);
    o[12] = 0.3731763325901154f * z * (5.0f * zz - 3.0f);
    o[13] = -0.45704579946446572f * x * (5.0f * zz - 1.0f);
    o[14] = 1.4453057213202769f * z * (xx - yy);
    o[15] = -0.59004358992664352f * x * (xx - 3.0f * yy);
  }
}

// e^x on the hardware base-2 exponential: 2^(x log2 e), about 1 ulp.
__device__ __forceinline__ float exp_hw(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }

// softplus(x) = max(x, 0) + log1p(e^-|x|) on the hardware exponential and
// base-2 logarithm.  log1p(v) = log(w) v / (w - 1) with w = 1 + v rounded
// (Goldberg, "What every computer scientist should know about
// floating-point arithmetic", 1991): the ratio cancels the rounding of 1 + v,
// so small densities keep their relative accuracy; for w = 1, log1p(v) = v.
__device__ __forceinline__ float softplusf(float x) {
  const float v = exp_hw(-fabsf(x));
  const float w = 1.0f + v;
  const float l = w == 1.0f ? v : 0.6931471805599453f * __builtin_amdgcn_logf(w) * (v / (w - 1.0f));
  return fmaxf(x, 0.0f) + l;
}

// ---------------------------------------------------------------------------
// density MLP on one sample per lane (occupancy grid), weights broadcast from
// LDS: W0 [64][32] at 0, W1 [16][64] at 2048.
// ---------------------------------------------------------------------------

template <int NIN>
__device__ __forceinline__ float dot_row(const float* __restrict__ w, const float* x) {
  float acc = 0.0f;
#pragma unroll
  for (int i = 0; i < NIN; i += 4) {
    const float4 q = *reinterpret_cast<const float4*>(w + i);
    acc += q.x * x[i];
    if (i + 1 < NIN) acc += q.y * x[i + 1];
    if (i + 2 < NIN) acc += q.z * x[i + 2];
    if (i + 3 < NIN) acc += q.w * x[i + 3];
  }
  return acc;
}

// density MLP: 2*NL features -> 64 (ReLU) -> 16 raw outputs
template <int NL>
__device__ __forceinline__ void density_mlp(const float* __restrict__ W, const float* feat, float* raw) {
#pragma unroll
  for (int k = 0; k < 16; ++k) raw[k] = 0.0f;
  for (int j = 0; j < 64; ++j) {
    const float h = fmaxf(dot_row<2 * NL>(W + 0 + j * 32, feat), 0.0f);
#pragma unroll
    for (int k = 0; k < 16; ++k) raw[k] += W[2048 + k * 64 + j] * h;
  }
}

// ---------------------------------------------------------------------------
// watertight ray-triangle test (Woop, Benthin, Wald, JCGT 2013) in FP32,
// evaluated without FMA contraction so that a shared edge gives the two
// triangles exactly opposite edge functions.
// ---------------------------------------------------------------------------
struct RayPre {
  V3 o, d, inv;
  int kx, ky, kz;
  float Sx, Sy, Sz;
};

__device__ __forceinline__ RayPre ray_pre(V3 o, V3 d) {
  RayPre r;
  r.o = o;
  r.d = d;
  const float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
  r.kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
  r.kx = r.kz == 2 ? 0 : r.kz + 1;
  r.ky = r.kx == 2 ? 0 : r.kx + 1;
  if (comp(d, r.kz) < 0.0f) { const int t = r.kx; r.kx = r.ky; r.ky = t; }
  const float dz = comp(d, r.kz);
  r.Sx = comp(d, r.kx) / dz;
  r.Sy = comp(d, r.ky) / dz;
  r.Sz = 1.0f / dz;
  // box-test reciprocals; a zero component becomes a huge finite value so no NaN appears
  r.inv = v3(1.0f / (d.x != 0.0f ? d.x : copysignf(1e-30f, d.x)),
             1.0f / (d.y != 0.0f ? d.y : copysignf(1e-30f, d.y)),
             1.0f / (d.z != 0.0f ? d.z : copysignf(1e-30f, d.z)));
  return r;
}

// returns t (or +inf on a miss); accepts 0 < t
__device__ __forceinline__ float tri_hit(const RayPre& r, float4 p0, float4 p1, float4 p2) {
#pragma clang fp contract(off)
  const V3 A = v3(p0.x, p0.y, p0.z) - r.o, B = v3(p1.x, p1.y, p1.z) - r.o, C = v3(p2.x, p2.y, p2.z) - r.o;
  const float Az = comp(A, r.kz), Bz = comp(B, r.kz), Cz = comp(C, r.kz);
  const float Ax = comp(A, r.kx) - r.Sx * Az, Ay = comp(A, r.ky) - r.Sy * Az;
  const float Bx = comp(B, r.kx) - r.Sx * Bz, By = comp(B, r.ky) - r.Sy * Bz;
  const float Cx = comp(C, r.kx) - r.Sx * Cz, Cy = comp(C, r.ky) - r.Sy * Cz;
  const float U = Cx * By - Cy * Bx;
  const float V = Ax * Cy - Ay * Cx;
  const float W = Bx * Ay - By * Ax;
  if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return INFINITY;
  const float det = U + V + W;
  if (det == 0.0f) return INFINITY;
  const float T = U * (r.Sz * Az) + V * (r.Sz * Bz) + W * (r.Sz * Cz);
  const float t = T / det;
  return t > 0.0f ? t : INFINITY;
}

// Conservative slab test of one box against [0, tmax] (tmax scaled by
// 1 + 2 gamma_3 after Ize 2013); returns the entry distance or +inf.
__device__ __forceinline__ float box_hit(const RayPre& r, float lx, float ly, float lz, float hx,
                                         float hy, float hz, float tmax) {
  const float tx0 = (lx - r.o.x) * r.inv.x, tx1 = (hx - r.o.x) * r.inv.x;
  const float ty0 = (ly - r.o.y) * r.inv.y, ty1 = (hy - r.o.y) * r.inv.y;
  const float tz0 = (lz - r.o.z) * r.inv.z, tz1 = (hz - r.o.z) * r.inv.z;
  const float tn = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), 0.0f));
  const float tf = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fminf(fmaxf(tz0, tz1), tmax));
  return tn <= tf * 1.0000003576f ? tn : INFINITY;
}

// Closest hit (ANY = false): lexicographic minimum of (t, original id) over
// 0 < t <= tmax.  Any hit (ANY = true): returns >= 0 for the first hit with
// 0 < t < tmax.  stack: this thread's LDS stack, entry k at stack[k * stride];
// tstack (closest hit only): the entry distance of each pending node, so that
// a node whose box starts beyond the best hit found since it was pushed is
// dropped without loading it (its children start no earlier than it does).
template <bool ANY>
__device__ __forceinline__ int bvh_trace(const BvhView& B, const RayPre& r, float tmax, float& t_best,
                                         int* stack, float* tstack, int stride) {
  int best = -1, best_id = 0x7fffffff;
  t_best = tmax;
  int sp = 0;
  int node = 0;
  if (B.n_prims == 0) return -1;
  while (true) {
    const BvhNode n = B.nodes[node];
    const float lim = ANY ? tmax : t_best;
    const float t0 = n.d.x < 0 ? INFINITY : box_hit(r, n.a.x, n.a.y, n.a.z, n.a.w, n.b.x, n.b.y, lim);
    const float t1 = n.d.y < 0 ? INFINITY : box_hit(r, n.b.z, n.b.w, n.c.x, n.c.y, n.c.z, n.c.w, lim);
    int next = -1;
    // leaves are tested at once; inner children are visited near-first
    int inner[2], ninner = 0;
    float tin[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const float tc = c == 0 ? t0 : t1;
      if (tc == INFINITY) continue;
      const int child = c == 0 ? n.d.x : n.d.y, cnt = c == 0 ? n.d.z : n.d.w;
      if (cnt > 0) {
        for (int p = child; p < child + cnt; ++p) {
          const float4 q0 = B.tris[3 * p], q1 = B.tris[3 * p + 1], q2 = B.tris[3 * p + 2];
          const float t = tri_hit(r, q0, q1, q2);
          if (ANY) {
            if (t < tmax) { t_best = t; return p; }
          } else if (t <= tmax) {
            const int id = __float_as_int(q0.w);
            if (t < t_best || (t == t_best && id < best_id)) { t_best = t; best = p; best_id = id; }
          }
        }
      } else {
        inner[ninner] = child;
        tin[ninner] = tc;
        ++ninner;
      }
    }
    if (ninner == 2) {
      const bool swap = tin[1] < tin[0];
      next = swap ? inner[1] : inner[0];
      stack[sp * stride] = swap ? inner[0] : inner[1];
      if constexpr (!ANY) tstack[sp * stride] = swap ? tin[0] : tin[1];
      ++sp;
    } else if (ninner == 1) {
      next = inner[0];
    }
    if (next < 0) {
      if constexpr (ANY) {
        if (sp == 0) break;
        --sp;
        next = stack[sp * stride];
      } else {
        // the box test accepts entry distances up to its limit times 1.0000003576
        const float reach = t_best * 1.0000003576f;
        while (sp > 0) {
          --sp;
          if (tstack[sp * stride] <= reach) {
            next = stack[sp * stride];
            break;
          }
        }
        if (next < 0) break;
      }
    }
    node = next;
  }
  return best;
}

}  // namespace mr
