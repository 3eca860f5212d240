// Matrix-core (MFMA) evaluation of the field MLPs on 16-sample tiles.
//
// One wave evaluates 16 samples at a time.  Lane l serves sample j = l % 16
// and, for the hash encoding, the level group g = l / 16 (levels
// g*NL/4 .. (g+1)*NL/4 - 1).  The features a lane gathers are exactly the
// B-operand values it owns in v_mfma_f32_16x16x32_bf16 (eight K values per
// lane, lane l holding k = 8 (l / 16) .. 8 (l / 16) + 7) or, where a layer's
// K is 16, v_mfma_f32_16x16x16bf16 (four K values per lane) for the product
// W (M = output rows) x X^T (N = 16 samples).  A 16x16 accumulator leaves
// row 4g + v, column j in register v of lane l, which is again the B layout of
// the next layer up to a fixed permutation of K; the weight fragments staged
// in LDS are written in that permuted order once, on the host.
//
// Two MLP precisions share that shape.  BF16: operands rounded to BF16, FP32
// accumulation.  FP32: every FP32 weight and input is held as three BF16
// pieces that add up to it exactly, and six of the nine piece products are
// accumulated in FP32; what is dropped is at most 2^-26 of each product,
// below the 2^-24 rounding of an FP32 multiply, so the result has FP32
// accuracy at the BF16 instruction rate (six BF16 instructions in place of
// the eight v_mfma_f32_16x16x4f32 a K of 32 takes, each of those twice as
// long).  The per-ray SH product (sh_rows) stays on v_mfma_f32_16x16x4f32.
#pragma once
#include "mr_device.h"

namespace mr {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef short s4v __attribute__((ext_vector_type(4)));

// K values per lane of one BF16 fragment of each layer kind (layer kinds:
// 0 density layer 1 over the features, 1 layers over 64 hidden units, 2
// colour layer 1 over the 16 raw outputs): 8 (the 16x16x32 instruction)
// where a step can take 32 K values, 4 (16x16x16) where the layer's K is 16.
__host__ __device__ constexpr int bf_kpl(int kind, int nf) { return kind == 2 ? 4 : (kind == 0 && nf % 8 ? 4 : 8); }

// Fragment layout sizes (in 32-bit words) for a field shape.  Both MLP
// precisions use the BF16 fragment shape; BF16 weights are one piece, FP32
// weights three BF16 pieces w = w0 + w1 + w2 (exact: each residual has at
// most 16, then 8, significant bits), stored one after the other per layer.
template <int NL, int SH, int CL, bool BF>
struct FragLayout {
  static constexpr int NF = NL / 2;                          // features per lane (2 per level, NL/4 levels)
  static constexpr int NP = BF ? 1 : 3;                      // BF16 pieces per weight
  static constexpr int KP1 = bf_kpl(0, NF);                  // K values per lane, density layer 1
  static constexpr int KP2 = bf_kpl(1, NF);                  // over 64 hidden units
  static constexpr int KPC = bf_kpl(2, NF);                  // over the 16 raw outputs
  static constexpr int KS1 = NF / KP1;                       // K steps, density layer 1
  static constexpr int KS2 = 16 / KP2;                       // K steps over 64 hidden units
  static constexpr int KSC = 4 / KPC;                        // K steps over the 16 raw outputs
  static constexpr int W1 = KP1 / 2;                         // words per lane per fragment
  static constexpr int W2 = KP2 / 2;
  static constexpr int WC = KPC / 2;
  static constexpr int P1 = 4 * KS1 * 64 * W1;               // words of one piece of each layer
  static constexpr int P2 = KS2 * 64 * W2;
  static constexpr int PC = 4 * KSC * 64 * WC;
  static constexpr int PC2 = 4 * KS2 * 64 * W2;
  static constexpr int L1 = 0;                               // [piece][4 mt][KS1] fragments
  static constexpr int L2 = L1 + NP * P1;                    // [piece][KS2]
  static constexpr int C1 = L2 + NP * P2;                    // [piece][4 mt][KSC]
  static constexpr int C2 = C1 + NP * PC;                    // [piece][4 mt][KS2] (two hidden colour layers)
  static constexpr int OUT = C2 + (CL == 2 ? NP * PC2 : 0);  // FP32 [3][64]
  static constexpr int SHW = OUT + 192;                      // FP32 [4 mt][SH/4][64]: SH columns of colour layer 1
  static constexpr int TOTAL = SHW + 64 * SH;
};

// K index carried by (step ks, lane group g, element e) for each layer kind.
__host__ __device__ inline int frag_k(int kind, int nf, int ks, int g, int e) {
  const int kp = bf_kpl(kind, nf);
  if (kind == 0) {
    // lane group g holds levels g, g + 4, g + 8, ... (register r: level 4 (r / 2) + g, feature r % 2)
    const int r = kp * ks + e;
    return 8 * (r >> 1) + 2 * g + (r & 1);
  }
  // the previous layer's outputs in C layout: unit 16 mt + 4 g + v (raw
  // output 4 g + v) in register v of tile mt; q counts the lane's registers
  // in the order the steps take them
  const int q = kp * ks + e;
  if (kind == 1) return (q >> 2) * 16 + 4 * g + (q & 3);
  return 4 * g + q;
}

__device__ __forceinline__ f4v mma(float a, float b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4v mma(uint2 a, uint2 b, f4v c) {
  // four bf16 values per operand, element 0 in the low half of .x
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4v, a), __builtin_bit_cast(s4v, b), c, 0, 0,
                                                   0);
}
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
__device__ __forceinline__ f4v mma(uint4 a, uint4 b, f4v c) {
  // eight bf16 values per operand (K = 32), element 0 in the low half of .x
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b), c,
                                                 0, 0, 0);
}

// Two FP32 values to bf16 (round to nearest even), the first in the low half:
// one v_cvt_pk_bf16_f32 on gfx950.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack2_bf16(float a, float b) {
  const f32x2_t v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}
__device__ __forceinline__ uint2 pack_bf16(float a, float b, float c, float d) {
  return make_uint2(pack2_bf16(a, b), pack2_bf16(c, d));
}
__device__ __forceinline__ uint4 pack_bf16(const f4v& lo, const f4v& hi) {
  return make_uint4(pack2_bf16(lo[0], lo[1]), pack2_bf16(lo[2], lo[3]), pack2_bf16(hi[0], hi[1]),
                    pack2_bf16(hi[2], hi[3]));
}

// FP32 values as three BF16 pieces, x = x0 + x1 + x2 exactly (each step
// rounds to nearest even, and a residual has at most 16, then 8, significant
// bits).  A product of two split values keeps the six piece products down to
// 2^-16 of its size and drops at most 2^-26 of it, under the 2^-24 rounding
// of an FP32 product; the matrix cores form each BF16 product exactly and sum
// in FP32 (the bf16x6 scheme of Henry, Tang and Heinecke, ARITH 2019).
__device__ __forceinline__ void split3(float a, float b, uint32_t& p0, uint32_t& p1, uint32_t& p2) {
  p0 = pack2_bf16(a, b);
  const float ra = a - __uint_as_float(p0 << 16), rb = b - __uint_as_float(p0 & 0xFFFF0000u);
  p1 = pack2_bf16(ra, rb);
  p2 = pack2_bf16(ra - __uint_as_float(p1 << 16), rb - __uint_as_float(p1 & 0xFFFF0000u));
}
__device__ __forceinline__ void split3(float a, float b, float c, float d, uint2& p0, uint2& p1, uint2& p2) {
  split3(a, b, p0.x, p1.x, p2.x);
  split3(c, d, p0.y, p1.y, p2.y);
}
__device__ __forceinline__ void split3(const f4v& lo, const f4v& hi, uint4& p0, uint4& p1, uint4& p2) {
  split3(lo[0], lo[1], p0.x, p1.x, p2.x);
  split3(lo[2], lo[3], p0.y, p1.y, p2.y);
  split3(hi[0], hi[1], p0.z, p1.z, p2.z);
  split3(hi[2], hi[3], p0.w, p1.w, p2.w);
}
// acc + W X over the six piece products of order <= 2, smallest first
template <typename V>
__device__ __forceinline__ f4v mma6(const V& w0, const V& w1, const V& w2, const V& x0, const V& x1, const V& x2,
                                    f4v acc) {
  acc = mma(w0, x2, acc);
  acc = mma(w2, x0, acc);
  acc = mma(w1, x1, acc);
  acc = mma(w0, x1, acc);
  acc = mma(w1, x0, acc);
  return mma(w0, x0, acc);
}

// ReLU on the bit pattern: positive floats order like positive integers and
// every value with the sign bit set becomes +0, so max_i32(bits, 0) is max(x,
// 0) in one instruction (fmaxf on a matrix-core result first quiets a
// possible signalling NaN, a second instruction per value).
__device__ __forceinline__ float relu(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

// Hash features of the lane's levels for one point (2 per level).  Lane
// group g takes levels g, g + 4, g + 8, ...: at each step ll the four
// groups hold four consecutive levels, so the dense coarse levels fall
// together and the dense-or-hashed choice is uniform across the wave at all
// but one step (it is per lane).
template <int NL, typename TabT>
__device__ __forceinline__ void encode_group(const FieldView& F, const TabT* __restrict__ table, float px, float py,
                                             float pz, int g, float* fe) {
  constexpr int LPG = NL / 4;
  float xh, yh, zh;
  to_unit(F, px, py, pz, xh, yh, zh);
  const size_t T = (size_t)F.table_mask + 1u;
#pragma unroll
  for (int ll = 0; ll < LPG; ++ll) {
    const int l = ll * 4 + g;
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
    fe[2 * ll] = f0;
    fe[2 * ll + 1] = f1;
  }
}

// The two features of level l at a unit-cube point (one level of encode_group).
template <typename TabT>
__device__ __forceinline__ void encode_level(const FieldView& F, const TabT* __restrict__ table, float xh, float yh,
                                             float zh, int l, float& f0, float& f1) {
  const size_t T = (size_t)F.table_mask + 1u;
  uint32_t idx[8];
  float w[8];
  level_corners(F, l, xh, yh, zh, idx, w);
  const TabT* tab = table + (size_t)l * T * 2;
  float2 e[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) e[c] = load_entry<TabT>(tab, idx[c]);
  f0 = 0.0f;
  f1 = 0.0f;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    f0 += w[c] * e[c].x;
    f1 += w[c] * e[c].y;
  }
}

// The MLPs on a 16-sample tile.  fe: this lane's features (its level group,
// its sample); u[mt][v]: the colour layer-1 contribution of the SH inputs for
// hidden row mt*16 + 4g + v (per lane's sample); W: fragments in LDS.
// Returns sigma and rgb of sample j on every lane, and raw in C layout
// (register v = raw output 4g + v of sample j).
template <int NL, int SH, int CL, bool BF>
__device__ __forceinline__ void mlp_tile(const uint32_t* __restrict__ W, const float* fe, const float (&u)[4][4],
                                         float density_offset, int lane, float& sigma, float rgb[3], f4v& raw) {
  using LY = FragLayout<NL, SH, CL, BF>;
  const int g = lane >> 4, j = lane & 15;
  const f4v zero = {0.0f, 0.0f, 0.0f, 0.0f};
  // density layer 1: 64 hidden x 16 samples
  f4v h[4] = {zero, zero, zero, zero};
  if constexpr (LY::KP1 == 8) {
    const uint4* Wb = reinterpret_cast<const uint4*>(W);
#pragma unroll
    for (int ks = 0; ks < LY::KS1; ++ks) {
      const f4v lo = {fe[8 * ks], fe[8 * ks + 1], fe[8 * ks + 2], fe[8 * ks + 3]};
      const f4v hi = {fe[8 * ks + 4], fe[8 * ks + 5], fe[8 * ks + 6], fe[8 * ks + 7]};
      if constexpr (BF) {
        const uint4 b = pack_bf16(lo, hi);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) h[mt] = mma(Wb[LY::L1 / 4 + (mt * LY::KS1 + ks) * 64 + lane], b, h[mt]);
      } else {
        uint4 x0, x1, x2;
        split3(lo, hi, x0, x1, x2);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
          const int o = LY::L1 / 4 + (mt * LY::KS1 + ks) * 64 + lane;
          h[mt] = mma6(Wb[o], Wb[o + LY::P1 / 4], Wb[o + LY::P1 / 2], x0, x1, x2, h[mt]);
        }
      }
    }
  } else {
    const uint2* Wb = reinterpret_cast<const uint2*>(W);
#pragma unroll
    for (int ks = 0; ks < LY::KS1; ++ks) {
      if constexpr (BF) {
        const uint2 b = pack_bf16(fe[4 * ks], fe[4 * ks + 1], fe[4 * ks + 2], fe[4 * ks + 3]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) h[mt] = mma(Wb[LY::L1 / 2 + (mt * LY::KS1 + ks) * 64 + lane], b, h[mt]);
      } else {
        uint2 x0, x1, x2;
        split3(fe[4 * ks], fe[4 * ks + 1], fe[4 * ks + 2], fe[4 * ks + 3], x0, x1, x2);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
          const int o = LY::L1 / 2 + (mt * LY::KS1 + ks) * 64 + lane;
          h[mt] = mma6(Wb[o], Wb[o + LY::P1 / 2], Wb[o + LY::P1], x0, x1, x2, h[mt]);
        }
      }
    }
  }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int v = 0; v < 4; ++v) h[mt][v] = relu(h[mt][v]);
  // density layer 2: 16 raw outputs, two K steps of 32 hidden units
  f4v rp[2] = {zero, zero};
  {
    const uint4* Wb = reinterpret_cast<const uint4*>(W);
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int o = LY::L2 / 4 + ks * 64 + lane;
      if constexpr (BF) {
        rp[ks] = mma(Wb[o], pack_bf16(h[2 * ks], h[2 * ks + 1]), rp[ks]);
      } else {
        uint4 x0, x1, x2;
        split3(h[2 * ks], h[2 * ks + 1], x0, x1, x2);
        rp[ks] = mma6(Wb[o], Wb[o + LY::P2 / 4], Wb[o + LY::P2 / 2], x0, x1, x2, rp[ks]);
      }
    }
  }
  raw = rp[0] + rp[1];
  sigma = softplusf(__shfl(raw[0], j, 64) + density_offset);
  // colour layer 1: SH part precomputed in u, raw part on the matrix cores
  f4v c[4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int v = 0; v < 4; ++v) c[mt][v] = u[mt][v];
  {
    const uint2* Wb = reinterpret_cast<const uint2*>(W);
    if constexpr (BF) {
      const uint2 b = pack_bf16(raw[0], raw[1], raw[2], raw[3]);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) c[mt] = mma(Wb[LY::C1 / 2 + mt * 64 + lane], b, c[mt]);
    } else {
      uint2 x0, x1, x2;
      split3(raw[0], raw[1], raw[2], raw[3], x0, x1, x2);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        const int o = LY::C1 / 2 + mt * 64 + lane;
        c[mt] = mma6(Wb[o], Wb[o + LY::PC / 2], Wb[o + LY::PC], x0, x1, x2, c[mt]);
      }
    }
  }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int v = 0; v < 4; ++v) c[mt][v] = relu(c[mt][v]);
  if constexpr (CL == 2) {
    f4v c2[4] = {zero, zero, zero, zero};
    const uint4* Wb = reinterpret_cast<const uint4*>(W);
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      if constexpr (BF) {
        const uint4 b = pack_bf16(c[2 * ks], c[2 * ks + 1]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) c2[mt] = mma(Wb[LY::C2 / 4 + (mt * 2 + ks) * 64 + lane], b, c2[mt]);
      } else {
        uint4 x0, x1, x2;
        split3(c[2 * ks], c[2 * ks + 1], x0, x1, x2);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
          const int o = LY::C2 / 4 + (mt * 2 + ks) * 64 + lane;
          c2[mt] = mma6(Wb[o], Wb[o + LY::PC2 / 4], Wb[o + LY::PC2 / 2], x0, x1, x2, c2[mt]);
        }
      }
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) c[mt][v] = relu(c2[mt][v]);
  }
  // 3-wide output layer on the vector units, reduced over the four lane groups
  const float* Wo = reinterpret_cast<const float*>(W) + LY::OUT;
  float o[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    float s = 0.0f;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) s += Wo[ch * 64 + mt * 16 + 4 * g + v] * c[mt][v];
    s += __shfl_xor(s, 16, 64);
    s += __shfl_xor(s, 32, 64);
    o[ch] = s;
  }
  rgb[0] = exp_hw(o[0]);
  rgb[1] = exp_hw(o[1]);
  rgb[2] = exp_hw(o[2]);
}

// SH contribution to colour layer 1 for hidden rows mt*16 + 4g + v: the
// product Wc1[:, 16:16+SH] x SH(d_j), where d_j is the direction lane (g, j)
// passes for column j (one ray for all columns, or one ray per column), as
// FP32 MFMAs whose B operand column j is SH(d_j) (lane group g supplies
// component 4 ks + g), so the result lands in the C layout.
template <int NL, int SH, int CL, bool BF>
__device__ __forceinline__ void sh_rows(const uint32_t* __restrict__ W, float dx, float dy, float dz, int lane,
                                        float (&u)[4][4]) {
  using LY = FragLayout<NL, SH, CL, BF>;
  const float* Ws = reinterpret_cast<const float*>(W) + LY::SHW;
  float shv[16];
  sh_eval<SH>(dx, dy, dz, shv);
  const int g = lane >> 4;
  float b[SH / 4];
#pragma unroll
  for (int ks = 0; ks < SH / 4; ++ks) {
    const float s0 = shv[4 * ks], s1 = shv[4 * ks + 1], s2 = shv[4 * ks + 2], s3 = shv[4 * ks + 3];
    b[ks] = g == 0 ? s0 : (g == 1 ? s1 : (g == 2 ? s2 : s3));
  }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f4v acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < SH / 4; ++ks) acc = mma(Ws[(mt * (SH / 4) + ks) * 64 + lane], b[ks], acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) u[mt][v] = acc[v];
  }
}

// Inclusive product scan over the 16 lanes of a row (lane j of the row gets
// v_0 * ... * v_j).
__device__ __forceinline__ float scan16_mul(float v, int j) {
#pragma unroll
  for (int off = 1; off < 16; off <<= 1) {
    const float u = __shfl_up(v, off, 16);
    if (j >= off) v *= u;
  }
  return v;
}

// Sum over the 16 lanes of a row, in every lane of it.
__device__ __forceinline__ float sum16(float v) {
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off, 16);
  return v;
}

// Parameter range [t0, t1] of the ray inside the field's box (field frame);
// false when the ray misses it.
__device__ __forceinline__ bool slab_box(const FieldView& F, float ox, float oy, float oz, float dx, float dy, float dz,
                                         float& t0, float& t1) {
  float lo = -INFINITY, hi = INFINITY;
  const float o[3] = {ox, oy, oz}, d[3] = {dx, dy, dz};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (d[k] == 0.0f) {
      if (o[k] < F.amin[k] || o[k] > F.amax[k]) return false;
      continue;
    }
    const float inv = 1.0f / d[k];
    float a = (F.amin[k] - o[k]) * inv, b = (F.amax[k] - o[k]) * inv;
    if (a > b) { const float t = a; a = b; b = t; }
    lo = fmaxf(lo, a);
    hi = fminf(hi, b);
  }
  t0 = lo;
  t1 = hi;
  return hi > lo;
}

// Occupancy bit of the grid cell holding a field-frame point.
__device__ __forceinline__ bool occ_lookup(const FieldView& F, float px, float py, float pz) {
  float xh, yh, zh;
  to_unit(F, px, py, pz, xh, yh, zh);
  const int R = F.occ_res;
  const int cx = min((int)(xh * R), R - 1), cy = min((int)(yh * R), R - 1), cz = min((int)(zh * R), R - 1);
  const int64_t c = ((int64_t)cz * R + cy) * R + cx;
  return (F.occ[c >> 5] >> (c & 31)) & 1u;
}

}  // namespace mr
