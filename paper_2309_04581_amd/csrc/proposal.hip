// Learned proposal sampler: a small density-only hash grid + MLP whose
// weights along a segment place the fine field samples (32 + 32 instead of a
// dense uniform grid), trained on the plain marcher's weight histograms with
// the project's own forward, backward and Adam kernels.
//
// The paper marches every segment with the field (Eq. 10-11) and does not use
// a proposal network; this sampler follows the proposal loss of Mip-NeRF 360
// (Barron et al., CVPR 2022).  Proposal weights w_j = T_j alpha_j on n_p
// uniform intervals of [lo, hi], dilated to max(w_{j-1}, w_j, w_{j+1}) and
// mixed half and half with a uniform density (plus 1e-3/n_p), give a
// piecewise-constant density; the n_f + 1 edges of the fine intervals are its
// inverse CDF at u = k/n_f.  The loss per segment is
// sum_j max(0, h_j - w_j)^2 / (h_j + 1e-7) against the histogram h of the
// plain marcher's weights over the same n_p bins.
#include <cmath>
#include <cstring>
#include <vector>

#include "mr_field_kernels.h"
#include "mr_mfma.h"
#include "mr_render.h"

using namespace mr;

namespace {

constexpr int kPropLevels = 5;
constexpr int kPropIn = 10, kPropHidden = 16, kPropMlp = kPropIn * kPropHidden + kPropHidden;

__device__ __forceinline__ float wscan_mul(float v, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const float u = __shfl_up(v, off, 64);
    if (lane >= off) v *= u;
  }
  return v;
}
__device__ __forceinline__ float wscan_add(float v, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const float u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  return v;
}
__device__ __forceinline__ float wsum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ float sc16_mul(float v, int j) {
#pragma unroll
  for (int off = 1; off < 16; off <<= 1) {
    const float u = __shfl_up(v, off, 16);
    if (j >= off) v *= u;
  }
  return v;
}
__device__ __forceinline__ float s16(float v) {
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off, 16);
  return v;
}

__device__ __forceinline__ bool seg_box(const FieldView& F, float ox, float oy, float oz, float dx, float dy, float dz,
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

__device__ __forceinline__ bool occ_bit(const FieldView& F, float px, float py, float pz) {
  float xh, yh, zh;
  to_unit(F, px, py, pz, xh, yh, zh);
  const int R = F.occ_res;
  const int cx = min((int)(xh * R), R - 1), cy = min((int)(yh * R), R - 1), cz = min((int)(zh * R), R - 1);
  const int64_t c = ((int64_t)cz * R + cy) * R + cx;
  return (F.occ[c >> 5] >> (c & 31)) & 1u;
}

// Proposal density at one point (one sample per lane); optionally returns the
// hash features and the hidden pre-activations for the backward pass.
template <typename TabT>
__device__ __forceinline__ float prop_density(const FieldView& P, const TabT* __restrict__ table,
                                              const float* __restrict__ W, float px, float py, float pz, float* feat,
                                              float* hpre, float& z) {
  hash_encode<kPropLevels, TabT>(P, table, px, py, pz, feat);
  float acc = 0.0f;
#pragma unroll
  for (int i = 0; i < kPropHidden; ++i) {
    float h = 0.0f;
#pragma unroll
    for (int c = 0; c < kPropIn; ++c) h += W[i * kPropIn + c] * feat[c];
    hpre[i] = h;
    acc += W[kPropIn * kPropHidden + i] * fmaxf(h, 0.0f);
  }
  z = acc;
  return softplusf(acc + P.density_offset);
}

// Forward-only proposal density for the march.  The hidden loop stays rolled
// so the 176 weights are read from LDS as they are used instead of being held
// in registers across the whole segment.
template <typename TabT>
__device__ __forceinline__ float prop_sigma(const FieldView& P, const TabT* __restrict__ table,
                                           const float* __restrict__ W, float px, float py, float pz) {
  float feat[kPropIn];
  hash_encode<kPropLevels, TabT>(P, table, px, py, pz, feat);
  float acc = 0.0f;
#pragma unroll 1
  for (int i = 0; i < kPropHidden; ++i) {
    float h = 0.0f;
#pragma unroll
    for (int c = 0; c < kPropIn; ++c) h += W[i * kPropIn + c] * feat[c];
    acc += W[kPropIn * kPropHidden + i] * fmaxf(h, 0.0f);
  }
  return softplusf(acc + P.density_offset);
}

// ---------------------------------------------------------------------------
// proposal-sampled march (one wave per ray)
// ---------------------------------------------------------------------------
template <int NL, int SH, int CL, typename TabT, bool BF, typename PTabT, bool SHADOW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_march_prop(RayQueue q, const int* __restrict__ count, int* __restrict__ work,
                                                    FieldView F, const TabT* __restrict__ table,
                                                    const uint32_t* __restrict__ frags, FieldView Pf,
                                                    const PTabT* __restrict__ ptable, MarchParams P, BvhView B,
                                                    int n_prop, int n_fine, unsigned long long* __restrict__ stats) {
  using LY = FragLayout<NL, SH, CL, BF>;
  __shared__ __align__(16) uint32_t sW[LY::TOTAL];
  __shared__ float sP[kPropMlp];
  __shared__ int sstack[4 * 16 * kStack];   // shadow-ray stacks: 16 lanes per wave
  for (int i = threadIdx.x; i < LY::TOTAL; i += blockDim.x) sW[i] = frags[i];
  for (int i = threadIdx.x; i < kPropMlp; i += blockDim.x) sP[i] = Pf.mlp[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
  const int cnt = *count;
  const bool use_occ = P.use_occupancy && F.occ;
  unsigned long long nsamp = 0;
  WorkQueue wq(work, cnt, P.chunk, P.batch);
  for (int base = wq.next(lane); base >= 0; base = wq.next(lane))
  for (int bi = 0; bi < wq.batch; ++bi) {
    const int r = wq.map(base + bi);
    if (r >= cnt) break;
    float ox = q.ox[r], oy = q.oy[r], oz = q.oz[r];
    float dx = q.dx[r], dy = q.dy[r], dz = q.dz[r];
    to_field_frame(F, ox, oy, oz, dx, dy, dz);   // the proposal shares the field's frame
    const int seg = q.depth[r] & 0xFFFF;
    const float t_a = seg == 0 ? P.t_near : 0.0f;
    float box0, box1;
    if (!seg_box(F, ox, oy, oz, dx, dy, dz, box0, box1)) continue;
    const float lo = fmaxf(t_a, box0);
    const float hi = fminf(fminf(t_a + P.span, q.hit_t[r]), box1);
    if (!(hi > lo)) continue;
    // proposal weights on n_prop uniform intervals
    const float Dp = (hi - lo) / (float)n_prop;
    float alpha_p = 0.0f;
    if (lane < n_prop) {
      const float tm = lo + ((float)lane + 0.5f) * Dp;
      const float sp = prop_sigma<PTabT>(Pf, ptable, sP, ox + tm * dx, oy + tm * dy, oz + tm * dz);
      alpha_p = -expm1f(-sp * Dp);
    }
    const float inclT = wscan_mul(1.0f - alpha_p, lane);
    float exclT = __shfl_up(inclT, 1, 64);
    if (lane == 0) exclT = 1.0f;
    // dilate over adjacent bins and mix half and half with a uniform density
    const float wraw = lane < n_prop ? exclT * alpha_p : 0.0f;
    float wl = __shfl_up(wraw, 1, 64), wr = __shfl_down(wraw, 1, 64);
    if (lane == 0) wl = 0.0f;
    if (lane >= n_prop - 1) wr = 0.0f;
    const float wdil = lane < n_prop ? fmaxf(wraw, fmaxf(wl, wr)) : 0.0f;
    const float wmean = wsum(wdil) / (float)n_prop;
    const float wp = lane < n_prop ? wdil + wmean + 1e-3f / (float)n_prop : 0.0f;
    const float cdf = wscan_add(wp, lane);
    const float tot = __shfl(cdf, n_prop - 1, 64);
    // edges of the fine intervals by inverse CDF (lane e holds edge e)
    const float u = (float)lane / (float)n_fine * tot;
    int blo = 0, bhi = n_prop - 1;
#pragma unroll
    for (int it = 0; it < 6; ++it) {
      const int mid = (blo + bhi) >> 1;
      const float cm = __shfl(cdf, mid, 64);
      if (blo < bhi) {
        if (cm < u) blo = mid + 1;
        else bhi = mid;
      }
    }
    const float prev = __shfl(cdf, max(blo - 1, 0), 64);
    const float wj = __shfl(wp, blo, 64);
    float edge = lo + ((float)blo + ((blo > 0 ? u - prev : u) / wj)) * Dp;
    if (lane == 0) edge = lo;
    if (lane >= n_fine) edge = hi;
    // fine samples, 16 per tile
    float u_sh[4][4];
    sh_rows<NL, SH, CL, BF>(sW, dx, dy, dz, lane, u_sh);
    float Tseg = 1.0f, acc0 = 0.0f, acc1 = 0.0f, acc2 = 0.0f;
    for (int kb = 0; kb < n_fine; kb += 16) {
      const int k = kb + j;
      const float a = __shfl(edge, min(k, 63), 64);
      const float bn = __shfl(edge, min(k + 1, 63), 64);
      const float b = k + 1 >= n_fine ? hi : bn;
      bool valid = k < n_fine && b > a;
      const float tm = 0.5f * (a + b), D = b - a;
      const float px = ox + tm * dx, py = oy + tm * dy, pz = oz + tm * dz;
      if (valid && use_occ) valid = occ_bit(F, px, py, pz);
      if (__ballot(valid) == 0ull) continue;
      float fe[LY::NF];
      encode_group<NL, TabT>(F, table, px, py, pz, g, fe);
      float sigma, rgb[3];
      f4v raw;
      mlp_tile<NL, SH, CL, BF>(sW, fe, u_sh, F.density_offset, lane, sigma, rgb, raw);
      const float alpha = valid ? -expm1f(-sigma * D) : 0.0f;
      const float incl = sc16_mul(1.0f - alpha, j);
      float excl = __shfl_up(incl, 1, 16);
      if (j == 0) excl = 1.0f;
      float msk = 1.0f;
      if constexpr (SHADOW)
        msk = sample_shadow(F, B, P, valid, px, py, pz, lane, sstack + (threadIdx.x >> 6) * 16 * kStack + j);
      const float w = Tseg * excl * alpha * msk;
      acc0 += w * rgb[0];
      acc1 += w * rgb[1];
      acc2 += w * rgb[2];
      Tseg *= __shfl(incl, 15, 16);
      if (g == 0 && valid) ++nsamp;
    }
    acc0 = s16(acc0);
    acc1 = s16(acc1);
    acc2 = s16(acc2);
    if (lane == 0) {
      const float tr = q.tr[r], tg = q.tg[r], tb = q.tb[r];
      q.lr[r] += tr * acc0;
      q.lg[r] += tg * acc1;
      q.lb[r] += tb * acc2;
      q.tr[r] = tr * Tseg;
      q.tg[r] = tg * Tseg;
      q.tb[r] = tb * Tseg;
    }
  }
  if (stats) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) nsamp += __shfl_xor(nsamp, off, 64);
    if (lane == 0 && nsamp) atomicAdd(stats + 0, nsamp);
  }
}

// ---------------------------------------------------------------------------
// proposal-sampled march, 16-ray packets (n_prop = 32, n_fine <= 32): a wave
// takes 16 consecutive queue rays; lane (g, j) evaluates proposal intervals
// 8g .. 8g+7 of ray j, the transmittance and CDF over the 32 intervals are a
// local scan plus a scan over the four lane groups, the ray's CDF goes to a
// per-wave LDS area where the lanes invert it for the fine edges, and the
// fine samples of the 16 rays are stepped together as with the plain packets
// ---------------------------------------------------------------------------
constexpr int kPkBins = 32;

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Waves per SIMD of the packet march: three where the registers allow it
// without spilling (FP16 tables, BF16 MLPs, no shadow mask: 168 registers,
// and 47 KB of LDS lets three blocks share a compute unit), two elsewhere.
// The camera segment of the mid frame took 3.59 ms at two and 3.00 at three.
template <typename TabT, bool BF, typename PTabT, bool SHADOW>
constexpr int prop_pk_waves() {
  return (sizeof(TabT) == 2 && BF && sizeof(PTabT) == 2 && !SHADOW) ? 3 : 2;
}

template <int NL, int SH, int CL, typename TabT, bool BF, typename PTabT, bool SHADOW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(prop_pk_waves<TabT, BF, PTabT, SHADOW>()))) void k_march_prop_pk(
    RayQueue q, const int* __restrict__ count, int* __restrict__ work, FieldView F, const TabT* __restrict__ table,
    const uint32_t* __restrict__ frags, FieldView Pf, const PTabT* __restrict__ ptable, MarchParams P, BvhView B,
    int n_fine, unsigned long long* __restrict__ stats) {
  using LY = FragLayout<NL, SH, CL, BF>;
  __shared__ __align__(16) uint32_t sW[LY::TOTAL];
  __shared__ float sP[kPropMlp];
  __shared__ int sstack[4 * 16 * kStack];   // shadow-ray stacks: 16 lanes per wave
  __shared__ float sCdf[4][16][kPkBins], sBin[4][16][kPkBins], sEdge[4][16][kPkBins + 1];
  for (int i = threadIdx.x; i < LY::TOTAL; i += blockDim.x) sW[i] = frags[i];
  for (int i = threadIdx.x; i < kPropMlp; i += blockDim.x) sP[i] = Pf.mlp[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15, wv = threadIdx.x >> 6;
  const int cnt = *count;
  const bool use_occ = P.use_occupancy && F.occ;
  constexpr float kInvBins = 1.0f / (float)kPkBins;
  unsigned long long nsamp = 0;
  WorkQueue wq(work, cnt, P.chunk, 16);
  for (int base = wq.next(lane); base >= 0; base = wq.next(lane)) {
    const int r = wq.map(base + j);
    bool live = r < cnt;
    float ox = 0.0f, oy = 0.0f, oz = 0.0f, dx = 0.0f, dy = 0.0f, dz = 1.0f, lo = 0.0f, hi = 0.0f;
    if (live) {
      ox = q.ox[r]; oy = q.oy[r]; oz = q.oz[r];
      dx = q.dx[r]; dy = q.dy[r]; dz = q.dz[r];
      to_field_frame(F, ox, oy, oz, dx, dy, dz);   // the proposal shares the field's frame
      const float t_a = (q.depth[r] & 0xFFFF) == 0 ? P.t_near : 0.0f;
      float box0, box1;
      live = seg_box(F, ox, oy, oz, dx, dy, dz, box0, box1);
      if (live) {
        lo = fmaxf(t_a, box0);
        hi = fminf(fminf(t_a + P.span, q.hit_t[r]), box1);
        live = hi > lo;
      }
    }
    if (__ballot(live) == 0ull) continue;
    // proposal opacities of this lane's 8 intervals
    const float Dp = (hi - lo) / (float)kPkBins;
    float al[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      al[p] = 0.0f;
      if (live) {
        const float tm = lo + ((float)(8 * g + p) + 0.5f) * Dp;
        al[p] = -expm1f(-prop_sigma<PTabT>(Pf, ptable, sP, ox + tm * dx, oy + tm * dy, oz + tm * dz) * Dp);
      }
    }
    // weights T_i alpha_i: local exclusive products times the product of the
    // lower lane groups' totals
    float w[8], run = 1.0f;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      w[p] = run * al[p];
      run *= 1.0f - al[p];
    }
    float below = 1.0f;
#pragma unroll
    for (int gg = 0; gg < 3; ++gg) {
      const float t = __shfl(run, gg * 16 + j, 64);
      if (gg < g) below *= t;
    }
#pragma unroll
    for (int p = 0; p < 8; ++p) w[p] *= below;
    // dilate over adjacent intervals, mix half and half with a uniform density
    float wl = __shfl(w[7], ((g + 3) & 3) * 16 + j, 64), wr = __shfl(w[0], ((g + 1) & 3) * 16 + j, 64);
    if (g == 0) wl = 0.0f;
    if (g == 3) wr = 0.0f;
    float wd[8], part = 0.0f;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const float a = p > 0 ? w[p - 1] : wl, b = p < 7 ? w[p + 1] : wr;
      wd[p] = fmaxf(w[p], fmaxf(a, b));
      part += wd[p];
    }
    float wsum_all = part + __shfl_xor(part, 16, 64);
    wsum_all += __shfl_xor(wsum_all, 32, 64);
    const float add = wsum_all * kInvBins + 1e-3f * kInvBins;
    float csum = 0.0f;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      wd[p] += add;
      csum += wd[p];
    }
    float off = 0.0f;
#pragma unroll
    for (int gg = 0; gg < 3; ++gg) {
      const float t = __shfl(csum, gg * 16 + j, 64);
      if (gg < g) off += t;
    }
    float c = off;
    wave_lds_sync();
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      c += wd[p];
      sCdf[wv][j][8 * g + p] = c;
      sBin[wv][j][8 * g + p] = wd[p];
    }
    const float tot = __shfl(c, 48 + j, 64);   // the last CDF value of ray j
    wave_lds_sync();
    // fine edges by inverse CDF at u = e / n_fine (lane group g takes e = g mod 4)
    for (int e = g; e <= n_fine; e += 4) {
      const float u = (float)e / (float)n_fine * tot;
      int blo = 0, bhi = kPkBins - 1;
#pragma unroll
      for (int it = 0; it < 5; ++it) {
        const int mid = (blo + bhi) >> 1;
        if (sCdf[wv][j][mid] < u) blo = mid + 1;
        else bhi = mid;
      }
      const float prev = blo > 0 ? sCdf[wv][j][blo - 1] : 0.0f;
      float edge = lo + ((float)blo + (u - prev) / sBin[wv][j][blo]) * Dp;
      if (e == 0) edge = lo;
      if (e >= n_fine) edge = hi;
      sEdge[wv][j][e] = edge;
    }
    wave_lds_sync();
    float u_sh[4][4];
    sh_rows<NL, SH, CL, BF>(sW, dx, dy, dz, lane, u_sh);
    float T = 1.0f, acc0 = 0.0f, acc1 = 0.0f, acc2 = 0.0f;
    for (int k = 0; k < n_fine; ++k) {
      const float a = sEdge[wv][j][k], b = sEdge[wv][j][k + 1];
      bool valid = live && b > a;
      const float tm = 0.5f * (a + b), D = b - a;
      const float px = ox + tm * dx, py = oy + tm * dy, pz = oz + tm * dz;
      if (valid && use_occ) valid = occ_bit(F, px, py, pz);
      if (__ballot(valid) == 0ull) continue;
      float fe[LY::NF];
      encode_group<NL, TabT>(F, table, px, py, pz, g, fe);
      float sigma, rgb[3];
      f4v raw;
      mlp_tile<NL, SH, CL, BF>(sW, fe, u_sh, F.density_offset, lane, sigma, rgb, raw);
      const float alpha = valid ? -expm1f(-sigma * D) : 0.0f;
      float msk = 1.0f;
      if constexpr (SHADOW) msk = sample_shadow(F, B, P, valid, px, py, pz, lane, sstack + wv * 16 * kStack + j);
      const float wt = T * alpha * msk;
      acc0 += wt * rgb[0];
      acc1 += wt * rgb[1];
      acc2 += wt * rgb[2];
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
    wave_lds_sync();
  }
  if (stats) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) nsamp += __shfl_xor(nsamp, off, 64);
    if (lane == 0 && nsamp) atomicAdd(stats + 0, nsamp);
  }
}

// ---------------------------------------------------------------------------
// training targets: the plain marcher's weights of the camera segment,
// histogrammed over n_bins equal bins of [lo, hi] by interval overlap
// ---------------------------------------------------------------------------
template <int NL, int SH, int CL, typename TabT, bool BF>
__global__ __launch_bounds__(256) void k_prop_targets(FieldView F, const TabT* __restrict__ table,
                                                      const uint32_t* __restrict__ frags, int64_t n,
                                                      const float* __restrict__ o, const float* __restrict__ d,
                                                      float t_near, float t_far, int n_samples, int n_bins,
                                                      float* __restrict__ lohi, float* __restrict__ target) {
  using LY = FragLayout<NL, SH, CL, BF>;
  __shared__ __align__(16) uint32_t sW[LY::TOTAL];
  for (int i = threadIdx.x; i < LY::TOTAL; i += blockDim.x) sW[i] = frags[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t r = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); r < n; r += waves) {
    const float ox = o[3 * r], oy = o[3 * r + 1], oz = o[3 * r + 2];
    const float dx = d[3 * r], dy = d[3 * r + 1], dz = d[3 * r + 2];
    float hist = 0.0f;   // lane b < n_bins accumulates bin b
    float box0, box1, lo = 0.0f, hi = 0.0f;
    if (seg_box(F, ox, oy, oz, dx, dy, dz, box0, box1)) {
      lo = fmaxf(t_near, box0);
      hi = fminf(t_far, box1);
    }
    if (hi > lo) {
      const float delta = (t_far - t_near) / (float)n_samples;
      const float bw = (hi - lo) / (float)n_bins;
      const int k0 = max(0, (int)floorf((lo - t_near) / delta) - 1);
      const int k1 = min(n_samples, (int)ceilf((hi - t_near) / delta) + 1);
      float u_sh[4][4];
      sh_rows<NL, SH, CL, BF>(sW, dx, dy, dz, lane, u_sh);
      float Tseg = 1.0f;
      for (int kb = k0; kb < k1; kb += 16) {
        const int k = kb + j;
        const float a = fmaxf(t_near + (float)k * delta, lo);
        const float b = fminf(t_near + (float)(k + 1) * delta, hi);
        const bool valid = k < k1 && b > a;
        if (__ballot(valid) == 0ull) continue;
        const float tm = 0.5f * (a + b), D = b - a;
        float fe[LY::NF];
        encode_group<NL, TabT>(F, table, ox + tm * dx, oy + tm * dy, oz + tm * dz, g, fe);
        float sigma, rgb[3];
        f4v raw;
        mlp_tile<NL, SH, CL, BF>(sW, fe, u_sh, F.density_offset, lane, sigma, rgb, raw);
        const float alpha = valid ? -expm1f(-sigma * D) : 0.0f;
        const float incl = sc16_mul(1.0f - alpha, j);
        float excl = __shfl_up(incl, 1, 16);
        if (j == 0) excl = 1.0f;
        const float w = Tseg * excl * alpha;
        Tseg *= __shfl(incl, 15, 16);
        // bins touched by this tile
        const float ta = __shfl(a, 0, 64), tb = __shfl(b, 15, 64);
        const int bmin = max(0, (int)floorf((ta - lo) / bw) - 1);
        const int bmax = min(n_bins - 1, (int)floorf((tb - lo) / bw) + 1);
        for (int bb = bmin; bb <= bmax; ++bb) {
          const float c0 = lo + (float)bb * bw, c1 = lo + (float)(bb + 1) * bw;
          const float ov = fminf(b, c1) - fmaxf(a, c0);
          const float part = (valid && ov > 0.0f) ? w * ov / D : 0.0f;
          const float sbin = s16(part);
          if (lane == bb) hist += sbin;
        }
      }
    }
    if (lane == 0) {
      lohi[2 * r] = hi > lo ? lo : 0.0f;
      lohi[2 * r + 1] = hi > lo ? hi : 0.0f;
    }
    if (lane < n_bins) target[r * n_bins + lane] = hist;
  }
}

// ---------------------------------------------------------------------------
// proposal loss and gradient (one wave per segment, one bin per lane)
// ---------------------------------------------------------------------------
// The gradient of a dense level 0 of up to 17^3 entries is summed in LDS per
// block and added to the global gradient once per block: every sample hits
// that level, and the samples of one segment share most of its corners.
constexpr int kPropL0Lds = 2 * 17 * 17 * 17;
// The MLP has no biases and h_i = sum_c W1[i][c] f_c, so both weight
// gradients follow from one 16 x 10 matrix per batch,
//   M[i][c] = sum_s dz(s) [h_i(s) > 0] f_c(s):
//   dL/dW1[i][c] = W2[i] M[i][c],   dL/dW2[i] = sum_c W1[i][c] M[i][c].
// Each wave accumulates M on the matrix cores over the segments it takes
// (K = the 64 bins of a segment, four per step); the per-lane factors go
// through a per-wave LDS stage whose row strides (17, 11) keep both the
// row-wise writes and the column-wise operand reads free of bank conflicts.
constexpr int kStA = 17, kStF = 11, kStageWave = 64 * (kStA + kStF);

__global__ __launch_bounds__(256) void k_prop_grad(FieldView P, const float* __restrict__ table,
                                                   const float* __restrict__ mlp, int64_t n,
                                                   const float* __restrict__ o, const float* __restrict__ d,
                                                   const float* __restrict__ lohi, const float* __restrict__ target,
                                                   int n_bins, float inv_n, float* __restrict__ g_table,
                                                   float* __restrict__ g_mlp, float* __restrict__ loss) {
  __shared__ float sW[kPropMlp];
  __shared__ float sM[16 * 16];
  __shared__ float sL0[kPropL0Lds];
  __shared__ float sStage[4 * kStageWave];
  for (int i = threadIdx.x; i < kPropMlp; i += blockDim.x) sW[i] = mlp[i];
  for (int i = threadIdx.x; i < 16 * 16; i += blockDim.x) sM[i] = 0.0f;
  const int n1 = P.res[0] + 1;
  const int n_l0 = (P.dense_mask & 1u) && 2 * n1 * n1 * n1 <= kPropL0Lds ? 2 * n1 * n1 * n1 : 0;
  for (int i = threadIdx.x; i < n_l0; i += blockDim.x) sL0[i] = 0.0f;
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
  float* sA = sStage + (threadIdx.x >> 6) * kStageWave;
  float* sF = sA + 64 * kStA;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
  const size_t T = (size_t)P.table_mask + 1u;
  float wave_loss = 0.0f;
  f4v accM = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int64_t s = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); s < n; s += waves) {
    const float lo = lohi[2 * s], hi = lohi[2 * s + 1];
    if (!(hi > lo)) continue;
    const float D = (hi - lo) / (float)n_bins;
    const bool act = lane < n_bins;
    float feat[kPropIn], hpre[kPropHidden], z = 0.0f, sigma = 0.0f, alpha = 0.0f;
    float px = 0.0f, py = 0.0f, pz = 0.0f;
    if (act) {
      const float tm = lo + ((float)lane + 0.5f) * D;
      px = o[3 * s] + tm * d[3 * s];
      py = o[3 * s + 1] + tm * d[3 * s + 1];
      pz = o[3 * s + 2] + tm * d[3 * s + 2];
      sigma = prop_density<float>(P, table, sW, px, py, pz, feat, hpre, z);
      alpha = -expm1f(-sigma * D);
    }
    const float inclT = wscan_mul(1.0f - alpha, lane);
    float Tj = __shfl_up(inclT, 1, 64);
    if (lane == 0) Tj = 1.0f;
    const float w = act ? Tj * alpha : 0.0f;
    const float h = act ? target[s * n_bins + lane] : 0.0f;
    const float rres = h - w;
    float gl = 0.0f;
    if (act && rres > 0.0f) {
      wave_loss += rres * rres / (h + 1e-7f);
      gl = -2.0f * rres / (h + 1e-7f) * inv_n;
    }
    // dL/dsigma_k = g_k T_k D exp(-sigma_k D) - D sum_{j > k} g_j w_j
    const float gw = gl * w;
    const float incl_gw = wscan_add(gw, lane);
    const float suffix = __shfl(incl_gw, 63, 64) - incl_gw;
    float dz = 0.0f;
    if (act) {
      const float dsig = gl * Tj * D * expf(-sigma * D) - D * suffix;
      dz = dsig / (1.0f + expf(-(z + P.density_offset)));
    }
    if (__ballot(dz != 0.0f) == 0ull) continue;
    // M += A B with A[i][s] = dz(s) [h_i(s) > 0], B[s][c] = f_c(s)
#pragma unroll
    for (int i = 0; i < kPropHidden; ++i) sA[lane * kStA + i] = (dz != 0.0f && hpre[i] > 0.0f) ? dz : 0.0f;
#pragma unroll
    for (int c = 0; c < kPropIn; ++c) sF[lane * kStF + c] = dz != 0.0f ? feat[c] : 0.0f;
    wave_lds_sync();
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int r = 16 * g + t;   // bin of K row g in step t
      const float a = sA[r * kStA + j];
      const float b = j < kPropIn ? sF[r * kStF + j] : 0.0f;
      accM = mma(a, b, accM);
    }
    wave_lds_sync();
    if (dz == 0.0f) continue;
    float df[kPropIn];
#pragma unroll
    for (int c = 0; c < kPropIn; ++c) df[c] = 0.0f;
#pragma unroll
    for (int i = 0; i < kPropHidden; ++i) {
      if (hpre[i] > 0.0f) {
        const float dh = dz * sW[kPropIn * kPropHidden + i];
#pragma unroll
        for (int c = 0; c < kPropIn; ++c) df[c] += dh * sW[i * kPropIn + c];
      }
    }
    // scatter to the table entries of the 8 corners of every level
    float xh, yh, zh;
    to_unit(P, px, py, pz, xh, yh, zh);
#pragma unroll
    for (int l = 0; l < kPropLevels; ++l) {
      uint32_t idx[8];
      float wc[8];
      level_corners(P, l, xh, yh, zh, idx, wc);
      if (l == 0 && n_l0) {
        // two branches rather than one pointer, so these stay LDS atomics
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          atomicAdd(sL0 + 2 * idx[c], wc[c] * df[0]);
          atomicAdd(sL0 + 2 * idx[c] + 1, wc[c] * df[1]);
        }
      } else {
        float* gt = g_table + (size_t)l * T * 2;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          atomicAdd(gt + 2 * (size_t)idx[c], wc[c] * df[2 * l]);
          atomicAdd(gt + 2 * (size_t)idx[c] + 1, wc[c] * df[2 * l + 1]);
        }
      }
    }
  }
  wave_loss = wsum(wave_loss);
  if (lane == 0 && wave_loss != 0.0f) atomicAdd(loss, wave_loss * inv_n);
  // accumulator register v of lane (g, j) holds M[4 g + v][j]
#pragma unroll
  for (int v = 0; v < 4; ++v)
    if (j < kPropIn && accM[v] != 0.0f) atomicAdd(&sM[(4 * g + v) * 16 + j], accM[v]);
  __syncthreads();
  for (int i = threadIdx.x; i < kPropMlp; i += blockDim.x) {
    float gv = 0.0f;
    if (i < kPropIn * kPropHidden) {
      gv = sW[kPropIn * kPropHidden + i / kPropIn] * sM[(i / kPropIn) * 16 + i % kPropIn];
    } else {
      const int u = i - kPropIn * kPropHidden;
#pragma unroll
      for (int c = 0; c < kPropIn; ++c) gv += sW[u * kPropIn + c] * sM[u * 16 + c];
    }
    if (gv != 0.0f) atomicAdd(g_mlp + i, gv);
  }
  for (int i = threadIdx.x; i < n_l0; i += blockDim.x)
    if (sL0[i] != 0.0f) atomicAdd(g_table + i, sL0[i]);
}

__global__ void k_fill(float* __restrict__ p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// Adam step on FP32 master parameters; refreshes the render copy of the table.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int64_t n, float lr, float b1, float b2, float eps, float c1, float c2,
                       __half* __restrict__ half_copy, float* __restrict__ float_copy) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    if (half_copy) half_copy[i] = __float2half_rn(pi);
    if (float_copy) float_copy[i] = pi;
  }
}

template <int NL, int SH, int CL, typename TabT, bool BF, typename PTabT, bool SHADOW>
mr_status launch_prop_mode(const mr_field* f, const mr_field* p, RayQueue q, const int* count, int* work,
                           const MarchParams& P, const BvhView& B, int n_prop, int n_fine, bool packets,
                           unsigned long long* stats, int blocks_per_cu, int64_t n, hipStream_t st) {
  const uint32_t* fr = BF ? f->frag_bf16_dev : f->frag_f32_dev;
  const TabT* tab = reinterpret_cast<const TabT*>(f->table_dev);
  const PTabT* ptab = reinterpret_cast<const PTabT*>(p->table_dev);
  if (packets && n_prop == kPkBins && n_fine <= kPkBins) {
    auto* k = k_march_prop_pk<NL, SH, CL, TabT, BF, PTabT, SHADOW>;
    const int blocks = persistent_blocks(reinterpret_cast<const void*>(k), 256, blocks_per_cu, (n + 63) / 64);
    hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, st, q, count, work, f->view, tab, fr, p->view, ptab, P, B,
                       n_fine, stats);
  } else {
    auto* k = k_march_prop<NL, SH, CL, TabT, BF, PTabT, SHADOW>;
    const int blocks = persistent_blocks(reinterpret_cast<const void*>(k), 256, blocks_per_cu, (n + 3) / 4);
    hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, st, q, count, work, f->view, tab, fr, p->view, ptab, P, B,
                       n_prop, n_fine, stats);
  }
  MR_HIP(hipGetLastError());
  return MR_OK;
}

template <int NL, int SH, int CL, typename TabT, bool BF, typename PTabT>
mr_status launch_prop(const mr_field* f, const mr_field* p, RayQueue q, const int* count, int* work,
                      const MarchParams& P, const BvhView& B, int n_prop, int n_fine, bool packets,
                      unsigned long long* stats, int blocks_per_cu, int64_t n, hipStream_t st) {
  if (P.shadows)
    return launch_prop_mode<NL, SH, CL, TabT, BF, PTabT, true>(f, p, q, count, work, P, B, n_prop, n_fine, packets,
                                                               stats, blocks_per_cu, n, st);
  return launch_prop_mode<NL, SH, CL, TabT, BF, PTabT, false>(f, p, q, count, work, P, B, n_prop, n_fine, packets,
                                                              stats, blocks_per_cu, n, st);
}

template <int NL, int SH, int CL, typename TabT, bool BF>
mr_status launch_targets(const mr_field* f, int64_t n, const float* o, const float* d, float t_near, float t_far,
                         int n_samples, int n_bins, float* lohi, float* target, hipStream_t st) {
  const uint32_t* fr = BF ? f->frag_bf16_dev : f->frag_f32_dev;
  const int blocks = (int)std::min<int64_t>((n + 3) / 4, (int64_t)device_cus() * 8);
  hipLaunchKernelGGL((k_prop_targets<NL, SH, CL, TabT, BF>), dim3(blocks), dim3(256), 0, st, f->view,
                     reinterpret_cast<const TabT*>(f->table_dev), fr, n, o, d, t_near, t_far, n_samples, n_bins, lohi,
                     target);
  MR_HIP(hipGetLastError());
  return MR_OK;
}

mr_status grad_into(const mr_field* p, int64_t n, const float* o, const float* d, const float* lohi,
                    const float* target, int n_bins, float* loss, float* g_table, float* g_mlp, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3(1024), dim3(256), 0, st, g_table, p->n_table, 0.0f);
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(256), 0, st, g_mlp, (int64_t)kPropMlp, 0.0f);
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st, loss, (int64_t)1, 0.0f);
  MR_HIP(hipGetLastError());
  const int blocks = (int)std::min<int64_t>((n + 3) / 4, (int64_t)device_cus() * 8);
  hipLaunchKernelGGL(k_prop_grad, dim3(blocks), dim3(256), 0, st, p->view, p->master_dev, p->mlp_dev, n, o, d, lohi,
                     target, n_bins, 1.0f / (float)n, g_table, g_mlp, loss);
  MR_HIP(hipGetLastError());
  return MR_OK;
}

mr_status check_prop(const mr_field* p, int64_t n, const float* o, const float* d, const float* lohi, const float* t,
                     int n_bins) {
  if (!p || p->view.c_layers != 0) return fail(MR_ERR_INVALID_ARG, "not a proposal field");
  if (n < 1) return fail(MR_ERR_INVALID_ARG, "need at least one segment");
  if (!o || !d || !lohi || !t) return fail(MR_ERR_INVALID_ARG, "null array");
  if (n_bins < 1 || n_bins > 64) return fail(MR_ERR_INVALID_ARG, "n_bins must be in 1..64");
  return MR_OK;
}

}  // namespace

namespace mr {

mr_status dispatch_march_proposal(const mr_field* f, const mr_field* prop, RayQueue q, const int* count, int* work,
                                  const MarchParams& P, const BvhView& B, int n_prop, int n_fine, bool packets,
                                  unsigned long long* stats, int blocks_per_cu, int64_t n, hipStream_t st) {
  const auto& v = f->view;
  const bool h = v.table_dtype == MR_F16, bf = v.mlp_dtype == MR_BF16;
  const bool ph = prop->view.table_dtype == MR_F16;
#define PR(NL, SH, CL, TT, BFV)                                                                                      \
  return ph ? launch_prop<NL, SH, CL, TT, BFV, __half>(f, prop, q, count, work, P, B, n_prop, n_fine, packets, stats, blocks_per_cu, n, st) \
            : launch_prop<NL, SH, CL, TT, BFV, float>(f, prop, q, count, work, P, B, n_prop, n_fine, packets, stats, blocks_per_cu, n, st);
#define M(NL, SH, CL)                                                        \
  if (v.n_levels == NL && v.sh == SH && v.c_layers == CL) {                   \
    if (bf) {                                                                 \
      if (h) { PR(NL, SH, CL, __half, true) } else { PR(NL, SH, CL, float, true) } \
    } else {                                                                  \
      if (h) { PR(NL, SH, CL, __half, false) } else { PR(NL, SH, CL, float, false) } \
    }                                                                         \
  }
  M(8, 4, 1)
  M(16, 16, 2)
#undef M
#undef PR
  return fail(MR_ERR_UNSUPPORTED, "proposal sampling supports the 8-level/SH4/1-layer and 16-level/SH16/2-layer fields");
}

}  // namespace mr

extern "C" mr_status mr_proposal_targets(const mr_field* fine, int64_t n, const float* origins, const float* dirs,
                                         float t_near, float t_far, int32_t n_samples, int32_t n_bins, float* lohi,
                                         float* targets, void* stream) {
  if (!fine || fine->view.c_layers == 0) return fail(MR_ERR_INVALID_ARG, "fine must be a radiance field");
  if (!proposal_march_layout(fine->view.n_levels, fine->view.sh, fine->view.c_layers))
    return fail(MR_ERR_UNSUPPORTED, "training targets support the 8-level/SH4/1-layer and 16-level/SH16/2-layer fields");
  if (n < 0) return fail(MR_ERR_INVALID_ARG, "n < 0");
  if (n == 0) return MR_OK;
  if (!origins || !dirs || !lohi || !targets) return fail(MR_ERR_INVALID_ARG, "null array");
  if (!(t_far > t_near) || !(t_near >= 0.0f)) return fail(MR_ERR_INVALID_ARG, "need 0 <= t_near < t_far");
  if (n_samples < 1 || n_samples > 4096) return fail(MR_ERR_INVALID_ARG, "n_samples must be in 1..4096");
  if (n_bins < 1 || n_bins > 64) return fail(MR_ERR_INVALID_ARG, "n_bins must be in 1..64");
  hipStream_t st = (hipStream_t)stream;
  const auto& v = fine->view;
  const bool h = v.table_dtype == MR_F16, bf = v.mlp_dtype == MR_BF16;
#define T(NL, SH, CL)                                                                                          \
  if (v.n_levels == NL && v.sh == SH && v.c_layers == CL) {                                                     \
    if (bf) return h ? launch_targets<NL, SH, CL, __half, true>(fine, n, origins, dirs, t_near, t_far, n_samples, n_bins, lohi, targets, st) \
                     : launch_targets<NL, SH, CL, float, true>(fine, n, origins, dirs, t_near, t_far, n_samples, n_bins, lohi, targets, st); \
    return h ? launch_targets<NL, SH, CL, __half, false>(fine, n, origins, dirs, t_near, t_far, n_samples, n_bins, lohi, targets, st) \
             : launch_targets<NL, SH, CL, float, false>(fine, n, origins, dirs, t_near, t_far, n_samples, n_bins, lohi, targets, st); \
  }
  T(8, 4, 1)
  T(16, 16, 2)
#undef T
  return fail(MR_ERR_UNSUPPORTED, "field shape not instantiated for targets");
}

extern "C" mr_status mr_proposal_grad(const mr_field* prop, int64_t n, const float* origins, const float* dirs,
                                      const float* lohi, const float* targets, int32_t n_bins, float* loss,
                                      float* g_table, float* g_mlp, void* stream) {
  mr_status s = check_prop(prop, n, origins, dirs, lohi, targets, n_bins);
  if (s != MR_OK) return s;
  if (!loss || !g_table || !g_mlp) return fail(MR_ERR_INVALID_ARG, "null output");
  return grad_into(prop, n, origins, dirs, lohi, targets, n_bins, loss, g_table, g_mlp, (hipStream_t)stream);
}

extern "C" mr_status mr_proposal_train_step(mr_field* prop, int64_t n, const float* origins, const float* dirs,
                                            const float* lohi, const float* targets, int32_t n_bins,
                                            const mr_adam* adam, float* loss, void* stream) {
  mr_status s = check_prop(prop, n, origins, dirs, lohi, targets, n_bins);
  if (s != MR_OK) return s;
  if (!adam || !loss) return fail(MR_ERR_INVALID_ARG, "null adam or loss");
  if (!(adam->lr > 0.0f) || !(adam->beta1 >= 0.0f && adam->beta1 < 1.0f) ||
      !(adam->beta2 >= 0.0f && adam->beta2 < 1.0f) || !(adam->eps > 0.0f) || !std::isfinite(adam->lr) ||
      !std::isfinite(adam->eps))
    return fail(MR_ERR_INVALID_ARG, "bad Adam hyper-parameters (need lr > 0, 0 <= beta < 1, eps > 0, finite)");
  hipStream_t st = (hipStream_t)stream;
  if (!prop->opt_dev) {
    const int64_t tot = 3 * (prop->n_table + kPropMlp);    // grad, m, v
    if (hipMalloc(&prop->opt_dev, tot * sizeof(float)) != hipSuccess) return fail(MR_ERR_OOM, "optimizer state");
    hipLaunchKernelGGL(k_fill, dim3(1024), dim3(256), 0, st, prop->opt_dev, tot, 0.0f);
    MR_HIP(hipGetLastError());
    prop->opt_step = 0;
  }
  float* g_tab = prop->opt_dev;
  float* g_mlp = g_tab + prop->n_table;
  float* m_tab = g_mlp + kPropMlp;
  float* m_mlp = m_tab + prop->n_table;
  float* v_tab = m_mlp + kPropMlp;
  float* v_mlp = v_tab + prop->n_table;
  s = grad_into(prop, n, origins, dirs, lohi, targets, n_bins, loss, g_tab, g_mlp, st);
  if (s != MR_OK) return s;
  prop->opt_step += 1;
  const float c1 = 1.0f - std::pow(adam->beta1, (float)prop->opt_step);
  const float c2 = 1.0f - std::pow(adam->beta2, (float)prop->opt_step);
  __half* hcopy = prop->view.table_dtype == MR_F16 ? (__half*)prop->table_dev : nullptr;
  float* fcopy = prop->view.table_dtype == MR_F32 ? (float*)prop->table_dev : nullptr;
  hipLaunchKernelGGL(k_adam, dim3(2048), dim3(256), 0, st, prop->master_dev, g_tab, m_tab, v_tab, prop->n_table,
                     adam->lr, adam->beta1, adam->beta2, adam->eps, c1, c2, hcopy, fcopy);
  hipLaunchKernelGGL(k_adam, dim3(1), dim3(256), 0, st, prop->mlp_dev, g_mlp, m_mlp, v_mlp, (int64_t)kPropMlp,
                     adam->lr, adam->beta1, adam->beta2, adam->eps, c1, c2, (__half*)nullptr, (float*)nullptr);
  MR_HIP(hipGetLastError());
  return MR_OK;
}
