// Several fields of one layout, marched as one medium.
//
// Where two boxes share a stretch of a segment the fields cannot be marched
// one after another: an interval there takes the summed density
// sigma_1 + sigma_2 + ... and the density-weighted mean of the colours
// (Eq. 8-11 applied to the sum of the media, each field zero outside its own
// box).  The same march serves disjoint boxes, in one pass over the rays
// instead of one per field.  Per ray (later segments) one wave takes one ray.  The segment's uniform grid is cut at every
// box face the ray crosses between two grid points, so that each piece lies
// wholly inside or wholly outside each box, and each piece is composited at
// its midpoint.  A tile is 16 consecutive pieces (column j = piece j); every
// field whose box holds some piece of the tile evaluates the whole tile (hash
// encoding and matrix-core MLP tiles with that field's weights, read through
// the caches) and contributes where it holds the piece and, with occupancy
// on, its own grid marks the cell.  Transmittance is the 16-lane prefix
// product of the per-ray march, carried from tile to tile.
//
// On the camera segment a wave takes packets instead: 16 consecutive queue
// rays (column j = ray j) step through their pieces together, piece s of each
// ray at step s, so that neighbouring pixels sample the fields at nearly the
// same t and share cache lines, as in the single-field packet march.  Each
// ray walks its own boundary list with a cursor: the piece that starts at a
// ends at the next grid point or at the first of the ray's stretch bounds
// beyond a, whichever is nearer, which gives the per-ray walk's pieces.
#include <cstring>

#include "mr_mfma.h"
#include "mr_render.h"

using namespace mr;

namespace {

struct JointFields {
  int n;
  FieldView view[kMaxFields];
  const void* table[kMaxFields];     // FP32 or FP16 table of each field
  const uint32_t* frags[kMaxFields];  // its MFMA weight fragments
};
static_assert(sizeof(JointFields) <= 2560, "kernel argument size");

// Grid point k of a segment that starts at t_a: one rounding, and the same
// expression wherever a grid point is needed, so that a cut is compared with
// exactly the value that bounds the pieces.
__device__ __forceinline__ float grid_t(float t_a, int k, float delta) { return __fmaf_rn((float)k, delta, t_a); }

// Element m of the sorted boundary list of a segment: the grid points k0..k1
// (clipped to t_b) merged with the cut points.  Lane i < 2 n holds cut i (or
// +inf) and its place pos in the merged list.
__device__ __forceinline__ float boundary(int m, float cut, int pos, int n_cand, float t_a, float t_b, int k0,
                                          float delta) {
  int before = 0;
  float v = 0.0f;
  bool at_cut = false;
  for (int i = 0; i < n_cand; ++i) {
    const float ci = __shfl(cut, i, 64);
    const int pi = __shfl(pos, i, 64);
    if (ci != INFINITY) {
      if (pi < m) ++before;
      else if (pi == m) {
        at_cut = true;
        v = ci;
      }
    }
  }
  return at_cut ? v : fminf(grid_t(t_a, k0 + m - before, delta), t_b);
}

template <int NL, int SH, int CL, typename TabT, bool BF, bool SHADOW>
__device__ __forceinline__ void march_fields_ray(const RayQueue& q, int r, const JointFields& J, const MarchParams& P,
                                                 const BvhView& B, int* sstack, int lane, unsigned long long& nsamp) {
  using LY = FragLayout<NL, SH, CL, BF>;
  const int g = lane >> 4, j = lane & 15;
  const float delta = P.delta;
  const float ox = q.ox[r], oy = q.oy[r], oz = q.oz[r];
  const float dx = q.dx[r], dy = q.dy[r], dz = q.dz[r];
  const float t_a = (q.depth[r] & 0xFFFF) == 0 ? P.t_near : 0.0f;
  const float t_b = fminf(t_a + P.span, q.hit_t[r]);
  // field k's stretch [tin, tout] of the segment: lane 2k holds tin and lane
  // 2k + 1 tout; a field the segment misses has [+inf, -inf]
  float bnd = 0.0f, lo = INFINITY, hi = -INFINITY;
#pragma unroll 1
  for (int k = 0; k < J.n; ++k) {
    const FieldView& F = J.view[k];
    float fx = ox, fy = oy, fz = oz, ex = dx, ey = dy, ez = dz;
    to_field_frame(F, fx, fy, fz, ex, ey, ez);
    float b0, b1, tin = INFINITY, tout = -INFINITY;
    if (slab_box(F, fx, fy, fz, ex, ey, ez, b0, b1)) {
      const float a = fmaxf(t_a, b0), b = fminf(t_b, b1);
      if (b > a) {
        tin = a;
        tout = b;
      }
    }
    lo = fminf(lo, tin);
    hi = fmaxf(hi, tout);
    if (lane == 2 * k) bnd = tin;
    if (lane == 2 * k + 1) bnd = tout;
  }
  if (!(hi > lo)) return;
  const int k0 = max(0, (int)floorf((lo - t_a) / delta) - 1);
  const int k1 = min(P.n_samples, (int)ceilf((hi - t_a) / delta) + 1);
  const int n_cand = 2 * J.n;
  // a box face strictly between two grid points of [k0, k1] cuts the interval
  // it falls in; one on a grid point cuts nothing
  const float g0 = grid_t(t_a, k0, delta), g1 = fminf(grid_t(t_a, k1, delta), t_b);
  float cut = INFINITY;
  int below = 0;   // grid points of k0..k1 below the cut
  if (lane < n_cand && bnd > g0 && bnd < g1) {
    int kk = min(max((int)floorf((bnd - t_a) / delta), k0), k1 - 1);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      if (kk > k0 && grid_t(t_a, kk, delta) > bnd) --kk;
      else if (kk + 1 < k1 && grid_t(t_a, kk + 1, delta) <= bnd) ++kk;
    }
    if (grid_t(t_a, kk, delta) != bnd) {
      cut = bnd;
      below = kk - k0 + 1;
    }
  }
  // place of each cut in the merged list: grid points below it plus cuts
  // before it (ties in lane order)
  int rank = 0;
  for (int i = 0; i < n_cand; ++i) {
    const float ci = __shfl(cut, i, 64);
    rank += (ci < cut || (ci == cut && i < lane)) ? 1 : 0;
  }
  const int pos = below + rank;
  const int n_cuts = __popcll(__ballot(cut != INFINITY));
  const int total = k1 - k0 + n_cuts;   // pieces
  float Tseg = 1.0f, acc0 = 0.0f, acc1 = 0.0f, acc2 = 0.0f;
  for (int mb = 0; mb < total; mb += 16) {
    const int m = mb + j;
    const float a = boundary(m, cut, pos, n_cand, t_a, t_b, k0, delta);
    const float b = boundary(m + 1, cut, pos, n_cand, t_a, t_b, k0, delta);
    const bool piece = m < total && b > a;
    if (__ballot(piece) == 0ull) continue;
    const float tm = 0.5f * (a + b), D = b - a;
    float sig = 0.0f, s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
    int nf = 0;
#pragma unroll 1
    for (int k = 0; k < J.n; ++k) {
      const float tin = __shfl(bnd, 2 * k, 64), tout = __shfl(bnd, 2 * k + 1, 64);
      bool in = piece && a >= tin && b <= tout;
      if (__ballot(in) == 0ull) continue;
      const FieldView& F = J.view[k];
      float fx = ox, fy = oy, fz = oz, ex = dx, ey = dy, ez = dz;
      to_field_frame(F, fx, fy, fz, ex, ey, ez);
      const float px = fx + tm * ex, py = fy + tm * ey, pz = fz + tm * ez;
      if (in && P.use_occupancy && F.occ) in = occ_lookup(F, px, py, pz);
      if (__ballot(in) == 0ull) continue;
      float u[4][4];
      sh_rows<NL, SH, CL, BF>(J.frags[k], ex, ey, ez, lane, u);
      float fe[LY::NF];
      encode_group<NL, TabT>(F, reinterpret_cast<const TabT*>(J.table[k]), px, py, pz, g, fe);
      float sigma, rgb[3];
      f4v raw;
      mlp_tile<NL, SH, CL, BF>(J.frags[k], fe, u, F.density_offset, lane, sigma, rgb, raw);
      if (in) {
        sig += sigma;
        s0 += sigma * rgb[0];
        s1 += sigma * rgb[1];
        s2 += sigma * rgb[2];
        ++nf;
      }
    }
    const bool any = nf > 0;
    const float alpha = any ? -expm1f(-sig * D) : 0.0f;
    const float inv = sig > 0.0f ? 1.0f / sig : 0.0f;
    const float incl = scan16_mul(1.0f - alpha, j);
    float excl = __shfl_up(incl, 1, 16);
    if (j == 0) excl = 1.0f;
    float msk = 1.0f;
    if constexpr (SHADOW) msk = sample_shadow_world(B, P, any, ox + tm * dx, oy + tm * dy, oz + tm * dz, lane, sstack);
    const float w = Tseg * excl * alpha * msk * inv;
    acc0 += w * s0;
    acc1 += w * s1;
    acc2 += w * s2;
    Tseg *= __shfl(incl, 15, 16);
    if (g == 0) nsamp += (unsigned long long)nf;
  }
  acc0 = sum16(acc0);
  acc1 = sum16(acc1);
  acc2 = sum16(acc2);
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

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// One 16-ray packet; column j's ray is r (live: r is in the queue).  sb: the
// wave's LDS rows, row j holding ray j's stretch [tin, tout] per field.
template <int NL, int SH, int CL, typename TabT, bool BF, bool SHADOW>
__device__ __forceinline__ void march_fields_packet(const RayQueue& q, int r, bool live, const JointFields& J,
                                                    const MarchParams& P, const BvhView& B,
                                                    float (*sb)[2 * kMaxFields], int* sstack, int lane,
                                                    unsigned long long& nsamp) {
  using LY = FragLayout<NL, SH, CL, BF>;
  const int g = lane >> 4, j = lane & 15;
  const float delta = P.delta;
  float ox = 0.0f, oy = 0.0f, oz = 0.0f, dx = 0.0f, dy = 0.0f, dz = 1.0f, t_a = 0.0f, t_b = 0.0f;
  if (live) {
    ox = q.ox[r]; oy = q.oy[r]; oz = q.oz[r];
    dx = q.dx[r]; dy = q.dy[r]; dz = q.dz[r];
    t_a = (q.depth[r] & 0xFFFF) == 0 ? P.t_near : 0.0f;
    t_b = fminf(t_a + P.span, q.hit_t[r]);
  }
  float lo = INFINITY, hi = -INFINITY;
#pragma unroll 1
  for (int k = 0; k < J.n; ++k) {
    const FieldView& F = J.view[k];
    float fx = ox, fy = oy, fz = oz, ex = dx, ey = dy, ez = dz;
    to_field_frame(F, fx, fy, fz, ex, ey, ez);
    float b0, b1, tin = INFINITY, tout = -INFINITY;
    if (live && slab_box(F, fx, fy, fz, ex, ey, ez, b0, b1)) {
      const float a = fmaxf(t_a, b0), b = fminf(t_b, b1);
      if (b > a) {
        tin = a;
        tout = b;
      }
    }
    lo = fminf(lo, tin);
    hi = fmaxf(hi, tout);
    if (g == 0) {
      sb[j][2 * k] = tin;
      sb[j][2 * k + 1] = tout;
    }
  }
  wave_lds_sync();
  // cursor: the piece starts at a, in grid interval gi (G_gi <= a < G_gi+1)
  bool alive = live && hi > lo;
  int gi = 0;
  float a = 0.0f, end = 0.0f;
  if (alive) {
    const int k0 = max(0, (int)floorf((lo - t_a) / delta) - 1);
    const int k1 = min(P.n_samples, (int)ceilf((hi - t_a) / delta) + 1);
    gi = k0;
    a = fminf(grid_t(t_a, k0, delta), t_b);
    end = fminf(grid_t(t_a, k1, delta), t_b);
    alive = a < end;
  }
  const int n_bnd = 2 * J.n;
  float T = 1.0f, acc0 = 0.0f, acc1 = 0.0f, acc2 = 0.0f;
  while (__ballot(alive) != 0ull) {
    float b = a;
    if (alive) {
      // a bound on a grid point cuts nothing: it ends the piece there anyway
      const float gnext = fminf(grid_t(t_a, gi + 1, delta), t_b);
      float c = gnext;
      for (int i = 0; i < n_bnd; ++i) {
        const float v = sb[j][i];
        if (v > a && v < c) c = v;
      }
      b = c;
      if (b == gnext) ++gi;
    }
    const bool piece = alive && b > a;
    const float tm = 0.5f * (a + b), D = b - a;
    float sig = 0.0f, s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
    int nf = 0;
#pragma unroll 1
    for (int k = 0; k < J.n; ++k) {
      bool in = piece && a >= sb[j][2 * k] && b <= sb[j][2 * k + 1];
      if (__ballot(in) == 0ull) continue;
      const FieldView& F = J.view[k];
      float fx = ox, fy = oy, fz = oz, ex = dx, ey = dy, ez = dz;
      to_field_frame(F, fx, fy, fz, ex, ey, ez);
      const float px = fx + tm * ex, py = fy + tm * ey, pz = fz + tm * ez;
      if (in && P.use_occupancy && F.occ) in = occ_lookup(F, px, py, pz);
      if (__ballot(in) == 0ull) continue;
      float u[4][4];
      sh_rows<NL, SH, CL, BF>(J.frags[k], ex, ey, ez, lane, u);
      float fe[LY::NF];
      encode_group<NL, TabT>(F, reinterpret_cast<const TabT*>(J.table[k]), px, py, pz, g, fe);
      float sigma, rgb[3];
      f4v raw;
      mlp_tile<NL, SH, CL, BF>(J.frags[k], fe, u, F.density_offset, lane, sigma, rgb, raw);
      if (in) {
        sig += sigma;
        s0 += sigma * rgb[0];
        s1 += sigma * rgb[1];
        s2 += sigma * rgb[2];
        ++nf;
      }
    }
    const bool any = nf > 0;
    const float alpha = any ? -expm1f(-sig * D) : 0.0f;
    const float inv = sig > 0.0f ? 1.0f / sig : 0.0f;
    float msk = 1.0f;
    if constexpr (SHADOW) msk = sample_shadow_world(B, P, any, ox + tm * dx, oy + tm * dy, oz + tm * dz, lane, sstack);
    const float w = T * alpha * msk * inv;
    acc0 += w * s0;
    acc1 += w * s1;
    acc2 += w * s2;
    T *= 1.0f - alpha;
    if (g == 0) nsamp += (unsigned long long)nf;
    if (alive) {
      a = b;
      alive = a < end;
    }
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
  wave_lds_sync();   // the rows are rewritten by the next packet
}

template <int NL, int SH, int CL, typename TabT, bool BF, bool PK, bool SHADOW>
__global__ __launch_bounds__(256) void k_march_fields(RayQueue q, const int* __restrict__ count,
                                                      int* __restrict__ work, JointFields J, MarchParams P, BvhView B,
                                                      unsigned long long* __restrict__ stats) {
  __shared__ int sstack[SHADOW ? 4 * 16 * kStack : 1];   // shadow-ray stacks: 16 lanes per wave
  __shared__ float sbnd[PK ? 4 : 1][16][2 * kMaxFields];   // packets: each ray's stretch per field
  const int lane = threadIdx.x & 63;
  const int cnt = *count;
  int* stack = SHADOW ? sstack + (threadIdx.x >> 6) * 16 * kStack + (lane & 15) : sstack;
  unsigned long long nsamp = 0;
  if constexpr (PK) {
    WorkQueue wq(work, cnt, P.chunk, 16);
    for (int base = wq.next(lane); base >= 0; base = wq.next(lane)) {
      const int r = wq.map(base + (lane & 15));
      march_fields_packet<NL, SH, CL, TabT, BF, SHADOW>(q, r, r < cnt, J, P, B, sbnd[threadIdx.x >> 6], stack, lane,
                                                        nsamp);
    }
  } else {
    WorkQueue wq(work, cnt, P.chunk, P.batch);
    for (int base = wq.next(lane); base >= 0; base = wq.next(lane))
      for (int bi = 0; bi < wq.batch; ++bi) {
        const int r = wq.map(base + bi);
        if (r >= cnt) break;
        march_fields_ray<NL, SH, CL, TabT, BF, SHADOW>(q, r, J, P, B, stack, lane, nsamp);
      }
  }
  if (stats) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) nsamp += __shfl_xor(nsamp, off, 64);
    if (lane == 0 && nsamp) atomicAdd(stats + 0, nsamp);
  }
}

template <int NL, int SH, int CL, typename TabT, bool BF, bool PK, bool SHADOW>
mr_status launch_fields_mode(const JointFields& J, RayQueue q, const int* count, int* work, const MarchParams& P,
                             const BvhView& B, unsigned long long* stats, int blocks_per_cu, int64_t n,
                             hipStream_t st) {
  auto* k = k_march_fields<NL, SH, CL, TabT, BF, PK, SHADOW>;
  const int64_t cap = PK ? (n + 63) / 64 : (n + 3) / 4;
  const int blocks = persistent_blocks(reinterpret_cast<const void*>(k), 256, blocks_per_cu, cap);
  hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, st, q, count, work, J, P, B, stats);
  MR_HIP(hipGetLastError());
  return MR_OK;
}

template <int NL, int SH, int CL, typename TabT, bool BF>
mr_status launch_fields(const JointFields& J, RayQueue q, const int* count, int* work, const MarchParams& P,
                        const BvhView& B, bool packets, unsigned long long* stats, int blocks_per_cu, int64_t n,
                        hipStream_t st) {
  if (packets)
    return P.shadows ? launch_fields_mode<NL, SH, CL, TabT, BF, true, true>(J, q, count, work, P, B, stats,
                                                                            blocks_per_cu, n, st)
                     : launch_fields_mode<NL, SH, CL, TabT, BF, true, false>(J, q, count, work, P, B, stats,
                                                                             blocks_per_cu, n, st);
  return P.shadows ? launch_fields_mode<NL, SH, CL, TabT, BF, false, true>(J, q, count, work, P, B, stats,
                                                                           blocks_per_cu, n, st)
                   : launch_fields_mode<NL, SH, CL, TabT, BF, false, false>(J, q, count, work, P, B, stats,
                                                                            blocks_per_cu, n, st);
}

}  // namespace

namespace mr {

mr_status dispatch_march_fields(const mr_field* const* fields, int n_fields, RayQueue q, const int* count, int* work,
                                const MarchParams& P, const BvhView& B, bool packets, unsigned long long* stats,
                                int blocks_per_cu, int64_t n, hipStream_t st) {
  if (n_fields < 1 || n_fields > kMaxFields) return fail(MR_ERR_INVALID_ARG, "n_fields must be in 1..8");
  JointFields J;
  std::memset(&J, 0, sizeof(J));
  J.n = n_fields;
  const FieldView& v = fields[0]->view;
  const bool h = v.table_dtype == MR_F16, bf = v.mlp_dtype == MR_BF16;
  for (int k = 0; k < n_fields; ++k) {
    const FieldView& w = fields[k]->view;
    if (w.n_levels != v.n_levels || w.sh != v.sh || w.c_layers != v.c_layers || w.table_dtype != v.table_dtype ||
        w.mlp_dtype != v.mlp_dtype)
      return fail(MR_ERR_UNSUPPORTED, "fields whose boxes overlap must share one layout (levels, SH components, "
                                      "colour layers, table and MLP types)");
    J.view[k] = w;
    J.table[k] = fields[k]->table_dev;
    J.frags[k] = bf ? fields[k]->frag_bf16_dev : fields[k]->frag_f32_dev;
  }
#define M(NL, SH, CL)                                                                                      \
  if (v.n_levels == NL && v.sh == SH && v.c_layers == CL) {                                                 \
    if (bf)                                                                                                 \
      return h ? launch_fields<NL, SH, CL, __half, true>(J, q, count, work, P, B, packets, stats, blocks_per_cu, \
                                                         n, st)                                             \
               : launch_fields<NL, SH, CL, float, true>(J, q, count, work, P, B, packets, stats, blocks_per_cu, n, \
                                                        st);                                                \
    return h ? launch_fields<NL, SH, CL, __half, false>(J, q, count, work, P, B, packets, stats, blocks_per_cu, n, \
                                                        st)                                                 \
             : launch_fields<NL, SH, CL, float, false>(J, q, count, work, P, B, packets, stats, blocks_per_cu, n, st); \
  }
  M(8, 4, 1)
  M(16, 16, 2)
  M(16, 4, 1)
  M(8, 16, 2)
#undef M
  return fail(MR_ERR_UNSUPPORTED, "field shape not instantiated");
}

}  // namespace mr
