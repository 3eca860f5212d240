// Shared host/device definitions of the meshrf HIP library (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <string>
#include <vector>

#include "meshrf.h"

namespace mr {

constexpr int kMaxLevels = 16;
constexpr int kMaxMaterials = 16;
constexpr int kMaxLights = 8;
constexpr int kStack = 48;          // BVH traversal stack depth (tree depth is capped below it)
constexpr int kLeafSize = 4;
constexpr int kTraceBlock = 128;    // threads per block of the traversal kernels

// Radiance-field layouts (levels, SH components, colour hidden layers) that
// have march and query kernels, and the subset that the proposal-sampled march
// serves.  mr_field_create refuses every other layout and mr_render refuses a
// proposal render of a layout outside the subset, before any launch.
inline bool march_layout(int nl, int sh, int cl) {
  return (nl == 8 && sh == 4 && cl == 1) || (nl == 16 && sh == 16 && cl == 2) || (nl == 16 && sh == 4 && cl == 1) ||
         (nl == 8 && sh == 16 && cl == 2);
}
inline bool proposal_march_layout(int nl, int sh, int cl) {
  return (nl == 8 && sh == 4 && cl == 1) || (nl == 16 && sh == 16 && cl == 2);
}

// ---------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
mr_status fail(mr_status s, const std::string& msg);
#define MR_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return ::mr::fail(MR_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// field as seen by kernels (passed by value)
// ---------------------------------------------------------------------------
struct FieldView {
  int n_levels, feats, log2_table;
  uint32_t table_mask;
  int res[kMaxLevels];
  uint32_t dense_mask;             // bit l: level l is stored densely
  const float* table;              // FP32 [L][T][F] (table_dtype F32)
  const __half* table_h;           // FP16 [L][T][F] (table_dtype F16)
  const float* mlp;                // FP32 flat weights
  const uint16_t* mlp_bf16;        // bf16 bits of the same weights (mlp_dtype BF16)
  int d_in, d_hidden, d_out, c_in, c_hidden, c_layers, sh;
  int n_mlp;
  float density_offset;
  float amin[3], inv_ext[3], amax[3];
  const uint32_t* occ;             // occupancy bits (x fastest) or null
  int occ_res;
  int table_dtype, mlp_dtype;
  // placement in the world (mr_field_set_pose): a world point p is looked up
  // at R^T (p - c), a direction d at R^T d; pose = [R | c] row-major 3x4
  int has_pose;
  float pose[12];
};

// ---------------------------------------------------------------------------
// BVH as seen by kernels
// ---------------------------------------------------------------------------
struct BvhNode {       // both children's boxes live in the parent: 64 bytes
  float4 a;            // c0.lo.x c0.lo.y c0.lo.z c0.hi.x
  float4 b;            // c0.hi.y c0.hi.z c1.lo.x c1.lo.y
  float4 c;            // c1.lo.z c1.hi.x c1.hi.y c1.hi.z
  int4 d;              // child0, child1, count0, count1: count > 0 leaf of prims
                       // [child, child+count); count == 0 inner node; child < 0 empty
};

struct Material {
  int kind;
  float ior;
  float albedo[3];
  float emission[3];
};

struct BvhView {
  const BvhNode* nodes;
  const float4* tris;  // 3 per prim in leaf order: (v0, id bits), (v1, material bits), (v2, 0)
  int n_prims;
};

// Emitting triangles for light sampling, in face order: x = cumulative
// choice probability (the last is 1), y = the triangle's own probability,
// z = its position in leaf order (int bits).  A triangle is chosen with
// probability proportional to its summed emitted radiance; its area is read
// from the current vertices, so a refit keeps the table valid.
struct MeshView {
  BvhView bvh;
  int n_mat;
  int emissive;        // some material emits (hits then read their material even at the bounce limit)
  Material mat[kMaxMaterials];
  const float4* emit;  // [n_emit]
  int n_emit;
};

}  // namespace mr

struct mr_field {
  mr::FieldView view;
  mr_field_desc desc;
  int resolutions[mr::kMaxLevels];
  void* table_dev = nullptr;       // FP32 or FP16 copy
  float* mlp_dev = nullptr;        // FP32 weights
  uint16_t* mlp_bf16_dev = nullptr;
  uint32_t* frag_f32_dev = nullptr;    // MFMA weight fragments, FP32
  uint32_t* frag_bf16_dev = nullptr;   // MFMA weight fragments, bf16
  uint32_t* occ_dev = nullptr;
  int occ_res = 0;
  float* master_dev = nullptr;        // proposal fields: FP32 master table for training
  float* opt_dev = nullptr;           // proposal fields: gradients and Adam moments
  int64_t opt_step = 0;
  int64_t n_table = 0, n_mlp = 0;
};

struct mr_mesh {
  mr::MeshView view;
  mr::BvhNode* nodes_dev = nullptr;
  float4* tris_dev = nullptr;
  int4* prim_idx_dev = nullptr;     // (i0, i1, i2, original id) per prim in leaf order
  float4* emit_dev = nullptr;       // emitting triangles (MeshView::emit)
  int* refit_nodes_dev = nullptr;   // node ids, deepest level first
  int n_nodes = 0, depth = 0, n_leaves = 0, nv = 0, nf = 0;
  std::vector<int>* level_offsets = nullptr;   // host: offsets of each level in refit_nodes
};
