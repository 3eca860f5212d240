// Triangle meshes: binned-SAH BVH build on the host, bottom-up refit on the
// device, and a closest-hit query.  Implements the ray-casting function
// t(p, w) of Eq. 3 (first surface hit along a ray) for the inserted meshes,
// and the per-step vertex update of dynamic meshes (Sec. 3.2 hands new vertex
// positions to the renderer every step).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "mr_device.h"

using namespace mr;

namespace {

constexpr int kMaxDepth = 44;
// a traversal holds at most one pending sibling per level of its current path
static_assert(kMaxDepth < kStack, "BVH depth must stay below the traversal stack size");
constexpr int kBins = 32;

struct Box {
  float lo[3] = {INFINITY, INFINITY, INFINITY};
  float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  void grow(const Box& b) {
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], b.lo[k]);
      hi[k] = std::max(hi[k], b.hi[k]);
    }
  }
  void grow(const float* p) {
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], p[k]);
      hi[k] = std::max(hi[k], p[k]);
    }
  }
  float area() const {
    if (hi[0] < lo[0]) return 0.0f;
    const float x = hi[0] - lo[0], y = hi[1] - lo[1], z = hi[2] - lo[2];
    return 2.0f * (x * y + y * z + z * x);
  }
};

struct BuildNode {
  Box box;
  int child[2] = {-1, -1};
  int first = 0, count = 0;   // leaf when count > 0
};

struct Builder {
  const std::vector<Box>& pbox;
  std::vector<float> cen;       // 3 per prim
  std::vector<int> ids;
  std::vector<BuildNode> nodes;
  int max_depth = 0;

  Builder(const std::vector<Box>& b) : pbox(b) {
    const int n = (int)b.size();
    cen.resize(3 * n);
    ids.resize(n);
    std::iota(ids.begin(), ids.end(), 0);
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < 3; ++k) cen[3 * i + k] = 0.5f * (b[i].lo[k] + b[i].hi[k]);
  }

  int make_leaf(int begin, int end, const Box& box) {
    BuildNode nd;
    nd.box = box;
    nd.first = begin;
    nd.count = end - begin;
    nodes.push_back(nd);
    return (int)nodes.size() - 1;
  }

  int build(int begin, int end, int depth) {
    max_depth = std::max(max_depth, depth);
    Box box, cbox;
    for (int i = begin; i < end; ++i) {
      box.grow(pbox[ids[i]]);
      cbox.grow(&cen[3 * ids[i]]);
    }
    const int n = end - begin;
    if (n <= kLeafSize || depth >= kMaxDepth) return make_leaf(begin, end, box);
    // binned SAH over the three axes
    float best_cost = INFINITY;
    int best_axis = -1, best_split = -1;
    for (int ax = 0; ax < 3; ++ax) {
      const float ext = cbox.hi[ax] - cbox.lo[ax];
      if (!(ext > 0.0f)) continue;
      Box bb[kBins];
      int bc[kBins] = {0};
      const float scale = kBins / ext;
      for (int i = begin; i < end; ++i) {
        int b = (int)((cen[3 * ids[i] + ax] - cbox.lo[ax]) * scale);
        b = std::min(std::max(b, 0), kBins - 1);
        bc[b]++;
        bb[b].grow(pbox[ids[i]]);
      }
      float rarea[kBins];
      int rcount[kBins];
      Box acc;
      int cnt = 0;
      for (int b = kBins - 1; b > 0; --b) {
        acc.grow(bb[b]);
        cnt += bc[b];
        rarea[b] = acc.area();
        rcount[b] = cnt;
      }
      Box lacc;
      int lcnt = 0;
      for (int b = 0; b < kBins - 1; ++b) {
        lacc.grow(bb[b]);
        lcnt += bc[b];
        if (lcnt == 0 || rcount[b + 1] == 0) continue;
        const float cost = lacc.area() * lcnt + rarea[b + 1] * rcount[b + 1];
        if (cost < best_cost) {
          best_cost = cost;
          best_axis = ax;
          best_split = b;
        }
      }
    }
    int mid;
    if (best_axis < 0) {
      mid = begin + n / 2;   // all centroids coincide: split by index
    } else {
      const float leaf_cost = (float)n * box.area();
      if (n <= 2 * kLeafSize && best_cost + box.area() >= leaf_cost) return make_leaf(begin, end, box);
      const float ext = cbox.hi[best_axis] - cbox.lo[best_axis];
      const float scale = kBins / ext;
      auto it = std::partition(ids.begin() + begin, ids.begin() + end, [&](int p) {
        int b = (int)((cen[3 * p + best_axis] - cbox.lo[best_axis]) * scale);
        b = std::min(std::max(b, 0), kBins - 1);
        return b <= best_split;
      });
      mid = (int)(it - ids.begin());
      if (mid == begin || mid == end) mid = begin + n / 2;
    }
    BuildNode nd;
    nd.box = box;
    nodes.push_back(nd);
    const int me = (int)nodes.size() - 1;
    const int l = build(begin, mid, depth + 1);
    const int r = build(mid, end, depth + 1);
    nodes[me].child[0] = l;
    nodes[me].child[1] = r;
    return me;
  }
};

void put_box(BvhNode& n, int c, const Box& b) {
  float* a = reinterpret_cast<float*>(&n);   // a, b, c hold 12 floats: c0 lo/hi then c1 lo/hi
  const int o = 6 * c;
  a[o + 0] = b.lo[0];
  a[o + 1] = b.lo[1];
  a[o + 2] = b.lo[2];
  a[o + 3] = b.hi[0];
  a[o + 4] = b.hi[1];
  a[o + 5] = b.hi[2];
}

// ---------------------------------------------------------------------------
// device refit: copy new vertex positions into the leaf-ordered triangles,
// then recompute child boxes level by level, deepest first.
// ---------------------------------------------------------------------------
__global__ void k_refit_tris(const float* __restrict__ v, const int4* __restrict__ prim_idx, int n_prims,
                             float4* __restrict__ tris) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n_prims; p += gridDim.x * blockDim.x) {
    const int4 q = prim_idx[p];
    const float4 old0 = tris[3 * p], old1 = tris[3 * p + 1];
    tris[3 * p] = make_float4(v[3 * q.x], v[3 * q.x + 1], v[3 * q.x + 2], old0.w);
    tris[3 * p + 1] = make_float4(v[3 * q.y], v[3 * q.y + 1], v[3 * q.y + 2], old1.w);
    tris[3 * p + 2] = make_float4(v[3 * q.z], v[3 * q.z + 1], v[3 * q.z + 2], 0.0f);
  }
}

__device__ void child_box(const BvhNode* nodes, const float4* tris, int child, int count, float lo[3],
                          float hi[3]) {
  for (int k = 0; k < 3; ++k) {
    lo[k] = INFINITY;
    hi[k] = -INFINITY;
  }
  if (child < 0) return;
  if (count > 0) {
    for (int p = child; p < child + count; ++p)
      for (int j = 0; j < 3; ++j) {
        const float4 q = tris[3 * p + j];
        lo[0] = fminf(lo[0], q.x); lo[1] = fminf(lo[1], q.y); lo[2] = fminf(lo[2], q.z);
        hi[0] = fmaxf(hi[0], q.x); hi[1] = fmaxf(hi[1], q.y); hi[2] = fmaxf(hi[2], q.z);
      }
  } else {
    const BvhNode c = nodes[child];
    lo[0] = fminf(c.a.x, c.b.z); lo[1] = fminf(c.a.y, c.b.w); lo[2] = fminf(c.a.z, c.c.x);
    hi[0] = fmaxf(c.a.w, c.c.y); hi[1] = fmaxf(c.b.x, c.c.z); hi[2] = fmaxf(c.b.y, c.c.w);
  }
}

__global__ void k_refit_level(BvhNode* __restrict__ nodes, const float4* __restrict__ tris,
                              const int* __restrict__ ids, int count) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
    const int ni = ids[i];
    BvhNode n = nodes[ni];
    float l0[3], h0[3], l1[3], h1[3];
    child_box(nodes, tris, n.d.x, n.d.z, l0, h0);
    child_box(nodes, tris, n.d.y, n.d.w, l1, h1);
    n.a = make_float4(l0[0], l0[1], l0[2], h0[0]);
    n.b = make_float4(h0[1], h0[2], l1[0], l1[1]);
    n.c = make_float4(l1[2], h1[0], h1[1], h1[2]);
    nodes[ni] = n;
  }
}

__global__ __launch_bounds__(kTraceBlock) void k_closest(BvhView B, int64_t n, const float* __restrict__ o,
                                                         const float* __restrict__ d, float tmax,
                                                         float* __restrict__ t_hit, int32_t* __restrict__ tri) {
  __shared__ int stack[kStack * kTraceBlock];
  __shared__ float tstack[kStack * kTraceBlock];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const RayPre r = ray_pre(v3(o[3 * i], o[3 * i + 1], o[3 * i + 2]), v3(d[3 * i], d[3 * i + 1], d[3 * i + 2]));
    float t;
    const int p = bvh_trace<false>(B, r, tmax, t, stack + threadIdx.x, tstack + threadIdx.x, kTraceBlock);
    t_hit[i] = p >= 0 ? t : INFINITY;
    tri[i] = p >= 0 ? __float_as_int(B.tris[3 * p].w) : -1;
  }
}

}  // namespace

extern "C" mr_status mr_mesh_build_bvh(const float* host_vertices, int32_t nv, const int32_t* host_indices,
                                       int32_t nf, const int32_t* host_mat_ids, const mr_material* host_materials,
                                       int32_t n_materials, void* stream, mr_mesh** out) {
  if (!out) return fail(MR_ERR_INVALID_ARG, "null out");
  if (nv < 0 || nf < 0) return fail(MR_ERR_INVALID_ARG, "negative sizes");
  if (nf > 0 && (!host_vertices || !host_indices || !host_mat_ids))
    return fail(MR_ERR_INVALID_ARG, "null mesh arrays");
  if (n_materials < 1 || n_materials > kMaxMaterials || !host_materials)
    return fail(MR_ERR_INVALID_ARG, "n_materials must be in 1..16");
  for (int m = 0; m < n_materials; ++m) {
    const mr_material& mt = host_materials[m];
    if (mt.kind < MR_MIRROR || mt.kind > MR_DIFFUSE) return fail(MR_ERR_INVALID_ARG, "unknown material kind");
    if (mt.kind == MR_GLASS && !(mt.ior > 1.0f && std::isfinite(mt.ior)))
      return fail(MR_ERR_INVALID_ARG, "glass ior must be finite and > 1");
    for (int c = 0; c < 3; ++c)
      if (!(mt.albedo[c] >= 0.0f && mt.albedo[c] <= 1.0f)) return fail(MR_ERR_INVALID_ARG, "albedo outside [0, 1]");
    for (int c = 0; c < 3; ++c)
      if (!(mt.emission[c] >= 0.0f && std::isfinite(mt.emission[c])))
        return fail(MR_ERR_INVALID_ARG, "emission must be finite and >= 0");
  }
  for (int64_t i = 0; i < 3LL * nv; ++i)
    if (!std::isfinite(host_vertices[i])) return fail(MR_ERR_INVALID_ARG, "non-finite vertex");
  for (int64_t i = 0; i < 3LL * nf; ++i)
    if (host_indices[i] < 0 || host_indices[i] >= nv) return fail(MR_ERR_INVALID_ARG, "index out of range");
  for (int i = 0; i < nf; ++i)
    if (host_mat_ids[i] < 0 || host_mat_ids[i] >= n_materials) return fail(MR_ERR_INVALID_ARG, "material id out of range");

  std::vector<Box> pb(nf);
  for (int i = 0; i < nf; ++i)
    for (int j = 0; j < 3; ++j) pb[i].grow(host_vertices + 3 * host_indices[3 * i + j]);
  Builder B(pb);
  std::vector<BvhNode> flat;
  std::vector<int> depth_of;
  if (nf > 0) B.build(0, nf, 0);
  // flatten: inner build nodes become BvhNodes in preorder; leaves live in their parent
  std::vector<int> map(B.nodes.size(), -1);
  struct Item { int bn, depth; };
  BvhNode empty;
  std::memset(&empty, 0, sizeof(empty));
  if (nf == 0 || B.nodes[0].count > 0) {
    BvhNode root = empty;
    Box inv;
    put_box(root, 0, nf ? B.nodes[0].box : inv);
    put_box(root, 1, inv);
    root.d = make_int4(nf ? 0 : -1, -1, nf, 0);
    flat.push_back(root);
    depth_of.push_back(0);
  } else {
    std::vector<Item> st{{0, 0}};
    std::vector<std::pair<int, int>> fix;   // (flat index, child slot) waiting for a child's flat index
    // iterative preorder
    std::vector<std::pair<int, int>> order;
    while (!st.empty()) {
      Item it = st.back();
      st.pop_back();
      map[it.bn] = (int)flat.size();
      flat.push_back(empty);
      depth_of.push_back(it.depth);
      order.push_back({it.bn, it.depth});
      const BuildNode& bn = B.nodes[it.bn];
      for (int c = 1; c >= 0; --c) {
        const BuildNode& ch = B.nodes[bn.child[c]];
        if (ch.count == 0) st.push_back({bn.child[c], it.depth + 1});
      }
    }
    for (auto& pr : order) {
      const BuildNode& bn = B.nodes[pr.first];
      BvhNode& n = flat[map[pr.first]];
      int ch[2], cnt[2];
      for (int c = 0; c < 2; ++c) {
        const BuildNode& cb = B.nodes[bn.child[c]];
        put_box(n, c, cb.box);
        if (cb.count > 0) {
          ch[c] = cb.first;
          cnt[c] = cb.count;
        } else {
          ch[c] = map[bn.child[c]];
          cnt[c] = 0;
        }
      }
      n.d = make_int4(ch[0], ch[1], cnt[0], cnt[1]);
    }
  }
  // leaf-ordered triangles
  std::vector<float4> tris(3 * std::max(nf, 1));
  std::vector<int4> pidx(std::max(nf, 1));
  for (int p = 0; p < nf; ++p) {
    const int id = B.ids[p];
    const int* f = host_indices + 3 * id;
    const float* v0 = host_vertices + 3 * f[0];
    const float* v1 = host_vertices + 3 * f[1];
    const float* v2 = host_vertices + 3 * f[2];
    float idbits, matbits;
    std::memcpy(&idbits, &id, 4);
    std::memcpy(&matbits, &host_mat_ids[id], 4);
    tris[3 * p] = make_float4(v0[0], v0[1], v0[2], idbits);
    tris[3 * p + 1] = make_float4(v1[0], v1[1], v1[2], matbits);
    tris[3 * p + 2] = make_float4(v2[0], v2[1], v2[2], 0.0f);
    pidx[p] = make_int4(f[0], f[1], f[2], id);
  }
  // refit order: node ids grouped by depth, deepest first
  int maxd = 0;
  for (int dd : depth_of) maxd = std::max(maxd, dd);
  std::vector<int> refit;
  auto* offs = new std::vector<int>();
  for (int dd = maxd; dd >= 0; --dd) {
    offs->push_back((int)refit.size());
    for (int i = 0; i < (int)flat.size(); ++i)
      if (depth_of[i] == dd) refit.push_back(i);
  }
  offs->push_back((int)refit.size());

  mr_mesh* m = new mr_mesh();
  m->level_offsets = offs;
  m->n_nodes = (int)flat.size();
  m->depth = B.max_depth;
  m->n_leaves = 0;
  for (auto& bn : B.nodes)
    if (bn.count > 0) m->n_leaves++;
  m->nv = nv;
  m->nf = nf;
  hipStream_t st = (hipStream_t)stream;
  auto cleanup = [&](mr_status s, const char* msg) {
    mr_mesh_destroy(m);
    return fail(s, msg);
  };
  if (hipMalloc(&m->nodes_dev, flat.size() * sizeof(BvhNode)) != hipSuccess) return cleanup(MR_ERR_OOM, "bvh alloc");
  if (hipMalloc(&m->tris_dev, tris.size() * sizeof(float4)) != hipSuccess) return cleanup(MR_ERR_OOM, "tri alloc");
  if (hipMalloc(&m->prim_idx_dev, pidx.size() * sizeof(int4)) != hipSuccess) return cleanup(MR_ERR_OOM, "idx alloc");
  if (hipMalloc(&m->refit_nodes_dev, std::max<size_t>(refit.size(), 1) * sizeof(int)) != hipSuccess)
    return cleanup(MR_ERR_OOM, "refit alloc");
  bool ok = hipMemcpyAsync(m->nodes_dev, flat.data(), flat.size() * sizeof(BvhNode), hipMemcpyHostToDevice, st) == hipSuccess;
  ok = ok && hipMemcpyAsync(m->tris_dev, tris.data(), tris.size() * sizeof(float4), hipMemcpyHostToDevice, st) == hipSuccess;
  ok = ok && hipMemcpyAsync(m->prim_idx_dev, pidx.data(), pidx.size() * sizeof(int4), hipMemcpyHostToDevice, st) == hipSuccess;
  if (!refit.empty())
    ok = ok && hipMemcpyAsync(m->refit_nodes_dev, refit.data(), refit.size() * sizeof(int), hipMemcpyHostToDevice, st) == hipSuccess;
  // emitting triangles in face order, chosen by summed emitted radiance
  std::vector<int> leaf_of(std::max(nf, 1), -1);
  for (int p = 0; p < nf; ++p) leaf_of[B.ids[p]] = p;
  std::vector<float4> emit;
  double wsum = 0.0;
  for (int i = 0; i < nf; ++i) {
    const float* e = host_materials[host_mat_ids[i]].emission;
    wsum += (double)e[0] + (double)e[1] + (double)e[2];
  }
  if (wsum > 0.0) {
    double cum = 0.0;
    for (int i = 0; i < nf; ++i) {
      const float* e = host_materials[host_mat_ids[i]].emission;
      const double w = (double)e[0] + (double)e[1] + (double)e[2];
      if (!(w > 0.0)) continue;
      cum += w;
      float leafbits;
      std::memcpy(&leafbits, &leaf_of[i], 4);
      emit.push_back(make_float4((float)(cum / wsum), (float)(w / wsum), leafbits, 0.0f));
    }
    emit.back().x = 1.0f;
    if (hipMalloc(&m->emit_dev, emit.size() * sizeof(float4)) != hipSuccess) return cleanup(MR_ERR_OOM, "emitter alloc");
    ok = ok && hipMemcpyAsync(m->emit_dev, emit.data(), emit.size() * sizeof(float4), hipMemcpyHostToDevice, st) == hipSuccess;
  }
  ok = ok && hipStreamSynchronize(st) == hipSuccess;
  if (!ok) return cleanup(MR_ERR_DEVICE, "bvh upload");
  m->view.emit = m->emit_dev;
  m->view.n_emit = (int)emit.size();
  m->view.bvh.nodes = m->nodes_dev;
  m->view.bvh.tris = m->tris_dev;
  m->view.bvh.n_prims = nf;
  m->view.n_mat = n_materials;
  m->view.emissive = 0;
  for (int i = 0; i < n_materials; ++i) {
    m->view.mat[i].kind = host_materials[i].kind;
    m->view.mat[i].ior = host_materials[i].ior;
    for (int c = 0; c < 3; ++c) {
      m->view.mat[i].albedo[c] = host_materials[i].albedo[c];
      m->view.mat[i].emission[c] = host_materials[i].emission[c];
      if (host_materials[i].emission[c] > 0.0f) m->view.emissive = 1;
    }
  }
  *out = m;
  return MR_OK;
}

extern "C" mr_status mr_mesh_refit(mr_mesh* m, const float* vertices, void* stream) {
  if (!m) return fail(MR_ERR_INVALID_ARG, "null mesh");
  if (m->nf == 0) return MR_OK;
  if (!vertices) return fail(MR_ERR_INVALID_ARG, "null vertices");
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_refit_tris, dim3((m->nf + 255) / 256), dim3(256), 0, st, vertices, m->prim_idx_dev, m->nf,
                     m->tris_dev);
  MR_HIP(hipGetLastError());
  const auto& offs = *m->level_offsets;
  for (size_t l = 0; l + 1 < offs.size(); ++l) {
    const int cnt = offs[l + 1] - offs[l];
    if (cnt == 0) continue;
    hipLaunchKernelGGL(k_refit_level, dim3((cnt + 127) / 128), dim3(128), 0, st, m->nodes_dev, m->tris_dev,
                       m->refit_nodes_dev + offs[l], cnt);
    MR_HIP(hipGetLastError());
  }
  return MR_OK;
}

extern "C" mr_status mr_mesh_destroy(mr_mesh* m) {
  if (!m) return MR_OK;
  if (m->nodes_dev) (void)hipFree(m->nodes_dev);
  if (m->tris_dev) (void)hipFree(m->tris_dev);
  if (m->prim_idx_dev) (void)hipFree(m->prim_idx_dev);
  if (m->emit_dev) (void)hipFree(m->emit_dev);
  if (m->refit_nodes_dev) (void)hipFree(m->refit_nodes_dev);
  delete m->level_offsets;
  delete m;
  return MR_OK;
}

extern "C" mr_status mr_mesh_info(const mr_mesh* m, int32_t* n_nodes, int32_t* depth, int32_t* n_leaves) {
  if (!m) return fail(MR_ERR_INVALID_ARG, "null mesh");
  if (n_nodes) *n_nodes = m->n_nodes;
  if (depth) *depth = m->depth;
  if (n_leaves) *n_leaves = m->n_leaves;
  return MR_OK;
}

extern "C" mr_status mr_mesh_closest_hit(const mr_mesh* m, int64_t n, const float* origins, const float* dirs,
                                         float t_max, float* t_hit, int32_t* tri, void* stream) {
  if (!m) return fail(MR_ERR_INVALID_ARG, "null mesh");
  if (n < 0) return fail(MR_ERR_INVALID_ARG, "n < 0");
  if (n == 0) return MR_OK;
  if (!origins || !dirs || !t_hit || !tri) return fail(MR_ERR_INVALID_ARG, "null array");
  if (!(t_max > 0.0f)) return fail(MR_ERR_INVALID_ARG, "t_max must be > 0");
  hipStream_t st = (hipStream_t)stream;
  const int blocks = (int)std::min<int64_t>((n + kTraceBlock - 1) / kTraceBlock, 16384);
  hipLaunchKernelGGL(k_closest, dim3(blocks), dim3(kTraceBlock), 0, st, m->view.bvh, n, origins, dirs, t_max, t_hit,
                     tri);
  MR_HIP(hipGetLastError());
  return MR_OK;
}
