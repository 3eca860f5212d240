"""Thin ctypes binding of ``libmeshrf.so`` (the C ABI in ``include/meshrf.h``).

Only argument marshalling happens here: every step of the rendering path runs
in the library's HIP kernels.  PyTorch provides device memory and streams.
The functions named ``mr_*`` mirror the C entry points one to one; the small
classes below own handles and the device tensors that a call needs.

There is no fallback: if the library is missing, importing a function raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmeshrf.so")

MR_OK, MR_ERR_INVALID_ARG, MR_ERR_OOM, MR_ERR_DEVICE, MR_ERR_UNSUPPORTED, MR_ERR_STATE = range(6)
MR_F32, MR_F16, MR_BF16 = 0, 1, 2
MR_MIRROR, MR_GLASS, MR_DIFFUSE = 0, 1, 2
MR_SAMPLER_UNIFORM, MR_SAMPLER_PROPOSAL = 0, 1

EXPORTED = [
    "mr_autotune_candidates", "mr_autotune_render", "mr_autotune_search", "mr_camera_bounce_limits", "mr_field_build_occupancy", "mr_field_create",
    "mr_field_destroy", "mr_field_params", "mr_field_query", "mr_field_set_pose", "mr_graph_destroy",
    "mr_graph_launch", "mr_last_error", "mr_mesh_build_bvh", "mr_mesh_closest_hit", "mr_mesh_destroy",
    "mr_mesh_info", "mr_mesh_refit", "mr_probe_gather", "mr_probe_gather_region", "mr_mlp_fragments", "mr_profile_enable", "mr_profile_read",
    "mr_proposal_grad", "mr_proposal_targets", "mr_proposal_train_step", "mr_rays_from_cameras", "mr_render",
    "mr_render_fields", "mr_render_fields_workspace_size", "mr_render_graph_create",
    "mr_render_noalloc", "mr_render_status",
    "mr_render_workspace_size", "mr_version",
]


class MrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"meshrf status {status}: {msg}")
        self.status = status


class FieldDesc(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("feats_per_level", C.c_int32),
                ("log2_table_size", C.c_int32), ("host_resolutions", C.c_void_p),
                ("table_dtype", C.c_int32), ("mlp_dtype", C.c_int32),
                ("density_in", C.c_int32), ("density_hidden", C.c_int32),
                ("density_out", C.c_int32), ("color_in", C.c_int32),
                ("color_hidden", C.c_int32), ("color_hidden_layers", C.c_int32),
                ("sh_components", C.c_int32), ("density_offset", C.c_float),
                ("aabb_min", C.c_float * 3), ("aabb_max", C.c_float * 3)]


class Material(C.Structure):
    _fields_ = [("kind", C.c_int32), ("ior", C.c_float), ("albedo", C.c_float * 3),
                ("emission", C.c_float * 3)]


class Light(C.Structure):
    _fields_ = [("pos", C.c_float * 3), ("intensity", C.c_float * 3)]


class RenderOpts(C.Structure):
    _fields_ = [("t_near", C.c_float), ("t_far", C.c_float), ("n_samples", C.c_int32),
                ("sampler", C.c_int32), ("proposal", C.c_void_p), ("n_proposal", C.c_int32),
                ("n_fine", C.c_int32), ("use_occupancy", C.c_int32), ("rr_after", C.c_int32),
                ("t_min_throughput", C.c_float), ("seed", C.c_uint32),
                ("march_blocks_per_cu", C.c_int32), ("stage_blocks_per_cu", C.c_int32),
                ("stage_tile", C.c_int32), ("march_chunk", C.c_int32), ("march_batch", C.c_int32),
                ("march_packets", C.c_int32), ("sample_shadows", C.c_int32), ("shadow_mask", C.c_float),
                ("sample_emitters", C.c_int32), ("wait_polls", C.c_int32),
                ("light_depth_samples", C.c_int32)]


class LaunchCfg(C.Structure):
    _fields_ = [("march_blocks_per_cu", C.c_int32), ("stage_blocks_per_cu", C.c_int32),
                ("stage_tile", C.c_int32), ("march_chunk", C.c_int32), ("march_batch", C.c_int32),
                ("march_packets", C.c_int32)]


class Adam(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float)]


class RenderOut(C.Structure):
    _fields_ = [("radiance", C.c_void_p), ("throughput", C.c_void_p), ("bounces", C.c_void_p),
                ("hit_ids", C.c_void_p), ("hit_stride", C.c_int32), ("counters", C.c_void_p)]


_lib = None


def lib():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2309_04581_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        L.mr_last_error.restype = C.c_char_p
        L.mr_version.restype = C.c_char_p
        L.mr_render_workspace_size.restype = C.c_size_t
        L.mr_render_workspace_size.argtypes = [C.c_int64]
        L.mr_render_fields_workspace_size.restype = C.c_size_t
        L.mr_render_fields_workspace_size.argtypes = [C.c_int64, C.c_int32]
        for name in EXPORTED:
            if name not in ("mr_last_error", "mr_version", "mr_render_workspace_size",
                            "mr_render_fields_workspace_size"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(status):
    if status != MR_OK:
        raise MrError(status, lib().mr_last_error().decode())


def _ptr(t):
    """Device (or host) address of a tensor/array, or None."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return C.c_void_p(t.ctypes.data)
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


# ---------------------------------------------------------------------------
# C entry points, same names
# ---------------------------------------------------------------------------

def mr_version():
    return lib().mr_version().decode()


def mr_field_create(desc: FieldDesc, host_table: np.ndarray, host_mlp: np.ndarray, stream=None):
    h = C.c_void_p()
    _check(lib().mr_field_create(C.byref(desc), _ptr(host_table), _ptr(host_mlp), _stream(stream),
                                 C.byref(h)))
    return h


def mr_field_destroy(h):
    _check(lib().mr_field_destroy(h))


def mr_field_query(h, n, x, dirs, sigma, rgb=None, feat=None, raw=None, stream=None):
    _check(lib().mr_field_query(h, C.c_int64(n), _ptr(x), _ptr(dirs), _ptr(sigma), _ptr(rgb),
                                _ptr(feat), _ptr(raw), _stream(stream)))


def mr_field_build_occupancy(h, res, thresh, bits_out=None, stream=None):
    _check(lib().mr_field_build_occupancy(h, C.c_int32(res), C.c_float(thresh), _ptr(bits_out),
                                          _stream(stream)))


def mr_field_params(h):
    tab, mlp = C.c_void_p(), C.c_void_p()
    nt, nm = C.c_int64(), C.c_int64()
    _check(lib().mr_field_params(h, C.byref(tab), C.byref(mlp), C.byref(nt), C.byref(nm)))
    return tab.value, mlp.value, nt.value, nm.value


def mr_mesh_build_bvh(vertices, indices, mat_ids, materials, stream=None):
    v = np.ascontiguousarray(vertices, dtype=np.float32)
    f = np.ascontiguousarray(indices, dtype=np.int32)
    m = np.ascontiguousarray(mat_ids, dtype=np.int32)
    mats = (Material * len(materials))()
    for i, row in enumerate(materials):
        mats[i].kind = int(row[0])
        mats[i].ior = float(row[1])
        mats[i].albedo = (C.c_float * 3)(*[float(x) for x in row[2:5]])
        mats[i].emission = (C.c_float * 3)(*[float(x) for x in (list(row[5:8]) + [0.0] * 3)[:3]])
    h = C.c_void_p()
    _check(lib().mr_mesh_build_bvh(_ptr(v), C.c_int32(len(v)), _ptr(f), C.c_int32(len(f)), _ptr(m),
                                   mats, C.c_int32(len(materials)), _stream(stream), C.byref(h)))
    return h


def mr_mesh_refit(h, vertices, stream=None):
    _check(lib().mr_mesh_refit(h, _ptr(vertices), _stream(stream)))


def mr_mesh_destroy(h):
    _check(lib().mr_mesh_destroy(h))


def mr_mesh_info(h):
    a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().mr_mesh_info(h, C.byref(a), C.byref(b), C.byref(c)))
    return dict(n_nodes=a.value, depth=b.value, n_leaves=c.value)


def mr_mesh_closest_hit(h, n, origins, dirs, t_max, t_hit, tri, stream=None):
    _check(lib().mr_mesh_closest_hit(h, C.c_int64(n), _ptr(origins), _ptr(dirs), C.c_float(t_max),
                                     _ptr(t_hit), _ptr(tri), _stream(stream)))


def mr_render_workspace_size(n):
    return int(lib().mr_render_workspace_size(C.c_int64(n)))


def mr_render(field, mesh, n, origins, dirs, max_bounces, per_ray_max_bounces, lights, opts, out,
              workspace, workspace_bytes, stream=None):
    nl = len(lights)
    arr = (Light * max(nl, 1))()
    for i, row in enumerate(lights):
        arr[i].pos = (C.c_float * 3)(*[float(x) for x in row[:3]])
        arr[i].intensity = (C.c_float * 3)(*[float(x) for x in row[3:6]])
    _check(lib().mr_render(field, mesh, C.c_int64(n), _ptr(origins), _ptr(dirs),
                           C.c_int32(max_bounces), _ptr(per_ray_max_bounces), arr, C.c_int32(nl),
                           C.byref(opts), C.byref(out), _ptr(workspace), C.c_size_t(workspace_bytes),
                           _stream(stream)))


MR_NOALLOC_MAX_RAYS = 262144


def mr_render_noalloc(field, mesh, n, origins, dirs, max_bounces, per_ray_max_bounces, lights, opts, out,
                      gave_up=None, stream=None):
    """mr_render without a workspace (the library's fixed per-device array);
    gave_up: optional device int32 tensor of one element."""
    arr, nl = _lights_arr(lights)
    _check(lib().mr_render_noalloc(field, mesh, C.c_int64(n), _ptr(origins), _ptr(dirs),
                                   C.c_int32(max_bounces), _ptr(per_ray_max_bounces), arr, C.c_int32(nl),
                                   C.byref(opts), C.byref(out), _ptr(gave_up), _stream(stream)))


def mr_render_status(workspace, stream=None):
    """Number of packet-march waves whose bounded wait gave up in the last
    render on this workspace; raises MrError (MR_ERR_DEVICE) when not 0."""
    g = C.c_int64()
    _check(lib().mr_render_status(_ptr(workspace), C.byref(g), _stream(stream)))
    return g.value


def mr_render_fields_workspace_size(n, n_fields):
    return int(lib().mr_render_fields_workspace_size(C.c_int64(n), C.c_int32(n_fields)))


def mr_render_fields(fields, mesh, n, origins, dirs, max_bounces, per_ray_max_bounces, lights, opts, out,
                     workspace, workspace_bytes, stream=None, proposals=None):
    nl = len(lights)
    arr = (Light * max(nl, 1))()
    for i, row in enumerate(lights):
        arr[i].pos = (C.c_float * 3)(*[float(x) for x in row[:3]])
        arr[i].intensity = (C.c_float * 3)(*[float(x) for x in row[3:6]])
    hs = (C.c_void_p * max(len(fields), 1))(*fields)
    ps = (C.c_void_p * max(len(proposals), 1))(*proposals) if proposals is not None else None
    _check(lib().mr_render_fields(hs, ps, C.c_int32(len(fields)), mesh, C.c_int64(n), _ptr(origins), _ptr(dirs),
                                  C.c_int32(max_bounces), _ptr(per_ray_max_bounces), arr, C.c_int32(nl),
                                  C.byref(opts), C.byref(out), _ptr(workspace), C.c_size_t(workspace_bytes),
                                  _stream(stream)))


def mr_rays_from_cameras(host_cams, origins, dirs, cam_index=None, capacity=None, stream=None):
    cams = np.ascontiguousarray(host_cams, dtype=np.float32).reshape(-1, 12)
    cap = capacity if capacity is not None else origins.shape[0]
    _check(lib().mr_rays_from_cameras(_ptr(cams), C.c_int32(len(cams)), _ptr(origins), _ptr(dirs),
                                      _ptr(cam_index), C.c_int64(cap), _stream(stream)))


# ---------------------------------------------------------------------------
# owners of handles (allocation and bookkeeping only)
# ---------------------------------------------------------------------------

def field_desc(f, table_dtype=MR_F32, mlp_dtype=MR_F32):
    """The mr_field_desc of a parameter set; returns (desc, resolutions array
    the desc points into, to be kept alive with it)."""
    d = FieldDesc()
    res = np.ascontiguousarray(f.resolutions, dtype=np.int32)
    d.n_levels, d.feats_per_level, d.log2_table_size = f.n_levels, f.feats, f.log2_table
    d.host_resolutions = res.ctypes.data
    d.table_dtype, d.mlp_dtype = table_dtype, mlp_dtype
    if hasattr(f, "d_hidden"):
        d.density_in, d.density_hidden, d.density_out = f.d_in, f.d_hidden, f.d_out
        d.color_in, d.color_hidden = f.c_in, f.c_hidden
        d.color_hidden_layers, d.sh_components = f.c_layers, f.sh
    else:
        d.density_in, d.density_hidden, d.density_out = f.n_levels * f.feats, f.hidden, 1
    d.density_offset = float(f.density_offset)
    d.aabb_min = (C.c_float * 3)(*f.aabb_min)
    d.aabb_max = (C.c_float * 3)(*f.aabb_max)
    return d, res


def mr_mlp_fragments(f, bf16):
    """The MLP weight fragments mr_field_create stages for a radiance field
    (host only, no device): uint32 words, FP32 weights as three BF16 pieces
    (bf16 False) or one BF16 piece (bf16 True)."""
    d, res = field_desc(f, MR_F32, MR_BF16 if bf16 else MR_F32)
    mlp = np.ascontiguousarray(f.mlp, dtype=np.float32)
    words = C.c_int64()
    _check(lib().mr_mlp_fragments(C.byref(d), _ptr(mlp), C.c_int32(1 if bf16 else 0), None, C.c_int64(0),
                                  C.byref(words)))
    out = np.zeros(words.value, dtype=np.uint32)
    _check(lib().mr_mlp_fragments(C.byref(d), _ptr(mlp), C.c_int32(1 if bf16 else 0), _ptr(out),
                                  C.c_int64(out.size), C.byref(words)))
    del res
    return out


class Field:
    """A field handle created from a seeded parameter set (scene generator
    objects or anything with the same attributes)."""

    def __init__(self, f, table_dtype=MR_F32, mlp_dtype=MR_F32, stream=None):
        d, self._res = field_desc(f, table_dtype, mlp_dtype)
        self.desc = d
        self.src = f
        self.handle = mr_field_create(d, np.ascontiguousarray(f.table, dtype=np.float32),
                                      np.ascontiguousarray(f.mlp, dtype=np.float32), stream)
        if getattr(f, "pose", None) is not None:
            self.set_pose(f.pose)

    def query(self, x, dirs=None, want_rgb=True, want_feat=False, want_raw=False):
        import torch
        n = x.shape[0]
        dev = x.device
        sigma = torch.empty(n, device=dev, dtype=torch.float32)
        rgb = torch.empty(n, 3, device=dev, dtype=torch.float32) if want_rgb else None
        feat = (torch.empty(n, self.src.n_levels * self.src.feats, device=dev, dtype=torch.float32)
                if want_feat else None)
        raw = torch.empty(n, 16, device=dev, dtype=torch.float32) if want_raw else None
        mr_field_query(self.handle, n, x, dirs, sigma, rgb, feat, raw)
        return dict(sigma=sigma, rgb=rgb, feat=feat, raw=raw)

    def set_pose(self, pose):
        """Rigid placement [R | c] (3x4, field frame -> world) or None."""
        if pose is None:
            _check(lib().mr_field_set_pose(self.handle, None))
        else:
            p = np.ascontiguousarray(np.asarray(pose, dtype=np.float32).reshape(12))
            _check(lib().mr_field_set_pose(self.handle, p.ctypes.data_as(C.c_void_p)))

    def build_occupancy(self, res, thresh, export=False):
        import torch
        bits = torch.empty(res ** 3, dtype=torch.uint8, device="cuda") if export else None
        mr_field_build_occupancy(self.handle, res, thresh, bits)
        return bits

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.mr_field_destroy(h)
            self.handle = None


class Mesh:
    def __init__(self, m, stream=None):
        self.src = m
        self.handle = mr_mesh_build_bvh(m.vertices, m.indices, m.mat_ids, m.materials, stream)

    def info(self):
        return mr_mesh_info(self.handle)

    def refit(self, vertices):
        mr_mesh_refit(self.handle, vertices)

    def closest_hit(self, origins, dirs, t_max=1e30):
        import torch
        n = origins.shape[0]
        t = torch.empty(n, device=origins.device, dtype=torch.float32)
        tri = torch.empty(n, device=origins.device, dtype=torch.int32)
        mr_mesh_closest_hit(self.handle, n, origins, dirs, t_max, t, tri)
        return t, tri

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.mr_mesh_destroy(h)
            self.handle = None


def make_opts(scene, sampler=MR_SAMPLER_UNIFORM, proposal=None, n_proposal=32, n_fine=32,
              use_occupancy=False, shadow_mask=None, sample_emitters=False, light_depth_samples=0):
    o = RenderOpts()
    o.t_near, o.t_far, o.n_samples = scene.t_near, scene.t_far, scene.n_samples
    o.sampler = sampler
    o.proposal = proposal.handle if proposal is not None else None
    o.n_proposal, o.n_fine = n_proposal, n_fine
    o.use_occupancy = int(bool(use_occupancy))
    o.rr_after = scene.rr_after
    o.t_min_throughput = scene.t_min_throughput
    o.seed = scene.seed & 0xFFFFFFFF
    if shadow_mask is not None:
        o.sample_shadows, o.shadow_mask = 1, float(shadow_mask)
    o.sample_emitters = int(bool(sample_emitters))
    o.light_depth_samples = int(light_depth_samples)
    return o


class Renderer:
    """Holds the workspace and output tensors for repeated renders of n rays."""

    def __init__(self, n, max_bounces, with_hits=True, device="cuda"):
        import torch
        self.n, self.max_bounces = n, max_bounces
        self.ws_bytes = mr_render_workspace_size(n)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.radiance = torch.empty(n, 3, dtype=torch.float32, device=device)
        self.throughput = torch.empty(n, 3, dtype=torch.float32, device=device)
        self.bounces = torch.empty(n, dtype=torch.int32, device=device)
        self.hit_ids = (torch.empty(n, max_bounces + 1, dtype=torch.int32, device=device)
                        if with_hits else None)
        self.counters = torch.zeros(4, dtype=torch.int64, device=device)
        self.out = RenderOut()
        self.out.radiance = self.radiance.data_ptr()
        self.out.throughput = self.throughput.data_ptr()
        self.out.bounces = self.bounces.data_ptr()
        self.out.hit_ids = self.hit_ids.data_ptr() if with_hits else None
        self.out.hit_stride = max_bounces + 1
        self.out.counters = self.counters.data_ptr()

    def render(self, field, mesh, origins, dirs, lights, opts, per_ray_max_bounces=None, stream=None):
        mr_render(field.handle if field is not None else None,
                  mesh.handle if mesh is not None else None, self.n, origins, dirs,
                  self.max_bounces, per_ray_max_bounces, lights, opts, self.out, self.workspace,
                  self.ws_bytes, stream)
        return self

    def render_noalloc(self, field, mesh, origins, dirs, lights, opts, per_ray_max_bounces=None, gave_up=None,
                       stream=None):
        """The same render through mr_render_noalloc (the library's own array
        instead of this object's workspace)."""
        mr_render_noalloc(field.handle if field is not None else None,
                          mesh.handle if mesh is not None else None, self.n, origins, dirs,
                          self.max_bounces, per_ray_max_bounces, lights, opts, self.out, gave_up, stream)
        return self

    def status(self, stream=None):
        """mr_render_status of the last render into this workspace."""
        return mr_render_status(self.workspace, stream)

    def render_fields(self, fields, mesh, origins, dirs, lights, opts, per_ray_max_bounces=None, stream=None,
                      proposals=None):
        """Several fields in one scene (mr_render_fields), with one proposal
        per field for the proposal sampler; grows the workspace to the size
        the field count needs."""
        need = mr_render_fields_workspace_size(self.n, len(fields))
        if need > self.ws_bytes:
            import torch
            self.workspace = torch.empty(need, dtype=torch.uint8, device=self.workspace.device)
            self.ws_bytes = need
        mr_render_fields([f.handle for f in fields], mesh.handle if mesh is not None else None, self.n,
                         origins, dirs, self.max_bounces, per_ray_max_bounces, lights, opts, self.out,
                         self.workspace, self.ws_bytes, stream,
                         proposals=[p.handle for p in proposals] if proposals is not None else None)
        return self


def camera_rays(cams, device="cuda"):
    """Pinhole rays of packed camera records (float32 [n, 12])."""
    import torch
    cams = np.ascontiguousarray(cams, dtype=np.float32).reshape(-1, 12)
    n = int(sum(int(c[10]) * int(c[11]) for c in cams))
    o = torch.empty(n, 3, dtype=torch.float32, device=device)
    d = torch.empty(n, 3, dtype=torch.float32, device=device)
    ci = torch.empty(n, dtype=torch.int32, device=device)
    mr_rays_from_cameras(cams, o, d, ci, n)
    return o, d, ci


def mr_profile_enable(on=True):
    _check(lib().mr_profile_enable(C.c_int32(1 if on else 0)))


def mr_profile_read():
    ms = (C.c_double * 4)()
    n = (C.c_int64 * 4)()
    _check(lib().mr_profile_read(ms, n))
    return list(ms), list(n)


def mr_probe_gather(field, n_loads, seed, sink, stream=None):
    """Random-gather ceiling of the field's table: returns (ms, loads issued)."""
    ms = C.c_float()
    loads = C.c_int64()
    _check(lib().mr_probe_gather(field, C.c_int64(n_loads), C.c_uint32(seed), _ptr(sink), C.byref(ms),
                                 C.byref(loads), _stream(stream)))
    return ms.value, loads.value


def mr_probe_gather_region(field, log2_region, per_die, n_loads, seed, sink, stream=None):
    """The random-gather probe confined to 2^log2_region entries, shared by
    every block or one region per die: returns (ms, loads issued)."""
    ms = C.c_float()
    loads = C.c_int64()
    _check(lib().mr_probe_gather_region(field, C.c_int32(log2_region), C.c_int32(1 if per_die else 0),
                                        C.c_int64(n_loads), C.c_uint32(seed), _ptr(sink), C.byref(ms),
                                        C.byref(loads), _stream(stream)))
    return ms.value, loads.value


def mr_proposal_targets(fine, n, origins, dirs, t_near, t_far, n_samples, n_bins, lohi, targets, stream=None):
    _check(lib().mr_proposal_targets(fine, C.c_int64(n), _ptr(origins), _ptr(dirs), C.c_float(t_near),
                                     C.c_float(t_far), C.c_int32(n_samples), C.c_int32(n_bins),
                                     _ptr(lohi), _ptr(targets), _stream(stream)))


def mr_proposal_grad(prop, n, origins, dirs, lohi, targets, n_bins, loss, g_table, g_mlp, stream=None):
    _check(lib().mr_proposal_grad(prop, C.c_int64(n), _ptr(origins), _ptr(dirs), _ptr(lohi),
                                  _ptr(targets), C.c_int32(n_bins), _ptr(loss), _ptr(g_table),
                                  _ptr(g_mlp), _stream(stream)))


def mr_proposal_train_step(prop, n, origins, dirs, lohi, targets, n_bins, adam, loss, stream=None):
    _check(lib().mr_proposal_train_step(prop, C.c_int64(n), _ptr(origins), _ptr(dirs), _ptr(lohi),
                                        _ptr(targets), C.c_int32(n_bins), C.byref(adam), _ptr(loss),
                                        _stream(stream)))


class ProposalTrainer:
    """Targets and Adam steps for a proposal field (bookkeeping only: the
    targets, loss, gradients and updates are computed by the library)."""

    def __init__(self, proposal: "Field", n_bins=32, lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-15):
        import torch
        self.prop = proposal
        self.n_bins = n_bins
        self.adam = Adam()
        self.adam.lr, self.adam.beta1, self.adam.beta2, self.adam.eps = lr, beta1, beta2, eps
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")

    def targets(self, fine: "Field", origins, dirs, t_near, t_far, n_samples):
        import torch
        n = origins.shape[0]
        lohi = torch.empty(n, 2, dtype=torch.float32, device="cuda")
        tgt = torch.empty(n, self.n_bins, dtype=torch.float32, device="cuda")
        mr_proposal_targets(fine.handle, n, origins, dirs, t_near, t_far, n_samples, self.n_bins, lohi, tgt)
        return lohi, tgt

    def step(self, origins, dirs, lohi, targets):
        mr_proposal_train_step(self.prop.handle, origins.shape[0], origins, dirs, lohi, targets,
                               self.n_bins, self.adam, self.loss)
        return self.loss

    def train(self, origins, dirs, lohi, targets, steps, batch):
        """Cycle through consecutive slices of a training set (rows already in
        random order); returns the per-step loss history (device tensor)."""
        import torch
        n = origins.shape[0]
        hist = torch.empty(steps, dtype=torch.float32, device="cuda")
        nb = max(1, n // batch)
        for s in range(steps):
            b = (s % nb) * batch
            e = min(n, b + batch)
            self.step(origins[b:e], dirs[b:e], lohi[b:e], targets[b:e])
            hist[s:s + 1].copy_(self.loss)
        return hist


def _lights_arr(lights):
    nl = len(lights)
    arr = (Light * max(nl, 1))()
    for i, row in enumerate(lights):
        arr[i].pos = (C.c_float * 3)(*[float(x) for x in row[:3]])
        arr[i].intensity = (C.c_float * 3)(*[float(x) for x in row[3:6]])
    return arr, nl


def mr_render_graph_create(field, mesh, n, origins, dirs, max_bounces, per_ray_max_bounces, lights, opts, out,
                           workspace, workspace_bytes):
    arr, nl = _lights_arr(lights)
    g = C.c_void_p()
    _check(lib().mr_render_graph_create(field, mesh, C.c_int64(n), _ptr(origins), _ptr(dirs),
                                        C.c_int32(max_bounces), _ptr(per_ray_max_bounces), arr,
                                        C.c_int32(nl), C.byref(opts), C.byref(out), _ptr(workspace),
                                        C.c_size_t(workspace_bytes), C.byref(g)))
    return g


def mr_graph_launch(graph, stream=None):
    _check(lib().mr_graph_launch(graph, _stream(stream)))


def mr_graph_destroy(graph):
    _check(lib().mr_graph_destroy(graph))


def mr_autotune_render(field, mesh, n, origins, dirs, max_bounces, per_ray_max_bounces, lights, opts, out,
                       workspace, workspace_bytes, candidates, reps=2, stream=None):
    """candidates: sequence of (march_blocks_per_cu, stage_blocks_per_cu, stage_tile, march_chunk,
    march_batch, march_packets)."""
    arr, nl = _lights_arr(lights)
    cands = (LaunchCfg * len(candidates))()
    for i, c in enumerate(candidates):
        (cands[i].march_blocks_per_cu, cands[i].stage_blocks_per_cu, cands[i].stage_tile,
         cands[i].march_chunk, cands[i].march_batch, cands[i].march_packets) = c
    best = C.c_int32()
    ms = C.c_float()
    _check(lib().mr_autotune_render(field, mesh, C.c_int64(n), _ptr(origins), _ptr(dirs), C.c_int32(max_bounces),
                                    _ptr(per_ray_max_bounces), arr, C.c_int32(nl), C.byref(opts), C.byref(out),
                                    _ptr(workspace), C.c_size_t(workspace_bytes), cands, C.c_int32(len(cands)),
                                    C.c_int32(reps), C.byref(best), C.byref(ms), _stream(stream)))
    return tuple(candidates[best.value]), ms.value


def mr_autotune_candidates(n):
    """The library's candidate values per launch axis for a queue of n rays:
    a list of six lists in mr_launch_cfg order."""
    counts = (C.c_int32 * 6)()
    values = (C.c_int32 * 36)()
    _check(lib().mr_autotune_candidates(C.c_int64(n), counts, values))
    return [[values[6 * k + i] for i in range(counts[k])] for k in range(6)]


def mr_autotune_search(field, mesh, n, origins, dirs, max_bounces, per_ray_max_bounces, lights, opts, out,
                       workspace, workspace_bytes, reps=1, passes=2, stream=None):
    """Coordinate-descent launch-shape search in the library; returns
    (best shape as a 6-tuple, its ms, the starting shape's ms, shapes timed)."""
    arr, nl = _lights_arr(lights)
    best = LaunchCfg()
    ms, ms0, nt = C.c_float(), C.c_float(), C.c_int32()
    _check(lib().mr_autotune_search(field, mesh, C.c_int64(n), _ptr(origins), _ptr(dirs), C.c_int32(max_bounces),
                                    _ptr(per_ray_max_bounces), arr, C.c_int32(nl), C.byref(opts), C.byref(out),
                                    _ptr(workspace), C.c_size_t(workspace_bytes), C.c_int32(reps), C.c_int32(passes),
                                    C.byref(best), C.byref(ms), C.byref(ms0), C.byref(nt), _stream(stream)))
    shape = (best.march_blocks_per_cu, best.stage_blocks_per_cu, best.stage_tile, best.march_chunk,
             best.march_batch, best.march_packets)
    return shape, ms.value, ms0.value, nt.value


def apply_launch(opts, shape):
    """Set the six launch fields of a RenderOpts from a shape tuple."""
    (opts.march_blocks_per_cu, opts.stage_blocks_per_cu, opts.stage_tile, opts.march_chunk, opts.march_batch,
     opts.march_packets) = shape
    return opts


def mr_camera_bounce_limits(cam_index, n, cam_limits, out, stream=None):
    lim = np.ascontiguousarray(cam_limits, dtype=np.int32)
    _check(lib().mr_camera_bounce_limits(_ptr(cam_index), C.c_int64(n), _ptr(lim), C.c_int32(len(lim)),
                                         _ptr(out), _stream(stream)))


def autotune_key(*parts):
    """Cache key of a launch shape: the device architecture and a hash of the
    workload's description (any reprs or byte strings)."""
    import hashlib
    import torch
    h = hashlib.sha256()
    for p in parts:
        h.update(p if isinstance(p, bytes) else repr(p).encode())
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    return f"{arch}/{h.hexdigest()[:16]}"


def autotune_cached(cache_path, key, tune):
    """Launch shape from a JSON cache keyed by (arch, workload); on a miss
    `tune()` runs the autotuner and returns (shape, ms); the result is stored.
    Returns (shape, ms, hit)."""
    import json
    cache = {}
    if os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
    if key in cache:
        return tuple(cache[key]["best"]), cache[key]["ms"], True
    best, ms = tune()
    cache[key] = {"best": list(best), "ms": ms}
    with open(cache_path, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    return best, ms, False
