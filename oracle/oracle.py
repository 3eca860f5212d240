"""ctypes front end of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg call this; the product path never does.  It takes plain
numpy arrays and scene objects by attribute, and imports nothing from the
HIP package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with the host C compiler (plain -O2, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, SRC,
                               "-lm", "-lpthread"])
        os.replace(tmp, LIB)
    return LIB


class _Field(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("feats", C.c_int32), ("log2_table", C.c_int32),
                ("res", C.c_void_p), ("table", C.c_void_p),
                ("d_in", C.c_int32), ("d_hidden", C.c_int32), ("d_out", C.c_int32),
                ("c_in", C.c_int32), ("c_hidden", C.c_int32), ("c_layers", C.c_int32),
                ("sh", C.c_int32), ("mlp", C.c_void_p), ("density_offset", C.c_double),
                ("aabb_min", C.c_double * 3), ("aabb_max", C.c_double * 3),
                ("has_pose", C.c_int32), ("pose", C.c_double * 12)]


class _Mesh(C.Structure):
    _fields_ = [("nv", C.c_int32), ("nf", C.c_int32), ("vertices", C.c_void_p),
                ("indices", C.c_void_p), ("mat_ids", C.c_void_p), ("n_mat", C.c_int32),
                ("materials", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("t_near", C.c_double), ("t_far", C.c_double), ("n_samples", C.c_int32),
                ("max_bounces", C.c_int32), ("rr_after", C.c_int32),
                ("t_min_throughput", C.c_double), ("seed", C.c_uint32),
                ("tie_eps", C.c_double), ("tie_rel", C.c_double),
                ("occ_res", C.c_int32), ("occ", C.c_void_p),
                ("proposal", C.c_void_p), ("n_prop", C.c_int32), ("n_fine", C.c_int32),
                ("sample_shadows", C.c_int32), ("shadow_mask", C.c_double),
                ("sample_emitters", C.c_int32), ("n_fields", C.c_int32), ("fields", C.c_void_p),
                ("field_occ", C.c_void_p), ("field_occ_res", C.c_void_p),
                ("field_proposals", C.c_void_p), ("force_hits", C.c_void_p), ("flip", C.c_void_p),
                ("light_depth_samples", C.c_int32)]


class _Out(C.Structure):
    _fields_ = [("radiance", C.c_void_p), ("throughput", C.c_void_p), ("bounces", C.c_void_p),
                ("hit_ids", C.c_void_p), ("tie", C.c_void_p), ("samples", C.c_void_p),
                ("segments", C.c_void_p), ("invalid", C.c_void_p), ("n_flagged", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = C.CDLL(LIB)
        _lib.orc_proposal_loss.restype = C.c_double
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def n_threads_default():
    return max(1, min(64, len(os.sched_getaffinity(0))))


class OField:
    """Keeps the numpy buffers of a field alive next to its C struct."""

    def __init__(self, f):
        self.res = np.ascontiguousarray(f.resolutions, dtype=np.int32)
        self.table = np.ascontiguousarray(f.table, dtype=np.float32)
        self.mlp = np.ascontiguousarray(f.mlp, dtype=np.float32)
        s = _Field()
        s.n_levels, s.feats = int(f.n_levels), int(f.feats)
        s.log2_table = int(f.log2_table)
        s.res, s.table, s.mlp = _p(self.res), _p(self.table), _p(self.mlp)
        if hasattr(f, "d_hidden"):
            s.d_in, s.d_hidden, s.d_out = int(f.d_in), int(f.d_hidden), int(f.d_out)
            s.c_in, s.c_hidden, s.c_layers, s.sh = (int(f.c_in), int(f.c_hidden),
                                                    int(f.c_layers), int(f.sh))
        else:                                  # density-only proposal field
            s.d_in, s.d_hidden, s.d_out = int(f.n_levels * f.feats), int(f.hidden), 1
            s.c_in = s.c_hidden = s.c_layers = s.sh = 0
        s.density_offset = float(f.density_offset)
        s.aabb_min = (C.c_double * 3)(*f.aabb_min)
        s.aabb_max = (C.c_double * 3)(*f.aabb_max)
        pose = getattr(f, "pose", None)
        s.has_pose = int(pose is not None)
        if pose is not None:
            s.pose = (C.c_double * 12)(*np.asarray(pose, dtype=np.float64).reshape(12))
        self.s = s

    @property
    def ptr(self):
        return C.byref(self.s)


class OMesh:
    def __init__(self, m):
        self.v = np.ascontiguousarray(m.vertices, dtype=np.float32)
        self.f = np.ascontiguousarray(m.indices, dtype=np.int32)
        self.mat = np.ascontiguousarray(m.mat_ids, dtype=np.int32)
        self.mats = np.ascontiguousarray(m.materials, dtype=np.float32)
        s = _Mesh()
        s.nv, s.nf = len(self.v), len(self.f)
        s.vertices, s.indices, s.mat_ids = _p(self.v), _p(self.f), _p(self.mat)
        s.n_mat, s.materials = len(self.mats), _p(self.mats)
        self.s = s

    @property
    def ptr(self):
        return C.byref(self.s)


# ---------------------------------------------------------------------------
# building blocks
# ---------------------------------------------------------------------------

def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def hash_index(res, log2_table, v):
    vv = (C.c_int64 * 3)(*[int(x) for x in v])
    idx = C.c_uint32()
    dense = lib().orc_hash_index(C.c_int32(res), C.c_int32(log2_table), vv, C.byref(idx))
    return int(idx.value), bool(dense)


def sh(n, d):
    d = np.asarray(d, dtype=np.float64)
    o = np.zeros(16, dtype=np.float64)
    lib().orc_sh(C.c_int32(n), d.ctypes.data_as(C.c_void_p), _p(o))
    return o[:n]


def intersect(o, d, v0, v1, v2):
    arr = [np.ascontiguousarray(x, dtype=np.float64) for x in (o, d, v0, v1, v2)]
    t = C.c_double()
    bary = np.zeros(3)
    hit = lib().orc_intersect(*[_p(a) for a in arr], C.byref(t), _p(bary))
    return bool(hit), float(t.value), bary


def closest_hit(mesh, o, d, t_max=np.inf, tie_eps=1e-5):
    om = OMesh(mesh)
    o = np.ascontiguousarray(o, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    t = C.c_double()
    bary = np.zeros(3)
    tie = C.c_int()
    hid = lib().orc_closest_hit(om.ptr, _p(o), _p(d), C.c_double(t_max), C.c_double(tie_eps),
                                C.byref(t), _p(bary), C.byref(tie))
    return int(hid), float(t.value), bary, bool(tie.value)


def rays_from_camera(cam_row):
    """FP64 pinhole rays of one packed camera record (float32[12])."""
    cam = np.ascontiguousarray(cam_row, dtype=np.float32)
    W, H = int(cam[10]), int(cam[11])
    o = np.zeros((W * H, 3))
    d = np.zeros((W * H, 3))
    lib().orc_rays_from_camera(_p(cam), _p(o), _p(d))
    return o, d


def field_batch(field, x, d=None, n_threads=None):
    of = OField(field)
    x = np.ascontiguousarray(x, dtype=np.float32)
    n = len(x)
    d = None if d is None else np.ascontiguousarray(d, dtype=np.float32)
    sigma = np.zeros(n)
    has_rgb = getattr(field, "c_layers", 0) > 0 and d is not None
    rgb = np.zeros((n, 3)) if has_rgb else None
    feat = np.zeros((n, field.n_levels * field.feats))
    d_out = getattr(field, "d_out", 1)
    raw = np.zeros((n, d_out))
    lib().orc_field_batch(of.ptr, C.c_int64(n), _p(x), _p(d), _p(sigma), _p(rgb), _p(feat),
                          _p(raw), C.c_int32(n_threads or n_threads_default()))
    return dict(sigma=sigma, rgb=rgb, feat=feat, raw=raw)


def occupancy(field, res, thresh, n_threads=None):
    of = OField(field)
    bits = np.zeros(res ** 3, dtype=np.uint8)
    margin = np.zeros(res ** 3)
    lib().orc_build_occupancy(of.ptr, C.c_int32(res), C.c_double(thresh), _p(bits), _p(margin),
                              C.c_int32(n_threads or n_threads_default()))
    return bits, margin


def render(scene, origins, dirs, ray_ids=None, max_bounces=None, n_threads=None,
           tie_eps=1e-5, tie_rel=1e-4, occupancy_bits=None, proposal=None, n_prop=32,
           n_fine=32, field=..., mesh=..., shadow_mask=None, sample_emitters=False, fields=None,
           field_occupancy=None, field_proposals=None, force_hits=None, flip=None, light_depth_samples=0,
           _gmax=None):
    """Render FP32 input rays through the whole path in FP64.

    shadow_mask: None = no per-sample shadows; else every field sample that a
    mesh hides from a light has its emitted radiance multiplied by this value
    once per such light (Sec. 3.1 "Shadow rays").
    sample_emitters: light sampling toward emitting triangles at diffuse hits
    (Eq. 12's L_e as area lights); light_depth_samples: grid intervals per
    segment length for the optical depth along the light samples' shadow
    segments (0 = n_samples).
    fields: several fields marched together (the scene's own field is then
    not used); field_occupancy: per field an occupancy bit array or None;
    field_proposals: per field its proposal (the proposal sampler with
    several fields, boxes disjoint; n_prop and n_fine apply to each).

    force_hits, flip: outcomes of tie rays (see orc_opts): per ray and
    segment a triangle to take instead of the closest hit when single
    precision can reach it, and per ray a bit mask over its flagged scalar
    decisions whose other branch to take.

    Returns a dict with radiance, throughput, bounces, hit_ids (segments),
    tie flags, per-ray sample and segment counts, invalid (a forced hit was
    not reachable) and n_flagged (flagged scalar decisions on the path), and
    rerun(idx, force_hits, flip): the same render of the rays idx with those
    options.
    """
    call = dict(tie_eps=tie_eps, tie_rel=tie_rel, occupancy_bits=occupancy_bits, proposal=proposal,
                n_prop=n_prop, n_fine=n_fine, field=field, mesh=mesh, shadow_mask=shadow_mask,
                sample_emitters=sample_emitters, light_depth_samples=light_depth_samples, fields=fields,
                field_occupancy=field_occupancy,
                field_proposals=field_proposals, n_threads=n_threads)
    field = scene.field if field is ... else field
    mesh = scene.mesh if mesh is ... else mesh
    origins = np.ascontiguousarray(origins, dtype=np.float32)
    dirs = np.ascontiguousarray(dirs, dtype=np.float32)
    n = len(origins)
    of = OField(field) if field is not None else None
    om = OMesh(mesh) if mesh is not None else None
    op = OField(proposal) if proposal is not None else None
    lights = np.ascontiguousarray(scene.lights, dtype=np.float32).reshape(-1, 6)
    ids = None if ray_ids is None else np.ascontiguousarray(ray_ids, dtype=np.int64)
    mbs = None if max_bounces is None else np.ascontiguousarray(max_bounces, dtype=np.int32)
    gmax = int(scene.max_bounces if mbs is None else max(scene.max_bounces, int(mbs.max(initial=0))))
    if _gmax is not None:
        gmax = int(_gmax)
    opt = _Opts()
    opt.t_near, opt.t_far = float(scene.t_near), float(scene.t_far)
    opt.n_samples, opt.max_bounces = int(scene.n_samples), gmax
    opt.rr_after = int(scene.rr_after)
    opt.t_min_throughput = float(scene.t_min_throughput)
    opt.seed = int(scene.seed) & 0xFFFFFFFF
    opt.tie_eps, opt.tie_rel = float(tie_eps), float(tie_rel)
    occ = None
    if occupancy_bits is not None:
        occ = np.ascontiguousarray(occupancy_bits, dtype=np.uint8)
        opt.occ_res = int(round(len(occ) ** (1 / 3)))
        opt.occ = _p(occ)
    if op is not None:
        opt.proposal = C.cast(C.pointer(op.s), C.c_void_p)
        opt.n_prop, opt.n_fine = int(n_prop), int(n_fine)
    if shadow_mask is not None:
        opt.sample_shadows, opt.shadow_mask = 1, float(shadow_mask)
    opt.sample_emitters = 1 if sample_emitters else 0
    opt.light_depth_samples = int(light_depth_samples)
    keep = []
    if fields is not None:
        if proposal is not None:
            raise ValueError("with several fields give field_proposals, one per field")
        ofs = [OField(f) for f in fields]
        ptrs = (C.c_void_p * len(ofs))(*[C.cast(C.pointer(x.s), C.c_void_p) for x in ofs])
        occs = (C.c_void_p * len(ofs))()
        ress = (C.c_int32 * len(ofs))()
        for k, bits in enumerate(field_occupancy or [None] * len(ofs)):
            if bits is not None:
                bits = np.ascontiguousarray(bits, dtype=np.uint8)
                keep.append(bits)
                occs[k] = bits.ctypes.data
                ress[k] = int(round(len(bits) ** (1 / 3)))
        keep += [ofs, ptrs, occs, ress]
        opt.n_fields = len(ofs)
        opt.fields = C.cast(ptrs, C.c_void_p)
        opt.field_occ = C.cast(occs, C.c_void_p)
        opt.field_occ_res = C.cast(ress, C.c_void_p)
        if field_proposals is not None:
            if len(field_proposals) != len(ofs):
                raise ValueError("one proposal per field")
            ops = [OField(pp) for pp in field_proposals]
            pptrs = (C.c_void_p * len(ops))(*[C.cast(C.pointer(x.s), C.c_void_p) for x in ops])
            keep += [ops, pptrs]
            opt.field_proposals = C.cast(pptrs, C.c_void_p)
            opt.n_prop, opt.n_fine = int(n_prop), int(n_fine)
        if of is None and ofs:
            of = ofs[0]
    if force_hits is not None:
        force_hits = np.ascontiguousarray(force_hits, dtype=np.int32)
        if force_hits.shape != (n, gmax + 1):
            raise ValueError(f"force_hits must be ({n}, {gmax + 1})")
        opt.force_hits = _p(force_hits)
    if flip is not None:
        flip = np.ascontiguousarray(flip, dtype=np.uint32)
        opt.flip = _p(flip)
    res = dict(radiance=np.zeros((n, 3)), throughput=np.zeros((n, 3)),
               bounces=np.zeros(n, dtype=np.int32),
               hit_ids=np.full((n, gmax + 1), -1, dtype=np.int32),
               tie=np.zeros(n, dtype=np.uint8), samples=np.zeros(n, dtype=np.int64),
               segments=np.zeros(n, dtype=np.int32), invalid=np.zeros(n, dtype=np.uint8),
               n_flagged=np.zeros(n, dtype=np.int32))
    out = _Out()
    for k in ("radiance", "throughput", "bounces", "hit_ids", "tie", "samples", "segments", "invalid",
              "n_flagged"):
        setattr(out, k, _p(res[k]))
    lib().orc_render(of.ptr if of else None, om.ptr if om else None, C.c_int64(n), _p(origins),
                     _p(dirs), _p(ids), _p(mbs), _p(lights), C.c_int32(len(lights)),
                     C.byref(opt), C.byref(out), C.c_int32(n_threads or n_threads_default()))
    res["tie"] = res["tie"].astype(bool)
    res["invalid"] = res["invalid"].astype(bool)

    def rerun(idx, force_hits=None, flip=None):
        idx = np.asarray(idx, dtype=np.int64)
        rid = idx if ids is None else ids[idx]
        return render(scene, origins[idx], dirs[idx], ray_ids=rid,
                      max_bounces=None if mbs is None else mbs[idx], force_hits=force_hits, flip=flip,
                      _gmax=gmax, **call)

    res["rerun"] = rerun
    return res


def proposal_weights(prop, o, d, lo, hi, n):
    op = OField(prop)
    o = np.ascontiguousarray(o, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    w = np.zeros(n)
    lib().orc_proposal_weights(op.ptr, _p(o), _p(d), C.c_double(lo), C.c_double(hi),
                               C.c_int32(n), _p(w))
    return w


def proposal_edges(w, n_fine, lo, hi):
    """Fine-interval edges (n_fine + 1) that the proposal sampler places on
    [lo, hi] for the proposal weights w (one per uniform interval)."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    e = np.zeros(n_fine + 1)
    lib().orc_proposal_edges(_p(w), C.c_int32(len(w)), C.c_int32(n_fine), C.c_double(lo),
                             C.c_double(hi), _p(e))
    return e


def proposal_loss(prop, o, d, lohi, target, grads=True, n_threads=None):
    """Mean proposal loss over segments and, optionally, its exact FP64
    gradient w.r.t. the table [L, T, F] and the flat MLP weights."""
    op = OField(prop)
    o = np.ascontiguousarray(o, dtype=np.float32)
    d = np.ascontiguousarray(d, dtype=np.float32)
    lohi = np.ascontiguousarray(lohi, dtype=np.float32)
    target = np.ascontiguousarray(target, dtype=np.float32)
    n_seg, n_bins = target.shape
    gt = np.zeros(prop.table.shape) if grads else None
    gm = np.zeros(prop.mlp.shape) if grads else None
    loss = lib().orc_proposal_loss(op.ptr, C.c_int64(n_seg), _p(o), _p(d), _p(lohi), _p(target),
                                   C.c_int32(n_bins), _p(gt), _p(gm),
                                   C.c_int32(n_threads or n_threads_default()))
    return float(loss), gt, gm


def proposal_grad_bound(prop, o, d, lohi, target, u=2.0 ** -24, K=64.0, lam=8.0):
    """Per-element tolerance on the rounding error of the proposal gradient
    computed in a format of unit roundoff u (FP32 by default), from a
    probabilistic rounding error analysis (Higham and Mary, 2019): the final
    sum over contributions, a running error bound of each contribution's
    chain (K roundings per node), the rounding of the sample positions
    carried into the trilinear weights, and the contributions that hinge on a
    ReLU whose sign is within rounding.  An element exceeds it with
    probability about 2 n exp(-lam^2 / 2) (n: its contributions).
    Returns (bound_table [L, T, F], bound_mlp)."""
    op = OField(prop)
    o = np.ascontiguousarray(o, dtype=np.float32)
    d = np.ascontiguousarray(d, dtype=np.float32)
    lohi = np.ascontiguousarray(lohi, dtype=np.float32)
    target = np.ascontiguousarray(target, dtype=np.float32)
    n_seg, n_bins = target.shape
    bt = np.zeros(prop.table.shape)
    bm = np.zeros(prop.mlp.shape)
    lib().orc_proposal_grad_bound(op.ptr, C.c_int64(n_seg), _p(o), _p(d), _p(lohi), _p(target),
                                  C.c_int32(n_bins), C.c_double(u), C.c_double(K), C.c_double(lam),
                                  _p(bt), _p(bm))
    return bt, bm


def scatter(mat, d, n, u):
    """One BSDF sample: returns (new direction, offset side, weight rgb, R)."""
    mat = np.ascontiguousarray(mat, dtype=np.float32)
    d = np.ascontiguousarray(d, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    nd, side, w = np.zeros(3), np.zeros(3), np.zeros(3)
    R = C.c_double(-1.0)
    lib().orc_scatter(_p(mat), _p(d), _p(n), _p(u), _p(nd), _p(side), _p(w), C.byref(R))
    return nd, side, w, float(R.value)


def fresnel(cos_i, eta_i, eta_t):
    f = lib().orc_fresnel
    f.restype = C.c_double
    return float(f(C.c_double(cos_i), C.c_double(eta_i), C.c_double(eta_t)))


def proposal_targets(field, o, d, t_near, t_far, n_samples, n_bins):
    """Plain-marcher weight histograms of the camera segment (training targets)."""
    of = OField(field)
    o = np.ascontiguousarray(o, dtype=np.float32)
    d = np.ascontiguousarray(d, dtype=np.float32)
    n = len(o)
    lohi = np.zeros((n, 2))
    tgt = np.zeros((n, n_bins))
    lib().orc_proposal_targets(of.ptr, C.c_int64(n), _p(o), _p(d), C.c_double(t_near),
                               C.c_double(t_far), C.c_int32(n_samples), C.c_int32(n_bins),
                               _p(lohi), _p(tgt))
    return lohi, tgt
