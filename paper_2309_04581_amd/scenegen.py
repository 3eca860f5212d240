"""Seeded synthetic scenes for the hybrid mesh + radiance-field marcher.

This module only *draws inputs*: random hash tables and MLP weights, triangle
meshes, cameras, point lights and render settings, all as plain numpy arrays.
It performs none of the rendering arithmetic (no hashing, no field evaluation,
no ray generation, no intersection, no shading), so that both the FP64 CPU
oracle and the HIP path can consume the very same data without sharing code.

The paper renders a pretrained Instant-NGP radiance field with inserted
meshes (Sec. 3.1 "Hybrid Rendering Algorithm", Algorithm 1; Sec. 3.3).  Its
captured scenes and trained weights are not available, so every workload here
is a seeded stand-in with the sizes of the published configuration it mimics:

* ``tiny``   64x64 camera, 8-level hash grid (2^14 entries, 2 features),
             32->64->16 density MLP, (16 + 4 SH) -> 64 -> 3 colour MLP,
             a 12-triangle mirror cube, 64 samples per ray, 4 bounces.
* ``mid``    800x800 camera, 16-level hash grid (2^19 entries), SH degree 4,
             two hidden colour layers, glass icosphere (20 480 triangles),
             mirror cube, diffuse floor, one point light, 256 samples, 8 bounces.
* ``multicam`` 16 cameras of uneven size on the tiny field and cube, four of
             them inside the mirror cube, up to 16 bounces, Russian roulette.
* ``cloth``  a 64x64-vertex diffuse cloth with a seeded sinusoidal motion.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# Material kinds (shared enumeration with the C ABI).
MIRROR, GLASS, DIFFUSE = 0, 1, 2

DEFAULT_PHILOX_SEED = 230904581


def level_resolutions(n_min: int, n_max: int, n_levels: int) -> np.ndarray:
    """Integer per-level grid resolutions of a geometric series n_min..n_max.

    Computed once here in FP64 and handed to both implementations as
    integers, so that neither has to take a floor of a rounded power.
    """
    if n_levels == 1:
        return np.array([n_min], dtype=np.int32)
    b = math.exp((math.log(n_max) - math.log(n_min)) / (n_levels - 1))
    return np.array([int(math.floor(n_min * b ** l + 1e-6)) for l in range(n_levels)],
                    dtype=np.int32)


@dataclasses.dataclass
class Field:
    """Hash grid + density MLP + colour MLP, all FP32, plus their shape."""
    n_levels: int
    feats: int
    log2_table: int
    resolutions: np.ndarray          # int32 [L]
    table: np.ndarray                # float32 [L, T, F]
    d_in: int                        # density MLP input width (features, zero padded)
    d_hidden: int
    d_out: int
    c_in: int                        # colour MLP input width (d_out + SH, zero padded)
    c_hidden: int
    c_layers: int                    # number of hidden colour layers (1 or 2)
    sh: int                          # number of SH components (4 or 16)
    mlp: np.ndarray                  # float32 flat, layers in forward order, [out][in]
    density_offset: float = 1.0
    aabb_min: tuple = (-1.0, -1.0, -1.0)
    aabb_max: tuple = (1.0, 1.0, 1.0)
    pose: object = None              # optional [R | c] 3x4 (field frame -> world), R a rotation

    @property
    def table_size(self) -> int:
        return 1 << self.log2_table

    def layer_shapes(self):
        """(out, in) of each layer in the flat ``mlp`` array, forward order."""
        shapes = [(self.d_hidden, self.d_in), (self.d_out, self.d_hidden),
                  (self.c_hidden, self.c_in)]
        for _ in range(self.c_layers - 1):
            shapes.append((self.c_hidden, self.c_hidden))
        shapes.append((3, self.c_hidden))
        return shapes


@dataclasses.dataclass
class Proposal:
    """Density-only proposal grid: hash grid + one hidden layer -> 1 output."""
    n_levels: int
    feats: int
    log2_table: int
    resolutions: np.ndarray
    table: np.ndarray                # float32 [L, T, F]
    hidden: int
    mlp: np.ndarray                  # float32 flat: [hidden][L*F], [1][hidden]
    density_offset: float = 0.0
    aabb_min: tuple = (-1.0, -1.0, -1.0)
    aabb_max: tuple = (1.0, 1.0, 1.0)


@dataclasses.dataclass
class Mesh:
    vertices: np.ndarray             # float32 [V, 3]
    indices: np.ndarray              # int32 [F, 3]
    mat_ids: np.ndarray              # int32 [F]
    materials: np.ndarray            # float32 [M, 8]: kind, ior, albedo rgb, emitted radiance rgb


@dataclasses.dataclass
class Camera:
    pos: tuple
    look_at: tuple
    fov_deg: float
    width: int
    height: int
    max_bounces: int = 4
    up: tuple = (0.0, 1.0, 0.0)


@dataclasses.dataclass
class Scene:
    name: str
    field: Optional[Field]
    mesh: Optional[Mesh]
    lights: np.ndarray               # float32 [n, 6]: pos xyz, intensity rgb
    cameras: List[Camera]
    t_near: float
    t_far: float
    n_samples: int
    max_bounces: int
    rr_after: int = -1
    t_min_throughput: float = 1e-4
    seed: int = DEFAULT_PHILOX_SEED
    occupancy_res: int = 0
    occupancy_thresh: float = 0.01

    @property
    def n_rays(self) -> int:
        return sum(c.width * c.height for c in self.cameras)


# ----------------------------------------------------------------------------
# field parameters
# ----------------------------------------------------------------------------

def _he_uniform(rng, out_dim, in_dim, fan_in):
    lim = math.sqrt(6.0 / fan_in)
    return rng.uniform(-lim, lim, size=(out_dim, in_dim)).astype(np.float32)


def make_field(*, n_levels, feats, log2_table, n_min, n_max, d_hidden, d_out,
               c_hidden, c_layers, sh, seed, table_amp=1e-4, density_offset=1.0,
               d_in=None, c_in=None) -> Field:
    """Draw a field: table U(-amp, amp) in flat [L][T][F] order, then
    He-uniform MLP weights in forward order, from one seeded generator."""
    rng = np.random.default_rng(seed)
    T = 1 << log2_table
    table = rng.uniform(-table_amp, table_amp, size=n_levels * T * feats)
    table = table.astype(np.float32).reshape(n_levels, T, feats)
    n_feat = n_levels * feats
    d_in = d_in or max(32, n_feat)
    c_real = d_out + sh
    c_in = c_in or max(32, c_real)
    layers = [_he_uniform(rng, d_hidden, d_in, d_in),
              _he_uniform(rng, d_out, d_hidden, d_hidden),
              _he_uniform(rng, c_hidden, c_in, c_real)]
    for _ in range(c_layers - 1):
        layers.append(_he_uniform(rng, c_hidden, c_hidden, c_hidden))
    layers.append(_he_uniform(rng, 3, c_hidden, c_hidden))
    mlp = np.concatenate([w.ravel() for w in layers]).astype(np.float32)
    return Field(n_levels=n_levels, feats=feats, log2_table=log2_table,
                 resolutions=level_resolutions(n_min, n_max, n_levels), table=table,
                 d_in=d_in, d_hidden=d_hidden, d_out=d_out, c_in=c_in,
                 c_hidden=c_hidden, c_layers=c_layers, sh=sh, mlp=mlp,
                 density_offset=density_offset)


def tiny_field(seed=1, table_amp=1e-4, density_offset=1.0) -> Field:
    """8 levels x 2 features, 2^14 entries, resolutions 16..256;
    density 32 -> 64 -> 16, colour (16 + 4 SH) -> 64 -> 3."""
    return make_field(n_levels=8, feats=2, log2_table=14, n_min=16, n_max=256,
                      d_hidden=64, d_out=16, c_hidden=64, c_layers=1, sh=4, seed=seed,
                      table_amp=table_amp, density_offset=density_offset)


def mid_field(seed=2, table_amp=1e-4, density_offset=1.0) -> Field:
    """16 levels x 2 features, 2^19 entries, resolutions 16..2048;
    density 32 -> 64 -> 16, colour (16 + 16 SH) -> 64 -> 64 -> 3."""
    return make_field(n_levels=16, feats=2, log2_table=19, n_min=16, n_max=2048,
                      d_hidden=64, d_out=16, c_hidden=64, c_layers=2, sh=16, seed=seed,
                      table_amp=table_amp, density_offset=density_offset)


def shell_field(seed=3, radius=0.5, width=0.08, gain=30.0, density_offset=-4.0) -> Field:
    """The tiny field layout with a thin spherical shell of density: the
    coarsest (dense) level stores exp(-((|p| - radius)/width)^2) at each grid
    vertex, the density MLP routes that feature to its first output with gain
    `gain`, and the other weights and levels are small seeded noise.  Far from
    the shell sigma = softplus(offset); on it sigma is about softplus(gain +
    offset).  A concentrated density for proposal-sampler experiments."""
    f = tiny_field(seed=seed, table_amp=1e-3, density_offset=density_offset)
    rng = np.random.default_rng(seed + 1000)
    N = int(f.resolutions[0])
    g = np.linspace(-1.0, 1.0, N + 1)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    vals = np.exp(-((r - radius) / width) ** 2).ravel()
    f.table[0, :vals.size, 0] = vals.astype(np.float32)
    f.table[0, :vals.size, 1] = 0.0
    W1 = f.mlp[:f.d_hidden * f.d_in].reshape(f.d_hidden, f.d_in)
    W1[:] = rng.uniform(-0.01, 0.01, size=W1.shape)
    W1[0, 0] = 1.0
    off = f.d_hidden * f.d_in
    W2 = f.mlp[off:off + f.d_out * f.d_hidden].reshape(f.d_out, f.d_hidden)
    W2[:] = rng.uniform(-0.01, 0.01, size=W2.shape)
    W2[0, 0] = gain
    return f


def make_proposal(seed=5, n_levels=5, feats=2, log2_table=17, n_min=16, n_max=256,
                  hidden=16, table_amp=1e-4, density_offset=0.0) -> Proposal:
    rng = np.random.default_rng(seed)
    T = 1 << log2_table
    table = rng.uniform(-table_amp, table_amp, size=n_levels * T * feats)
    table = table.astype(np.float32).reshape(n_levels, T, feats)
    n_in = n_levels * feats
    w1 = _he_uniform(rng, hidden, n_in, n_in)
    w2 = _he_uniform(rng, 1, hidden, hidden)
    return Proposal(n_levels=n_levels, feats=feats, log2_table=log2_table,
                    resolutions=level_resolutions(n_min, n_max, n_levels), table=table,
                    hidden=hidden, mlp=np.concatenate([w1.ravel(), w2.ravel()]),
                    density_offset=density_offset)


# ----------------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------------

def _materials(rows):
    """Material rows: kind, ior, albedo rgb, and optionally emitted radiance
    rgb (linear HDR; zero when left out)."""
    rows = [list(r) + [0.0] * (8 - len(r)) for r in rows]
    return np.array(rows, dtype=np.float32).reshape(-1, 8)


def cube_triangles(center, side):
    """Axis-aligned cube: 8 vertices, 12 triangles (two per face)."""
    c = np.asarray(center, dtype=np.float64)
    h = side / 2.0
    v = np.array([[x, y, z] for z in (-h, h) for y in (-h, h) for x in (-h, h)]) + c
    # vertex index = x_bit + 2*y_bit + 4*z_bit
    quads = [(0, 2, 3, 1), (4, 5, 7, 6),      # z-, z+
             (0, 1, 5, 4), (2, 6, 7, 3),      # y-, y+
             (0, 4, 6, 2), (1, 3, 7, 5)]      # x-, x+
    f = []
    for a, b, cc, d in quads:
        f.append((a, b, cc))
        f.append((a, cc, d))
    return v.astype(np.float32), np.array(f, dtype=np.int32)


def icosphere(level, radius=1.0, center=(0.0, 0.0, 0.0)):
    """Golden-ratio icosahedron, midpoint-subdivided ``level`` times and pushed
    to the sphere; faces wound counter-clockwise seen from outside."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    verts = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
             (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
             (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in verts]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    v = np.array(verts) * radius + np.asarray(center, dtype=np.float64)
    return v.astype(np.float32), np.array(faces, dtype=np.int32)


def floor_plane(y, half=1.0):
    v = np.array([[-half, y, -half], [half, y, -half], [half, y, half], [-half, y, half]],
                 dtype=np.float32)
    return v, np.array([[0, 2, 1], [0, 3, 2]], dtype=np.int32)


def merge_meshes(parts, materials):
    """parts: list of (vertices, indices, material index)."""
    vs, fs, ms, base = [], [], [], 0
    for v, f, m in parts:
        vs.append(v)
        fs.append(f + base)
        ms.append(np.full(len(f), m, dtype=np.int32))
        base += len(v)
    return Mesh(vertices=np.concatenate(vs).astype(np.float32),
                indices=np.concatenate(fs).astype(np.int32),
                mat_ids=np.concatenate(ms), materials=_materials(materials))


def mirror_cube_mesh(side=0.5, center=(0.0, 0.0, 0.0)) -> Mesh:
    v, f = cube_triangles(center, side)
    return merge_meshes([(v, f, 0)], [[MIRROR, 1.0, 1.0, 1.0, 1.0]])


def mid_mesh() -> Mesh:
    """Glass icosphere (level 5), mirror cube, diffuse floor; ids in that order."""
    sv, sf = icosphere(5, radius=0.35, center=(-0.4, -0.24, 0.0))
    cv, cf = cube_triangles((0.45, -0.35, 0.1), 0.5)
    pv, pf = floor_plane(-0.6)
    mats = [[GLASS, 1.5, 1.0, 1.0, 1.0], [MIRROR, 1.0, 1.0, 1.0, 1.0],
            [DIFFUSE, 1.0, 0.7, 0.7, 0.7]]
    return merge_meshes([(sv, sf, 0), (cv, cf, 1), (pv, pf, 2)], mats)


def cloth_params(seed=55):
    """Seeded wave parameters of the cloth motion (count, wave vectors,
    angular speeds, phases)."""
    rng = np.random.default_rng(seed)
    K = int(rng.integers(1, 4))
    ang = rng.uniform(0, 2 * math.pi, size=K)
    mag = rng.uniform(0.5, 3.0, size=K)
    k = np.stack([mag * np.cos(ang), mag * np.sin(ang)], axis=1)
    omega = rng.uniform(0.05, 0.3, size=K)
    phase = rng.uniform(0, 2 * math.pi, size=K)
    return K, k, omega, phase


def cloth_topology(n=64):
    """Row-major quads of an n x n vertex grid, each split by one fixed diagonal."""
    f = []
    for j in range(n - 1):
        for i in range(n - 1):
            a = j * n + i
            f.append((a, a + n, a + 1))
            f.append((a + 1, a + n, a + n + 1))
    return np.array(f, dtype=np.int32)


def cloth_vertices(frame, n=64, seed=55, amp=0.1, y0=-0.3, half=0.8):
    """Vertex positions of the cloth at ``frame`` (the simulated motion the
    renderer receives each frame; a prescribed sinusoid stands in for the
    position-based dynamics solver)."""
    K, k, omega, phase = cloth_params(seed)
    xs = np.linspace(-half, half, n)
    X, Z = np.meshgrid(xs, xs)                      # row j = z index, col i = x index
    dy = np.zeros_like(X)
    for q in range(K):
        dy += (amp / K) * np.sin(2 * math.pi * (k[q, 0] * X + k[q, 1] * Z)
                                 + omega[q] * frame + phase[q])
    v = np.stack([X, y0 + dy, Z], axis=-1).reshape(-1, 3)
    return v.astype(np.float32)


def cloth_mesh(frame=0, n=64, seed=55) -> Mesh:
    return merge_meshes([(cloth_vertices(frame, n, seed), cloth_topology(n), 0)],
                        [[DIFFUSE, 1.0, 0.7, 0.7, 0.7]])


def random_triangles(n, seed, scale=1.0) -> Mesh:
    """Random triangle soup inside [-scale, scale]^3 with random materials."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-0.8 * scale, 0.8 * scale, size=(n, 1, 3))
    v = (c + rng.uniform(-0.4 * scale, 0.4 * scale, size=(n, 3, 3))).reshape(-1, 3)
    f = np.arange(3 * n, dtype=np.int32).reshape(n, 3)
    mats = [[MIRROR, 1.0, 1.0, 1.0, 1.0], [GLASS, 1.5, 1.0, 1.0, 1.0],
            [DIFFUSE, 1.0, 0.7, 0.5, 0.3]]
    return Mesh(vertices=v.astype(np.float32), indices=f,
                mat_ids=rng.integers(0, 3, size=n).astype(np.int32),
                materials=_materials(mats))


# ----------------------------------------------------------------------------
# lights and cameras
# ----------------------------------------------------------------------------

def seeded_light(seed=22, intensity=10.0):
    rng = np.random.default_rng(seed)
    p = [rng.uniform(-0.8, 0.8), rng.uniform(0.6, 0.9), rng.uniform(-0.8, 0.8)]
    return np.array([p + [intensity] * 3], dtype=np.float32)


def no_lights():
    return np.zeros((0, 6), dtype=np.float32)


def front_camera(width, height, max_bounces, dist=2.5):
    return Camera(pos=(0.0, 0.0, -dist), look_at=(0.0, 0.0, 0.0), fov_deg=60.0,
                  width=width, height=height, max_bounces=max_bounces)


def multicam_cameras(seed=44, n=16):
    """16 cameras: sizes 256x256 .. 1920x1080 (first two fixed to the extremes),
    12 outside on a radius-2.5 sphere, 4 inside the mirror cube; per-camera
    bounce limits in [2, 16] with one inside camera at 16."""
    rng = np.random.default_rng(seed)
    cams = []
    for i in range(n):
        if i == 0:
            w, h = 256, 256
        elif i == 1:
            w, h = 1920, 1080
        else:
            w, h = int(rng.integers(256, 1921)), int(rng.integers(256, 1081))
        if i < 12:
            z = rng.uniform(-1, 1)
            phi = rng.uniform(0, 2 * math.pi)
            r = math.sqrt(max(0.0, 1 - z * z))
            # keep away from the poles so that "up" is never parallel to the view
            pos = (2.5 * r * math.cos(phi), 2.5 * 0.8 * z, 2.5 * r * math.sin(phi))
            look = (0.0, 0.0, 0.0)
        else:
            pos = tuple(rng.uniform(-0.2, 0.2, size=3))
            dvec = rng.normal(size=3)
            dvec[1] *= 0.3
            dvec /= np.linalg.norm(dvec)
            look = tuple(np.asarray(pos) + dvec)
        mb = int(rng.integers(2, 17))
        if i == 12:
            mb = 16
        cams.append(Camera(pos=tuple(float(x) for x in pos),
                           look_at=tuple(float(x) for x in look), fov_deg=60.0,
                           width=w, height=h, max_bounces=mb))
    return cams


def cameras_array(cams: List[Camera]) -> np.ndarray:
    """Packed camera records: float32 [n, 12] = pos(3), look_at(3), up(3),
    fov_deg, width, height."""
    a = np.zeros((len(cams), 12), dtype=np.float32)
    for i, c in enumerate(cams):
        a[i, 0:3] = c.pos
        a[i, 3:6] = c.look_at
        a[i, 6:9] = c.up
        a[i, 9] = c.fov_deg
        a[i, 10] = c.width
        a[i, 11] = c.height
    return a


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def tiny_scene(width=64, height=64, table_amp=1e-4, field_seed=1, with_field=True,
               with_mesh=True) -> Scene:
    return Scene(name="tiny",
                 field=tiny_field(field_seed, table_amp) if with_field else None,
                 mesh=mirror_cube_mesh() if with_mesh else None, lights=no_lights(),
                 cameras=[front_camera(width, height, 4)], t_near=0.05, t_far=4.0,
                 n_samples=64, max_bounces=4)


def mid_scene(width=800, height=800, table_amp=1e-4, n_samples=256,
              occupancy_res=128) -> Scene:
    return Scene(name="mid", field=mid_field(2, table_amp), mesh=mid_mesh(),
                 lights=seeded_light(22), cameras=[front_camera(width, height, 8)],
                 t_near=0.05, t_far=4.0, n_samples=n_samples, max_bounces=8,
                 occupancy_res=occupancy_res, occupancy_thresh=0.01)


def balls_mesh(n_balls, seed=66, radius=0.03, level=1):
    """n seeded icospheres (level 1: 80 triangles) of one radius with centres
    uniform in [-0.9, 0.9]^3, materials cycling glass, mirror, diffuse, over
    the mid scene's diffuse floor (ball i has triangle ids 80 i .. 80 i + 79,
    the floor comes last)."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-0.9, 0.9, size=(n_balls, 3))
    bv, bf = icosphere(level, radius=1.0)
    V = (bv[None].astype(np.float64) * radius + centres[:, None, :]).reshape(-1, 3)
    F = (bf[None] + (np.arange(n_balls) * len(bv))[:, None, None]).reshape(-1, 3)
    M = np.repeat(np.arange(n_balls) % 3, len(bf))
    pv, pf = floor_plane(-0.6)
    mats = [[GLASS, 1.5, 1.0, 1.0, 1.0], [MIRROR, 1.0, 1.0, 1.0, 1.0], [DIFFUSE, 1.0, 0.7, 0.7, 0.7]]
    return Mesh(vertices=np.concatenate([V, pv]).astype(np.float32),
                indices=np.concatenate([F, pf + len(V)]).astype(np.int32),
                mat_ids=np.concatenate([M, np.full(len(pf), 2)]).astype(np.int32),
                materials=_materials(mats))


def balls_scene(n_balls, width=900, height=450, seed=66) -> Scene:
    """Scaling workload after the paper's App. A (1 .. 10^4 inserted balls at
    900x450): the mid field and light with n_balls small spheres."""
    return Scene(name=f"balls{n_balls}", field=mid_field(2), mesh=balls_mesh(n_balls, seed),
                 lights=seeded_light(22), cameras=[front_camera(width, height, 8)], t_near=0.05,
                 t_far=4.0, n_samples=256, max_bounces=8, occupancy_res=128, occupancy_thresh=0.01)


def emitter_quad(y=0.95, half=0.4, radiance=(5.0, 5.0, 5.0)):
    """A black diffuse quad facing down at height y that emits radiance (an
    area light made of two triangles)."""
    v = np.array([[-half, y, -half], [half, y, -half], [half, y, half], [-half, y, half]], dtype=np.float32)
    f = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    return v, f, [DIFFUSE, 1.0, 0.0, 0.0, 0.0, *radiance]


def emitter_scene(width=800, height=800) -> Scene:
    """The mid scene with an emitting ceiling panel (Eq. 12 L_e): glass
    sphere, mirror cube and floor as in the mid scene, the panel last."""
    sv, sf = icosphere(5, radius=0.35, center=(-0.4, -0.24, 0.0))
    cv, cf = cube_triangles((0.45, -0.35, 0.1), 0.5)
    pv, pf = floor_plane(-0.6)
    ev, ef, em = emitter_quad()
    mats = [[GLASS, 1.5, 1.0, 1.0, 1.0], [MIRROR, 1.0, 1.0, 1.0, 1.0], [DIFFUSE, 1.0, 0.7, 0.7, 0.7], em]
    mesh = merge_meshes([(sv, sf, 0), (cv, cf, 1), (pv, pf, 2), (ev, ef, 3)], mats)
    return Scene(name="emitter", field=mid_field(2), mesh=mesh, lights=seeded_light(22),
                 cameras=[front_camera(width, height, 8)], t_near=0.05, t_far=4.0, n_samples=256,
                 max_bounces=8, occupancy_res=128, occupancy_thresh=0.01)


def fields_scene(n_fields=3, width=800, height=450, kind="mid", table_amp=1e-4, spacing=2.9, seed=77,
                 n_samples=None) -> Scene:
    """Several NeRF objects in one scene: n copies of the mid (or tiny) field
    layout with seeds 2, 3, ... (tiny: 1, 2, ...), each turned about y by a
    seeded angle in [-pi/4, pi/4] and set `spacing` apart along x (a box turned
    about y spans at most 2 sqrt 2 in x, so at the default spacing the boxes
    stay disjoint; below 2 neighbouring boxes always overlap), over a
    wide diffuse floor with a glass sphere and a mirror cube in front of them;
    camera 4.8 back.  The segment length covers the far boxes (t in [0.05,
    8.0]) with about the interval length of the single-field workloads (mid:
    516 samples, tiny: 128).  Scene.field is the first field; Scene.fields
    all."""
    rng = np.random.default_rng(seed)
    fields = []
    for k in range(n_fields):
        f = (mid_field(2 + k, table_amp) if kind == "mid" else tiny_field(1 + k, table_amp))
        x = (k - (n_fields - 1) / 2.0) * spacing
        f.pose = pose_matrix(rotation((0.0, 1.0, 0.0), rng.uniform(-math.pi / 4, math.pi / 4)), (x, 0.0, 0.0))
        fields.append(f)
    sv, sf = icosphere(4, radius=0.35, center=(-1.45, -0.75, -2.0))
    cv, cf = cube_triangles((1.45, -0.8, -2.0), 0.6)
    pv, pf = floor_plane(-1.1, half=7.0)
    mats = [[GLASS, 1.5, 1.0, 1.0, 1.0], [MIRROR, 1.0, 1.0, 1.0, 1.0], [DIFFUSE, 1.0, 0.7, 0.7, 0.7]]
    mesh = merge_meshes([(sv, sf, 0), (cv, cf, 1), (pv, pf, 2)], mats)
    cam = Camera(pos=(0.0, 0.4, -4.8), look_at=(0.0, 0.0, 0.0), fov_deg=60.0, width=width, height=height,
                 max_bounces=8)
    if n_samples is None:
        n_samples = 516 if kind == "mid" else 128
    sc = Scene(name=f"fields{n_fields}", field=fields[0], mesh=mesh,
               lights=np.array([[0.0, 2.5, -1.0, 40.0, 40.0, 40.0]], np.float32), cameras=[cam],
               t_near=0.05, t_far=8.0, n_samples=n_samples, max_bounces=8, occupancy_res=128,
               occupancy_thresh=0.01)
    sc.fields = fields
    return sc


def multicam_scene(seed=44) -> Scene:
    return Scene(name="multicam", field=tiny_field(1), mesh=mirror_cube_mesh(),
                 lights=no_lights(), cameras=multicam_cameras(seed), t_near=0.05,
                 t_far=4.0, n_samples=64, max_bounces=16, rr_after=3)


def cloth_scene(frame=0, width=800, height=800) -> Scene:
    return Scene(name="cloth", field=tiny_field(1), mesh=cloth_mesh(frame),
                 lights=no_lights(), cameras=[front_camera(width, height, 8)],
                 t_near=0.05, t_far=4.0, n_samples=256, max_bounces=8)


def rotation(axis, angle):
    """Rotation matrix about a unit axis (Rodrigues), float64."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])
    return np.eye(3) + math.sin(angle) * K + (1.0 - math.cos(angle)) * (K @ K)


def pose_matrix(R, c):
    """[R | c] as a 3x4 float64 array."""
    return np.concatenate([np.asarray(R, np.float64), np.asarray(c, np.float64).reshape(3, 1)], axis=1)


def sample_points(n, seed, lo=-1.0, hi=1.0):
    """Seeded FP32 query points and unit directions for field-level checks."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(lo, hi, size=(n, 3)).astype(np.float32)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return x, d.astype(np.float32)


def random_rays(n, seed, origin_radius=2.5):
    """Seeded FP32 rays from a sphere around the scene towards random points
    inside it (unit directions)."""
    rng = np.random.default_rng(seed)
    o = rng.normal(size=(n, 3))
    o = o / np.linalg.norm(o, axis=1, keepdims=True) * origin_radius
    tgt = rng.uniform(-0.9, 0.9, size=(n, 3))
    d = tgt - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o.astype(np.float32), d.astype(np.float32)
