"""Pins of the FP64 oracle against things other than itself: published
known-answer vectors, closed forms, library routines, brute force and
invariants.  CPU only."""
import copy
import math
import os

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2309_04581_amd import scenegen as sg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _built():
    orc.build(force=False)


# ---------------------------------------------------------------------------
# random numbers
# ---------------------------------------------------------------------------

def test_philox_known_answers():
    """Philox4x32-10 against the generator's published known-answer vectors."""
    n = 0
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        assert orc.philox(v[:4], v[4:6]) == v[6:]
        n += 1
    assert n == 3


# ---------------------------------------------------------------------------
# hash encoding
# ---------------------------------------------------------------------------

def _field_with_table(base, fill):
    f = sg.tiny_field()
    f.table = fill(f).astype(np.float32)
    return f


def test_resolutions_match_config():
    """Integer level resolutions of the two published grids (16..256, 16..2048)."""
    assert list(sg.level_resolutions(16, 256, 8)) == [16, 23, 35, 52, 78, 115, 172, 256]
    assert list(sg.level_resolutions(16, 2048, 16)) == [
        16, 22, 30, 42, 58, 80, 111, 153, 212, 294, 406, 561, 776, 1072, 1482, 2048]


def test_dense_levels_reproduce_linear_functions():
    """On a dense level filled with an affine function of the vertex
    coordinates, trilinear interpolation returns that function exactly."""
    f = sg.tiny_field()
    T = f.table_size
    a = np.array([0.25, -0.5, 0.125])
    for l, N in enumerate(f.resolutions):
        if (N + 1) ** 3 > T:
            continue
        g = np.arange(N + 1)
        vz, vy, vx = np.meshgrid(g, g, g, indexing="ij")
        vals = a[0] * vx + a[1] * vy + a[2] * vz + 3.0
        f.table[l, :(N + 1) ** 3, 0] = vals.ravel()
        f.table[l, :(N + 1) ** 3, 1] = -2.0 * vals.ravel()
    x, _ = sg.sample_points(500, seed=3, lo=-1.0, hi=1.0)
    feat = orc.field_batch(f, x)["feat"]
    dense = [l for l, N in enumerate(f.resolutions) if (N + 1) ** 3 <= T]
    assert dense == [0, 1]
    for l in dense:
        N = f.resolutions[l]
        xl = (x.astype(np.float64) + 1.0) / 2.0 * N
        want = xl @ a + 3.0
        np.testing.assert_allclose(feat[:, 2 * l], want, rtol=0, atol=1e-12)
        np.testing.assert_allclose(feat[:, 2 * l + 1], -2.0 * want, rtol=0, atol=1e-12)


def test_hashed_level_vertex_values_and_continuity():
    """At a grid vertex the feature is the stored entry of that vertex's slot
    (uint32 wrap-around hash, primes 1, 2654435761, 805459861 of the
    multiresolution hash encoding), and the encoding is continuous across cell
    faces (a wrong corner/weight pairing would jump there)."""
    rng = np.random.default_rng(7)
    f = sg.tiny_field()
    f.table = rng.uniform(-1, 1, size=f.table.shape).astype(np.float32)
    l = 7
    N = int(f.resolutions[l])
    T = f.table_size
    assert (N + 1) ** 3 > T
    for _ in range(50):
        v = rng.integers(1, N, size=3)
        h = (int(v[0]) ^ (int(v[1]) * 2654435761 % 2**32) ^ (int(v[2]) * 805459861 % 2**32)) % T
        idx, dense = orc.hash_index(N, f.log2_table, v)
        assert not dense and idx == h
        x = (v / N * 2.0 - 1.0).astype(np.float32)
        xd = x.astype(np.float64)
        # features of the level at the exact vertex: feed the FP64 point through xhat
        feat = orc.field_batch(f, x[None])["feat"][0]
        xl = (xd + 1.0) / 2.0 * N
        if np.all(np.abs(xl - np.round(xl)) < 1e-9):
            np.testing.assert_allclose(feat[2 * l:2 * l + 2], f.table[l, h], atol=1e-5)
    # continuity: points just either side of a cell face at the finest level
    for _ in range(50):
        p = rng.uniform(-0.9, 0.9, size=3)
        k = rng.integers(0, 3)
        xl = (p[k] + 1.0) / 2.0 * N
        p[k] = (math.floor(xl) + 1.0) / N * 2.0 - 1.0
        eps = 2e-7
        a, b = p.copy(), p.copy()
        a[k] -= eps
        b[k] += eps
        fa = orc.field_batch(f, a[None].astype(np.float32))["feat"][0]
        fb = orc.field_batch(f, b[None].astype(np.float32))["feat"][0]
        np.testing.assert_allclose(fa, fb, atol=5e-3)


def test_encoding_at_domain_faces_stays_in_table():
    """Points on the upper faces of the domain use the last cell (weight 1)."""
    f = sg.tiny_field()
    x = np.array([[1.0, 1.0, 1.0], [-1.0, -1.0, -1.0], [1.0, -1.0, 0.3]], dtype=np.float32)
    out = orc.field_batch(f, x)
    assert np.all(np.isfinite(out["feat"]))


# ---------------------------------------------------------------------------
# MLPs, SH, activations
# ---------------------------------------------------------------------------

def test_softplus_of_one_with_zero_table():
    """With an all-zero table the density is softplus(0 + 1) everywhere."""
    f = sg.tiny_field()
    f.table[:] = 0
    x, d = sg.sample_points(64, seed=4)
    s = orc.field_batch(f, x, d)["sigma"]
    np.testing.assert_allclose(s, 1.3132616875182228, rtol=0, atol=1e-15)


def _numpy_mlp(f, feat, d, sh_vals):
    layers = []
    off = 0
    for (o, i) in f.layer_shapes():
        layers.append(f.mlp[off:off + o * i].astype(np.float64).reshape(o, i))
        off += o * i
    x = np.zeros((len(feat), f.d_in))
    x[:, :feat.shape[1]] = feat
    h = np.maximum(x @ layers[0].T, 0)
    raw = h @ layers[1].T
    sigma = np.logaddexp(0.0, raw[:, 0] + f.density_offset)
    cin = np.zeros((len(feat), f.c_in))
    cin[:, :f.d_out] = raw
    cin[:, f.d_out:f.d_out + f.sh] = sh_vals
    h = np.maximum(cin @ layers[2].T, 0)
    for k in range(f.c_layers - 1):
        h = np.maximum(h @ layers[3 + k].T, 0)
    rgb = np.exp(h @ layers[-1].T)
    return sigma, rgb, raw


@pytest.mark.parametrize("kind", ["tiny", "mid"])
def test_mlp_matches_numpy_matmul(kind):
    """Density and colour MLPs against numpy matrix products in FP64."""
    f = sg.tiny_field(table_amp=1.0) if kind == "tiny" else sg.mid_field(table_amp=1.0)
    x, d = sg.sample_points(300, seed=5)
    out = orc.field_batch(f, x, d)
    shv = np.stack([orc.sh(f.sh, dd.astype(np.float64)) for dd in d])
    sigma, rgb, raw = _numpy_mlp(f, out["feat"], d, shv)
    np.testing.assert_allclose(out["sigma"], sigma, rtol=1e-12)
    np.testing.assert_allclose(out["raw"], raw, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(out["rgb"], rgb, rtol=1e-12)


def test_padded_inputs_do_not_matter():
    """Weights of zero-padded input columns never change the output."""
    f = sg.tiny_field(table_amp=1.0)
    x, d = sg.sample_points(50, seed=6)
    a = orc.field_batch(f, x, d)
    off = 0
    W1 = f.mlp[:f.d_hidden * f.d_in].reshape(f.d_hidden, f.d_in)
    W1[:, 16:] = 123.0                         # features occupy columns 0..15
    off = f.d_hidden * f.d_in + f.d_out * f.d_hidden
    Wc = f.mlp[off:off + f.c_hidden * f.c_in].reshape(f.c_hidden, f.c_in)
    Wc[:, 20:] = -77.0                         # 16 raw + 4 SH occupy 0..19
    b = orc.field_batch(f, x, d)
    np.testing.assert_array_equal(a["sigma"], b["sigma"])
    np.testing.assert_array_equal(a["rgb"], b["rgb"])


def _real_sh_scipy(l, m, d):
    from scipy.special import sph_harm_y
    x, y, z = d
    theta = math.acos(max(-1.0, min(1.0, z)))
    phi = math.atan2(y, x)
    if m == 0:
        return sph_harm_y(l, 0, theta, phi).real
    # scipy's complex harmonics carry the Condon-Shortley phase; Sloan's real
    # basis keeps it, so no extra (-1)^m here
    if m > 0:
        return math.sqrt(2) * sph_harm_y(l, m, theta, phi).real
    return math.sqrt(2) * sph_harm_y(l, -m, theta, phi).imag


def test_sh_matches_scipy_real_harmonics():
    """Orthonormal real SH of Sloan (Condon-Shortley phase kept) against scipy's
    complex harmonics, degree <= 3."""
    rng = np.random.default_rng(8)
    for _ in range(40):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        ours = orc.sh(16, d)
        ref = [_real_sh_scipy(l, m, d) for l in range(4) for m in range(-l, l + 1)]
        np.testing.assert_allclose(ours, ref, atol=1e-12)


def test_sh_orthonormal_by_quadrature():
    n = 200
    th = (np.arange(n) + 0.5) / n * math.pi
    ph = (np.arange(2 * n) + 0.5) / (2 * n) * 2 * math.pi
    T, P = np.meshgrid(th, ph, indexing="ij")
    dirs = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1).reshape(-1, 3)
    w = (np.sin(T) * (math.pi / n) * (2 * math.pi / (2 * n))).ravel()
    Y = np.stack([orc.sh(16, d) for d in dirs[::7]])
    G = (Y * w[::7, None] * 7).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=2e-2)


# ---------------------------------------------------------------------------
# intersection
# ---------------------------------------------------------------------------

def _moller_trumbore(o, d, v0, v1, v2):
    e1, e2 = v1 - v0, v2 - v0
    p = np.cross(d, e2)
    det = e1 @ p
    if abs(det) < 1e-300:
        return None
    s = o - v0
    u = (s @ p) / det
    q = np.cross(s, e1)
    v = (d @ q) / det
    t = (e2 @ q) / det
    if u < 0 or v < 0 or u + v > 1 or t <= 0:
        return None
    return t, 1 - u - v, u, v


def test_watertight_test_against_moller_trumbore():
    """Hit/miss, t and barycentrics against the textbook Moller-Trumbore test
    (a different algorithm), away from edges."""
    rng = np.random.default_rng(9)
    agree = 0
    for _ in range(3000):
        v = rng.uniform(-1, 1, size=(3, 3))
        o = rng.uniform(-2, 2, size=3)
        a, b = rng.uniform(-0.3, 1.3, size=2)         # aim near the triangle
        d = v[0] + a * (v[1] - v[0]) + b * (v[2] - v[0]) - o
        d /= np.linalg.norm(d)
        if rng.uniform() < 0.2:
            d = -d                                     # and sometimes away from it
        mt = _moller_trumbore(o, d, *v)
        hit, t, bary = orc.intersect(o, d, *v)
        if mt is not None and min(mt[1:]) < 1e-9:
            continue
        assert hit == (mt is not None)
        if hit:
            assert t == pytest.approx(mt[0], rel=1e-9, abs=1e-12)
            np.testing.assert_allclose(bary, mt[1:], atol=1e-9)
            agree += 1
    assert agree > 400


def test_closest_hit_brute_force_against_numpy():
    """Closest hit over a random soup equals the lexicographic (t, id) minimum
    of per-triangle Moller-Trumbore hits."""
    m = sg.random_triangles(64, seed=10)
    o, d = sg.random_rays(400, seed=11)
    n_hit = 0
    for k in range(len(o)):
        oo, dd = o[k].astype(np.float64), d[k].astype(np.float64)
        hits = []
        for i, f in enumerate(m.indices):
            r = _moller_trumbore(oo, dd, *m.vertices[f].astype(np.float64))
            if r is not None:
                hits.append((r[0], i))
        hid, t, _, tie = orc.closest_hit(m, oo, dd)
        if tie:
            continue
        if hits:
            want = min(hits)
            assert hid == want[1] and t == pytest.approx(want[0], rel=1e-9)
            n_hit += 1
        else:
            assert hid == -1
    assert n_hit > 50


def test_shared_edge_is_watertight_and_flagged():
    """A ray through the shared diagonal of a quad hits exactly one of the two
    triangles (lowest id on equal t) and is flagged as a tie."""
    m = sg.mirror_cube_mesh()
    # z- face diagonal of the cube of side 0.5 at the origin runs (-.25,-.25)-(.25,.25)
    o = np.array([0.1, 0.1, -2.0])
    d = np.array([0.0, 0.0, 1.0])
    hid, t, _, tie = orc.closest_hit(m, o, d)
    assert hid in (0, 1) and t == pytest.approx(1.75) and tie


def test_forced_hit_across_a_shared_edge_is_reachable_and_others_are_not():
    """Outcomes of a tie ray: a ray through the z- face diagonal of the mirror
    cube may hit either triangle of the face in single precision (both reflect
    the same way, so radiance is unchanged); a face the ray never meets, and
    no hit at all (the far face is a certain hit behind), are not reachable."""
    f = _constant_field()
    sc = _scene(f, sg.mirror_cube_mesh())
    d = np.array([0.0, 0.05, 1.0])
    d /= np.linalg.norm(d)
    o = np.array([0.1, 0.1 - 0.05 * 1.75, -2.0])     # meets z = -0.25 at x = y = 0.1
    o32, d32 = o[None].astype(np.float32), d[None].astype(np.float32)
    r = orc.render(sc, o32, d32)
    assert r["tie"][0] and r["hit_ids"][0, 0] in (0, 1)
    other = 1 - r["hit_ids"][0, 0]
    fh = r["hit_ids"].copy()
    fh[0, 0] = other
    a = r["rerun"]([0], force_hits=fh)
    assert not a["invalid"][0] and a["hit_ids"][0, 0] == other
    np.testing.assert_allclose(a["radiance"][0], r["radiance"][0], rtol=1e-12)
    np.testing.assert_allclose(a["throughput"][0], r["throughput"][0], rtol=1e-12)
    for bad in (10, -1):                 # x+ face; no hit although the z+ face is certain
        fb = r["hit_ids"].copy()
        fb[0, 0] = bad
        assert r["rerun"]([0], force_hits=fb)["invalid"][0], bad
    # forcing what the oracle chose anyway changes nothing
    same = r["rerun"]([0], force_hits=r["hit_ids"])
    assert not same["invalid"][0]
    np.testing.assert_array_equal(same["radiance"], r["radiance"])


def test_forced_hit_on_a_clear_ray_is_not_reachable():
    """Away from every edge there is one outcome: forcing the other triangle
    of the face, or no hit, marks the ray invalid."""
    sc = _scene(_constant_field(), sg.mirror_cube_mesh())
    o = np.array([[0.1, -0.12, -2.0]], np.float32)
    d = np.array([[0.0, 0.0, 1.0]], np.float32)
    r = orc.render(sc, o, d)
    assert not r["tie"][0] and r["hit_ids"][0, 0] in (0, 1)
    for bad in (1 - r["hit_ids"][0, 0], -1):
        fb = r["hit_ids"].copy()
        fb[0, 0] = bad
        assert r["rerun"]([0], force_hits=fb)["invalid"][0]


def test_flipping_a_flagged_decision_takes_its_other_branch():
    """A cut-off equal to the throughput after one diffuse bounce (albedo 0.7
    stored in FP32, just below 0.7) is a flagged decision: as it stands the
    path stops after the floor (one segment); with its bit set the path goes
    on and escapes (two segments).  Bits beyond the flagged decisions change
    nothing."""
    plane_v, plane_f = sg.floor_plane(-0.6)
    mesh = sg.merge_meshes([(plane_v, plane_f, 0)], [[sg.DIFFUSE, 1.0, 0.7, 0.7, 0.7]])
    sc = _scene(None, mesh, t_min_throughput=0.7)
    o = np.array([[0.0, 0.5, -2.0]], np.float32)
    tgt = np.array([0.1, -0.6, 0.2])
    d = ((tgt - o[0]) / np.linalg.norm(tgt - o[0]))[None].astype(np.float32)
    r = orc.render(sc, o, d)
    assert r["tie"][0] and r["n_flagged"][0] == 1 and r["segments"][0] == 1 and r["bounces"][0] == 1
    f1 = r["rerun"]([0], flip=np.array([1], np.uint32))
    assert f1["segments"][0] == 2 and f1["bounces"][0] == 1 and not f1["invalid"][0]
    np.testing.assert_array_equal(f1["throughput"], r["throughput"])
    f2 = r["rerun"]([0], flip=np.array([2], np.uint32))
    assert f2["segments"][0] == 1


# ---------------------------------------------------------------------------
# BSDFs
# ---------------------------------------------------------------------------

def test_fresnel_closed_forms():
    """Normal incidence R = ((1-1.5)/(1+1.5))^2 = 0.04; total internal
    reflection beyond asin(1/1.5) = 41.8103 deg from inside; R(90 deg) = 1."""
    assert orc.fresnel(1.0, 1.0, 1.5) == pytest.approx(0.04, abs=1e-15)
    assert orc.fresnel(1.0, 1.5, 1.0) == pytest.approx(0.04, abs=1e-15)
    crit = math.asin(1 / 1.5)
    assert math.degrees(crit) == pytest.approx(41.8103149, abs=1e-6)
    assert orc.fresnel(math.cos(crit + 1e-6), 1.5, 1.0) == 1.0
    assert orc.fresnel(math.cos(crit - 1e-3), 1.5, 1.0) < 1.0
    assert orc.fresnel(0.0, 1.0, 1.5) == pytest.approx(1.0)


def test_refraction_obeys_snell_and_reflection_law():
    rng = np.random.default_rng(12)
    glass = np.array([sg.GLASS, 1.5, 1, 1, 1], dtype=np.float32)
    mirror = np.array([sg.MIRROR, 1, 1, 1, 1], dtype=np.float32)
    for _ in range(200):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        # reflection: equal angles, in the plane of d and n
        nd, side, w, _ = orc.scatter(mirror, d, n, [0.5] * 4)
        assert np.dot(nd, n) == pytest.approx(-np.dot(d, n), abs=1e-14)
        assert np.linalg.det(np.stack([d, n, nd])) == pytest.approx(0, abs=1e-12)
        assert np.dot(side, d) < 0
        # refraction (u = 0.999999 forces the transmitted branch unless TIR)
        nd, side, w, R = orc.scatter(glass, d, n, [0.999999, 0, 0, 0])
        entering = np.dot(d, n) < 0
        n1, n2 = (1.0, 1.5) if entering else (1.5, 1.0)
        sin_i = np.linalg.norm(np.cross(d, n))
        sin_t = np.linalg.norm(np.cross(nd, n))
        if R < 1.0:
            assert n1 * sin_i == pytest.approx(n2 * sin_t, abs=1e-12)
            assert np.dot(nd, n) * np.dot(d, n) > 0          # crosses the surface
            assert np.dot(side, d) > 0
        np.testing.assert_array_equal(w, [1, 1, 1])


def test_mirror_reflection_is_an_exact_sign_flip_on_axis_faces():
    mirror = np.array([sg.MIRROR, 1, 1, 1, 1], dtype=np.float32)
    d = np.array([0.3, -0.2, 0.9327379053088815])
    for ax in range(3):
        n = np.zeros(3)
        n[ax] = 1.0
        nd, *_ = orc.scatter(mirror, d, n, [0] * 4)
        want = d.copy()
        want[ax] = -want[ax]
        np.testing.assert_array_equal(nd, want)


def test_cosine_sampling_statistics():
    """Cosine-weighted directions: E[cos] = 2/3, E[cos^2] = 1/2, all in the
    hemisphere facing the incoming ray; chi-square on 10 cos^2 bins."""
    diffuse = np.array([sg.DIFFUSE, 1, 0.7, 0.6, 0.5], dtype=np.float32)
    n = np.array([0.2, 0.9, -0.3])
    n /= np.linalg.norm(n)
    d = -n + np.array([0.1, 0.0, 0.05])
    d /= np.linalg.norm(d)
    cs = []
    for k in range(20000):
        u = [u for u in np.array(orc.philox([k, 0, 1, 0], [230904581, 0])) / 2**32]
        u = [(x * 2**32 // 256) / 2**24 for x in u]
        nd, side, w, _ = orc.scatter(diffuse, d, n, u)
        cs.append(np.dot(nd, n))
        assert abs(np.linalg.norm(nd) - 1) < 1e-12
    cs = np.array(cs)
    np.testing.assert_allclose(w, [0.7, 0.6, 0.5], rtol=1e-7)
    assert cs.min() > 0
    assert cs.mean() == pytest.approx(2 / 3, abs=0.01)
    assert (cs ** 2).mean() == pytest.approx(0.5, abs=0.01)
    hist, _ = np.histogram(cs ** 2, bins=10, range=(0, 1))     # cos^2 is uniform
    chi2 = ((hist - 2000) ** 2 / 2000).sum()
    assert chi2 < 27.9                                           # p = 0.001, 9 dof


# ---------------------------------------------------------------------------
# whole paths: closed forms and invariants
# ---------------------------------------------------------------------------

def _constant_field(sigma_offset=1.0):
    f = sg.tiny_field()
    f.table[:] = 0
    f.mlp[:] = 0
    f.density_offset = sigma_offset
    return f


def _scene(field, mesh, lights=None, **kw):
    sc = sg.tiny_scene()
    sc.field, sc.mesh = field, mesh
    sc.lights = sg.no_lights() if lights is None else lights
    for k, v in kw.items():
        setattr(sc, k, v)
    return sc


def _chord(o, d, t0, t1):
    """Length of [t0, t1] inside [-1, 1]^3 along o + t d."""
    lo, hi = t0, t1
    for k in range(3):
        if d[k] == 0:
            continue
        a, b = (-1 - o[k]) / d[k], (1 - o[k]) / d[k]
        lo, hi = max(lo, min(a, b)), min(hi, max(a, b))
    return max(0.0, hi - lo)


def test_constant_medium_transmittance_closed_form():
    """Constant sigma, colour exp(0) = 1, no mesh: T = exp(-sigma l) and
    L = 1 - T for the chord length l (midpoint quadrature is exact)."""
    f = _constant_field()
    sigma = math.log1p(math.e)
    sc = _scene(f, None)
    o, d = sg.random_rays(300, seed=13)
    r = orc.render(sc, o, d)
    for k in range(len(o)):
        ell = _chord(o[k].astype(np.float64), d[k].astype(np.float64), sc.t_near, sc.t_far)
        T = math.exp(-sigma * ell)
        np.testing.assert_allclose(r["throughput"][k], T, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(r["radiance"][k], 1 - T, rtol=1e-11, atol=1e-14)
    assert np.all(r["bounces"] == 0)


def test_mirror_cube_closed_form_path():
    """A ray onto the z- face of the mirror cube reflects to (dx, dy, -dz);
    its transmittance is exp(-sigma (l_in + l_out)) with the spawn offset."""
    f = _constant_field()
    sigma = math.log1p(math.e)
    sc = _scene(f, sg.mirror_cube_mesh())
    d = np.array([0.02, 0.01, 1.0])
    d /= np.linalg.norm(d)
    o = np.array([0.1, 0.05, -2.5])
    r = orc.render(sc, o[None].astype(np.float32), d[None].astype(np.float32))
    o32, d32 = o.astype(np.float32).astype(np.float64), d.astype(np.float32).astype(np.float64)
    t_hit = (-0.25 - o32[2]) / d32[2]
    p = o32 + t_hit * d32
    l_in = _chord(o32, d32, sc.t_near, t_hit)
    o2 = p + np.array([0, 0, -1e-4])
    d2 = d32 * np.array([1, 1, -1])
    l_out = _chord(o2, d2, 0.0, sc.t_far - sc.t_near)
    T = math.exp(-sigma * (l_in + l_out))
    assert r["bounces"][0] == 1 and r["hit_ids"][0, 0] in (0, 1) and r["hit_ids"][0, 1] == -1
    np.testing.assert_allclose(r["throughput"][0], T, rtol=1e-12)
    np.testing.assert_allclose(r["radiance"][0], 1 - T, rtol=1e-11)


def test_lit_diffuse_plane_closed_form():
    """Empty medium, one diffuse quad, one point light: L = (rho/pi) I cos/d^2;
    with a blocker between, L = 0."""
    plane_v, plane_f = sg.floor_plane(-0.6)
    mesh = sg.merge_meshes([(plane_v, plane_f, 0)], [[sg.DIFFUSE, 1.0, 0.7, 0.5, 0.3]])
    light = np.array([[0.3, 0.7, -0.2, 10.0, 8.0, 6.0]], dtype=np.float32)
    sc = _scene(None, mesh, light)
    o = np.array([[0.0, 0.5, -2.0]], dtype=np.float32)
    tgt = np.array([0.1, -0.6, 0.2])
    d = (tgt - o[0]) / np.linalg.norm(tgt - o[0])
    r = orc.render(sc, o, d[None].astype(np.float32))
    oo, dd = o[0].astype(np.float64), d.astype(np.float32).astype(np.float64)
    t = (float(np.float32(-0.6)) - oo[1]) / dd[1]            # plane height stored in FP32
    p = oo + t * dd
    wi = light[0, :3].astype(np.float64) - p
    cos = wi[1] / np.linalg.norm(wi)
    rho = np.array([0.7, 0.5, 0.3], dtype=np.float32).astype(np.float64)   # stored in FP32
    want = rho / math.pi * np.array([10.0, 8.0, 6.0]) * cos / (wi @ wi)
    np.testing.assert_allclose(r["radiance"][0], want, rtol=1e-12)
    np.testing.assert_allclose(r["throughput"][0], [0.7, 0.5, 0.3], rtol=1e-7)
    assert r["bounces"][0] == 1
    # a small blocker half way between the hit point and the light
    c = (p + light[0, :3]) / 2
    bv = np.array([c + [-0.1, 0, -0.1], c + [0.1, 0, -0.1], c + [0.0, 0, 0.15]], dtype=np.float32)
    mesh2 = sg.merge_meshes([(plane_v, plane_f, 0), (bv, np.array([[0, 1, 2]], np.int32), 0)],
                            [[sg.DIFFUSE, 1.0, 0.7, 0.5, 0.3]])
    r2 = orc.render(_scene(None, mesh2, light), o, d[None].astype(np.float32))
    assert r2["hit_ids"][0, 0] in (0, 1)
    np.testing.assert_array_equal(r2["radiance"][0], 0.0)


@pytest.mark.parametrize("mesh_kind", ["cube", "glass_and_mirror"])
def test_energy_telescopes_on_specular_paths(mesh_kind):
    """With colour exp(0) = 1 and only lossless specular surfaces, each
    sample moves T alpha from throughput to radiance: L + T = 1 per channel."""
    f = sg.tiny_field(table_amp=0.5)
    off = sum(o * i for o, i in f.layer_shapes()[:-1])
    f.mlp[off:] = 0.0                                   # colour output layer -> exp(0)
    if mesh_kind == "cube":
        mesh = sg.mirror_cube_mesh()
    else:
        sv, sf = sg.icosphere(2, radius=0.35, center=(-0.3, 0.0, 0.0))
        cv, cf = sg.cube_triangles((0.4, -0.1, 0.1), 0.4)
        mesh = sg.merge_meshes([(sv, sf, 0), (cv, cf, 1)],
                               [[sg.GLASS, 1.5, 1, 1, 1], [sg.MIRROR, 1, 1, 1, 1]])
    sc = _scene(f, mesh, t_min_throughput=0.0, max_bounces=8)
    o, d = sg.random_rays(500, seed=14)
    if mesh_kind == "cube":                           # and rays inside the mirror box
        oi, di = sg.sample_points(200, seed=24, lo=-0.2, hi=0.2)
        o, d = np.concatenate([o, oi]), np.concatenate([d, di])
    r = orc.render(sc, o, d)
    np.testing.assert_allclose(r["radiance"] + r["throughput"], 1.0, rtol=0, atol=1e-12)
    assert r["bounces"].max() >= 2


def test_throughput_bounded_and_diffuse_loss():
    """Throughput never exceeds 1; a diffuse bounce keeps rho of it."""
    sc = sg.mid_scene(width=8, height=8, n_samples=32)
    sc.field = sg.tiny_field()
    o, d = sg.random_rays(400, seed=15)
    r = orc.render(sc, o, d)
    assert np.all(r["throughput"] <= 1.0 + 1e-15) and np.all(r["throughput"] >= 0)
    assert np.all(np.isfinite(r["radiance"])) and np.all(r["radiance"] >= 0)


def test_no_light_radiance_bounded_by_field_maximum():
    """With the field as the only light and dissipative transport, radiance
    never exceeds the field's largest colour (Sec. 3.1, LDR remark)."""
    sc = sg.tiny_scene()
    sc.field = sg.tiny_field(table_amp=0.5)
    o, d = sg.random_rays(300, seed=16)
    r = orc.render(sc, o, d)
    x, dd = sg.sample_points(20000, seed=17)
    cmax = orc.field_batch(sc.field, x, dd)["rgb"].max()
    assert r["radiance"].max() <= cmax * 1.05


def test_camera_model():
    """Pinhole rays: left-right mirror symmetry, unit length, and the centre
    pixel of an odd-sized image looks straight at the origin (t = 2.25 to the
    cube's front face)."""
    cam = sg.cameras_array([sg.front_camera(65, 65, 4)])[0]
    o, d = orc.rays_from_camera(cam)
    D = d.reshape(65, 65, 3)
    np.testing.assert_allclose(D[:, ::-1, 0], -D[:, :, 0], atol=1e-15)
    np.testing.assert_allclose(D[:, ::-1, 1:], D[:, :, 1:], atol=1e-15)
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15)
    np.testing.assert_allclose(D[32, 32], [0, 0, 1], atol=1e-15)
    assert D[0, 32, 1] > 0                         # top row looks up
    hid, t, _, _ = orc.closest_hit(sg.mirror_cube_mesh(), o[32 * 65 + 32], D[32, 32])
    assert t == pytest.approx(2.25) and hid in (0, 1)
    # the corner ray makes the half field of view with the axis along x and y
    assert math.degrees(math.atan(D[32, 0, 0] / D[32, 0, 2])) == pytest.approx(
        -math.degrees(math.atan(math.tan(math.radians(30)) * 64 / 65)), abs=1e-9)


def test_occupancy_extremes():
    """An all-empty occupancy grid removes the medium; an all-full one changes nothing."""
    sc = sg.tiny_scene()
    o, d = sg.random_rays(100, seed=18)
    base = orc.render(sc, o, d)
    full = orc.render(sc, o, d, occupancy_bits=np.ones(8 ** 3, np.uint8))
    empty = orc.render(sc, o, d, occupancy_bits=np.zeros(8 ** 3, np.uint8))
    np.testing.assert_array_equal(base["radiance"], full["radiance"])
    np.testing.assert_array_equal(empty["radiance"], 0.0)


def test_occupancy_thresholds_subcell_maximum():
    """A cell is occupied iff some sub-cell centre reaches the threshold."""
    f = sg.tiny_field(table_amp=1.0)
    f.density_offset = -5.0                      # sigma spans ~0.004..0.013
    bits, margin = orc.occupancy(f, 8, 0.01)
    assert 0 < bits.mean() < 1
    np.testing.assert_array_equal(bits, (margin >= 0).astype(np.uint8))
    # re-evaluate one cell's probes directly
    c = int(np.argmax(margin))
    cx, cy, cz = c % 8, (c // 8) % 8, c // 64
    probes = np.array([[(cx + 0.25 + 0.5 * (s & 1)) / 8, (cy + 0.25 + 0.5 * ((s >> 1) & 1)) / 8,
                        (cz + 0.25 + 0.5 * ((s >> 2) & 1)) / 8] for s in range(8)]) * 2 - 1
    s = orc.field_batch(f, probes.astype(np.float32))["sigma"]
    assert s.max() - 0.01 == pytest.approx(margin[c], rel=1e-6)


def test_russian_roulette_keeps_expectation():
    """Roulette divides by q on survival: averaged over many paths, the
    estimator's radiance matches the no-roulette value."""
    f = sg.tiny_field(table_amp=0.5)
    mesh = sg.mid_mesh()
    base = _scene(f, mesh, sg.seeded_light(22), max_bounces=6, n_samples=16)
    o, d = sg.random_rays(1, seed=19)
    o = np.repeat(o, 4000, 0)
    d = np.repeat(d, 4000, 0)
    a = orc.render(base, o, d)
    rr = _scene(f, mesh, sg.seeded_light(22), max_bounces=6, n_samples=16, rr_after=1)
    b = orc.render(rr, o, d)
    # with q = min(1, max T) the survivor's largest channel becomes at most 1
    assert np.all(b["throughput"] >= 0.0) and np.all(b["throughput"] <= 1.0 + 1e-12)
    ma, mb = a["radiance"].mean(0), b["radiance"].mean(0)
    se = b["radiance"].std(0) / math.sqrt(len(o)) + a["radiance"].std(0) / math.sqrt(len(o))
    assert np.all(np.abs(ma - mb) <= 4 * se + 1e-12)


# ---------------------------------------------------------------------------
# proposal sampler and its gradient
# ---------------------------------------------------------------------------

def test_proposal_sampler_exact_for_constant_medium():
    """For a constant medium any partition of the segment gives the exact
    transmittance, so proposal sampling must reproduce exp(-sigma l)."""
    f = _constant_field()
    prop = sg.make_proposal(table_amp=1.0)
    sc = _scene(f, None)
    o, d = sg.random_rays(100, seed=20)
    a = orc.render(sc, o, d)
    b = orc.render(sc, o, d, proposal=prop, n_prop=32, n_fine=32)
    np.testing.assert_allclose(a["throughput"], b["throughput"], rtol=1e-12)
    np.testing.assert_allclose(a["radiance"], b["radiance"], rtol=1e-11)


def _prop_batch(n, seed):
    rng = np.random.default_rng(seed)
    o, d = sg.random_rays(n, seed)
    lohi = np.stack([np.full(n, 1.6), np.full(n, 3.2)], 1).astype(np.float32)
    tgt = rng.dirichlet(np.ones(32) * 0.3, size=n).astype(np.float32) * 0.9
    return o, d, lohi, tgt


def test_proposal_gradient_finite_differences():
    """FP64 analytic gradient of the proposal loss against central differences
    (h = 1e-6) on a seeded subset of table entries and MLP weights."""
    prop = sg.make_proposal(table_amp=0.3)
    prop.mlp = prop.mlp.astype(np.float64)
    prop.table = prop.table.astype(np.float64)
    o, d, lohi, tgt = _prop_batch(6, 21)

    class P64:
        pass

    loss, gt, gm = orc.proposal_loss(prop, o, d, lohi, tgt)
    assert loss > 0
    # which table entries are touched
    touched = np.argwhere(np.abs(gt) > 1e-6)
    rng = np.random.default_rng(22)
    sel = touched[rng.choice(len(touched), size=min(12, len(touched)), replace=False)]

    def loss_at(mut):
        p2 = sg.make_proposal(table_amp=0.3)
        mut(p2)
        return orc.proposal_loss(p2, o, d, lohi, tgt, grads=False)[0]

    # the oracle reads FP32 parameters, so perturb with a step FP32 resolves
    h = 1e-3
    for (l, t, c) in sel:
        def up(p2, s=+1):
            p2.table[l, t, c] += s * h
        lp = loss_at(lambda p2: up(p2, +1))
        lm = loss_at(lambda p2: up(p2, -1))
        base = sg.make_proposal(table_amp=0.3).table[l, t, c]
        hp = float(np.float32(base + h)) - float(base)
        hm = float(base) - float(np.float32(base - h))
        fd = (lp - lm) / (hp + hm)
        assert fd == pytest.approx(gt[l, t, c], rel=2e-2, abs=1e-7)
    for k in rng.choice(len(prop.mlp), size=12, replace=False):
        base = sg.make_proposal(table_amp=0.3).mlp[k]

        def mk(s):
            def m(p2):
                p2.mlp[k] += s * h
            return m
        lp, lm = loss_at(mk(+1)), loss_at(mk(-1))
        hp = float(np.float32(base + h)) - float(base)
        hm = float(base) - float(np.float32(base - h))
        fd = (lp - lm) / (hp + hm)
        assert fd == pytest.approx(gm[k], rel=2e-2, abs=1e-7)


def test_proposal_gradient_rounding_bound():
    """The per-element FP32 tolerance of the proposal gradient (the GPU parity
    tolerance) (a) covers the change of the exact gradient when every input of
    the chain moves by one FP32 ulp, with random sign: ray origins, directions,
    segment ranges, table entries and weights, which includes the position
    rounding carried into the trilinear weights; (b) stays a small fraction of
    the gradient, so an O(1) error in any term (the chain's partials, a lost
    contribution) still exceeds it; (c) grows with the unit roundoff."""
    prop = sg.make_proposal(table_amp=0.3)
    o, d, lohi, tgt = _prop_batch(200, 41)
    lohi = lohi + np.random.default_rng(43).uniform(-0.2, 0.2, lohi.shape).astype(np.float32)
    _, gt, gm = orc.proposal_loss(prop, o, d, lohi, tgt)
    bt, bm = orc.proposal_grad_bound(prop, o, d, lohi, tgt)
    rng = np.random.default_rng(42)

    def nudge(a):
        a = np.asarray(a, np.float32)
        up = rng.random(a.shape) < 0.5
        return np.where(up, np.nextafter(a, np.float32(np.inf)), np.nextafter(a, np.float32(-np.inf)))

    p2 = copy.deepcopy(prop)
    p2.table = nudge(prop.table)
    p2.mlp = nudge(prop.mlp)
    _, gt2, gm2 = orc.proposal_loss(p2, nudge(o), nudge(d), nudge(lohi), tgt)
    # one ulp is 2^-23 of the value at most: the tolerance for that unit
    bt_ulp, bm_ulp = orc.proposal_grad_bound(prop, o, d, lohi, tgt, u=2.0 ** -23)
    assert (np.abs(gt2 - gt) <= bt_ulp).all()
    assert (np.abs(gm2 - gm) <= bm_ulp).all()
    # the nudge is felt: it moves a share of the table gradient by more than
    # a hundredth of the tolerance
    assert (np.abs(gt2 - gt) > 0.01 * bt_ulp).mean() > 0.05
    nz = np.abs(gt) > 0
    assert np.median(bt[nz] / np.abs(gt[nz])) < 0.03
    assert np.median(bm / np.abs(gm)) < 0.03
    # one segment's contribution left out exceeds the tolerance somewhere
    _, gt1, gm1 = orc.proposal_loss(prop, o[1:], d[1:], lohi[1:], tgt[1:])
    n = len(o)
    assert (np.abs(gt1 * (n - 1) / n - gt) > bt).any()
    assert (np.abs(gm1 * (n - 1) / n - gm) > bm).any()
    bt2, bm2 = orc.proposal_grad_bound(prop, o, d, lohi, tgt, u=2.0 ** -11)
    assert (bt2 >= bt).all() and (bm2 > bm).all()


def test_proposal_loss_zero_when_proposal_dominates():
    prop = sg.make_proposal(table_amp=0.3)
    o, d, lohi, tgt = _prop_batch(4, 23)
    loss, gt, gm = orc.proposal_loss(prop, o, d, lohi, np.zeros_like(tgt))
    assert loss == 0.0 and not gt.any() and not gm.any()


def test_proposal_targets_sum_to_opacity():
    """The binned plain-marcher weights of a segment sum to 1 - T over it; for
    a constant medium that is 1 - exp(-sigma l) for the clipped chord l, and
    every bin is non-negative."""
    f = _constant_field()
    sigma = math.log1p(math.e)
    o, d = sg.random_rays(50, seed=25)
    lohi, tgt = orc.proposal_targets(f, o, d, 0.05, 4.0, 256, 32)
    for k in range(len(o)):
        ell = _chord(o[k].astype(np.float64), d[k].astype(np.float64), 0.05, 4.0)
        assert tgt[k].sum() == pytest.approx(1 - math.exp(-sigma * ell), rel=1e-12, abs=1e-15)
        if ell > 0:
            assert lohi[k, 1] - lohi[k, 0] == pytest.approx(ell, rel=1e-12)
    assert np.all(tgt >= 0)
    # a shell of density: the mass sits in the bins that cross the shell
    shell = sg.shell_field()
    o = np.array([[0.0, 0.0, -2.5]], np.float32)
    d = np.array([[0.0, 0.0, 1.0]], np.float32)
    lohi, tgt = orc.proposal_targets(shell, o, d, 0.05, 4.0, 256, 32)
    centers = lohi[0, 0] + (np.arange(32) + 0.5) * (lohi[0, 1] - lohi[0, 0]) / 32
    peak = centers[np.argmax(tgt[0])]
    assert abs(peak - 2.0) < 0.1                      # the front of the shell (|z| = 0.5) at t = 2


def _constant_proposal(offset):
    """A proposal field of constant density softplus(offset): with a zero
    table every feature is 0, so the MLP's output is 0 whatever its weights."""
    prop = sg.make_proposal(table_amp=1.0)
    prop.table[:] = 0
    prop.density_offset = offset
    return prop


def test_proposal_weights_constant_medium_closed_form():
    """On a constant medium the proposal weight of interval j of width D is
    the probability of the first interaction falling in it,
    exp(-sigma j D) (1 - exp(-sigma D)): transmittance before the interval
    times its opacity (Eq. 10-11 on a piecewise-constant density)."""
    offset = 1.5
    sigma = math.log1p(math.exp(offset))
    prop = _constant_proposal(offset)
    o, d = np.array([0.1, -0.2, -2.5]), np.array([0.0, 0.0, 1.0])
    lo, hi, n = 1.7, 3.3, 32                          # z from -0.8 to 0.8: inside the box
    w = orc.proposal_weights(prop, o, d, lo, hi, n)
    D = (hi - lo) / n
    for j in range(n):
        exact = math.exp(-sigma * j * D) * -math.expm1(-sigma * D)
        assert w[j] == pytest.approx(exact, rel=1e-12, abs=1e-300)
    assert w.sum() == pytest.approx(-math.expm1(-sigma * (hi - lo)), rel=1e-12)


def test_proposal_edges_hand_worked_step_density():
    """Four proposal intervals on [0, 4] with all weight in the second one.
    Worked by hand: dilation over neighbours gives (1, 1, 1, 0); the uniform
    half adds their mean 3/4 and the floor adds 1e-3/4, so the density is
    1.75025 on [0, 3] and 0.75025 on [3, 4], 6.001 in total.  The median sits
    where the mass reaches 3.0005, inside [1, 2] at 1 + 1.25025/1.75025; the
    quartiles at 1.50025/1.75025 and 2 + 1.00025/1.75025.  Without the
    dilation, without the mixture, or with a misplaced inverse, each of these
    moves by more than 0.05."""
    w = [0.0, 1.0, 0.0, 0.0]
    e2 = orc.proposal_edges(w, 2, 0.0, 4.0)
    np.testing.assert_allclose(e2, [0.0, 1.0 + 1.25025 / 1.75025, 4.0], rtol=0, atol=1e-13)
    e4 = orc.proposal_edges(w, 4, 0.0, 4.0)
    np.testing.assert_allclose(
        e4, [0.0, 1.50025 / 1.75025, 1.0 + 1.25025 / 1.75025, 2.0 + 1.00025 / 1.75025, 4.0],
        rtol=0, atol=1e-13)
    # the same density on [1, 3]: every interval half as wide
    e4s = orc.proposal_edges(w, 4, 1.0, 3.0)
    np.testing.assert_allclose(e4s, 1.0 + 0.5 * np.asarray(e4), rtol=0, atol=1e-13)
    # a density the dilation does not change (flat weights): the mixture is
    # flat too and the edges are uniform
    np.testing.assert_allclose(orc.proposal_edges([0.2] * 8, 4, 0.0, 2.0),
                               [0.0, 0.5, 1.0, 1.5, 2.0], rtol=0, atol=1e-13)
    # weight at the first interval only: the dilation reaches one neighbour,
    # density (1 + 1/2 + 1e-3/4) on [0, 2] and (1/2 + 1e-3/4) on [2, 4],
    # 4.001 in total; the median (2.0005) lies at 1 + 0.5/1.50025 in [1, 2]
    e = orc.proposal_edges([1.0, 0.0, 0.0, 0.0], 2, 0.0, 4.0)
    assert e[1] == pytest.approx(1.0 + (2.0005 - 1.50025) / 1.50025, abs=1e-13)


def test_proposal_edges_split_the_density_into_equal_masses():
    """The edges are quantiles: between consecutive edges lies 1/n_fine of
    the sampling density's mass, for seeded weights and interval counts,
    with the mass of each piece integrated exactly over the piecewise-constant
    density (dilated weights + their mean + 1e-3/n)."""
    rng = np.random.default_rng(31)
    for np_, nf in ((32, 32), (32, 7), (5, 16), (64, 33)):
        w = rng.exponential(size=np_) * (rng.uniform(size=np_) < 0.3)
        lo, hi = 0.4, 2.9
        e = orc.proposal_edges(w, nf, lo, hi)
        wd = np.array([max(w[max(j - 1, 0):j + 2]) for j in range(np_)])
        dens = wd + wd.mean() + 1e-3 / np_
        step = (hi - lo) / np_
        cum = np.concatenate([[0.0], np.cumsum(dens * step)])

        def mass(t):
            j = min(int((t - lo) / step), np_ - 1)
            return cum[j] + dens[j] * (t - (lo + j * step))
        masses = np.diff([mass(t) for t in e])
        np.testing.assert_allclose(masses, cum[-1] / nf, rtol=1e-9)
        assert e[0] == lo and e[-1] == hi and np.all(np.diff(e) > 0)


def test_proposal_march_composites_between_the_edges():
    """The proposal-sampled march composites the fine intervals between the
    edges that the (pinned) weights and edges give, each at its midpoint:
    checked on a non-constant field, one ray through the box, no mesh."""
    f = sg.tiny_field(table_amp=1.0)
    prop = sg.make_proposal(table_amp=1.0)
    sc = _scene(f, None)
    o = np.array([[0.13, -0.07, -2.5]], np.float32)
    d = np.array([[0.02, 0.01, 1.0]], np.float32)
    d /= np.linalg.norm(d)
    r = orc.render(sc, o, d, proposal=prop, n_prop=32, n_fine=24)
    o64, d64 = o[0].astype(np.float64), d[0].astype(np.float64)
    lo = max(sc.t_near, *[min((-1 - o64[k]) / d64[k], (1 - o64[k]) / d64[k]) for k in range(3)])
    hi = min(sc.t_far, *[max((-1 - o64[k]) / d64[k], (1 - o64[k]) / d64[k]) for k in range(3)])
    w = orc.proposal_weights(prop, o64, d64, lo, hi, 32)
    e = orc.proposal_edges(w, 24, lo, hi)
    mid = 0.5 * (e[1:] + e[:-1])
    q = orc.field_batch(f, (o64[None] + mid[:, None] * d64[None]).astype(np.float32),
                        np.repeat(d, len(mid), 0))
    # field_batch takes FP32 points: compare at the FP32 rounding of the positions
    T, L = np.ones(3), np.zeros(3)
    for k in range(len(mid)):
        a = -math.expm1(-q["sigma"][k] * (e[k + 1] - e[k]))
        L += T * a * q["rgb"][k]
        T *= 1 - a
    np.testing.assert_allclose(r["throughput"][0], T, rtol=1e-5)
    np.testing.assert_allclose(r["radiance"][0], L, rtol=1e-5)
    assert r["samples"][0] == 24


def test_proposal_targets_converge_to_the_exact_bin_integrals():
    """On a constant medium the exact weight mass of bin [a_j, b_j] of the
    clipped range [lo, hi] is exp(-sigma (a_j - lo)) - exp(-sigma (b_j - lo)).
    Splitting each plain interval's weight by overlap reaches it to O(delta^2)
    (under 1e-5 at 1 000 samples here, where a whole interval given to the
    bin of its midpoint is off by about 4e-3), and the error falls as the grid
    refines."""
    offset = 2.0
    sigma = math.log1p(math.exp(offset))
    f = _constant_field(offset)
    o = np.array([[0.1, 0.2, -2.5]], np.float32)
    d = np.array([[0.0, 0.0, 1.0]], np.float32)
    nb = 32
    errs = []
    for ns in (1000, 2000):
        lohi, tgt = orc.proposal_targets(f, o, d, 0.05, 4.0, ns, nb)
        lo, hi = lohi[0]
        assert (lo, hi) == pytest.approx((1.5, 3.5), abs=1e-12)
        bw = (hi - lo) / nb
        exact = np.array([math.exp(-sigma * j * bw) - math.exp(-sigma * (j + 1) * bw) for j in range(nb)])
        errs.append(np.abs(tgt[0] - exact).max())
    assert errs[0] < 1e-5 and errs[1] < 0.6 * errs[0]


# ---------------------------------------------------------------------------
# placement of the field (a moving NeRF object): world point p is looked up at
# R^T (p - c), direction d at R^T d
# ---------------------------------------------------------------------------

def _posed(f, R, c):
    g = sg.Field(**{k: getattr(f, k) for k in f.__dataclass_fields__})
    g.pose = sg.pose_matrix(R, c)
    return g


def test_pose_identity_changes_nothing():
    sc = sg.tiny_scene(table_amp=1.0)
    o, d = sg.random_rays(200, seed=31)
    a = orc.render(sc, o, d)
    sc.field = _posed(sc.field, np.eye(3), np.zeros(3))
    b = orc.render(sc, o, d)
    for k in ("radiance", "throughput", "bounces", "hit_ids"):
        np.testing.assert_array_equal(a[k], b[k])


def test_pose_rotated_box_chord_closed_form():
    """Constant medium rotated 45 degrees about y: the ray along +z through the
    centre crosses the box between two opposite vertical edges, a chord of
    2 sqrt(2); without the rotation the chord is 2."""
    f = _constant_field()
    sigma = math.log1p(math.e)
    o = np.array([[0.0, 0.0, -2.5]], np.float32)
    d = np.array([[0.0, 0.0, 1.0]], np.float32)
    plain = orc.render(_scene(f, None), o, d)
    np.testing.assert_allclose(plain["throughput"][0], math.exp(-2.0 * sigma), rtol=1e-12)
    rot = orc.render(_scene(_posed(f, sg.rotation((0, 1, 0), math.pi / 4), np.zeros(3)), None), o, d)
    np.testing.assert_allclose(rot["throughput"][0], math.exp(-2.0 * math.sqrt(2.0) * sigma), rtol=1e-12)
    np.testing.assert_allclose(rot["radiance"][0], 1.0 - math.exp(-2.0 * math.sqrt(2.0) * sigma), rtol=1e-11)


def test_pose_translated_box_closed_form():
    """A ray at x = 1.2 misses the box [-1, 1]^3; with the box moved by
    (0.5, 0, 0) it crosses 2 units of it."""
    f = _constant_field()
    sigma = math.log1p(math.e)
    o = np.array([[1.2, 0.0, -2.5]], np.float32)
    d = np.array([[0.0, 0.0, 1.0]], np.float32)
    miss = orc.render(_scene(f, None), o, d)
    np.testing.assert_array_equal(miss["throughput"][0], 1.0)
    np.testing.assert_array_equal(miss["radiance"][0], 0.0)
    hit = orc.render(_scene(_posed(f, np.eye(3), (0.5, 0.0, 0.0)), None), o, d)
    np.testing.assert_allclose(hit["throughput"][0], math.exp(-2.0 * sigma), rtol=1e-12)


def test_pose_random_rays_match_transformed_chords():
    """Constant medium under a general rotation and translation: every ray's
    transmittance is exp(-sigma l) for the chord of the ray mapped into the
    field's frame with numpy."""
    f = _constant_field()
    sigma = math.log1p(math.e)
    R, c = sg.rotation((1.0, 2.0, 3.0), 0.7), np.array([0.3, -0.2, 0.1])
    sc = _scene(_posed(f, R, c), None)
    o, d = sg.random_rays(300, seed=32)
    r = orc.render(sc, o, d)
    for k in range(len(o)):
        of = R.T @ (o[k].astype(np.float64) - c)
        df = R.T @ d[k].astype(np.float64)
        T = math.exp(-sigma * _chord(of, df, sc.t_near, sc.t_far))
        np.testing.assert_allclose(r["throughput"][k], T, rtol=1e-11, atol=1e-15)


def test_pose_rigid_motion_of_the_whole_scene_changes_nothing():
    """Moving field, mesh and camera rays by the same rigid motion leaves
    every ray's outcome unchanged: the field is looked up in its own frame
    with both points and directions mapped back."""
    sc = sg.tiny_scene(table_amp=1.0)
    cam = sg.cameras_array(sc.cameras)[0]
    o, d = orc.rays_from_camera(cam)
    idx = np.arange(0, len(o), 7)
    o, d = o[idx], d[idx]
    a = orc.render(sc, o.astype(np.float32), d.astype(np.float32))
    R, c = sg.rotation((0.2, 1.0, -0.4), 1.1), np.array([0.25, -0.125, 0.5])
    moved = copy.copy(sc)
    moved.field = _posed(sc.field, R, c)
    moved.mesh = copy.copy(sc.mesh)
    moved.mesh.vertices = (sc.mesh.vertices.astype(np.float64) @ R.T + c).astype(np.float32)
    ow, dw = o @ R.T + c, d @ R.T
    b = orc.render(moved, ow.astype(np.float32), dw.astype(np.float32))
    ok = ~(a["tie"] | b["tie"])
    assert ok.mean() > 0.95
    np.testing.assert_array_equal(a["hit_ids"][ok], b["hit_ids"][ok])
    np.testing.assert_array_equal(a["bounces"][ok], b["bounces"][ok])
    # FP32 rounding of the moved rays and vertices only
    np.testing.assert_allclose(b["radiance"][ok], a["radiance"][ok], rtol=2e-5, atol=1e-9)
    np.testing.assert_allclose(b["throughput"][ok], a["throughput"][ok], rtol=2e-5, atol=1e-9)


def test_pose_field_queries_exact_under_exact_motion():
    """A 90-degree turn about z and a dyadic shift are exact in FP32 and FP64:
    querying the moved field at moved points and directions gives the same
    values bit for bit."""
    f = sg.tiny_field(table_amp=1.0)
    R = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    c = np.array([0.25, -0.5, 0.125])
    rng = np.random.default_rng(33)
    x = (rng.integers(-4000, 4000, size=(500, 3)) / 4096.0).astype(np.float32)   # dyadic: shifts stay exact
    d = sg.sample_points(500, seed=34)[1]
    a = orc.field_batch(f, x, d)
    b = orc.field_batch(_posed(f, R, c), (x @ R.T + c).astype(np.float32), (d @ R.T).astype(np.float32))
    for k in ("sigma", "rgb", "feat"):
        np.testing.assert_array_equal(a[k], b[k])


# ---------------------------------------------------------------------------
# shadow mask per field sample (Sec. 3.1 "Shadow rays"): a sample a mesh hides
# from a light emits mask x its radiance
# ---------------------------------------------------------------------------

def _blocker_quad(y=1.5, half=0.5):
    v = np.array([[-half, y, -half], [half, y, -half], [half, y, half], [-half, y, half]], np.float32)
    f = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    return sg.merge_meshes([(v, f, 0)], [[sg.DIFFUSE, 1.0, 0.7, 0.7, 0.7]])


def test_sample_shadows_change_nothing_without_blockers_lights_or_strength():
    sc = sg.tiny_scene(table_amp=1.0)
    sc.lights = sg.seeded_light()
    o, d = sg.random_rays(200, seed=41)
    a = orc.render(sc, o, d)
    np.testing.assert_array_equal(a["radiance"], orc.render(sc, o, d, shadow_mask=1.0)["radiance"])
    no_mesh = orc.render(sc, o, d, mesh=None)
    np.testing.assert_array_equal(no_mesh["radiance"], orc.render(sc, o, d, mesh=None, shadow_mask=0.2)["radiance"])
    sc.lights = sg.no_lights()
    np.testing.assert_array_equal(orc.render(sc, o, d)["radiance"], orc.render(sc, o, d, shadow_mask=0.2)["radiance"])


def test_sample_shadow_closed_form_under_a_blocker():
    """Constant medium (sigma = softplus(1), colour 1) crossed along x at y = 0,
    z = 0; a quad at y = 1.5 over |x|, |z| < 0.5 and a light at (0, 5, 0): the
    segment from (x, 0, 0) to the light crosses y = 1.5 at (0.7 x, 1.5, 0), so
    exactly the samples with |x| < 0.5 / 0.7 are hidden.  L is the sum over the
    fixed grid of T alpha m with m = 0.25 for hidden midpoints."""
    f = _constant_field()
    sigma = math.log1p(math.e)
    light = np.array([[0.0, 5.0, 0.0, 10.0, 10.0, 10.0]], np.float32)
    sc = _scene(f, _blocker_quad(), light)
    o = np.array([[-2.5, 0.0, 0.0]], np.float32)
    d = np.array([[1.0, 0.0, 0.0]], np.float32)
    r = orc.render(sc, o, d, shadow_mask=0.25)
    assert r["tie"][0] == 0 and r["hit_ids"][0, 0] == -1
    delta = (sc.t_far - sc.t_near) / sc.n_samples
    lo, hi = 1.5, 3.5                    # the box chord x in [-1, 1]
    T, L = 1.0, 0.0
    for k in range(sc.n_samples):
        a, b = sc.t_near + k * delta, sc.t_near + (k + 1) * delta
        a, b = max(a, lo), min(b, hi)
        if not b > a:
            continue
        x = -2.5 + 0.5 * (a + b)
        m = 0.25 if abs(0.7 * x) < 0.5 else 1.0
        alpha = 1.0 - math.exp(-sigma * (b - a))
        L += T * alpha * m
        T *= 1.0 - alpha
    np.testing.assert_allclose(r["radiance"][0], L, rtol=1e-12)
    np.testing.assert_allclose(r["throughput"][0], T, rtol=1e-12)
    plain = orc.render(sc, o, d)
    assert plain["radiance"][0, 0] > r["radiance"][0, 0] * 1.2


def test_sample_shadow_masks_multiply_over_lights():
    """Lights at (0, 5, 0) and (0, 6, 0) over the quad: the first hides
    |x| < 0.5 / 0.7, the second |x| < 0.5 / 0.75 (the segment crosses y = 1.5
    at 0.7 x and 0.75 x), so with mask 0.5 the middle samples get 0.25, the
    samples hidden from the first light only 0.5, the others 1."""
    f = _constant_field()
    sigma = math.log1p(math.e)
    lights = np.array([[0.0, 5.0, 0.0, 1, 1, 1], [0.0, 6.0, 0.0, 1, 1, 1]], np.float32)
    sc = _scene(f, _blocker_quad(), lights)
    o = np.array([[-2.5, 0.0, 0.0]], np.float32)
    d = np.array([[1.0, 0.0, 0.0]], np.float32)
    r = orc.render(sc, o, d, shadow_mask=0.5)
    assert r["tie"][0] == 0
    delta = (sc.t_far - sc.t_near) / sc.n_samples
    T, L = 1.0, 0.0
    for k in range(sc.n_samples):
        a, b = max(sc.t_near + k * delta, 1.5), min(sc.t_near + (k + 1) * delta, 3.5)
        if not b > a:
            continue
        x = -2.5 + 0.5 * (a + b)
        m = (0.5 if abs(0.7 * x) < 0.5 else 1.0) * (0.5 if abs(0.75 * x) < 0.5 else 1.0)
        alpha = 1.0 - math.exp(-sigma * (b - a))
        L += T * alpha * m
        T *= 1.0 - alpha
    np.testing.assert_allclose(r["radiance"][0], L, rtol=1e-12)


# ---------------------------------------------------------------------------
# emitted radiance of surfaces (Eq. 12, L_e, with the segment's attenuation)
# ---------------------------------------------------------------------------

def _emitter_quad(z=0.5, half=0.6, le=(4.0, 2.0, 1.0), kind=sg.DIFFUSE, albedo=0.0):
    v = np.array([[-half, -half, z], [half, -half, z], [half, half, z], [-half, half, z]], np.float32)
    f = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    return v, f, [kind, 1.0, albedo, albedo, albedo, *le]


def test_emitter_seen_directly_and_through_a_constant_medium():
    """A black diffuse quad at z = 0.5 emitting (4, 2, 1): through empty
    space the camera ray collects exactly L_e; through the constant medium
    (sigma = softplus(1), colour 1) it collects (1 - T) + T L_e with T the
    transmittance of the chord in front of the quad."""
    v, f, mat = _emitter_quad()
    mesh = sg.merge_meshes([(v, f, 0)], [mat])
    o = np.array([[0.05, 0.02, -2.5]], np.float32)
    d = np.array([[0.0, 0.0, 1.0]], np.float32)
    empty = orc.render(_scene(None, mesh), o, d)
    np.testing.assert_allclose(empty["radiance"][0], [4.0, 2.0, 1.0], rtol=1e-15)
    assert empty["bounces"][0] == 1 and np.all(empty["throughput"][0] == 0)
    f0 = _constant_field()
    sigma = math.log1p(math.e)
    fog = orc.render(_scene(f0, mesh), o, d)
    T = math.exp(-sigma * 1.5)                     # the box from z = -1 to the quad at z = 0.5
    np.testing.assert_allclose(fog["radiance"][0], (1 - T) + T * np.array([4.0, 2.0, 1.0]), rtol=1e-12)


def test_emitter_seen_through_a_mirror_and_at_the_bounce_limit():
    """A mirror turns the camera ray onto the emitter (weight 1): L = L_e;
    with max_bounces = 0 a camera ray that stops on the emitter still
    collects its L_e."""
    v, f, mat = _emitter_quad(z=-1.5, le=(3.0, 3.0, 3.0))
    mv = np.array([[-0.7, -0.7, 0.8], [0.7, -0.7, 0.8], [0.7, 0.7, 0.8], [-0.7, 0.7, 0.8]], np.float32)
    mesh = sg.merge_meshes([(v, f, 0), (mv, f, 1)], [mat, [sg.MIRROR, 1.0, 1.0, 1.0, 1.0]])
    o = np.array([[0.05, 0.02, -1.0]], np.float32)
    d = np.array([[0.0, 0.0, 1.0]], np.float32)
    r = orc.render(_scene(None, mesh), o, d)
    np.testing.assert_allclose(r["radiance"][0], 3.0, rtol=1e-15)
    assert r["bounces"][0] == 2
    v2, f2, mat2 = _emitter_quad()
    direct = orc.render(_scene(None, sg.merge_meshes([(v2, f2, 0)], [mat2]), max_bounces=0),
                        np.array([[0.05, 0.02, -2.5]], np.float32), d)
    np.testing.assert_allclose(direct["radiance"][0], [4.0, 2.0, 1.0], rtol=1e-15)
    assert direct["bounces"][0] == 0


# ---------------------------------------------------------------------------
# light sampling toward emitting triangles (Eq. 12's L_e as area lights)
# ---------------------------------------------------------------------------

def _corner_form_factor(x, z, h):
    """Form factor from a differential area to a parallel rectangle [0, x] x
    [0, z] at height h with one corner straight above it (the classical
    closed form of radiative transfer)."""
    X, Z = x / h, z / h
    a, b = math.sqrt(1 + X * X), math.sqrt(1 + Z * Z)
    return (X / a * math.atan(Z / a) + Z / b * math.atan(X / b)) / (2 * math.pi)


def _floor_under_emitters(emitters, albedo=0.5, extra=()):
    """Diffuse floor y = 0 (its diagonal misses the origin) and emitting
    rectangles [x0, x1] x [z0, z1] at height h facing down, each with its
    radiance; the camera ray comes in low from +x and hits the floor at the
    origin."""
    fv = np.array([[-4, 0, -3], [5, 0, -3], [5, 0, 6], [-4, 0, 6]], np.float32)
    quad = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    parts, mats = [(fv, quad, 0)], [[sg.DIFFUSE, 1.0, albedo, albedo, albedo]]
    for (x0, x1, z0, z1, h, le) in emitters:
        v = np.array([[x0, h, z0], [x1, h, z0], [x1, h, z1], [x0, h, z1]], np.float32)
        parts.append((v, quad, len(mats)))
        mats.append([sg.DIFFUSE, 1.0, 0.0, 0.0, 0.0, *le])
    for v, f, mat in extra:
        parts.append((v, f, len(mats)))
        mats.append(mat)
    mesh = sg.merge_meshes(parts, mats)
    o = np.array([[3.0, 0.3, 0.0]], np.float32)
    d = -o / np.linalg.norm(o)
    return _scene(None, mesh, max_bounces=1), o, d.astype(np.float32)


def _mean_and_err(sc, o, d, n, **kw):
    r = orc.render(sc, np.repeat(o, n, 0), np.repeat(d, n, 0), ray_ids=np.arange(n), **kw)
    # the emitter choice is a tie when u0 W falls within the relative band of
    # a cumulative weight (about 2e-4 of the draws per boundary)
    assert r["tie"].mean() < 0.005
    L = r["radiance"]
    return L.mean(0), L.std(0) / math.sqrt(n), r


@pytest.mark.parametrize("sample_emitters", [True, False])
def test_light_from_a_square_emitter_matches_the_form_factor(sample_emitters):
    """Floor point under the centre of a unit square at height 1 emitting
    (2, 1, 0.5), albedo 0.5: the reflected radiance is albedo L_e F with F the
    closed-form form factor (4 corner rectangles).  Both estimators, the
    light sample and the cosine-sampled bounce that reaches the emitter, must
    agree with it within 5 standard errors over 20 000 paths; with light
    sampling the bounce's own hit of the emitter adds nothing (else the mean
    doubles)."""
    sc, o, d = _floor_under_emitters([(-0.5, 0.5, -0.5, 0.5, 1.0, (2.0, 1.0, 0.5))])
    F = 4 * _corner_form_factor(0.5, 0.5, 1.0)
    want = 0.5 * np.array([2.0, 1.0, 0.5]) * F
    mean, err, _ = _mean_and_err(sc, o, d, 20000, sample_emitters=sample_emitters)
    assert np.all(err > 0)
    assert np.all(np.abs(mean - want) < 5 * err), (mean, want, err)
    assert np.all(err < 0.02 * want)


def _dark_constant_field(sigma_offset=1.0):
    """Constant density softplus(offset) whose colour is exp(-180), zero for
    every purpose: with a zero table the colour layer sees only SH(d), whose
    first component is the constant Y00; every hidden unit is Y00 and each of
    the 64 output weights is -10."""
    f = _constant_field(sigma_offset)
    shapes = f.layer_shapes()
    off = sum(o * i for o, i in shapes[:2])
    Wc1 = f.mlp[off:off + shapes[2][0] * shapes[2][1]].reshape(shapes[2])
    Wc1[:, f.d_out] = 1.0
    off = sum(o * i for o, i in shapes[:-1])
    f.mlp[off:off + 3 * f.c_hidden] = -10.0
    return f


@pytest.mark.parametrize("sample_emitters,light_depth_samples", [(True, 0), (True, 8), (False, 0)])
def test_light_from_an_emitter_through_a_constant_medium(sample_emitters, light_depth_samples):
    """A floor point and a square emitter (2, 1, 0.5) 0.8 above it, both
    inside an absorbing constant medium (sigma = softplus(1), colour 0).  The
    reflected radiance is T_cam (albedo / pi) times the integral over the
    emitter of L_e cos_p cos_x / d^2 exp(-sigma l), where l is the path from
    the spawn point to the emitter point and T_cam the camera chord's
    transmittance.  A midpoint quadrature of 400 x 400 gives the integral.
    Both estimators must agree with it within 5 standard errors: the light
    sample carries the medium's transmittance along its shadow segment, and
    the bounce that reaches the emitter is attenuated by its own march.
    Without the factor the light-sampled mean would be 3.4 times too
    large.  The midpoint rule is exact for a constant density, so a coarse
    grid for the light samples' depth (8 intervals per segment length)
    gives the same."""
    sc, o, d = _floor_under_emitters([(-0.5, 0.5, -0.5, 0.5, 0.8, (2.0, 1.0, 0.5))])
    sc.field = _dark_constant_field()
    sigma = math.log1p(math.e)
    o64, d64 = o[0].astype(np.float64), d[0].astype(np.float64)
    t_floor = -o64[1] / d64[1]
    p = o64 + t_floor * d64
    t_in = (1.0 - o64[0]) / d64[0]                 # the camera ray enters the box at x = 1
    T_cam = math.exp(-sigma * (t_floor - t_in))
    n = 400
    g = (np.arange(n) + 0.5) / n - 0.5
    X, Z = np.meshgrid(g, g, indexing="ij")
    x = np.stack([X.ravel(), np.full(X.size, np.float32(0.8)), Z.ravel()], 1)
    so = p + np.array([0.0, 1e-4, 0.0])
    w = x - p
    dist = np.linalg.norm(w, axis=1)
    cos_p = w[:, 1] / dist
    integral = np.sum(cos_p * cos_p / dist ** 2 * np.exp(-sigma * np.linalg.norm(x - so, axis=1))) / n ** 2
    want = T_cam * 0.5 / math.pi * np.array([2.0, 1.0, 0.5]) * integral
    mean, err, r = _mean_and_err(sc, o, d, 20000, sample_emitters=sample_emitters,
                                 light_depth_samples=light_depth_samples)
    assert np.all(np.abs(mean - want) < 5 * err), (mean, want, err)
    assert np.all(err < 0.03 * want)


def test_light_sampling_weights_emitters_of_different_radiance():
    """Two emitters of different radiance and size, side by side at height 1:
    the chosen emitter's probability (by summed radiance) and its area enter
    the estimate so that the mean is albedo (L_1 F_1 + L_2 F_2), each F from
    the closed form; an offset rectangle is a difference of corner ones."""
    sc, o, d = _floor_under_emitters([(-0.5, 0.5, -0.5, 0.5, 1.0, (2.0, 1.0, 0.5)),
                                      (0.8, 1.4, -0.3, 0.3, 1.0, (1.0, 3.0, 1.0))])
    F1 = 4 * _corner_form_factor(0.5, 0.5, 1.0)
    F2 = 2 * (_corner_form_factor(1.4, 0.3, 1.0) - _corner_form_factor(0.8, 0.3, 1.0))
    want = 0.5 * (np.array([2.0, 1.0, 0.5]) * F1 + np.array([1.0, 3.0, 1.0]) * F2)
    mean, err, _ = _mean_and_err(sc, o, d, 20000, sample_emitters=True)
    assert np.all(np.abs(mean - want) < 5 * err), (mean, want, err)


def test_light_sample_blocked_by_a_mesh_is_zero():
    """A black square at y = 0.5 covering the whole cone from the floor point
    to the emitter: every light sample is blocked and the bounce ends on the
    black square, so the radiance is exactly 0."""
    blocker = (np.array([[-2, 0.5, -2], [2, 0.5, -2], [2, 0.5, 2], [-2, 0.5, 2]], np.float32),
               np.array([[0, 1, 2], [0, 2, 3]], np.int32), [sg.DIFFUSE, 1.0, 0.0, 0.0, 0.0])
    sc, o, d = _floor_under_emitters([(-0.5, 0.5, -0.5, 0.5, 1.0, (2.0, 1.0, 0.5))], extra=[blocker])
    _, _, r = _mean_and_err(sc, o, d, 2000, sample_emitters=True)
    assert np.all(r["radiance"] == 0.0)


def test_light_sampling_without_emitters_changes_nothing():
    """With no emitting triangle the option changes no bit of the output
    (its random numbers have a stream of their own), and a path that reaches
    an emitter through a mirror still collects L_e."""
    sc, o, d = _floor_under_emitters([])
    sc.lights = np.array([[0.2, 1.0, 0.1, 3.0, 2.0, 1.0]], np.float32)
    sc.max_bounces = 3
    oo, dd = np.repeat(o, 64, 0), np.repeat(d, 64, 0)
    a = orc.render(sc, oo, dd, ray_ids=np.arange(64), sample_emitters=True)
    b = orc.render(sc, oo, dd, ray_ids=np.arange(64))
    for k in ("radiance", "throughput", "bounces", "hit_ids"):
        np.testing.assert_array_equal(a[k], b[k])
    assert a["radiance"].max() > 0
    v, f, mat = _emitter_quad(z=-1.5, le=(3.0, 3.0, 3.0))
    mv = np.array([[-0.7, -0.7, 0.8], [0.7, -0.7, 0.8], [0.7, 0.7, 0.8], [-0.7, 0.7, 0.8]], np.float32)
    mesh = sg.merge_meshes([(v, f, 0), (mv, f, 1)], [mat, [sg.MIRROR, 1.0, 1.0, 1.0, 1.0]])
    r = orc.render(_scene(None, mesh), np.array([[0.05, 0.02, -1.0]], np.float32),
                   np.array([[0.0, 0.0, 1.0]], np.float32), sample_emitters=True)
    np.testing.assert_allclose(r["radiance"][0], 3.0, rtol=1e-15)


# ---------------------------------------------------------------------------
# several fields in one scene (density sum, density-weighted colour)
# ---------------------------------------------------------------------------

Y00 = 0.28209479177387814


def _tinted_field(sigma_offset, rgb, center=None):
    """Zero table: sigma = softplus(sigma_offset) everywhere in the box and a
    colour fixed by the weights from SH component Y00 (the colour MLP's
    input column d_out) through hidden unit 0 to the output layer.  Returns
    the field and its exact colour, exp(w Y00) of the stored FP32 weights."""
    f = _constant_field(sigma_offset)
    shapes = f.layer_shapes()
    assert len(shapes) == 4
    offs = np.cumsum([0] + [o * i for o, i in shapes])
    W = f.mlp[offs[2]:offs[3]].reshape(shapes[2])
    W[0, f.d_out] = 1.0
    V = f.mlp[offs[3]:offs[4]].reshape(shapes[3])
    V[:, 0] = np.log(np.asarray(rgb, np.float64)) / Y00
    colour = np.exp(V[:, 0].astype(np.float64) * Y00)
    if center is not None:
        f.pose = sg.pose_matrix(np.eye(3), center)
    return f, colour


def _fields_render(fields, o, d, **kw):
    sc = _scene(None, None, t_far=8.0, n_samples=64, max_bounces=0)
    return orc.render(sc, o, d, fields=fields, **kw)


def test_one_field_through_the_several_fields_march_is_the_single_field_march():
    """The several-fields march with one (posed) field agrees with the
    single-field march on the tiny scene's rays."""
    sc = sg.tiny_scene(table_amp=1.0)
    sc.field.pose = sg.pose_matrix(sg.rotation((0.2, 1.0, 0.1), 0.4), (0.1, -0.05, 0.0))
    o, d = orc.rays_from_camera(sg.cameras_array(sc.cameras)[0])
    o, d = o.astype(np.float32), d.astype(np.float32)
    a = orc.render(sc, o, d)
    b = orc.render(sc, o, d, fields=[sc.field])
    np.testing.assert_allclose(b["radiance"], a["radiance"], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(b["throughput"], a["throughput"], rtol=1e-12, atol=1e-15)
    np.testing.assert_array_equal(b["samples"], a["samples"])


def test_two_disjoint_fields_composite_front_to_back():
    """Field A in [-1, 1]^3 and field B moved to z in [1.5, 3.5], different
    densities and colours, ray along +z: L = c_A (1 - T_A) + T_A c_B (1 - T_B)
    with T = exp(-sigma * 2); the reverse ray sees B first."""
    fa, ca = _tinted_field(1.0, (0.9, 0.3, 0.2))
    fb, cb = _tinted_field(-0.5, (0.1, 0.6, 1.7), center=(0.0, 0.0, 2.5))
    sa, sb = math.log1p(math.exp(1.0)), math.log1p(math.exp(-0.5))
    Ta, Tb = math.exp(-2 * sa), math.exp(-2 * sb)
    o = np.array([[0.05, 0.02, -2.5], [0.05, 0.02, 5.5]], np.float32)
    d = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]], np.float32)
    r = _fields_render([fa, fb], o, d)
    np.testing.assert_allclose(r["radiance"][0], ca * (1 - Ta) + Ta * cb * (1 - Tb), rtol=1e-12)
    np.testing.assert_allclose(r["radiance"][1], cb * (1 - Tb) + Tb * ca * (1 - Ta), rtol=1e-12)
    np.testing.assert_allclose(r["throughput"], Ta * Tb, rtol=1e-12)
    r2 = _fields_render([fb, fa], o, d)                 # the list order does not matter
    np.testing.assert_allclose(r2["radiance"], r["radiance"], rtol=1e-13)


def test_overlapping_fields_add_density_and_mix_colour():
    """Field B moved to z in [0.2, 2.2] overlaps A on [0.2, 1]: there the
    density is sigma_A + sigma_B and the colour (sigma_A c_A + sigma_B c_B) /
    (sigma_A + sigma_B); the three pieces composite in closed form, exactly,
    because the grid is cut at the box faces."""
    fa, ca = _tinted_field(1.0, (0.9, 0.3, 0.2))
    fb, cb = _tinted_field(-0.5, (0.1, 0.6, 1.7), center=(0.0, 0.0, 1.2))
    sa, sb = math.log1p(math.exp(1.0)), math.log1p(math.exp(-0.5))
    o = np.array([[0.05, 0.02, -2.5]], np.float32)
    d = np.array([[0.0, 0.0, 1.0]], np.float32)
    r = _fields_render([fa, fb], o, d)
    T1, T2, T3 = math.exp(-sa * 1.2), math.exp(-(sa + sb) * 0.8), math.exp(-sb * 1.2)
    cmix = (sa * ca + sb * cb) / (sa + sb)
    want = ca * (1 - T1) + T1 * cmix * (1 - T2) + T1 * T2 * cb * (1 - T3)
    np.testing.assert_allclose(r["radiance"][0], want, rtol=1e-12)
    np.testing.assert_allclose(r["throughput"][0], T1 * T2 * T3, rtol=1e-12)


def test_field_outside_the_segment_changes_nothing():
    """A second field beyond the first surface hit, or behind the camera,
    leaves every output bit of the one-field render unchanged."""
    fa, _ = _tinted_field(1.0, (0.9, 0.3, 0.2))
    fb, _ = _tinted_field(0.0, (1.0, 1.0, 1.0), center=(0.0, 0.0, -6.0))
    o = np.array([[0.05, 0.02, -2.5], [0.3, -0.2, -2.5]], np.float32)
    d = np.array([[0.0, 0.0, 1.0], [0.1, 0.0, 0.995]], np.float32)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    a = _fields_render([fa], o, d)
    b = _fields_render([fa, fb], o, d)
    for k in ("radiance", "throughput", "samples"):
        np.testing.assert_array_equal(a[k], b[k])


def test_one_field_with_its_proposal_is_the_single_field_proposal_march():
    """Several-fields proposal path with one field equals the single-field
    proposal render bit for bit (the same march, in field order)."""
    sc = sg.tiny_scene(table_amp=1.0)
    sc.field.pose = sg.pose_matrix(sg.rotation((0.2, 1.0, 0.1), 0.4), (0.1, -0.05, 0.0))
    prop = sg.make_proposal(table_amp=0.5)
    o, d = orc.rays_from_camera(sg.cameras_array(sc.cameras)[0])
    o, d = o.astype(np.float32), d.astype(np.float32)
    a = orc.render(sc, o, d, proposal=prop, n_prop=32, n_fine=32)
    b = orc.render(sc, o, d, fields=[sc.field], field_proposals=[prop], n_prop=32, n_fine=32)
    for k in ("radiance", "throughput", "samples"):
        np.testing.assert_array_equal(a[k], b[k])


def test_two_disjoint_fields_with_proposals_composite_in_closed_form():
    """Each constant field sampled by its own (untrained) proposal: the
    proposal sampler is exact for a constant medium, so the front-to-back
    closed form holds exactly, in both ray directions and list orders."""
    fa, ca = _tinted_field(1.0, (0.9, 0.3, 0.2))
    fb, cb = _tinted_field(-0.5, (0.1, 0.6, 1.7), center=(0.0, 0.0, 2.5))
    pa, pb = sg.make_proposal(table_amp=0.5), sg.make_proposal(seed=9, table_amp=0.8)
    sa, sb = math.log1p(math.exp(1.0)), math.log1p(math.exp(-0.5))
    Ta, Tb = math.exp(-2 * sa), math.exp(-2 * sb)
    o = np.array([[0.05, 0.02, -2.5], [0.05, 0.02, 5.5]], np.float32)
    d = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]], np.float32)
    r = _fields_render([fa, fb], o, d, field_proposals=[pa, pb], n_prop=32, n_fine=24)
    np.testing.assert_allclose(r["radiance"][0], ca * (1 - Ta) + Ta * cb * (1 - Tb), rtol=1e-12)
    np.testing.assert_allclose(r["radiance"][1], cb * (1 - Tb) + Tb * ca * (1 - Ta), rtol=1e-12)
    np.testing.assert_allclose(r["throughput"], Ta * Tb, rtol=1e-12)
    r2 = _fields_render([fb, fa], o, d, field_proposals=[pb, pa], n_prop=32, n_fine=24)
    np.testing.assert_allclose(r2["radiance"], r["radiance"], rtol=1e-13)
    assert r["samples"][0] == 2 * 24
