"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances: hit triangle ids, bounce counts and occupancy bits are compared
bit-exactly on rays (cells) the oracle does not flag as ties; radiance and
throughput per channel within |a - b| <= 1e-4 |b| + 1e-7 (FP32 arithmetic
against FP64); field values with the bounds derived at each test."""
import copy
import functools
import math

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2309_04581_amd import scenegen as sg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = 1e-4
ATOL = 1e-7
# BF16 MLPs: every layer input is rounded to 8 significant bits (2^-9
# relative), and the colour is exp of the last layer, so the rounding of its
# 64 inputs moves a sample's colour by a random walk of 2^-9 |w h| terms; 2^-8
# covers two such roundings (the largest seen over 4 000 full-size rays of
# the proposal workload is 2.7e-3).
BF16_RTOL = 2.0 ** -8
# Posed (rotated) field boxes: FP32 locates a box-face crossing to about two
# ulp of t (t <= 4 on these cameras: 2 x 2.4e-7), and a crossing moves the
# radiance by sigma c (<= 2 for these fields) times that, twice per box; a ray
# that clips a box corner (a chord of ~1e-3, two samples) sees this as a
# relative error of 2e-4, so these cases add 4e-6 to the absolute floor.
CLIP_ATOL = 4e-6


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    orc.build(force=False)
    from paper_2309_04581_amd import meshrf
    meshrf.lib()


def mr():
    from paper_2309_04581_amd import meshrf
    return meshrf


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def assert_close_rel(got, want, rtol=RTOL, atol=ATOL, what=""):
    got, want = np.asarray(got, np.float64), np.asarray(want, np.float64)
    bad = np.abs(got - want) > rtol * np.abs(want) + atol
    if bad.any():
        i = np.argwhere(bad)[0]
        raise AssertionError(f"{what}: {bad.sum()} of {bad.size} outside tolerance; first at {tuple(i)}: "
                             f"got {got[tuple(i)]!r} want {want[tuple(i)]!r}")


def away_from_grid_planes(field, x, margin=1e-3):
    """Points whose every level coordinate is at least `margin` cells from a grid plane."""
    xh = (x.astype(np.float64) + 1.0) / 2.0
    ok = np.ones(len(x), bool)
    for N in field.resolutions:
        f = xh * N
        ok &= np.all(np.abs(f - np.round(f)) > margin, axis=1)
    return ok


def oracle_camera_rays(scene):
    cams = sg.cameras_array(scene.cameras)
    os_, ds_ = zip(*[orc.rays_from_camera(c) for c in cams])
    return np.concatenate(os_).astype(np.float32), np.concatenate(ds_).astype(np.float32)


def gpu_render(scene, o, d, field=None, mesh=None, table_dtype=0, mlp_dtype=0, use_occupancy=False,
               occ_res=0, max_bounces=None, per_ray=None, packets=0, **opts_kw):
    M = mr()
    fld = field if field is not None else (M.Field(scene.field, table_dtype, mlp_dtype) if scene.field is not None else None)
    msh = mesh if mesh is not None else (M.Mesh(scene.mesh) if scene.mesh is not None else None)
    if use_occupancy:
        fld.build_occupancy(occ_res, scene.occupancy_thresh)
    mb = scene.max_bounces if max_bounces is None else max_bounces
    R = M.Renderer(len(o), mb)
    opts = M.make_opts(scene, use_occupancy=use_occupancy, **opts_kw)
    opts.march_packets = packets
    R.render(fld, msh, dev(o), dev(d), scene.lights, opts,
             per_ray_max_bounces=None if per_ray is None else dev(per_ray, torch.int32))
    torch.cuda.synchronize()
    return dict(radiance=host(R.radiance), throughput=host(R.throughput), bounces=host(R.bounces),
                hit_ids=host(R.hit_ids), counters=host(R.counters))


def compare_render(g, r, what, rtol=RTOL, atol=ATOL, max_tie_frac=0.05):
    tie = r["tie"]
    ok = ~tie
    assert tie.mean() <= max_tie_frac, f"{what}: tie fraction {tie.mean():.4f}"
    np.testing.assert_array_equal(g["hit_ids"][ok], r["hit_ids"][ok], err_msg=f"{what}: hit ids")
    np.testing.assert_array_equal(g["bounces"][ok], r["bounces"][ok], err_msg=f"{what}: bounces")
    assert_close_rel(g["radiance"][ok], r["radiance"][ok], rtol, atol, what + " radiance")
    assert_close_rel(g["throughput"][ok], r["throughput"][ok], rtol, atol, what + " throughput")
    assert np.all(np.isfinite(g["radiance"])) and np.all(g["throughput"] <= 1.0 + 1e-6)
    assert np.all((g["hit_ids"] >= -1))
    if "rerun" in r:
        unmatched, tried = tie_outcomes_unmatched(g, r, rtol, atol)
        assert not unmatched, (f"{what}: {len(unmatched)} of {int(tie.sum())} tie rays reach no outcome of the "
                               f"oracle's candidates (first: ray {unmatched[0]})")
    return int(tie.sum())


def tie_outcomes_unmatched(g, r, rtol=RTOL, atol=ATOL, max_bits=6):
    """Tie rays must match one of the oracle's candidate outcomes: each is
    re-rendered by the oracle with the GPU's triangle per segment forced
    (accepted only where single precision can reach it) and with every
    combination of its first max_bits flagged scalar decisions (occupancy,
    shadow visibility, Fresnel, roulette, cut-off, emitter choice) taken
    either way.  Returns the tie rays no combination matches (hit ids and
    bounces exactly, radiance and throughput to the tolerance) and the number
    of combinations rendered."""
    idx = np.nonzero(r["tie"])[0]
    if len(idx) == 0:
        return [], 0
    stride = r["hit_ids"].shape[1]
    gh = g["hit_ids"][idx]
    fh = np.full((len(idx), stride), -1, np.int32)
    w = min(stride, gh.shape[1])
    fh[:, :w] = gh[:, :w]
    base = r["rerun"](idx, force_hits=fh, flip=np.zeros(len(idx), np.uint32))
    rows, masks = [], []
    for i, k in enumerate(np.minimum(base["n_flagged"], max_bits)):
        rows += [i] * (1 << int(k))
        masks += list(range(1 << int(k)))
    rows = np.array(rows)
    v = r["rerun"](idx[rows], force_hits=fh[rows], flip=np.array(masks, np.uint32))
    gi = {k: np.asarray(g[k])[idx][rows] for k in ("radiance", "throughput", "bounces")}

    def close(a, b):
        a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
        return np.all(np.abs(a - b) <= rtol * np.abs(b) + atol, axis=1)

    good = (~v["invalid"]) & (v["bounces"] == gi["bounces"]) & np.all(v["hit_ids"] == fh[rows], axis=1)
    good &= close(gi["radiance"], v["radiance"]) & close(gi["throughput"], v["throughput"])
    matched = np.zeros(len(idx), bool)
    np.logical_or.at(matched, rows, good)
    return [int(i) for i in idx[~matched]], len(rows)


# ---------------------------------------------------------------------------
# field queries: hash indices/features, density MLP, colour MLP
# ---------------------------------------------------------------------------

U32 = 2.0 ** -24


def feature_bound(field, amp):
    """Per-feature error bound of FP32 encoding against FP64 on the same FP32
    point: the level coordinate x_l = xhat N_l carries an absolute rounding
    error of about 2 N_l u (u = 2^-24), which moves each of the 8 trilinear
    weights by at most 3 times that; entries are bounded by amp.  Factor 4 of
    headroom for the interpolation sums."""
    b = []
    for N in field.resolutions:
        e = 4 * 8 * 3 * 2 * N * U32 * amp + 16 * U32 * amp
        b += [e] * field.feats
    return np.array(b)


def mlp_bounds(field, dfeat):
    """First-order propagation of feature errors through the MLPs (ReLU and
    softplus are 1-Lipschitz, exp turns an absolute error into a relative
    one): returns bounds for raw outputs, sigma and the log of rgb."""
    shapes = field.layer_shapes()
    Ws, off = [], 0
    for o, i in shapes:
        Ws.append(np.abs(field.mlp[off:off + o * i].astype(np.float64).reshape(o, i)))
        off += o * i
    df = np.zeros(field.d_in)
    df[:len(dfeat)] = dfeat
    draw = Ws[1] @ (Ws[0] @ df)
    dcin = np.zeros(field.c_in)
    dcin[:field.d_out] = draw
    h = Ws[2] @ dcin
    for k in range(field.c_layers - 1):
        h = Ws[3 + k] @ h
    dout = Ws[-1] @ h
    return draw, draw[0], dout


def lattice_points(field, n, seed):
    """FP32 points whose level coordinates xhat*N_l are exact in FP32 (xhat =
    j/4096, N_l <= 2048) and never integers, so FP32 and FP64 select the same
    8 corners with the same weights; directions seeded unit vectors."""
    rng = np.random.default_rng(seed)
    j = rng.integers(1, 4096, size=(4 * n, 3))
    ok = np.ones(len(j), bool)
    for N in field.resolutions:
        ok &= np.all((j * int(N)) % 4096 != 0, axis=1)
    j = j[ok][:n]
    x = (j / 4096.0 * 2.0 - 1.0).astype(np.float32)
    d = rng.normal(size=(len(x), 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return x, d.astype(np.float32)


@pytest.mark.parametrize("kind,amp", [("tiny", 1e-4), ("tiny", 1.0), ("mid", 1e-4), ("mid", 1.0)])
def test_field_query_matches_oracle(kind, amp):
    """Features, raw density outputs, sigma and rgb against the FP64 oracle on
    lattice points where both sides interpolate between the same corners with
    the same weights (indices are therefore compared exactly through the
    features).  Tolerances: features 1e-5 relative + 16 ulp of the table
    amplitude (8-term sums of rounded weight products); raw outputs 1e-4
    relative + 1e-5 of their range (FP32 dot products of <= 64 terms); sigma
    2e-5 relative; rgb 1e-4 relative."""
    M = mr()
    f = sg.tiny_field(table_amp=amp) if kind == "tiny" else sg.mid_field(table_amp=amp)
    x, d = lattice_points(f, 4000, seed=101)
    F = M.Field(f)
    out = F.query(dev(x), dev(d), want_feat=True, want_raw=True)
    ref = orc.field_batch(f, x, d)
    assert_close_rel(host(out["feat"]), ref["feat"], 1e-5, 16 * U32 * amp, "features")
    raw_scale = np.abs(ref["raw"]).max()
    assert_close_rel(host(out["raw"]), ref["raw"], 1e-4, 1e-5 * raw_scale, "raw density outputs")
    assert_close_rel(host(out["sigma"]), ref["sigma"], 2e-5, 1e-7, "sigma")
    assert_close_rel(host(out["rgb"]), ref["rgb"], 1e-4, 1e-7, "rgb")


@pytest.mark.parametrize("k", [-20, 20])
def test_fp32_engine_scales_exactly_with_power_of_two_weights(k):
    """The FP32 engine holds weights and layer inputs as exact BF16 splits.
    Scaling the density layer-1 weights by 2^k scales every piece, product and
    FP32 partial sum by 2^k, and ReLU and the second layer are positively
    homogeneous, so the raw density outputs scale by exactly 2^k (bit for
    bit), and at 2^k they still match the FP64 oracle at the FP32 tolerance
    (raw outputs 1e-4 relative + 1e-5 of their range)."""
    M = mr()
    f = sg.mid_field(table_amp=1.0)
    x, d = lattice_points(f, 4000, seed=131)
    base = M.Field(f).query(dev(x), dev(d), want_feat=False, want_raw=True)
    mlp = f.mlp.astype(np.float32).copy()
    mlp[:64 * f.d_in] *= np.float32(2.0 ** k)
    f2 = copy.copy(f)
    f2.mlp = mlp
    out = M.Field(f2).query(dev(x), dev(d), want_feat=False, want_raw=True)
    np.testing.assert_array_equal(host(out["raw"]), host(base["raw"]) * np.float32(2.0 ** k))
    ref = orc.field_batch(f2, x, d)
    raw_scale = np.abs(ref["raw"]).max()
    assert_close_rel(host(out["raw"]), ref["raw"], 1e-4, 1e-5 * raw_scale, f"raw density outputs at 2^{k}")


def test_largest_table_query_and_render_match_oracle():
    """The largest table mr_field_create accepts: 2^24 entries per level and
    16 levels, 2 GiB of FP32, so byte offsets into it pass 2^31.  Features,
    raw outputs, sigma and rgb on lattice points (tolerances as in
    test_field_query_matches_oracle; a wrong index would move a feature by
    the table amplitude), and a 24x20 render of the mid scene with that field
    against the FP64 oracle."""
    M = mr()
    f = sg.make_field(n_levels=16, feats=2, log2_table=24, n_min=16, n_max=2048, d_hidden=64, d_out=16,
                      c_hidden=64, c_layers=2, sh=16, seed=9, table_amp=1e-4)
    assert f.table.nbytes == 2 << 30
    x, d = lattice_points(f, 4000, seed=141)
    F = M.Field(f)
    out = F.query(dev(x), dev(d), want_feat=True, want_raw=True)
    ref = orc.field_batch(f, x, d)
    assert_close_rel(host(out["feat"]), ref["feat"], 1e-5, 16 * U32 * 1e-4, "features")
    raw_scale = np.abs(ref["raw"]).max()
    assert_close_rel(host(out["raw"]), ref["raw"], 1e-4, 1e-5 * raw_scale, "raw density outputs")
    assert_close_rel(host(out["sigma"]), ref["sigma"], 2e-5, 1e-7, "sigma")
    assert_close_rel(host(out["rgb"]), ref["rgb"], 1e-4, 1e-7, "rgb")
    sc = sg.mid_scene(width=24, height=20)
    sc.field = f
    o, dd = oracle_camera_rays(sc)
    r = orc.render(sc, o, dd)
    g = gpu_render(sc, o, dd, field=F)
    compare_render(g, r, "mid 24x20, 2^24-entry table")


@pytest.mark.parametrize("offset", [-9.0, -5.0, 5.0])
def test_field_query_sigma_over_the_softplus_range(offset):
    """Amplitude-1 tiny field with its density offset moved so that sigma
    spans small (softplus of -12 .. -6: the log1p term is the whole value)
    and large values; sigma within 2e-5 relative of the oracle's."""
    M = mr()
    f = sg.tiny_field(table_amp=1.0)
    f.density_offset = offset
    x, d = lattice_points(f, 4000, seed=107)
    out = M.Field(f).query(dev(x), dev(d), want_feat=False, want_raw=False)
    ref = orc.field_batch(f, x, d)
    assert ref["sigma"].min() < 1e-2 or offset > 0
    assert_close_rel(host(out["sigma"]), ref["sigma"], 2e-5, 1e-12, f"sigma offset {offset}")
    assert_close_rel(host(out["rgb"]), ref["rgb"], 1e-4, 1e-7, f"rgb offset {offset}")


@pytest.mark.parametrize("kind", ["tiny", "mid"])
def test_field_query_random_points_literal_field(kind):
    """Arbitrary FP32 points on the configured fields (table U(-1e-4, 1e-4)):
    here FP32 rounds the level coordinate (about 2 N_l ulp), and the error is
    bounded by propagating that through the trilinear weights and the MLPs."""
    M = mr()
    amp = 1e-4
    f = sg.tiny_field() if kind == "tiny" else sg.mid_field()
    x, d = sg.sample_points(5000, seed=111)
    keep = away_from_grid_planes(f, x)
    x, d = x[keep], d[keep]
    F = M.Field(f)
    out = F.query(dev(x), dev(d), want_feat=True, want_raw=True)
    ref = orc.field_batch(f, x, d)
    fb = feature_bound(f, amp)
    draw, dsig, dout = mlp_bounds(f, fb)
    assert_close_rel(host(out["feat"]), ref["feat"], 1e-5, fb[None, :], "features")
    raw_scale = np.abs(ref["raw"]).max()
    assert_close_rel(host(out["raw"]), ref["raw"], 1e-4, draw[None, :] + 1e-5 * raw_scale, "raw")
    assert_close_rel(host(out["sigma"]), ref["sigma"], 2e-5, dsig + 1e-7, "sigma")
    assert_close_rel(host(out["rgb"]), ref["rgb"], 1e-4 + dout[None, :], 1e-7, "rgb")


def test_field_query_ragged_and_empty():
    M = mr()
    f = sg.tiny_field(table_amp=1.0)
    F = M.Field(f)
    for n in (1, 63, 65, 257):
        x, d = sg.sample_points(n, seed=n)
        out = F.query(dev(x), dev(d))
        ref = orc.field_batch(f, x, d)
        assert_close_rel(host(out["sigma"]), ref["sigma"], 1e-5, 1e-6, f"sigma n={n}")
    M.mr_field_query(F.handle, 0, None, None, None)


# ---------------------------------------------------------------------------
# ray casting
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("which", ["cube", "soup", "mid", "cloth"])
def test_bvh_closest_hit_equals_brute_force(which):
    M = mr()
    mesh = {"cube": sg.mirror_cube_mesh, "soup": lambda: sg.random_triangles(64, seed=5),
            "mid": sg.mid_mesh, "cloth": lambda: sg.cloth_mesh(3)}[which]()
    o, d = sg.random_rays(3000, seed=102)
    sc = sg.tiny_scene()
    sc.max_bounces = 0
    r = orc.render(sc, o, d, field=None, mesh=mesh)
    G = M.Mesh(mesh)
    t, tri = G.closest_hit(dev(o), dev(d), t_max=sc.t_far)
    tri = host(tri)
    ok = ~r["tie"]
    # 20k small icosphere triangles: ~2% of random rays pass within 1e-5 of an edge
    assert r["tie"].mean() < 0.05
    np.testing.assert_array_equal(tri[ok], r["hit_ids"][ok, 0])
    assert (tri >= 0).sum() > 100 or which == "cube"


def test_refit_matches_brute_force_on_new_vertices():
    M = mr()
    m0 = sg.cloth_mesh(0)
    G = M.Mesh(m0)
    o, d = sg.random_rays(3000, seed=103)
    sc = sg.tiny_scene()
    sc.max_bounces = 0
    for frame in (5, 40):
        m = sg.cloth_mesh(frame)
        G.refit(dev(m.vertices))
        t, tri = G.closest_hit(dev(o), dev(d), t_max=sc.t_far)
        r = orc.render(sc, o, d, field=None, mesh=m)
        ok = ~r["tie"]
        np.testing.assert_array_equal(host(tri)[ok], r["hit_ids"][ok, 0])
        assert (host(tri) >= 0).sum() > 200


def test_camera_rays_match_oracle():
    M = mr()
    cams = sg.cameras_array(sg.multicam_cameras()[:3] + [sg.front_camera(65, 33, 4)])
    cams[:3, 10:12] = [[40, 30], [17, 9], [64, 64]]
    o, d, ci = M.camera_rays(cams)
    want = [orc.rays_from_camera(c) for c in cams]
    wo = np.concatenate([w[0] for w in want])
    wd = np.concatenate([w[1] for w in want])
    np.testing.assert_allclose(host(o), wo, atol=1e-6)
    np.testing.assert_allclose(host(d), wd, atol=2e-6)
    sizes = [int(c[10] * c[11]) for c in cams]
    np.testing.assert_array_equal(host(ci), np.repeat(np.arange(len(cams)), sizes))


# ---------------------------------------------------------------------------
# whole paths
# ---------------------------------------------------------------------------

# march_packets settings: default (camera segment as 16-ray packets), none,
# every segment
PACKETS = [0, -1, 99]


@functools.lru_cache(maxsize=None)
def _oracle_image(name):
    sc = sg.tiny_scene() if name == "tiny" else sg.mid_scene(width=48, height=40)
    o, d = oracle_camera_rays(sc)
    return sc, o, d, orc.render(sc, o, d)


@pytest.mark.parametrize("packets", PACKETS)
def test_render_tiny_scene_matches_oracle(packets):
    """The 64x64 camera, 8-level field, mirror cube, 64 samples, 4 bounces."""
    sc, o, d, r = _oracle_image("tiny")
    g = gpu_render(sc, o, d, packets=packets)
    ties = compare_render(g, r, f"tiny packets={packets}")
    assert ties < 40
    assert g["bounces"].max() == 1 and (g["hit_ids"][:, 0] >= 0).sum() > 100


def test_render_tiny_high_amplitude_field():
    """Table U(-1, 1): every gather matters (the literal field is nearly
    homogeneous).  FP32 sample positions differ from FP64 ones by ~1e-7 and
    the finest level has 256 cells per unit with features O(1); radiance is
    still compared at the 1e-4 relative bar."""
    sc = sg.tiny_scene(table_amp=1.0)
    o, d = oracle_camera_rays(sc)
    r = orc.render(sc, o, d)
    g = gpu_render(sc, o, d)
    compare_render(g, r, "tiny high amplitude")


@pytest.mark.parametrize("packets", PACKETS)
def test_render_mid_scene_small_image_matches_oracle(packets):
    """Glass icosphere, mirror cube, lit diffuse floor, 16-level field,
    256 samples, 8 bounces, on a 48x40 image of the same camera (the image
    width is not a multiple of 16, so packets straddle rows)."""
    sc, o, d, r = _oracle_image("mid")
    g = gpu_render(sc, o, d, packets=packets)
    compare_render(g, r, f"mid 48x40 packets={packets}")
    assert g["bounces"].max() >= 3
    assert (g["hit_ids"] >= 0).sum() > 500


@pytest.mark.parametrize("use_occupancy", [False, True])
def test_render_mid_scene_full_size_sampled(use_occupancy):
    """800x800 at full settings, with the occupancy grid as the benchmark
    times it (128^3, threshold 0.01, the oracle's own grid on its side: every
    cell is occupied by a margin far above FP32 noise); 4 000 seeded rays
    re-rendered one by one by the oracle."""
    sc = sg.mid_scene()
    M = mr()
    o, d, _ = M.camera_rays(sg.cameras_array(sc.cameras))
    F, G = M.Field(sc.field), M.Mesh(sc.mesh)
    bits = None
    if use_occupancy:
        F.build_occupancy(sc.occupancy_res, sc.occupancy_thresh)
        bits, margin = orc.occupancy(sc.field, sc.occupancy_res, sc.occupancy_thresh)
        assert np.abs(margin).min() > 1e-3
    R = M.Renderer(o.shape[0], sc.max_bounces)
    R.render(F, G, o, d, sc.lights, M.make_opts(sc, use_occupancy=use_occupancy))
    g = dict(radiance=host(R.radiance), throughput=host(R.throughput), bounces=host(R.bounces),
             hit_ids=host(R.hit_ids))
    rng = np.random.default_rng(104)
    idx = np.sort(rng.choice(o.shape[0], 4000, replace=False))
    oo, dd = host(o)[idx], host(d)[idx]
    r = orc.render(sc, oo, dd, ray_ids=idx, occupancy_bits=bits)
    sub = {k: v[idx] for k, v in g.items()}
    compare_render(sub, r, "mid 800x800 sample")
    # whole-image properties
    assert np.all(g["throughput"] <= 1 + 1e-6) and np.all(g["radiance"] >= 0)
    assert np.all(g["bounces"] <= sc.max_bounces)


def test_render_energy_telescopes_on_gpu():
    """colour exp(0) = 1, lossless specular surfaces, no cut-off: L + T = 1."""
    f = sg.tiny_field(table_amp=0.5)
    off = sum(a * b for a, b in f.layer_shapes()[:-1])
    f.mlp[off:] = 0.0
    sv, sf = sg.icosphere(2, radius=0.35, center=(-0.3, 0.0, 0.0))
    cv, cf = sg.cube_triangles((0.4, -0.1, 0.1), 0.4)
    mesh = sg.merge_meshes([(sv, sf, 0), (cv, cf, 1)], [[sg.GLASS, 1.5, 1, 1, 1], [sg.MIRROR, 1, 1, 1, 1]])
    sc = sg.tiny_scene()
    sc.field, sc.mesh, sc.t_min_throughput, sc.max_bounces = f, mesh, 0.0, 8
    o, d = sg.random_rays(4000, seed=105)
    g = gpu_render(sc, o, d)
    np.testing.assert_allclose(g["radiance"] + g["throughput"], 1.0, atol=2e-5)
    assert g["bounces"].max() >= 3


def test_render_edge_cases():
    """Single ray, rays that miss the field box, no mesh, no field, zero bounces."""
    sc = sg.tiny_scene()
    # rays pointing away from the box: L = 0, T = 1 exactly
    o = np.array([[0, 0, -2.5], [3, 3, 3]], np.float32)
    d = np.array([[0, 0, -1], [0.5773503, 0.5773503, 0.5773503]], np.float32)
    g = gpu_render(sc, o, d)
    np.testing.assert_array_equal(g["radiance"], 0.0)
    np.testing.assert_array_equal(g["throughput"], 1.0)
    np.testing.assert_array_equal(g["hit_ids"], -1)
    # single ray through the cube front face
    o1 = np.array([[0.05, 0.02, -2.5]], np.float32)
    d1 = np.array([[0, 0, 1]], np.float32)
    r = orc.render(sc, o1, d1)
    g = gpu_render(sc, o1, d1)
    compare_render(g, r, "single ray", max_tie_frac=1.0)
    assert g["bounces"][0] == 1
    # no mesh
    o, d = sg.random_rays(300, seed=106)
    sc2 = sg.tiny_scene(with_mesh=False)
    compare_render(gpu_render(sc2, o, d), orc.render(sc2, o, d), "no mesh")
    # no field (empty medium) with a lit diffuse floor
    sc3 = sg.mid_scene(width=8, height=8)
    sc3.field = None
    r = orc.render(sc3, o, d)
    compare_render(gpu_render(sc3, o, d), r, "empty medium")
    # zero bounces: stop at the first surface
    sc4 = sg.tiny_scene()
    sc4.max_bounces = 0
    r = orc.render(sc4, o, d)
    g = gpu_render(sc4, o, d)
    compare_render(g, r, "zero bounces")
    assert g["bounces"].max() == 0


def test_render_per_ray_bounce_limits():
    sc = sg.tiny_scene()
    sc.max_bounces = 6
    oi, di = sg.sample_points(500, seed=107, lo=-0.2, hi=0.2)     # inside the mirror box
    mb = (np.arange(500) % 7).astype(np.int32)
    r = orc.render(sc, oi, di, max_bounces=mb)
    g = gpu_render(sc, oi, di, per_ray=mb)
    compare_render(g, r, "per-ray limits")
    np.testing.assert_array_equal(g["bounces"][~r["tie"]], mb[~r["tie"]])


def test_render_is_deterministic():
    sc = sg.mid_scene(width=40, height=40, n_samples=64)
    o, d = oracle_camera_rays(sc)
    a = gpu_render(sc, o, d)
    b = gpu_render(sc, o, d)
    for k in ("radiance", "throughput", "bounces", "hit_ids", "counters"):
        np.testing.assert_array_equal(a[k], b[k])


def test_russian_roulette_matches_oracle():
    sc = sg.multicam_scene()
    sc.max_bounces = 12
    oi, di = sg.sample_points(2000, seed=108, lo=-0.2, hi=0.2)
    r = orc.render(sc, oi, di)
    g = gpu_render(sc, oi, di)
    compare_render(g, r, "roulette")
    assert (g["bounces"] > 3).any() and (g["bounces"] < 12).any()


# ---------------------------------------------------------------------------
# occupancy grid
# ---------------------------------------------------------------------------

def _sparse_field():
    f = sg.tiny_field(table_amp=1.0)
    f.density_offset = -5.0
    return f


def test_occupancy_grid_matches_oracle():
    M = mr()
    f = _sparse_field()
    F = M.Field(f)
    bits = host(F.build_occupancy(32, 0.01, export=True))
    ref, margin = orc.occupancy(f, 32, 0.01)
    certain = np.abs(margin) > 1e-5
    np.testing.assert_array_equal(bits[certain], ref[certain])
    assert 0.02 < ref.mean() < 0.98


def _unambiguous_threshold(field, res, near=0.01):
    """A threshold close to `near` in the widest gap between the cells' maximum
    densities, so that no cell sits within FP32 noise of it."""
    _, m = orc.occupancy(field, res, near)
    v = np.sort(m + near)
    w = v[(v > near * 0.9) & (v < near * 1.1)]
    gaps = np.diff(w)
    k = int(np.argmax(gaps))
    return float((w[k] + w[k + 1]) / 2)


def test_render_with_occupancy_matches_oracle():
    sc = sg.tiny_scene()
    sc.field = _sparse_field()
    sc.occupancy_thresh = _unambiguous_threshold(sc.field, 32)
    ref_bits, margin = orc.occupancy(sc.field, 32, sc.occupancy_thresh)
    assert np.abs(margin).min() > 5e-7
    o, d = oracle_camera_rays(sc)
    r = orc.render(sc, o, d, occupancy_bits=ref_bits)
    g = gpu_render(sc, o, d, use_occupancy=True, occ_res=32)
    compare_render(g, r, "occupancy", rtol=1e-3, atol=1e-6)
    full = orc.render(sc, o, d)
    assert np.abs(full["radiance"] - r["radiance"]).max() > 1e-4   # skipping changed the image


# ---------------------------------------------------------------------------
# placement of the field (a moving NeRF object)
# ---------------------------------------------------------------------------

def _posed(f, R, c):
    g = sg.Field(**{k: getattr(f, k) for k in f.__dataclass_fields__})
    g.pose = sg.pose_matrix(R, c)
    return g


@pytest.mark.parametrize("amp,rtol", [(1e-4, RTOL), (1.0, 1e-3)])
def test_render_with_field_pose_matches_oracle(amp, rtol):
    """Tiny scene with the field turned 0.9 rad about (1, 2, -1) and moved by
    (0.2, -0.1, 0.15): hit ids exact, radiance within 1e-4 relative (1e-3 for
    the amplitude-1 table, where FP32 positions matter at the finest level)
    plus 1e-6 absolute: the FP32 change of frame rounds the ray origin (|o| <=
    2.6) by about 3e-7, which moves both ends of the box-clipped chord by that
    much; with sigma = 1.31 and colour O(1) a ray that grazes an edge of the
    turned box, chord ~1e-4, carries ~8e-7 absolute error at any chord
    length."""
    sc = sg.tiny_scene(table_amp=amp)
    sc.field = _posed(sc.field, sg.rotation((1.0, 2.0, -1.0), 0.9), (0.2, -0.1, 0.15))
    o, d = oracle_camera_rays(sc)
    r = orc.render(sc, o, d)
    g = gpu_render(sc, o, d)
    compare_render(g, r, f"posed field amp={amp}", rtol=rtol, atol=1e-6)


def test_field_query_under_exact_motion_is_bit_equal():
    """A 90-degree turn about z and a dyadic shift are exact in FP32: the
    posed field queried at moved points and directions returns the unposed
    field's values bit for bit."""
    M = mr()
    f = sg.tiny_field(table_amp=1.0)
    R = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    c = np.array([0.25, -0.5, 0.125])
    rng = np.random.default_rng(35)
    x = (rng.integers(-4000, 4000, size=(3000, 3)) / 4096.0).astype(np.float32)
    d = sg.sample_points(3000, seed=36)[1]
    a = M.Field(f).query(dev(x), dev(d), want_feat=True)
    b = M.Field(_posed(f, R, c)).query(dev((x @ R.T + c).astype(np.float32)), dev((d @ R.T).astype(np.float32)),
                                       want_feat=True)
    for k in ("sigma", "rgb", "feat"):
        np.testing.assert_array_equal(host(a[k]), host(b[k]))


def test_set_pose_rejects_non_rotations():
    M = mr()
    F = M.Field(sg.tiny_field())
    with pytest.raises(M.MrError):
        F.set_pose(sg.pose_matrix(1.01 * np.eye(3), np.zeros(3)))            # scaled
    with pytest.raises(M.MrError):
        F.set_pose(sg.pose_matrix(np.diag([1.0, 1.0, -1.0]), np.zeros(3)))   # reflection
    F.set_pose(sg.pose_matrix(sg.rotation((0, 0, 1), 0.3), (0.1, 0.0, 0.0)))
    F.set_pose(None)


# ---------------------------------------------------------------------------
# shadow mask per field sample (Sec. 3.1 "Shadow rays")
# ---------------------------------------------------------------------------

def _shadow_render(sc, o, d, mask, packets=0):
    M = mr()
    F, G = M.Field(sc.field), M.Mesh(sc.mesh)
    R = M.Renderer(len(o), sc.max_bounces)
    opts = M.make_opts(sc, shadow_mask=mask)
    opts.march_packets = packets
    R.render(F, G, dev(o), dev(d), sc.lights, opts)
    torch.cuda.synchronize()
    return dict(radiance=host(R.radiance), throughput=host(R.throughput), bounces=host(R.bounces),
                hit_ids=host(R.hit_ids))


@pytest.mark.parametrize("packets", PACKETS)
def test_sample_shadows_tiny_match_oracle(packets):
    """Tiny scene with a light above the mirror cube: samples the cube hides
    from the light emit 0.2 of their radiance."""
    sc = sg.tiny_scene(table_amp=1.0)
    sc.lights = np.array([[0.1, 1.6, -0.2, 10.0, 10.0, 10.0]], np.float32)
    o, d = oracle_camera_rays(sc)
    r = orc.render(sc, o, d, shadow_mask=0.2)
    plain = orc.render(sc, o, d)
    assert (np.abs(r["radiance"] - plain["radiance"]) > 1e-3 * plain["radiance"]).any(axis=1).mean() > 0.05
    g = _shadow_render(sc, o, d, 0.2, packets)
    compare_render(g, r, f"tiny sample shadows packets={packets}", rtol=1e-3, atol=1e-6)


def test_sample_shadows_mid_small_image_match_oracle():
    """Glass sphere, mirror cube and floor under the mid scene's light, 32x24.
    Every sample's shadow ray is a geometric decision that can sit within the
    tie margin of one of the sphere's 30 000 small-triangle edges, so more
    rays are ties here (about 4%, cap 15%); non-tie rays must match."""
    sc = sg.mid_scene(width=32, height=24)
    o, d = oracle_camera_rays(sc)
    r = orc.render(sc, o, d, shadow_mask=0.1)
    g = _shadow_render(sc, o, d, 0.1)
    compare_render(g, r, "mid 32x24 sample shadows", max_tie_frac=0.15)


def test_sample_shadows_with_field_pose_match_oracle():
    """Shadow rays start at the samples' world positions when the field is
    placed elsewhere."""
    sc = sg.tiny_scene(table_amp=1.0)
    sc.lights = np.array([[0.1, 1.6, -0.2, 10.0, 10.0, 10.0]], np.float32)
    sc.field = _posed(sc.field, sg.rotation((0.0, 1.0, 0.3), 0.5), (0.1, 0.2, 0.0))
    o, d = oracle_camera_rays(sc)
    r = orc.render(sc, o, d, shadow_mask=0.2)
    compare_render(_shadow_render(sc, o, d, 0.2), r, "posed sample shadows", rtol=1e-3, atol=1e-6)


def test_sample_shadow_options_validated():
    M = mr()
    sc = sg.tiny_scene()
    sc.lights = np.array([[0.1, 1.6, -0.2, 1.0, 1.0, 1.0]], np.float32)
    o, d = oracle_camera_rays(sc)
    F, G = M.Field(sc.field), M.Mesh(sc.mesh)
    R = M.Renderer(len(o), sc.max_bounces)
    with pytest.raises(M.MrError):
        R.render(F, G, dev(o), dev(d), sc.lights, M.make_opts(sc, shadow_mask=1.5))
    with pytest.raises(M.MrError):
        R.render(F, G, dev(o), dev(d), sc.lights, M.make_opts(sc, shadow_mask=-0.1))


def test_scaling_workload_small_matches_oracle():
    """The App. A-style workload (many small inserted spheres) at 200 spheres
    and 40x20: 16 002 triangles, glass, mirror and diffuse, 8 bounces."""
    sc = sg.balls_scene(200, width=40, height=20)
    o, d = oracle_camera_rays(sc)
    r = orc.render(sc, o, d)
    g = gpu_render(sc, o, d)
    compare_render(g, r, "200 spheres 40x20")
    assert (g["hit_ids"][:, 0] >= 0).mean() > 0.1


# ---------------------------------------------------------------------------
# emitted radiance of surfaces (Eq. 12 L_e)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("packets", PACKETS)
def test_emitters_match_oracle(packets):
    """Tiny scene with an emitting quad behind the mirror cube (seen directly
    and in the cube's faces): hit ids exact, radiance within 1e-4."""
    sc = sg.tiny_scene()
    v = np.array([[-0.9, -0.9, 0.9], [0.9, -0.9, 0.9], [0.9, 0.9, 0.9], [-0.9, 0.9, 0.9]], np.float32)
    f = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    cv, cf = sg.cube_triangles((0.0, 0.0, 0.0), 0.5)
    sc.mesh = sg.merge_meshes([(cv, cf, 0), (v, f, 1)], [[sg.MIRROR, 1.0, 1.0, 1.0, 1.0],
                                                          [sg.DIFFUSE, 1.0, 0.2, 0.2, 0.2, 3.0, 2.0, 1.0]])
    o, d = oracle_camera_rays(sc)
    r = orc.render(sc, o, d)
    assert (r["radiance"][:, 0] > 1.0).mean() > 0.2
    compare_render(gpu_render(sc, o, d, packets=packets), r, f"emitters packets={packets}")


@pytest.mark.parametrize("sample_emitters,light_depth_samples", [(False, 0), (True, 0), (True, 32)])
def test_emitter_scene_small_image_matches_oracle(sample_emitters, light_depth_samples):
    """The mid scene with its emitting ceiling panel at 32x24, with and
    without light sampling toward the panel at the floor's diffuse hits, the
    light samples' optical depth on the march's grid or on a coarse one (32
    intervals per segment length)."""
    sc = sg.emitter_scene(width=32, height=24)
    o, d = oracle_camera_rays(sc)
    r = orc.render(sc, o, d, sample_emitters=sample_emitters, light_depth_samples=light_depth_samples)
    compare_render(gpu_render(sc, o, d, sample_emitters=sample_emitters, light_depth_samples=light_depth_samples),
                   r, f"emitter scene 32x24 sample_emitters={sample_emitters} depth={light_depth_samples}")


# ---------------------------------------------------------------------------
# light sampling toward emitting triangles (Eq. 12's L_e as area lights)
# ---------------------------------------------------------------------------

def _one_ray_many_paths(sc, o, d, n):
    return np.repeat(o, n, 0), np.repeat(d, n, 0)


@pytest.mark.parametrize("two,sample_emitters", [(False, True), (False, False), (True, True)])
def test_emitter_sampling_paths_match_oracle(two, sample_emitters):
    """20 000 paths of one camera ray onto a diffuse floor under one or two
    emitting rectangles (ray i draws the Philox streams of id i on both
    sides): every path's light sample or bounce matches the oracle's, and the
    GPU mean is the closed-form albedo L_e F (5 standard errors)."""
    from test_oracle_pins import _corner_form_factor, _floor_under_emitters
    em = [(-0.5, 0.5, -0.5, 0.5, 1.0, (2.0, 1.0, 0.5))]
    if two:
        em.append((0.8, 1.4, -0.3, 0.3, 1.0, (1.0, 3.0, 1.0)))
    sc, o1, d1 = _floor_under_emitters(em)
    o, d = _one_ray_many_paths(sc, o1, d1, 20000)
    r = orc.render(sc, o, d, sample_emitters=sample_emitters)
    g = gpu_render(sc, o, d, sample_emitters=sample_emitters)
    compare_render(g, r, f"emitter paths two={two} sample_emitters={sample_emitters}", rtol=1e-4, atol=1e-7,
                   max_tie_frac=0.005)
    want = 0.5 * np.array([2.0, 1.0, 0.5]) * 4 * _corner_form_factor(0.5, 0.5, 1.0)
    if two:
        want = want + 0.5 * np.array([1.0, 3.0, 1.0]) * 2 * (_corner_form_factor(1.4, 0.3, 1.0) -
                                                              _corner_form_factor(0.8, 0.3, 1.0))
    mean, err = g["radiance"].mean(0), g["radiance"].std(0) / math.sqrt(len(o))
    assert np.all(np.abs(mean - want) < 5 * err), (mean, want, err)


def test_emitter_sampling_after_refit_matches_oracle():
    """The emitter table holds probabilities by radiance only and reads areas
    from the current vertices: grow the emitter to 1.5 times its size with a
    refit and compare against the oracle on the moved mesh."""
    from test_oracle_pins import _floor_under_emitters
    sc, o1, d1 = _floor_under_emitters([(-0.5, 0.5, -0.5, 0.5, 1.0, (2.0, 1.0, 0.5))])
    o, d = _one_ray_many_paths(sc, o1, d1, 4000)
    M = mr()
    G = M.Mesh(sc.mesh)
    moved = copy.deepcopy(sc.mesh)
    moved.vertices[4:, [0, 2]] *= 1.5
    G.refit(dev(moved.vertices))
    sc2 = copy.copy(sc)
    sc2.mesh = moved
    r = orc.render(sc2, o, d, sample_emitters=True)
    compare_render(gpu_render(sc2, o, d, mesh=G, sample_emitters=True), r, "emitter sampling after refit",
                   rtol=1e-4, atol=1e-7, max_tie_frac=0.005)


# ---------------------------------------------------------------------------
# several fields in one scene (mr_render_fields)
# ---------------------------------------------------------------------------

def _fields_gpu(sc, o, d, fields=None, packets=0, use_occupancy=False, occ_res=0, proposals=None, table_dtype=0,
                mlp_dtype=0, **kw):
    M = mr()
    Fs = [M.Field(f, table_dtype=table_dtype, mlp_dtype=mlp_dtype)
          for f in (fields if fields is not None else sc.fields)]
    Ps = [M.Field(p, table_dtype=M.MR_F32) for p in proposals] if proposals is not None else None
    if Ps is not None:
        kw = dict(kw, sampler=M.MR_SAMPLER_PROPOSAL)
    if use_occupancy:
        for F in Fs:
            F.build_occupancy(occ_res, sc.occupancy_thresh)
    G = M.Mesh(sc.mesh)
    R = M.Renderer(len(o), sc.max_bounces)
    opts = M.make_opts(sc, use_occupancy=use_occupancy, **kw)
    opts.march_packets = packets
    R.render_fields(Fs, G, dev(o), dev(d), sc.lights, opts, proposals=Ps)
    torch.cuda.synchronize()
    return dict(radiance=host(R.radiance), throughput=host(R.throughput), bounces=host(R.bounces),
                hit_ids=host(R.hit_ids), counters=host(R.counters))


@pytest.mark.parametrize("spacing", [2.9, 1.2], ids=["disjoint", "overlapping"])
def test_light_samples_cross_several_fields(spacing):
    """Light sampling toward an emitting panel above three fields (amplitude-1
    tiny fields, turned; disjoint boxes, or 1.2 apart so that they overlap):
    each light sample's shadow segment is attenuated by the summed optical
    depth of the fields it crosses, against the oracle."""
    sc = sg.fields_scene(3, 48, 27, kind="tiny", table_amp=1.0, spacing=spacing)
    ev, ef, em = sg.emitter_quad(y=0.9, half=0.8, radiance=(6.0, 5.0, 4.0))
    m = sc.mesh
    sc.mesh = sg.Mesh(vertices=np.concatenate([m.vertices, ev]),
                      indices=np.concatenate([m.indices, ef + len(m.vertices)]),
                      mat_ids=np.concatenate([m.mat_ids, np.full(len(ef), len(m.materials), np.int32)]),
                      materials=np.concatenate([m.materials, sg._materials([em])]))
    o, d = oracle_camera_rays(sc)
    r = orc.render(sc, o, d, fields=sc.fields, sample_emitters=True)
    g = _fields_gpu(sc, o, d, sample_emitters=True)
    compare_render(g, r, f"3 fields spacing {spacing}, light samples toward an emitter")
    # the light samples reach the floor through the fields: some radiance comes from the panel
    plain = _fields_gpu(sc, o, d)
    assert (g["radiance"] != plain["radiance"]).any()


@pytest.mark.parametrize("n_fields,packets", [(2, 0), (3, 0), (3, -1)])
def test_several_fields_with_proposals_match_oracle(n_fields, packets):
    """Each field sampled by its own proposal (32 + 32 samples per segment,
    FP32 proposal tables): the passes use the proposal march per field and
    are composited in box order, against the oracle's front-to-back march of
    the disjoint fields."""
    sc = sg.fields_scene(n_fields, 48, 27, kind="tiny", table_amp=1.0)
    props = [sg.make_proposal(seed=5 + k, table_amp=0.5) for k in range(n_fields)]
    o, d = oracle_camera_rays(sc)
    r = orc.render(sc, o, d, fields=sc.fields, field_proposals=props, n_prop=32, n_fine=32)
    assert (r["samples"] > 0).mean() > 0.3
    g = _fields_gpu(sc, o, d, packets=packets, proposals=props)
    compare_render(g, r, f"{n_fields} fields with proposals packets={packets}", rtol=1e-3, atol=1e-6)
    assert int(g["counters"][0]) == int(r["samples"].sum())


@pytest.mark.parametrize("n_fields,packets", [(2, 0), (3, 0), (3, -1), (3, 99)])
def test_several_fields_match_oracle(n_fields, packets):
    """Two or three amplitude-1 tiny fields, turned and set side by side over
    a floor with a glass sphere and a mirror cube, 48x27: one march pass per
    field composited in box order against the oracle's summed medium; the
    field-sample count equals the oracle's."""
    sc = sg.fields_scene(n_fields, 48, 27, kind="tiny", table_amp=1.0)
    o, d = oracle_camera_rays(sc)
    r = orc.render(sc, o, d, fields=sc.fields)
    assert (r["samples"] > 0).mean() > 0.3
    g = _fields_gpu(sc, o, d, packets=packets)
    compare_render(g, r, f"{n_fields} fields packets={packets}", rtol=1e-3, atol=1e-6)
    assert int(g["counters"][0]) == int(r["samples"].sum())


def test_several_fields_with_occupancy_and_sample_shadows_match_oracle():
    """Three copies of the sparse field (its occupancy threshold in a gap of
    the cells' densities), each with its own grid, and the per-sample shadow
    mask toward the scene's light."""
    sc = sg.fields_scene(3, 48, 27, kind="tiny")
    base = _sparse_field()
    fields = []
    for f in sc.fields:
        g = copy.deepcopy(base)
        g.pose = f.pose
        fields.append(g)
    sc.fields = fields
    sc.occupancy_thresh = _unambiguous_threshold(base, 32)
    bits, margin = orc.occupancy(base, 32, sc.occupancy_thresh)
    assert np.abs(margin).min() > 5e-7
    o, d = oracle_camera_rays(sc)
    r = orc.render(sc, o, d, fields=fields, field_occupancy=[bits] * 3, shadow_mask=0.2)
    g = _fields_gpu(sc, o, d, use_occupancy=True, occ_res=32, shadow_mask=0.2)
    compare_render(g, r, "3 sparse fields, occupancy, sample shadows", rtol=1e-3, atol=1e-6)


def _overlap_fraction(fields, o, d):
    """Fraction of the rays whose line crosses a stretch shared by two boxes."""
    spans = []
    for f in fields:
        P = np.asarray(f.pose, np.float64)
        of, df = (o - P[:, 3]) @ P[:, :3], d @ P[:, :3]
        with np.errstate(divide="ignore", invalid="ignore"):
            t0 = (np.asarray(f.aabb_min, np.float64) - of) / df
            t1 = (np.asarray(f.aabb_max, np.float64) - of) / df
        spans.append((np.nanmax(np.minimum(t0, t1), axis=1), np.nanmin(np.maximum(t0, t1), axis=1)))
    both = np.zeros(len(o), bool)
    for i in range(len(fields)):
        for j in range(i + 1, len(fields)):
            both |= np.minimum(spans[i][1], spans[j][1]) > np.maximum(spans[i][0], spans[j][0])
    return both.mean()


@pytest.mark.parametrize("n_fields,spacing,packets", [(2, 1.2, 0), (3, 1.2, 0), (3, 1.2, -1), (3, 1.2, 99),
                                                      (3, 0.0, 0), (8, 0.5, 0), (8, 0.5, -1)])
def test_overlapping_fields_match_oracle(n_fields, spacing, packets):
    """Boxes that overlap (1.2 apart, all on one centre with different turns,
    which makes their y faces coincide, or the most fields, 0.5 apart): the
    fields are marched together over the summed medium (density sum,
    density-weighted colour, the grid cut at every box face), against the
    oracle's march of the same sum; the count of field evaluations equals the
    oracle's.  Packets on the camera segment (default), on no segment or on
    every segment."""
    sc = sg.fields_scene(n_fields, 48, 27, kind="tiny", table_amp=1.0, spacing=spacing)
    o, d = oracle_camera_rays(sc)
    assert _overlap_fraction(sc.fields, o.astype(np.float64), d.astype(np.float64)) > 0.04
    r = orc.render(sc, o, d, fields=sc.fields)
    assert (r["samples"] > 0).mean() > 0.15
    g = _fields_gpu(sc, o, d, packets=packets)
    compare_render(g, r, f"{n_fields} overlapping fields spacing={spacing} packets={packets}", rtol=1e-3, atol=1e-6)
    assert int(g["counters"][0]) == int(r["samples"].sum())


@pytest.mark.parametrize("packets", [0, 99])
def test_overlapping_fields_with_occupancy_and_sample_shadows_match_oracle(packets):
    """Three overlapping copies of the sparse field, each with its own
    occupancy grid, and the per-sample shadow mask toward the light; packets
    on the camera segment or on every segment."""
    sc = sg.fields_scene(3, 48, 27, kind="tiny", spacing=1.0)
    base = _sparse_field()
    fields = []
    for f in sc.fields:
        g = copy.deepcopy(base)
        g.pose = f.pose
        fields.append(g)
    sc.fields = fields
    sc.occupancy_thresh = _unambiguous_threshold(base, 32)
    bits, margin = orc.occupancy(base, 32, sc.occupancy_thresh)
    assert np.abs(margin).min() > 5e-7
    o, d = oracle_camera_rays(sc)
    assert _overlap_fraction(fields, o.astype(np.float64), d.astype(np.float64)) > 0.04
    r = orc.render(sc, o, d, fields=fields, field_occupancy=[bits] * 3, shadow_mask=0.2)
    g = _fields_gpu(sc, o, d, use_occupancy=True, occ_res=32, shadow_mask=0.2, packets=packets)
    compare_render(g, r, f"3 overlapping sparse fields, occupancy, sample shadows, packets={packets}", rtol=1e-3,
                   atol=1e-6)
    assert int(g["counters"][0]) == int(r["samples"].sum())


@pytest.mark.parametrize("seed", range(6))
def test_overlapping_fields_random_placements_match_oracle(seed):
    """2 to 5 tiny-layout fields of table amplitude 1 at seeded placements:
    any rotation axis and angle, centres within 0.9 of the origin (so boxes
    overlap, often three or more at a time), and a seeded sample count
    (64 to 200 per segment), in the several-fields scene at 40x24."""
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(2, 6))
    sc = sg.fields_scene(n, 40, 24, kind="tiny", table_amp=1.0, n_samples=int(rng.integers(64, 201)))
    for f in sc.fields:
        axis = rng.normal(size=3)
        f.pose = sg.pose_matrix(sg.rotation(axis, rng.uniform(-math.pi, math.pi)), rng.uniform(-0.9, 0.9, 3))
    o, d = oracle_camera_rays(sc)
    assert _overlap_fraction(sc.fields, o.astype(np.float64), d.astype(np.float64)) > 0.05
    r = orc.render(sc, o, d, fields=sc.fields)
    g = _fields_gpu(sc, o, d)
    compare_render(g, r, f"{n} fields at random placements, seed {seed}", rtol=1e-3, atol=1e-6)
    assert int(g["counters"][0]) == int(r["samples"].sum())


@pytest.mark.parametrize("shadow_mask", [None, 0.3])
def test_overlapping_fields_around_meshes_match_oracle(shadow_mask):
    """Two tiny-layout fields (table amplitude 1), turned and shifted so that
    their boxes overlap over most of the mid scene's meshes: bounce segments
    start inside one box or both, and the glass sphere's interior paths run
    through the shared stretch; 48x40, 128 samples, 8 bounces, with and
    without the per-sample shadow mask."""
    sc = sg.mid_scene(48, 40, n_samples=128)
    fa, fb = sg.tiny_field(1, 1.0), sg.tiny_field(2, 1.0)
    fa.pose = sg.pose_matrix(sg.rotation((0.0, 1.0, 0.0), 0.3), (-0.3, 0.0, 0.0))
    fb.pose = sg.pose_matrix(sg.rotation((0.2, 1.0, 0.1), -0.4), (0.35, 0.1, 0.0))
    sc.fields = [fa, fb]
    o, d = oracle_camera_rays(sc)
    assert _overlap_fraction(sc.fields, o.astype(np.float64), d.astype(np.float64)) > 0.3
    kw = {} if shadow_mask is None else dict(shadow_mask=shadow_mask)
    r = orc.render(sc, o, d, fields=sc.fields, **kw)
    g = _fields_gpu(sc, o, d, **kw)
    assert g["bounces"].max() >= 3
    compare_render(g, r, f"2 overlapping fields around the mid meshes, mask={shadow_mask}", rtol=1e-3, atol=1e-6)
    assert int(g["counters"][0]) == int(r["samples"].sum())


def test_overlapping_mid_fields_full_size_sampled():
    """Three mid-layout fields (16 levels, 2^19-entry tables) 1.2 apart, so
    that neighbouring boxes overlap, at the several-fields benchmark's settings
    (800x450, 516 samples per segment, 8 bounces, each field's 128^3 occupancy
    grid; the oracle uses its own grids, every cell occupied by a wide
    margin); 4 000 seeded rays re-rendered one by one by the oracle."""
    sc = sg.fields_scene(3, spacing=1.2)
    M = mr()
    o, d, _ = M.camera_rays(sg.cameras_array(sc.cameras))
    assert _overlap_fraction(sc.fields, host(o).astype(np.float64), host(d).astype(np.float64)) > 0.05
    Fs = [M.Field(f) for f in sc.fields]
    bits = []
    for F, f in zip(Fs, sc.fields):
        F.build_occupancy(sc.occupancy_res, sc.occupancy_thresh)
        b, margin = orc.occupancy(f, sc.occupancy_res, sc.occupancy_thresh)
        assert np.abs(margin).min() > 1e-3
        bits.append(b)
    G = M.Mesh(sc.mesh)
    R = M.Renderer(o.shape[0], sc.max_bounces)
    R.render_fields(Fs, G, o, d, sc.lights, M.make_opts(sc, use_occupancy=True))
    torch.cuda.synchronize()
    g = dict(radiance=host(R.radiance), throughput=host(R.throughput), bounces=host(R.bounces),
             hit_ids=host(R.hit_ids))
    rng = np.random.default_rng(106)
    idx = np.sort(rng.choice(o.shape[0], 4000, replace=False))
    r = orc.render(sc, host(o)[idx], host(d)[idx], ray_ids=idx, fields=sc.fields, field_occupancy=bits)
    assert (r["samples"] > 0).mean() > 0.2
    compare_render({k: v[idx] for k, v in g.items()}, r, "3 overlapping mid fields 800x450 sample", atol=CLIP_ATOL)
    assert np.all(g["throughput"] <= 1 + 1e-6) and np.all(g["radiance"] >= 0)


def test_several_mid_fields_full_size_sampled():
    """The several-fields benchmark at full size: three mid-layout fields 2.9
    apart (disjoint boxes, one pass per field), 800x450, 516 samples per
    segment, 8 bounces, each field's 128^3 occupancy grid (the oracle uses its
    own grids); 4 000 seeded rays re-rendered one by one by the oracle."""
    sc = sg.fields_scene(3)
    M = mr()
    o, d, _ = M.camera_rays(sg.cameras_array(sc.cameras))
    Fs = [M.Field(f) for f in sc.fields]
    bits = []
    for F, f in zip(Fs, sc.fields):
        F.build_occupancy(sc.occupancy_res, sc.occupancy_thresh)
        b, margin = orc.occupancy(f, sc.occupancy_res, sc.occupancy_thresh)
        assert np.abs(margin).min() > 1e-3
        bits.append(b)
    G = M.Mesh(sc.mesh)
    R = M.Renderer(o.shape[0], sc.max_bounces)
    R.render_fields(Fs, G, o, d, sc.lights, M.make_opts(sc, use_occupancy=True))
    torch.cuda.synchronize()
    g = dict(radiance=host(R.radiance), throughput=host(R.throughput), bounces=host(R.bounces),
             hit_ids=host(R.hit_ids))
    rng = np.random.default_rng(107)
    idx = np.sort(rng.choice(o.shape[0], 4000, replace=False))
    r = orc.render(sc, host(o)[idx], host(d)[idx], ray_ids=idx, fields=sc.fields, field_occupancy=bits)
    assert (r["samples"] > 0).mean() > 0.2
    compare_render({k: v[idx] for k, v in g.items()}, r, "3 disjoint mid fields 800x450 sample")
    assert np.all(g["throughput"] <= 1 + 1e-6) and np.all(g["radiance"] >= 0)


def test_several_mid_fields_proposal_fp16_full_size_sampled():
    """The several-fields benchmark's proposal configuration at full size:
    three mid-layout fields with FP16 tables + BF16 MLPs, each sampled by its
    own proposal (FP16 table, 32 + 32 samples), occupancy grids.  The oracle
    runs on the parameters as the GPU holds them (tables rounded to FP16,
    BF16-held layers rounded) with seeded proposals (trained weights would come
    from the GPU); 4 000 seeded rays; radiance within 2^-8 relative (the BF16
    rounding of layer inputs) and 1e-5 absolute."""
    import bench
    sc = sg.fields_scene(3)
    M = mr()
    o, d, _ = M.camera_rays(sg.cameras_array(sc.cameras))
    props = [sg.make_proposal(seed=11 + k) for k in range(3)]
    Fs = [M.Field(f, table_dtype=M.MR_F16, mlp_dtype=M.MR_BF16) for f in sc.fields]
    rounded = [bench._rounded_field(sg, f) for f in sc.fields]
    bits = []
    for F, f in zip(Fs, rounded):
        F.build_occupancy(sc.occupancy_res, sc.occupancy_thresh)
        b, margin = orc.occupancy(f, sc.occupancy_res, sc.occupancy_thresh)
        assert np.abs(margin).min() > 1e-3
        bits.append(b)
    Ps = [M.Field(p, table_dtype=M.MR_F16) for p in props]
    G = M.Mesh(sc.mesh)
    R = M.Renderer(o.shape[0], sc.max_bounces)
    opts = M.make_opts(sc, sampler=M.MR_SAMPLER_PROPOSAL, use_occupancy=True)
    R.render_fields(Fs, G, o, d, sc.lights, opts, proposals=Ps)
    torch.cuda.synchronize()
    g = dict(radiance=host(R.radiance), throughput=host(R.throughput), bounces=host(R.bounces),
             hit_ids=host(R.hit_ids))
    propr = []
    for p in props:
        q = copy.deepcopy(p)
        q.table = p.table.astype(np.float16).astype(np.float32)
        propr.append(q)
    rng = np.random.default_rng(108)
    idx = np.sort(rng.choice(o.shape[0], 4000, replace=False))
    r = orc.render(sc, host(o)[idx], host(d)[idx], ray_ids=idx, fields=rounded, field_occupancy=bits,
                   field_proposals=propr, n_prop=32, n_fine=32)
    assert (r["samples"] > 0).mean() > 0.2
    compare_render({k: v[idx] for k, v in g.items()}, r, "3 mid fields, proposals, fp16 800x450 sample",
                   rtol=BF16_RTOL, atol=1e-5)
    assert np.all(g["throughput"] <= 1 + 1e-6) and np.all(g["radiance"] >= 0)


def test_several_fields_of_different_layouts_match_oracle():
    """Disjoint fields of different layouts under the uniform sampler take one
    pass per field (the joint march needs one layout): a tiny field with an
    FP32 table beside two with FP16 tables, against the oracle with those
    tables rounded to FP16."""
    M = mr()
    sc = sg.fields_scene(3, 48, 27, kind="tiny", table_amp=1.0)
    o, d = oracle_camera_rays(sc)
    rounded = [sc.fields[0]] + [copy.deepcopy(f) for f in sc.fields[1:]]
    for f in rounded[1:]:
        f.table = f.table.astype(np.float16).astype(np.float32)
    r = orc.render(sc, o, d, fields=rounded)
    Fs = [M.Field(sc.fields[0])] + [M.Field(f, table_dtype=M.MR_F16) for f in sc.fields[1:]]
    G = M.Mesh(sc.mesh)
    R = M.Renderer(len(o), sc.max_bounces)
    R.render_fields(Fs, G, dev(o), dev(d), sc.lights, M.make_opts(sc))
    torch.cuda.synchronize()
    g = dict(radiance=host(R.radiance), throughput=host(R.throughput), bounces=host(R.bounces),
             hit_ids=host(R.hit_ids), counters=host(R.counters))
    compare_render(g, r, "3 fields of two layouts", rtol=1e-3, atol=1e-6)
    assert int(g["counters"][0]) == int(r["samples"].sum())


def test_one_field_list_is_mr_render():
    """mr_render_fields with one field is mr_render, bit for bit."""
    sc = sg.tiny_scene(table_amp=1.0)
    o, d = oracle_camera_rays(sc)
    a = gpu_render(sc, o, d)
    b = _fields_gpu(sc, o, d, fields=[sc.field])
    for k in ("radiance", "throughput", "bounces", "hit_ids"):
        np.testing.assert_array_equal(a[k], b[k])


def test_several_fields_validated():
    """Overlapping boxes with the proposal sampler or with fields of different
    layouts, the proposal sampler without one proposal per field (or with a
    field that is no proposal), more than 8 fields and a missing occupancy
    grid are refused; overlapping boxes under the uniform sampler and boxes
    that touch are accepted."""
    M = mr()
    sc = sg.tiny_scene()
    o, d = oracle_camera_rays(sc)
    G = M.Mesh(sc.mesh)
    R = M.Renderer(len(o), sc.max_bounces)

    def placed(x, angle=0.0):
        f = copy.deepcopy(sc.field)
        f.pose = sg.pose_matrix(sg.rotation((0.0, 1.0, 0.0), angle), (x, 0.0, 0.0))
        return M.Field(f)
    opts = M.make_opts(sc)
    R.render_fields([placed(0.0), placed(2.0)], G, dev(o), dev(d), sc.lights, opts)    # touching
    R.render_fields([placed(0.0), placed(1.9)], G, dev(o), dev(d), sc.lights, opts)    # overlapping
    R.render_fields([placed(0.0), placed(2.3, math.pi / 4)], G, dev(o), dev(d), sc.lights, opts)
    R.render_fields([placed(0.0), placed(2.5, math.pi / 4)], G, dev(o), dev(d), sc.lights, opts)
    def placed_f16(x):
        f = copy.deepcopy(sc.field)
        f.pose = sg.pose_matrix(np.eye(3), (x, 0.0, 0.0))
        return M.Field(f, table_dtype=M.MR_F16)
    with pytest.raises(M.MrError, match="layout"):   # an FP16 table overlapping an FP32 one
        R.render_fields([placed(0.0), placed_f16(1.0)], G, dev(o), dev(d), sc.lights, opts)
    R.render_fields([placed(0.0), placed_f16(3.0)], G, dev(o), dev(d), sc.lights, opts)   # disjoint: accepted
    P = M.Field(sg.make_proposal(), table_dtype=M.MR_F32)
    popts = M.make_opts(sc, sampler=M.MR_SAMPLER_PROPOSAL, proposal=P)
    with pytest.raises(M.MrError, match="overlap"):
        R.render_fields([placed(0.0), placed(1.9)], G, dev(o), dev(d), sc.lights, popts, proposals=[P, P])
    with pytest.raises(M.MrError, match="one proposal per field"):
        R.render_fields([placed(0.0), placed(3.0)], G, dev(o), dev(d), sc.lights, popts)
    R.render_fields([placed(0.0), placed(3.0)], G, dev(o), dev(d), sc.lights, popts, proposals=[P, P])
    with pytest.raises(M.MrError):   # a full field is no proposal
        R.render_fields([placed(0.0), placed(3.0)], G, dev(o), dev(d), sc.lights, popts,
                        proposals=[P, placed(6.0)])
    with pytest.raises(M.MrError):
        R.render_fields([placed(3.0 * k) for k in range(9)], G, dev(o), dev(d), sc.lights, opts)
    with pytest.raises(M.MrError):
        R.render_fields([placed(0.0), placed(3.0)], G, dev(o), dev(d), sc.lights, M.make_opts(sc, use_occupancy=True))
