"""Learned proposal sampler on the GPU against the FP64 oracle: training
targets, loss and gradient, proposal-sampled rendering, and what training
gains over the untrained proposal and over uniform sampling at equal budget."""
import functools
import math

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2309_04581_amd import scenegen as sg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from test_gpu_parity import BF16_RTOL, assert_close_rel, compare_render, dev, host, mr, oracle_camera_rays  # noqa: E402,E501


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    orc.build(force=False)


def psnr_tonemapped(a, b):
    """PSNR of Reinhard L/(1+L) followed by the sRGB transfer curve, peak 1."""
    def psi(L):
        x = np.clip(L / (1.0 + L), 0.0, 1.0)
        return np.where(x <= 0.0031308, 12.92 * x, 1.055 * np.power(x, 1 / 2.4) - 0.055)
    mse = np.mean((psi(np.asarray(a, np.float64)) - psi(np.asarray(b, np.float64))) ** 2)
    return math.inf if mse == 0 else 10.0 * math.log10(1.0 / mse)


def test_targets_match_oracle():
    M = mr()
    f = sg.shell_field()
    o, d = sg.random_rays(600, seed=301)
    F = M.Field(f)
    P = M.Field(sg.make_proposal(), table_dtype=M.MR_F16)
    T = M.ProposalTrainer(P)
    lohi, tgt = T.targets(F, dev(o), dev(d), 0.05, 4.0, 256)
    rl, rt = orc.proposal_targets(f, o, d, 0.05, 4.0, 256, 32)
    assert_close_rel(host(lohi), rl, 1e-6, 1e-6, "segment ranges")
    assert_close_rel(host(tgt), rt, 2e-3, 2e-5, "target histograms")
    np.testing.assert_allclose(host(tgt).sum(1), rt.sum(1), rtol=1e-3, atol=1e-5)


# bins per segment: the trained proposal's 32 (also at the training batch of
# 2^14 segments, in the launch shape the training step uses), a full 64-lane
# wave, and a count that leaves part of the last matrix-core K group empty
@pytest.mark.parametrize("n_bins,n", [(32, 512), (32, 1 << 14), (64, 3000), (20, 3000)])
def test_proposal_gradient_matches_oracle(n_bins, n):
    """GPU loss and gradient (FP32; MLP weight gradient accumulated on the
    matrix cores, table gradient by atomics) against the FP64 analytic
    gradient, which is itself pinned to finite differences on the CPU."""
    M = mr()
    prop = sg.make_proposal(table_amp=0.3)
    rng = np.random.default_rng(302 + n_bins)
    o, d = sg.random_rays(n, seed=303)
    lohi = np.stack([rng.uniform(1.4, 1.8, n), rng.uniform(3.0, 3.4, n)], 1).astype(np.float32)
    tgt = (rng.dirichlet(np.ones(n_bins) * 0.3, size=n) * 0.9).astype(np.float32)
    P = M.Field(prop, table_dtype=M.MR_F16)
    loss = torch.zeros(1, device="cuda")
    gt = torch.zeros(prop.table.size, device="cuda")
    gm = torch.zeros(prop.mlp.size, device="cuda")
    M.mr_proposal_grad(P.handle, n, dev(o), dev(d), dev(lohi), dev(tgt), n_bins, loss, gt, gm)
    rl, rgt, rgm = orc.proposal_loss(prop, o, d, lohi, tgt)
    assert float(host(loss)[0]) == pytest.approx(rl, rel=1e-4)
    # per-element FP32 rounding tolerance of this gradient (probabilistic
    # rounding error analysis; pinned in the oracle tests)
    bt, bm = orc.proposal_grad_bound(prop, o, d, lohi, tgt)
    gmh = host(gm).astype(np.float64)
    gth = host(gt).reshape(prop.table.shape).astype(np.float64)
    for name, got, ref, tol in (("MLP", gmh, rgm, bm), ("table", gth, rgt, bt)):
        err = np.abs(got - ref)
        bad = np.flatnonzero(err > tol)
        print(f"{name} gradient: largest error / rounding bound {np.max(err / np.maximum(tol, 1e-300)):.3f}")
        assert bad.size == 0, (f"{name} gradient: {bad.size} elements beyond the rounding bound, e.g. "
                               f"{[(int(i), got.flat[i], ref.flat[i], tol.flat[i]) for i in bad[:4]]}")
    assert (np.abs(rgt) > 0).sum() > 1000


@functools.lru_cache(maxsize=None)
def _proposal_oracle(fieldkind, n_fine):
    sc = sg.tiny_scene()
    if fieldkind == "shell":
        sc.field = sg.shell_field()
    prop = sg.make_proposal(table_amp=0.5)
    o, d = oracle_camera_rays(sc)
    return sc, prop, o, d, orc.render(sc, o, d, proposal=prop, n_prop=32, n_fine=n_fine)


# (field, fine samples, march_packets): the camera segment in 16-ray packets
# (default), no packets, packets on every segment, and 24 fine samples per
# segment in packets
@pytest.mark.parametrize("fieldkind,n_fine,packets", [("tiny", 32, 0), ("shell", 32, 0), ("tiny", 32, -1),
                                                      ("shell", 32, -1), ("shell", 32, 99), ("shell", 24, 0)])
def test_proposal_sampled_render_matches_oracle(fieldkind, n_fine, packets):
    """32 proposal + n_fine fine samples per segment, same proposal parameters
    on both sides (FP32 table): hit ids/bounces exact, radiance within 1e-4
    (1e-3 for the shell field, whose density varies within a cell)."""
    M = mr()
    sc, prop, o, d, r = _proposal_oracle(fieldkind, n_fine)
    F, G = M.Field(sc.field), M.Mesh(sc.mesh)
    P = M.Field(prop, table_dtype=M.MR_F32)
    R = M.Renderer(len(o), sc.max_bounces)
    opts = M.make_opts(sc, sampler=M.MR_SAMPLER_PROPOSAL, proposal=P, n_fine=n_fine)
    opts.march_packets = packets
    R.render(F, G, dev(o), dev(d), sc.lights, opts)
    g = dict(radiance=host(R.radiance), throughput=host(R.throughput), bounces=host(R.bounces),
             hit_ids=host(R.hit_ids))
    tol = 1e-4 if fieldkind == "tiny" else 1e-3
    compare_render(g, r, f"proposal {fieldkind} n_fine={n_fine} packets={packets}", rtol=tol, atol=1e-6)


def test_training_gains_over_untrained_and_uniform():
    """Train on the shell field's plain-marcher histograms; the trained
    proposal's 32 + 32 samples must beat (PSNR against the 256-sample plain
    image) both the untrained proposal and 64 uniform samples."""
    M = mr()
    sc = sg.tiny_scene()
    sc.field = sg.shell_field()
    sc.mesh = None
    F = M.Field(sc.field)
    P = M.Field(sg.make_proposal(), table_dtype=M.MR_F16)
    T = M.ProposalTrainer(P)
    to, td = sg.random_rays(1 << 16, seed=304)
    to, td = dev(to), dev(td)
    lohi, tgt = T.targets(F, to, td, sc.t_near, sc.t_far, 256)
    o, d = oracle_camera_rays(sc)
    o, d = dev(o), dev(d)

    def render(sampler, prop=None, n_samples=256):
        sc.n_samples = n_samples
        R = M.Renderer(o.shape[0], sc.max_bounces)
        R.render(F, None, o, d, sc.lights, M.make_opts(sc, sampler=sampler, proposal=prop))
        return host(R.radiance)

    plain = render(M.MR_SAMPLER_UNIFORM, n_samples=256)
    uniform64 = render(M.MR_SAMPLER_UNIFORM, n_samples=64)
    untrained = render(M.MR_SAMPLER_PROPOSAL, P)
    hist = host(T.train(to, td, lohi, tgt, steps=400, batch=1 << 14))
    trained = render(M.MR_SAMPLER_PROPOSAL, P)
    p_u64, p_un, p_tr = (psnr_tonemapped(x, plain) for x in (uniform64, untrained, trained))
    print(f"loss {hist[0]:.4g} -> {hist[-1]:.4g}; PSNR vs 256-sample plain: uniform-64 {p_u64:.2f} dB, "
          f"untrained proposal {p_un:.2f} dB, trained proposal {p_tr:.2f} dB")
    assert hist[-20:].mean() < 0.2 * hist[:20].mean()
    assert p_tr >= 40.0
    assert p_tr > p_un + 3.0
    assert p_tr > p_u64 + 3.0


def test_proposal_render_with_field_pose_matches_oracle():
    """The proposal is evaluated in the frame of the field it samples for:
    shell field turned and moved, 32 + 32 samples, against the oracle."""
    M = mr()
    sc = sg.tiny_scene()
    f = sg.shell_field()
    f.pose = sg.pose_matrix(sg.rotation((0.3, 1.0, 0.2), 0.6), (0.1, 0.05, -0.1))
    sc.field = f
    prop = sg.make_proposal(table_amp=0.5)
    o, d = oracle_camera_rays(sc)
    r = orc.render(sc, o, d, proposal=prop, n_prop=32, n_fine=32)
    F, G = M.Field(sc.field), M.Mesh(sc.mesh)
    P = M.Field(prop, table_dtype=M.MR_F32)
    R = M.Renderer(len(o), sc.max_bounces)
    R.render(F, G, dev(o), dev(d), sc.lights, M.make_opts(sc, sampler=M.MR_SAMPLER_PROPOSAL, proposal=P))
    g = dict(radiance=host(R.radiance), throughput=host(R.throughput), bounces=host(R.bounces),
             hit_ids=host(R.hit_ids))
    compare_render(g, r, "proposal posed shell", rtol=1e-3, atol=1e-6)


# (field, march_packets): the proposal march in packets on the camera segment
# only (default), per ray on every segment, and in packets on every segment
@pytest.mark.parametrize("fieldkind,packets", [("tiny", 0), ("tiny", -1), ("shell", 99)])
def test_proposal_render_with_sample_shadows_matches_oracle(fieldkind, packets):
    """Per-sample shadow mask (Sec. 3.1) with the proposal sampler: each fine
    sample the mirror cube hides from the light above it emits 0.2 of its
    radiance; 32 + 32 samples, against the oracle."""
    M = mr()
    sc = sg.tiny_scene(table_amp=1.0)
    if fieldkind == "shell":
        sc.field = sg.shell_field()
    sc.lights = np.array([[0.1, 1.6, -0.2, 10.0, 10.0, 10.0]], np.float32)
    prop = sg.make_proposal(table_amp=0.5)
    o, d = oracle_camera_rays(sc)
    r = orc.render(sc, o, d, proposal=prop, n_prop=32, n_fine=32, shadow_mask=0.2)
    plain = orc.render(sc, o, d, proposal=prop, n_prop=32, n_fine=32)
    assert (np.abs(r["radiance"] - plain["radiance"]) > 1e-3 * plain["radiance"]).any(axis=1).mean() > 0.05
    F, G = M.Field(sc.field), M.Mesh(sc.mesh)
    P = M.Field(prop, table_dtype=M.MR_F32)
    R = M.Renderer(len(o), sc.max_bounces)
    opts = M.make_opts(sc, sampler=M.MR_SAMPLER_PROPOSAL, proposal=P, shadow_mask=0.2)
    opts.march_packets = packets
    R.render(F, G, dev(o), dev(d), sc.lights, opts)
    g = dict(radiance=host(R.radiance), throughput=host(R.throughput), bounces=host(R.bounces),
             hit_ids=host(R.hit_ids))
    tol = 1e-4 if fieldkind == "tiny" else 1e-3
    compare_render(g, r, f"proposal {fieldkind} sample shadows packets={packets}", rtol=tol, atol=1e-6)


@pytest.mark.parametrize("table_amp", [1e-4, 1.0])
def test_proposal_render_with_light_sampling_matches_oracle(table_amp):
    """The emitter scene (mid meshes and field, ceiling panel) at 32x24 under
    the proposal sampler with light sampling toward the panel: the fine
    samples come from the seeded proposal, the light samples' transmittance
    from the uniform grid of the march, against the oracle."""
    M = mr()
    sc = sg.emitter_scene(width=32, height=24)
    if table_amp != 1e-4:
        sc.field = sg.mid_field(2, table_amp)
    prop = sg.make_proposal(table_amp=0.5)
    o, d = oracle_camera_rays(sc)
    r = orc.render(sc, o, d, proposal=prop, n_prop=32, n_fine=32, sample_emitters=True)
    F, G = M.Field(sc.field), M.Mesh(sc.mesh)
    P = M.Field(prop, table_dtype=M.MR_F32)
    R = M.Renderer(len(o), sc.max_bounces)
    R.render(F, G, dev(o), dev(d), sc.lights,
             M.make_opts(sc, sampler=M.MR_SAMPLER_PROPOSAL, proposal=P, sample_emitters=True))
    g = dict(radiance=host(R.radiance), throughput=host(R.throughput), bounces=host(R.bounces),
             hit_ids=host(R.hit_ids))
    tol = 1e-4 if table_amp < 1e-3 else 1e-3
    compare_render(g, r, f"proposal + light sampling amp {table_amp}", rtol=tol, atol=1e-6)


def test_proposal_fp16_full_size_sampled():
    """The benchmark's second configuration at full size: 800x800 mid scene,
    FP16 table + BF16 MLPs, FP16 proposal table, 32 + 32 samples, occupancy
    grid, default packets.  The oracle runs on the parameters as the GPU holds
    them (table and proposal table rounded to FP16, BF16-held layers rounded)
    with a seeded proposal (trained weights would come from the GPU); 4 000
    seeded rays.  Hit ids and bounces exact off ties; radiance within 2^-8
    relative (the BF16 rounding of layer inputs) and 1e-5 absolute."""
    import bench
    M = mr()
    sc = sg.mid_scene()
    prop = sg.make_proposal()
    o, d, _ = M.camera_rays(sg.cameras_array(sc.cameras))
    F = M.Field(sc.field, table_dtype=M.MR_F16, mlp_dtype=M.MR_BF16)
    F.build_occupancy(sc.occupancy_res, sc.occupancy_thresh)
    P = M.Field(prop, table_dtype=M.MR_F16)
    G = M.Mesh(sc.mesh)
    R = M.Renderer(o.shape[0], sc.max_bounces)
    R.render(F, G, o, d, sc.lights, M.make_opts(sc, sampler=M.MR_SAMPLER_PROPOSAL, proposal=P, use_occupancy=True))
    g = dict(radiance=host(R.radiance), throughput=host(R.throughput), bounces=host(R.bounces),
             hit_ids=host(R.hit_ids))
    scr = sg.mid_scene()
    scr.field = bench._rounded_field(sg, sc.field)
    propr = sg.make_proposal()
    propr.table = prop.table.astype(np.float16).astype(np.float32)
    bits, margin = orc.occupancy(scr.field, sc.occupancy_res, sc.occupancy_thresh)
    assert np.abs(margin).min() > 1e-3
    rng = np.random.default_rng(106)
    idx = np.sort(rng.choice(o.shape[0], 4000, replace=False))
    r = orc.render(scr, host(o)[idx], host(d)[idx], ray_ids=idx, occupancy_bits=bits, proposal=propr,
                   n_prop=32, n_fine=32)
    compare_render({k: v[idx] for k, v in g.items()}, r, "proposal fp16 800x800 sample", rtol=BF16_RTOL,
                   atol=1e-5)
    assert np.all(g["throughput"] <= 1 + 1e-6) and np.all(g["radiance"] >= 0)
