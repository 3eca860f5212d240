#!/usr/bin/env python3
"""Throughput of the hybrid surface-volumetric marcher on one MI355X.

Workload (mid scene): 800x800 pinhole camera, 16-level hash grid (2^19
entries, 2 features, resolutions 16..2048, FP32), density MLP 32->64->16,
colour MLP (16 + 16 SH)->64->64->3, 128^3 occupancy grid (cells with density
>= 0.01 somewhere are marched), 256 uniform samples per segment on
[0.05, 4.0], glass icosphere (20 480 triangles) + mirror cube + diffuse floor
(20 494 triangles, SAH BVH), one point light with one shadow ray per diffuse
hit, up to 8 bounces.  Synthetic seeded inputs stand in for the paper's
captured scenes.

One step = camera ray generation + the whole bounce loop (closest hit, march,
shade/compaction per bounce) for all 640 000 primary rays, with field, mesh
and workspace resident in HBM.  Prints one JSON line.
"""
import argparse
import dataclasses
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rays/sec (full bounce paths) plain FP32 vs proposal+FP16 at >=40 dB PSNR"
HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3   # MI355X published dense FP32 matrix peak
BF16_MFMA_PEAK_TFLOPS = 2500.0  # MI355X published dense BF16 matrix peak
PROPOSAL_MACS = 10 * 16 + 16 * 1        # proposal MLP 10 -> 16 -> 1 per proposal sample


# Sources that make up the march kernels and their launches: the fabric traffic
# taken with rocprofv3 counters is reported only while they are unchanged since
# the counters were taken.  (The public header only declares the C ABI; the
# march takes nothing from it but enum constants.)
MARCH_SOURCES = ["march_mfma.hip", "mr_mfma.h", "mr_field_kernels.h", "mr_device.h", "mr_render.h",
                 "mr_common.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_march_mid_fabric_traffic.md")


def march_sources_sha256():
    h = hashlib.sha256()
    for f in MARCH_SOURCES:
        with open(os.path.join(ROOT, "paper_2309_04581_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


TRAFFIC_KEYS = ("traffic_bytes_per_launch", "camera_segment_fabric_bytes", "bounce_segments_fabric_bytes")


def measured_traffic(key="traffic_bytes_per_launch"):
    """Fabric bytes of the march (L2-to-memory read requests counted by size,
    32 / 64 / 128 bytes, plus write requests) from the committed counter
    summary: per launch, or one step's bytes on the camera segment or on the
    bounce segments; None when the march sources have changed since it was
    taken."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as fh:
            for ln in fh:
                if ":" in ln and ln.split(":", 1)[0].strip() in TRAFFIC_KEYS + ("march_sources_sha256",):
                    k, v = ln.split(":", 1)
                    kv[k.strip()] = v.strip().strip("`")
        if kv.get("march_sources_sha256") != march_sources_sha256():
            return None
        return int(float(kv[key]))
    except (OSError, KeyError, ValueError):
        return None


def field_macs(f):
    """Real multiply-accumulates per field sample (density + colour MLPs),
    counting only the non-padded inputs."""
    nfeat = f.n_levels * f.feats
    macs = nfeat * f.d_hidden + f.d_hidden * f.d_out
    macs += (f.d_out + f.sh) * f.c_hidden + (f.c_layers - 1) * f.c_hidden * f.c_hidden + 3 * f.c_hidden
    return macs


def split_macs(f):
    """Multiply-accumulates per sample that run on the matrix cores as FP32
    split into three BF16 pieces (six BF16 products each): the density layers
    and the hidden colour layers; the SH columns of colour layer 1 are a
    per-ray FP32 product and the 3-wide output layer runs on the vector units."""
    nfeat = f.n_levels * f.feats
    return nfeat * f.d_hidden + f.d_hidden * f.d_out + f.d_out * f.c_hidden + (f.c_layers - 1) * f.c_hidden * f.c_hidden


def gather_bytes(f, bytes_per_value=4):
    return f.n_levels * 8 * f.feats * bytes_per_value


def gather_probe(M, sg, F_mid):
    """Random-gather ceilings (mr_probe_gather): 2^28 table-entry loads at
    pseudo-random positions from the mid table (FP32, 64 MiB: Infinity Cache),
    its FP16 copy (32 MiB) and the tiny table (FP32, 1 MiB: L2)."""
    import torch
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    F16 = M.Field(sg.mid_field(), table_dtype=M.MR_F16, mlp_dtype=M.MR_BF16)
    Ft = M.Field(sg.tiny_field())
    out = {}
    for name, F, eb in (("mid_fp32_64MiB", F_mid, 8), ("mid_fp16_32MiB", F16, 4), ("tiny_fp32_1MiB", Ft, 8)):
        M.mr_probe_gather(F.handle, 1 << 26, 11, sink)          # warm the caches
        ms, loads = M.mr_probe_gather(F.handle, 1 << 28, 12, sink)
        out[name] = {"GB_per_s": round(loads * eb / (ms / 1e3) / 1e9, 1),
                     "Gloads_per_s": round(loads / (ms / 1e3) / 1e9, 2), "entry_bytes": eb}
    # the same loads confined to a region of the mid table, shared by every die
    # or one region per die (blocks go to the eight dies in turn): the rate as
    # a function of what each die's L2 has to hold
    reg = {}
    for lg in (17, 19, 20, 21):
        for per_die in (False, True):
            if per_die and lg + 3 > 23:
                continue
            M.mr_probe_gather_region(F_mid.handle, lg, per_die, 1 << 25, 13, sink)
            ms, loads = M.mr_probe_gather_region(F_mid.handle, lg, per_die, 1 << 27, 14, sink)
            key = f"{(8 << lg) >> 20}MiB_{'per_die' if per_die else 'shared'}"
            reg[key] = round(loads / (ms / 1e3) / 1e9, 2)
    out["mid_fp32_region_Gloads_per_s"] = reg
    return out


def psnr_tonemapped(a, b):
    """PSNR after Reinhard L/(1+L) and the sRGB transfer curve, peak 1."""
    import numpy as np

    def psi(L):
        x = np.clip(L / (1.0 + L), 0.0, 1.0)
        return np.where(x <= 0.0031308, 12.92 * x, 1.055 * np.power(x, 1 / 2.4) - 0.055)
    mse = float(np.mean((psi(np.asarray(a, np.float64)) - psi(np.asarray(b, np.float64))) ** 2))
    return float("inf") if mse == 0 else 10.0 * math.log10(1.0 / mse)


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def proposal_variant(M, sg, sc, F_plain, G, cams, n, plain_img, steps, warmup, train_steps):
    """Proposal (32 + 32) with FP16 table and BF16 MLPs on the same workload,
    trained on the plain marcher's histograms; PSNR against the plain image."""
    import torch
    F16 = M.Field(sc.field, table_dtype=M.MR_F16, mlp_dtype=M.MR_BF16)
    F16.build_occupancy(sc.occupancy_res, sc.occupancy_thresh)
    P = M.Field(sg.make_proposal(), table_dtype=M.MR_F16)
    T = M.ProposalTrainer(P)
    to, td = sg.random_rays(1 << 18, seed=505)
    to = torch.from_numpy(to).cuda()
    td = torch.from_numpy(td).cuda()
    lohi, tgt = T.targets(F_plain, to, td, sc.t_near, sc.t_far, sc.n_samples)
    t0 = time.perf_counter()
    hist = T.train(to, td, lohi, tgt, steps=train_steps, batch=1 << 14).cpu().numpy()
    train_s = time.perf_counter() - t0
    o = torch.empty(n, 3, device="cuda")
    d = torch.empty(n, 3, device="cuda")
    R = M.Renderer(n, sc.max_bounces, with_hits=False)
    opts_default = M.make_opts(sc, sampler=M.MR_SAMPLER_PROPOSAL, proposal=P, use_occupancy=True)
    # launch shape from the library's autotuner, as for the plain frame
    key = M.autotune_key("mid-proposal", sc.field.resolutions.tobytes(), len(sc.mesh.indices), n, sc.max_bounces,
                         cams.tobytes(), sc.occupancy_res)
    cache = os.path.join(os.environ.get("XDG_CACHE_HOME", os.path.expanduser("~/.cache")), "meshrf_autotune.json")
    os.makedirs(os.path.dirname(cache), exist_ok=True)
    search = {}

    def tune():
        t_s = time.perf_counter()
        M.mr_rays_from_cameras(cams, o, d, None, n)
        shape, tms, ms0, nt = M.mr_autotune_search(F16.handle, G.handle, n, o, d, sc.max_bounces, None, sc.lights,
                                                   opts_default, R.out, R.workspace, R.ws_bytes, reps=2, passes=2)
        search.update({"shapes_timed": nt, "search_s": round(time.perf_counter() - t_s, 2),
                       "default_ms_in_search": round(ms0, 3), "tuned_ms_in_search": round(tms, 3)})
        return shape, tms
    shape, _, hit = M.autotune_cached(cache, key, tune)
    opts = M.apply_launch(M.make_opts(sc, sampler=M.MR_SAMPLER_PROPOSAL, proposal=P, use_occupancy=True), shape)

    def step_default():
        M.mr_rays_from_cameras(cams, o, d, None, n)
        R.render(F16, G, o, d, sc.lights, opts_default)
    ms_default = timed(step_default, steps, warmup)

    def step():
        M.mr_rays_from_cameras(cams, o, d, None, n)
        R.render(F16, G, o, d, sc.lights, opts)
    ms = timed(step, steps, warmup)
    img = R.radiance.cpu().numpy()
    names = ("march_blocks_per_cu", "stage_blocks_per_cu", "stage_tile", "march_chunk", "march_batch",
             "march_packets")
    launch = {"shape": dict(zip(names, shape)), "autotuned": True, "cache_hit": hit, **search,
              "default_shape": {"value": round(n / (ms_default / 1e3), 1), "unit": "rays/s",
                                "ms_per_step": round(ms_default, 3)}}
    stage_ms, stage_n, counters = profiled(M, step, steps, R)
    fine = int(counters[0])
    prop = fine                             # 32 proposal intervals and 32 fine samples per marched segment
    march_ms = stage_ms[1] + stage_ms[3]            # later segments + camera segment
    march_s = march_ms / steps / 1e3
    flops = 2.0 * (field_macs(sc.field) * fine + PROPOSAL_MACS * prop)
    gbytes = (gather_bytes(sc.field, 2) * fine + 5 * 8 * 2 * 2 * prop) / 1e9
    roof = {"kernel": "k_march_prop_pk (camera segment) + k_march_prop (later segments)", "bound": "mfma",
            "achieved": round(flops / march_s / 1e12, 2), "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(flops / march_s / 1e12 / BF16_MFMA_PEAK_TFLOPS, 4),
            "gather_GB_per_s": round(gbytes / march_s, 1), "peak_hbm": HBM_PEAK_GBS,
            "fine_samples_per_step": fine, "proposal_samples_per_step": prop,
            "launch_ms": round(march_ms / max(1, stage_n[1] + stage_n[3]), 4),
            "stage_ms_per_step": {"closest_hit": round(stage_ms[0] / steps, 3), "march": round(march_ms / steps, 3),
                                  "shade": round(stage_ms[2] / steps, 3)},
            "camera_segment": {"kernel": "k_march_prop_pk", "ms_per_step": round(stage_ms[3] / steps, 3)},
            "bounce_segments": {"kernel": "k_march_prop", "ms_per_step": round(stage_ms[1] / steps, 3)}}
    # the uniform sampler on the same FP16 / BF16 engine: 256 samples (the plain count) and 64
    # (the proposal's budget of 32 + 32)
    uniform = {}
    for ns in (256, 64):
        scu = dataclasses.replace(sc, n_samples=ns)
        uopts = M.make_opts(scu, use_occupancy=True)

        def ustep():
            M.mr_rays_from_cameras(cams, o, d, None, n)
            R.render(F16, G, o, d, sc.lights, uopts)
        ums = timed(ustep, steps, 1)
        uniform[f"uniform_{ns}"] = {"value": round(n / (ums / 1e3), 1), "unit": "rays/s", "ms_per_step": round(ums, 3),
                                    "psnr_db_vs_plain_fp32": round(psnr_tonemapped(R.radiance.cpu().numpy(),
                                                                                   plain_img), 2)}
    # the same trained proposal with the per-sample shadow mask (0.2)
    opts_sh = M.make_opts(sc, sampler=M.MR_SAMPLER_PROPOSAL, proposal=P, use_occupancy=True, shadow_mask=0.2)

    def step_sh():
        M.mr_rays_from_cameras(cams, o, d, None, n)
        R.render(F16, G, o, d, sc.lights, opts_sh)
    ms_sh = timed(step_sh, steps, 1)
    return {"value": round(n / (ms / 1e3), 1), "unit": "rays/s", "ms_per_step": round(ms, 3),
            "launch_shape": launch,
            "with_sample_shadows": {"value": round(n / (ms_sh / 1e3), 1), "unit": "rays/s",
                                    "ms_per_step": round(ms_sh, 3), "mask": 0.2},
            "psnr_db_vs_plain_fp32": round(psnr_tonemapped(img, plain_img), 2),
            "samples": "32 proposal + 32 fine per segment", "table": "fp16", "mlp": "bf16 (MFMA, fp32 accumulate)",
            "roofline": roof, "fp16_bf16_engine_uniform_sampler": uniform,
            "train": {"steps": train_steps, "batch_segments": 1 << 14, "loss_first": float(hist[0]),
                      "loss_last": float(hist[-1]), "seconds": round(train_s, 2)}}


def profiled(M, step, steps, R):
    """The steps once more with per-stage event timing on (a pass of its own,
    so that timed headline steps carry no events): per-stage ms and launches,
    and the render counters of the last step."""
    import torch
    torch.cuda.synchronize()
    M.mr_profile_read()
    M.mr_profile_enable(True)
    try:
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
    finally:
        M.mr_profile_enable(False)
    stage_ms, stage_n = M.mr_profile_read()
    return stage_ms, stage_n, R.counters.cpu().numpy()


def shell_proposal(M, sg, steps, train_steps):
    """Where the samples go matters here: a field whose density sits on a thin
    spherical shell (the tiny layout; sigma = softplus(-4) off the shell, about
    softplus(26) on it) among the mid scene's meshes and light, 800x800, 8
    bounces.  The 256-sample plain FP32 image is the reference; 64 uniform
    samples and the trained proposal's 32 + 32 take the same budget of field
    evaluations, in FP32 and on the FP16 / BF16 engine."""
    import torch
    sc = dataclasses.replace(sg.mid_scene(), field=sg.shell_field(), name="shell")
    cams = sg.cameras_array(sc.cameras)
    n = sc.n_rays
    F = M.Field(sc.field)
    F16 = M.Field(sc.field, table_dtype=M.MR_F16, mlp_dtype=M.MR_BF16)
    for f in (F, F16):
        f.build_occupancy(sc.occupancy_res, sc.occupancy_thresh)
    G = M.Mesh(sc.mesh)
    P = M.Field(sg.make_proposal(), table_dtype=M.MR_F16)
    T = M.ProposalTrainer(P)
    to, td = sg.random_rays(1 << 18, seed=508)
    to, td = torch.from_numpy(to).cuda(), torch.from_numpy(td).cuda()
    lohi, tgt = T.targets(F, to, td, sc.t_near, sc.t_far, sc.n_samples)
    hist = T.train(to, td, lohi, tgt, steps=train_steps, batch=1 << 14).cpu().numpy()
    o = torch.empty(n, 3, device="cuda")
    d = torch.empty(n, 3, device="cuda")
    R = M.Renderer(n, sc.max_bounces, with_hits=False)

    def run(field, opts):
        def step():
            M.mr_rays_from_cameras(cams, o, d, None, n)
            R.render(field, G, o, d, sc.lights, opts)
        ms = timed(step, steps, 1)
        return ms, R.radiance.cpu().numpy()
    ms_ref, ref = run(F, M.make_opts(sc, use_occupancy=True))
    out = {"plain_256_fp32": {"value": round(n / (ms_ref / 1e3), 1), "unit": "rays/s", "ms_per_step": round(ms_ref, 3)}}
    sc64 = dataclasses.replace(sc, n_samples=64)
    for name, field, opts in (
            ("uniform_64_fp32", F, M.make_opts(sc64, use_occupancy=True)),
            ("proposal_32_32_fp32", F, M.make_opts(sc, sampler=M.MR_SAMPLER_PROPOSAL, proposal=P, use_occupancy=True)),
            ("uniform_64_fp16_bf16", F16, M.make_opts(sc64, use_occupancy=True)),
            ("proposal_32_32_fp16_bf16", F16,
             M.make_opts(sc, sampler=M.MR_SAMPLER_PROPOSAL, proposal=P, use_occupancy=True))):
        ms, img = run(field, opts)
        out[name] = {"value": round(n / (ms / 1e3), 1), "unit": "rays/s", "ms_per_step": round(ms, 3),
                     "psnr_db_vs_plain_256_fp32": round(psnr_tonemapped(img, ref), 2)}
    out["train"] = {"steps": train_steps, "batch_segments": 1 << 14, "loss_first": float(hist[0]),
                    "loss_last": float(hist[-1])}
    return out


def _rounded_field(sg, f):
    """The field's parameters as the FP16-table / BF16-MLP engine holds them:
    table rounded to FP16; density layers, the raw-feature columns of colour
    layer 1 and the hidden colour layer rounded to BF16 (round-to-nearest-even);
    the SH columns of colour layer 1 and the 3-wide output layer stay FP32 (the
    engine applies them in FP32, once per ray and on the vector units)."""
    import numpy as np

    def bf16(a):
        u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
        return ((((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32)).view(np.float32)

    g = sg.Field(**{k: getattr(f, k) for k in f.__dataclass_fields__})
    g.table = f.table.astype(np.float16).astype(np.float32)
    mlp = np.array(f.mlp, dtype=np.float32, copy=True)
    off = 0
    for i, (o, n) in enumerate(f.layer_shapes()):
        W = mlp[off:off + o * n].reshape(o, n)
        if i == 2:
            W[:, :f.d_out] = bf16(W[:, :f.d_out])
        elif i < len(f.layer_shapes()) - 1:
            W[:] = bf16(W)
        off += o * n
    g.mlp = mlp
    return g


def precision_report(M, sg):
    """Tiny workload, FP32 and FP16 table + BF16 MLPs, against the FP64 oracle
    on the master (FP32) parameters (total error) and, for FP16/BF16, on the
    rounded parameters (arithmetic error only); for the configured field
    (table amplitude 1e-4, nearly homogeneous) and its amplitude-1 twin."""
    import copy
    import numpy as np
    import torch
    from oracle import oracle as orc
    out = {}
    for label, amp in (("table_amp_1e-4", 1e-4), ("table_amp_1", 1.0)):
        sc = sg.tiny_scene(table_amp=amp)
        cam = sg.cameras_array(sc.cameras)[0]
        o, d = orc.rays_from_camera(cam)
        o, d = o.astype(np.float32), d.astype(np.float32)
        t0 = time.perf_counter()
        ref = orc.render(sc, o, d)
        oracle_s = time.perf_counter() - t0
        scr = copy.copy(sc)
        scr.field = _rounded_field(sg, sc.field)
        ref_r = orc.render(scr, o, d)
        res = {"oracle_full_image": {"rays": len(o), "seconds": round(oracle_s, 3),
                                     "rays_per_s": round(len(o) / oracle_s, 1), "cores": orc.n_threads_default()}}
        for name, td, md in (("fp32", M.MR_F32, M.MR_F32), ("fp16_table_bf16_mlp", M.MR_F16, M.MR_BF16)):
            F, G = M.Field(sc.field, td, md), M.Mesh(sc.mesh)
            R = M.Renderer(len(o), sc.max_bounces)
            R.render(F, G, torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda(), sc.lights, M.make_opts(sc))
            torch.cuda.synchronize()
            L = R.radiance.cpu().numpy().astype(np.float64)
            hits = R.hit_ids.cpu().numpy()
            entry = {}
            for which, rr in (("vs_master_params", ref), ("vs_rounded_params", ref_r)):
                if which == "vs_rounded_params" and name == "fp32":
                    continue
                ok = ~rr["tie"]
                rel = np.abs(L[ok] - rr["radiance"][ok]) / np.abs(rr["radiance"][ok])
                entry[which] = {"max_rel_err": float(rel.max()), "mean_rel_err": float(rel.mean()),
                                "hit_ids_bit_exact_non_tie": bool(np.array_equal(hits[ok], rr["hit_ids"][ok])),
                                "tie_rays": int((~ok).sum())}
            res[name] = entry
        out[label] = res
    return out


def tuned(M, opts, shape):
    """The plain mid frame's autotuned launch shape on a variant of that frame."""
    return M.apply_launch(opts, shape) if shape is not None else opts


def moving_field(M, sg, sc, F, G, cams, n, steps, shape=None):
    """The mid workload with the field as a moving object: a different rigid
    placement (turning about y, drifting along x) on every step, set with
    mr_field_set_pose between renders."""
    import torch
    o = torch.empty(n, 3, device="cuda")
    d = torch.empty(n, 3, device="cuda")
    R = M.Renderer(n, sc.max_bounces, with_hits=False)
    opts = tuned(M, M.make_opts(sc, use_occupancy=True), shape)
    poses = [sg.pose_matrix(sg.rotation((0.0, 1.0, 0.0), 0.05 * k), (0.02 * k, 0.0, 0.0)) for k in range(16)]
    state = {"k": 0}

    def step():
        F.set_pose(poses[state["k"] % len(poses)])
        state["k"] += 1
        M.mr_rays_from_cameras(cams, o, d, None, n)
        R.render(F, G, o, d, sc.lights, opts)
    try:
        ms = timed(step, steps, 1)
    finally:
        F.set_pose(None)
    return {"value": round(n / (ms / 1e3), 1), "unit": "rays/s", "ms_per_step": round(ms, 3),
            "motion": "turn 0.05 rad about y and move 0.02 along x per step",
            "launch_shape": "the plain mid frame's autotuned shape" if shape is not None else "default"}


def sample_shadows(M, sg, sc, F, G, cams, n, steps, mask=0.2, shape=None):
    """The mid workload with the paper's per-sample shadow mask: every field
    sample sends a ray to the light (one any-hit traversal per sample)."""
    import torch
    o = torch.empty(n, 3, device="cuda")
    d = torch.empty(n, 3, device="cuda")
    R = M.Renderer(n, sc.max_bounces, with_hits=False)
    opts = tuned(M, M.make_opts(sc, use_occupancy=True, shadow_mask=mask), shape)

    def step():
        M.mr_rays_from_cameras(cams, o, d, None, n)
        R.render(F, G, o, d, sc.lights, opts)
    ms = timed(step, steps, 1)
    c = R.counters.cpu().numpy()
    return {"value": round(n / (ms / 1e3), 1), "unit": "rays/s", "ms_per_step": round(ms, 3),
            "shadow_rays_per_s": round(int(c[0]) * len(sc.lights) / (ms / 1e3), 1), "mask": mask,
            "launch_shape": "the plain mid frame's autotuned shape" if shape is not None else "default"}


def scaling(M, sg, steps):
    """After the paper's App. A: rays/s and frame time with 1 .. 10^4 inserted
    spheres (80 triangles each) at 900x450 over the mid field, and with the
    image size swept at 100 spheres; the host BVH build time and the device
    bytes of BVH, triangles and render workspace per configuration."""
    import torch
    sc0 = sg.balls_scene(1)
    F = M.Field(sc0.field)
    F.build_occupancy(sc0.occupancy_res, sc0.occupancy_thresh)

    def run(sc):
        cams = sg.cameras_array(sc.cameras)
        n = sc.n_rays
        t0 = time.perf_counter()
        G = M.Mesh(sc.mesh)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        o = torch.empty(n, 3, device="cuda")
        d = torch.empty(n, 3, device="cuda")
        R = M.Renderer(n, sc.max_bounces, with_hits=False)
        opts = M.make_opts(sc, use_occupancy=True)

        def step():
            M.mr_rays_from_cameras(cams, o, d, None, n)
            R.render(F, G, o, d, sc.lights, opts)
        ms = timed(step, steps, 1)
        info = G.info()
        nodes = info["n_nodes"]
        tris = len(sc.mesh.indices)
        return {"rays": n, "triangles": tris, "bvh_depth": info["depth"], "ms_per_frame": round(ms, 3),
                "rays_per_s": round(n / (ms / 1e3), 1), "bvh_build_s": round(build_s, 3),
                "device_mib": round((nodes * 64 + tris * 48 + R.ws_bytes) / 2 ** 20, 1)}
    out = {"spheres_900x450": {}, "pixels_at_100_spheres": {}}
    for nb in (1, 10, 100, 1000, 10000):
        out["spheres_900x450"][str(nb)] = run(sg.balls_scene(nb))
    for w, h in ((225, 112), (450, 225), (900, 450), (1800, 900)):
        out["pixels_at_100_spheres"][f"{w}x{h}"] = run(sg.balls_scene(100, w, h))
    return out


def emitters(M, sg, steps, shape=None):
    """The mid workload with an emitting ceiling panel (Eq. 12 L_e) next to the
    point light: 800x800, 8 bounces, plain FP32."""
    import torch
    sc = sg.emitter_scene()
    cams = sg.cameras_array(sc.cameras)
    n = sc.n_rays
    F, G = M.Field(sc.field), M.Mesh(sc.mesh)
    F.build_occupancy(sc.occupancy_res, sc.occupancy_thresh)
    o = torch.empty(n, 3, device="cuda")
    d = torch.empty(n, 3, device="cuda")
    R = M.Renderer(n, sc.max_bounces, with_hits=False)
    opts = tuned(M, M.make_opts(sc, use_occupancy=True), shape)

    def step():
        M.mr_rays_from_cameras(cams, o, d, None, n)
        R.render(F, G, o, d, sc.lights, opts)
    ms = timed(step, steps, 1)
    mean = [round(float(x), 5) for x in R.radiance.mean(0).cpu().numpy()]
    # light sampling toward the panel's triangles at every diffuse hit
    opts_ls = tuned(M, M.make_opts(sc, use_occupancy=True, sample_emitters=True), shape)

    def step_ls():
        M.mr_rays_from_cameras(cams, o, d, None, n)
        R.render(F, G, o, d, sc.lights, opts_ls)
    ms_ls = timed(step_ls, steps, 1)
    mean_ls = [round(float(x), 5) for x in R.radiance.mean(0).cpu().numpy()]
    # the same with the light samples' optical depth on a coarse grid (32 intervals per segment length)
    opts_c = tuned(M, M.make_opts(sc, use_occupancy=True, sample_emitters=True, light_depth_samples=32), shape)

    def step_c():
        M.mr_rays_from_cameras(cams, o, d, None, n)
        R.render(F, G, o, d, sc.lights, opts_c)
    ms_c = timed(step_c, steps, 1)
    return {"value": round(n / (ms / 1e3), 1), "unit": "rays/s", "ms_per_step": round(ms, 3), "mean_radiance": mean,
            "with_light_sampling": {"value": round(n / (ms_ls / 1e3), 1), "unit": "rays/s",
                                    "ms_per_step": round(ms_ls, 3), "mean_radiance": mean_ls,
                                    "light_depth_grid": "the march's, 256 intervals per segment length"},
            "with_light_sampling_coarse_depth": {
                "value": round(n / (ms_c / 1e3), 1), "unit": "rays/s", "ms_per_step": round(ms_c, 3),
                "mean_radiance": [round(float(x), 5) for x in R.radiance.mean(0).cpu().numpy()],
                "light_depth_grid": "32 intervals per segment length"},
            "launch_shape": "the plain mid frame's autotuned shape" if shape is not None else "default"}


def several_fields(M, sg, steps, n_fields=3, train_steps=0):
    """Several NeRF objects in one scene (mr_render_fields): three mid-layout
    fields (64 MiB tables each), turned and side by side, over a floor with a
    glass sphere and a mirror cube, 800x450, 8 bounces, plain FP32 with each
    field's occupancy grid; then the same fields 1.2 apart, where neighbouring
    boxes overlap and the fields are marched together."""
    import torch
    sc = sg.fields_scene(n_fields)
    cams = sg.cameras_array(sc.cameras)
    n = sc.n_rays
    Fs = [M.Field(f) for f in sc.fields]
    for F in Fs:
        F.build_occupancy(sc.occupancy_res, sc.occupancy_thresh)
    G = M.Mesh(sc.mesh)
    o = torch.empty(n, 3, device="cuda")
    d = torch.empty(n, 3, device="cuda")
    R = M.Renderer(n, sc.max_bounces, with_hits=False)
    opts = M.make_opts(sc, use_occupancy=True)

    def step():
        M.mr_rays_from_cameras(cams, o, d, None, n)
        R.render_fields(Fs, G, o, d, sc.lights, opts)
    ms = timed(step, steps, 1)
    c = R.counters.cpu().numpy()
    out = {"value": round(n / (ms / 1e3), 1), "unit": "rays/s", "ms_per_step": round(ms, 3), "fields": n_fields,
           "rays": n, "samples_per_step": int(c[0]), "samples_per_s": round(int(c[0]) / (ms / 1e3), 1)}
    plain_img = R.radiance.cpu().numpy()
    # the same fields 1.2 apart: neighbouring boxes overlap, and all fields are
    # marched together over the summed medium (one ray per wave)
    sco = sg.fields_scene(n_fields, spacing=1.2)
    Fo = [M.Field(f) for f in sco.fields]
    for F in Fo:
        F.build_occupancy(sco.occupancy_res, sco.occupancy_thresh)
    oopts = M.make_opts(sco, use_occupancy=True)

    def step_o():
        M.mr_rays_from_cameras(cams, o, d, None, n)
        R.render_fields(Fo, G, o, d, sco.lights, oopts)
    ms_o = timed(step_o, steps, 1)
    c = R.counters.cpu().numpy()
    out["overlapping"] = {"value": round(n / (ms_o / 1e3), 1), "unit": "rays/s", "ms_per_step": round(ms_o, 3),
                          "spacing": 1.2, "field_samples_per_step": int(c[0]),
                          "field_samples_per_s": round(int(c[0]) / (ms_o / 1e3), 1)}
    del Fo
    if train_steps > 0:
        # each field sampled by its own proposal (32 + 32), trained on that field
        # in its own frame; FP16 tables + BF16 MLPs; PSNR against the plain image
        import dataclasses
        F16s, props = [], []
        for k, f in enumerate(sc.fields):
            F16 = M.Field(f, table_dtype=M.MR_F16, mlp_dtype=M.MR_BF16)
            F16.build_occupancy(sc.occupancy_res, sc.occupancy_thresh)
            F16s.append(F16)
            local = M.Field(dataclasses.replace(f, pose=None))
            P = M.Field(sg.make_proposal(), table_dtype=M.MR_F16)
            T = M.ProposalTrainer(P)
            to, td = sg.random_rays(1 << 18, seed=507 + k)
            to, td = torch.from_numpy(to).cuda(), torch.from_numpy(td).cuda()
            lohi, tgt = T.targets(local, to, td, 0.05, 4.0, 256)
            T.train(to, td, lohi, tgt, steps=train_steps, batch=1 << 14)
            props.append(P)
        popts = M.make_opts(sc, sampler=M.MR_SAMPLER_PROPOSAL, use_occupancy=True)

        def step_p():
            M.mr_rays_from_cameras(cams, o, d, None, n)
            R.render_fields(F16s, G, o, d, sc.lights, popts, proposals=props)
        ms_p = timed(step_p, steps, 1)
        out["proposal_fp16"] = {"value": round(n / (ms_p / 1e3), 1), "unit": "rays/s", "ms_per_step": round(ms_p, 3),
                                "psnr_db_vs_plain_fp32": round(psnr_tonemapped(R.radiance.cpu().numpy(), plain_img), 2),
                                "samples": "32 proposal + 32 fine per field and segment", "train_steps": train_steps}
    return out


def multicam(M, sg, steps):
    """16 cameras of uneven size and bounce depth in one queue, replayed as a
    graph, with the launch shape (march and stage grids, stage tile, march
    queue chunk and batch, packet segments) chosen by the library's autotuner
    (coordinate descent over its own candidates, cached per architecture and
    workload); the default shape is timed beside it."""
    import numpy as np
    import torch
    sc = sg.multicam_scene()
    cams = sg.cameras_array(sc.cameras)
    o, d, ci = M.camera_rays(cams)
    n = o.shape[0]
    limits = np.array([c.max_bounces for c in sc.cameras], np.int32)
    mb = torch.empty(n, dtype=torch.int32, device="cuda")
    M.mr_camera_bounce_limits(ci, n, limits, mb)
    F, G = M.Field(sc.field), M.Mesh(sc.mesh)
    mbmax = int(limits.max())
    R = M.Renderer(n, mbmax, with_hits=False)
    opts = M.make_opts(sc)
    key = M.autotune_key("multicam", cams.tobytes(), limits.tobytes(), sc.field.resolutions.tobytes(),
                         len(sc.mesh.indices), sc.n_samples, sc.rr_after)
    cache = os.path.join(os.environ.get("XDG_CACHE_HOME", os.path.expanduser("~/.cache")), "meshrf_autotune.json")
    os.makedirs(os.path.dirname(cache), exist_ok=True)
    search = {}

    def tune():
        t0 = time.perf_counter()
        shape, ms, ms0, nt = M.mr_autotune_search(F.handle, G.handle, n, o, d, mbmax, mb, sc.lights, opts, R.out,
                                                  R.workspace, R.ws_bytes, reps=1, passes=2)
        search.update({"shapes_timed": nt, "search_s": round(time.perf_counter() - t0, 2),
                       "default_ms_in_search": round(ms0, 3)})
        return shape, ms
    shape, tuned_ms, hit = M.autotune_cached(cache, key, tune)

    def graph_ms(o_):
        g = M.mr_render_graph_create(F.handle, G.handle, n, o, d, mbmax, mb, sc.lights, o_, R.out,
                                     R.workspace, R.ws_bytes)
        try:
            return timed(lambda: M.mr_graph_launch(g), steps, 1)
        finally:
            M.mr_graph_destroy(g)
    ms_default = graph_ms(opts)
    ms = graph_ms(M.apply_launch(M.make_opts(sc), shape))
    c = R.counters.cpu().numpy()
    names = ("march_blocks_per_cu", "stage_blocks_per_cu", "stage_tile", "march_chunk", "march_batch",
             "march_packets")
    return {"value": round(n / (ms / 1e3), 1), "unit": "rays/s", "rays": n, "ms_per_frame": round(ms, 3),
            "segments_per_s": round(int(c[1]) / (ms / 1e3), 1), "graph": True,
            "autotuned": {"shape": dict(zip(names, shape)), "cache_hit": hit, "key": key, **search,
                          "candidates": dict(zip(names, M.mr_autotune_candidates(n)))},
            "default_shape": {"value": round(n / (ms_default / 1e3), 1), "unit": "rays/s",
                              "ms_per_frame": round(ms_default, 3)},
            "bounce_histogram": np.bincount(R.bounces.cpu().numpy(), minlength=17).tolist()}


def cloth(M, sg, frames, train_steps):
    """Cloth of 7 938 triangles with a BVH refit every frame, 800x800, 8
    bounces, on the tiny field: plain FP32 (256 samples) and proposal (32 + 32,
    trained on the tiny field's plain-marcher histograms) with FP16 table +
    BF16 MLPs; PSNR of the proposal image against the plain one per frame."""
    import numpy as np
    import torch
    sc = sg.cloth_scene(0)
    cams = sg.cameras_array(sc.cameras)
    n = sc.n_rays
    F, G = M.Field(sc.field), M.Mesh(sc.mesh)
    F16 = M.Field(sc.field, table_dtype=M.MR_F16, mlp_dtype=M.MR_BF16)
    P = M.Field(sg.make_proposal(), table_dtype=M.MR_F16)
    T = M.ProposalTrainer(P)
    to, td = sg.random_rays(1 << 18, seed=506)
    to = torch.from_numpy(to).cuda()
    td = torch.from_numpy(td).cuda()
    lohi, tgt = T.targets(F, to, td, sc.t_near, sc.t_far, sc.n_samples)
    T.train(to, td, lohi, tgt, steps=train_steps, batch=1 << 14)
    o = torch.empty(n, 3, device="cuda")
    d = torch.empty(n, 3, device="cuda")
    M.mr_rays_from_cameras(cams, o, d, None, n)
    R = M.Renderer(n, sc.max_bounces, with_hits=False)
    plain = M.make_opts(sc)
    prop = M.make_opts(sc, sampler=M.MR_SAMPLER_PROPOSAL, proposal=P)
    verts = [torch.from_numpy(sg.cloth_vertices(f)).cuda() for f in range(frames)]

    def run(field, opts):
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for f in range(frames):
            G.refit(verts[f])
            R.render(field, G, o, d, sc.lights, opts)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / frames

    run(F, plain)
    ms_plain = run(F, plain)
    ms_prop = run(F16, prop)
    # the refits alone (7 938 triangles, device bottom-up pass per frame)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for f in range(frames):
        G.refit(verts[f])
    b.record()
    torch.cuda.synchronize()
    ms_refit = a.elapsed_time(b) / frames
    psnr = []
    for f in range(frames):
        G.refit(verts[f])
        R.render(F, G, o, d, sc.lights, plain)
        ref = R.radiance.cpu().numpy()
        R.render(F16, G, o, d, sc.lights, prop)
        psnr.append(psnr_tonemapped(R.radiance.cpu().numpy(), ref))
    return {"plain_fp32": {"value": round(n / (ms_plain / 1e3), 1), "unit": "rays/s",
                           "ms_per_frame_incl_refit": round(ms_plain, 3)},
            "proposal_fp16": {"value": round(n / (ms_prop / 1e3), 1), "unit": "rays/s",
                              "ms_per_frame_incl_refit": round(ms_prop, 3),
                              "psnr_db_per_frame": [round(x, 2) for x in psnr],
                              "psnr_db_min": round(min(psnr), 2)},
            "refit_ms_per_frame": round(ms_refit, 4), "frames": frames, "triangles": int(len(sc.mesh.indices))}


def _err_entry(L, hits, rr):
    import numpy as np
    ok = ~rr["tie"]
    ref = rr["radiance"][ok]
    rel = np.abs(L[ok] - ref) / np.maximum(np.abs(ref), 1e-30)
    return {"rays": int(len(ok)), "max_rel_err": float(rel.max()), "mean_rel_err": float(rel.mean()),
            "hit_ids_bit_exact_non_tie": bool(np.array_equal(hits[ok], rr["hit_ids"][ok])),
            "tie_rays": int((~ok).sum())}


def error_vs_oracle(M, sg, n_rays=2000):
    """Error of the GPU against the FP64 oracle per configuration, on seeded
    samples of n_rays rays of each full-size image: relative radiance error
    (max, mean) over the rays the oracle does not flag as ties, and whether
    their hit ids agree bit for bit.  FP16/BF16 engines are compared with the
    oracle on the master parameters (total error) and on the parameters as
    the engine holds them (arithmetic only).  The proposal configurations use
    a seeded proposal (the oracle takes no input that the GPU produced)."""
    import copy
    import numpy as np
    import torch
    from oracle import oracle as orc
    out = {}
    rng = np.random.default_rng(31)

    def gpu(sc, F, G, opts, o, d):
        R = M.Renderer(len(o), sc.max_bounces)
        R.render(F, G, o, d, sc.lights, opts)
        torch.cuda.synchronize()
        return R.radiance.cpu().numpy().astype(np.float64), R.hit_ids.cpu().numpy()

    def rays(sc):
        o = torch.empty(sc.n_rays, 3, device="cuda")
        d = torch.empty(sc.n_rays, 3, device="cuda")
        M.mr_rays_from_cameras(sg.cameras_array(sc.cameras), o, d, None, sc.n_rays)
        idx = np.sort(rng.choice(sc.n_rays, n_rays, replace=False))
        return o, d, idx, o.cpu().numpy()[idx], d.cpu().numpy()[idx]

    # mid scene: plain FP32 and the FP16 / BF16 engine, uniform 256 and seeded proposal 32 + 32
    sc = sg.mid_scene()
    o, d, idx, oh, dh = rays(sc)
    G = M.Mesh(sc.mesh)
    F32 = M.Field(sc.field)
    F16 = M.Field(sc.field, table_dtype=M.MR_F16, mlp_dtype=M.MR_BF16)
    for f in (F32, F16):
        f.build_occupancy(sc.occupancy_res, sc.occupancy_thresh)
    occ, _ = orc.occupancy(sc.field, sc.occupancy_res, sc.occupancy_thresh)
    scr = copy.copy(sc)
    scr.field = _rounded_field(sg, sc.field)
    occr, _ = orc.occupancy(scr.field, sc.occupancy_res, sc.occupancy_thresh)
    ref = orc.render(sc, oh, dh, ray_ids=idx, occupancy_bits=occ)
    ref_r = orc.render(scr, oh, dh, ray_ids=idx, occupancy_bits=occr)
    L, h = gpu(sc, F32, G, M.make_opts(sc, use_occupancy=True), o, d)
    out["mid_uniform256_fp32"] = {"vs_master_params": _err_entry(L[idx], h[idx], ref)}
    L, h = gpu(sc, F16, G, M.make_opts(sc, use_occupancy=True), o, d)
    out["mid_uniform256_fp16_table_bf16_mlp"] = {"vs_master_params": _err_entry(L[idx], h[idx], ref),
                                                 "vs_rounded_params": _err_entry(L[idx], h[idx], ref_r)}
    prop = sg.make_proposal(table_amp=0.5)
    propr = copy.deepcopy(prop)
    propr.table = prop.table.astype(np.float16).astype(np.float32)
    P = M.Field(prop, table_dtype=M.MR_F16)
    popts = M.make_opts(sc, sampler=M.MR_SAMPLER_PROPOSAL, proposal=P, use_occupancy=True)
    L, h = gpu(sc, F16, G, popts, o, d)
    rp = orc.render(sc, oh, dh, ray_ids=idx, occupancy_bits=occ, proposal=prop, n_prop=32, n_fine=32)
    rpr = orc.render(scr, oh, dh, ray_ids=idx, occupancy_bits=occr, proposal=propr, n_prop=32, n_fine=32)
    out["mid_proposal32x32_fp16_table_bf16_mlp_seeded_proposal"] = {
        "vs_master_params": _err_entry(L[idx], h[idx], rp), "vs_rounded_params": _err_entry(L[idx], h[idx], rpr)}
    # cloth (frame 0 and frame 37 after refits): plain FP32 and the seeded proposal on the FP16 / BF16 engine
    for frame in (0, 37):
        sc = sg.cloth_scene(frame)
        o, d, idx, oh, dh = rays(sc)
        G = M.Mesh(sg.cloth_scene(0).mesh)
        for f in range(1, frame + 1):
            G.refit(torch.from_numpy(sg.cloth_vertices(f)).cuda())
        Fc = M.Field(sc.field)
        Fc16 = M.Field(sc.field, table_dtype=M.MR_F16, mlp_dtype=M.MR_BF16)
        scr = copy.copy(sc)
        scr.field = _rounded_field(sg, sc.field)
        L, h = gpu(sc, Fc, G, M.make_opts(sc), o, d)
        out[f"cloth_frame{frame}_uniform256_fp32"] = {
            "vs_master_params": _err_entry(L[idx], h[idx], orc.render(sc, oh, dh, ray_ids=idx))}
        L, h = gpu(sc, Fc16, G, M.make_opts(sc, sampler=M.MR_SAMPLER_PROPOSAL, proposal=P), o, d)
        out[f"cloth_frame{frame}_proposal32x32_fp16_table_bf16_mlp_seeded_proposal"] = {
            "vs_master_params": _err_entry(L[idx], h[idx], orc.render(sc, oh, dh, ray_ids=idx, proposal=prop)),
            "vs_rounded_params": _err_entry(L[idx], h[idx], orc.render(scr, oh, dh, ray_ids=idx, proposal=propr))}
    out["sample"] = f"{n_rays} seeded rays per full-size image (800x800), re-rendered by the oracle one by one"
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sc, o, d, frac, frac_one_core=512):
    from oracle import oracle as orc
    import numpy as np
    n = len(o)
    rng = np.random.default_rng(7)
    m = max(1, n // frac)
    idx = np.sort(rng.choice(n, m, replace=False))
    threads = orc.n_threads_default()
    occ, _ = orc.occupancy(sc.field, sc.occupancy_res, sc.occupancy_thresh, n_threads=threads)   # not timed
    t0 = time.perf_counter()
    orc.render(sc, o[idx], d[idx], ray_ids=idx, n_threads=threads, occupancy_bits=occ)
    dt = time.perf_counter() - t0
    m1 = max(1, n // frac_one_core)
    idx1 = idx[:m1]
    t0 = time.perf_counter()
    orc.render(sc, o[idx1], d[idx1], ray_ids=idx1, n_threads=1, occupancy_bits=occ)
    dt1 = time.perf_counter() - t0
    return {"value": m / dt, "unit": "rays/s", "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
            "host_cpus_seen": os.cpu_count(),
            "sample": f"seeded uniform 1/{frac} ray subset ({m} of {n} rays), FP64 brute force with the "
                      f"oracle's own occupancy grid (built untimed), {dt:.1f} s",
            "one_core": {"value": m1 / dt1, "unit": "rays/s", "cores": 1,
                         "sample": f"the first {m1} rays of the same subset, {dt1:.1f} s"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-frac", type=int, default=8, help="oracle runs on 1/frac of the rays")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="headline workload only")
    ap.add_argument("--train-steps", type=int, default=1000)
    ap.add_argument("--cloth-frames", type=int, default=100)
    ap.add_argument("--segment-samples", action="store_true",
                    help="print the headline render's field samples per bounce segment and exit")
    ap.add_argument("--proposal-only", action="store_true",
                    help="only the proposal + FP16/BF16 frame (for profiler passes)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB device copy first (reference dispatch for memory counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the path is not sharded "
                                   "across GPUs (each GPU would render its own share of the rays)"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2309_04581_amd import meshrf as M
    from paper_2309_04581_amd import scenegen as sg

    torch.cuda.set_device(0)
    sc = sg.mid_scene()
    cams = sg.cameras_array(sc.cameras)
    n = sc.n_rays
    F, G = M.Field(sc.field), M.Mesh(sc.mesh)
    F.build_occupancy(sc.occupancy_res, sc.occupancy_thresh)
    o = torch.empty(n, 3, device="cuda")
    d = torch.empty(n, 3, device="cuda")
    R = M.Renderer(n, sc.max_bounces, with_hits=False)
    opts = M.make_opts(sc, use_occupancy=True)

    def step():
        M.mr_rays_from_cameras(cams, o, d, None, n)
        R.render(F, G, o, d, sc.lights, opts)

    if args.segment_samples:
        # renders with the bounce limit raised one segment at a time: the paths
        # are the same, so the differences are the samples of each segment
        cum = []
        for mb in range(sc.max_bounces + 1):
            Rs = M.Renderer(n, mb, with_hits=False)
            M.mr_rays_from_cameras(cams, o, d, None, n)
            Rs.render(F, G, o, d, sc.lights, opts)
            torch.cuda.synchronize()
            cum.append(int(Rs.counters.cpu().numpy()[0]))
        print(json.dumps({"samples_per_segment": [cum[0]] + [cum[i] - cum[i - 1] for i in range(1, len(cum))]}))
        return
    if args.proposal_only:
        # the proposal + FP16/BF16 frame alone (with its training), for counter passes
        step()
        torch.cuda.synchronize()
        out = proposal_variant(M, sg, sc, F, G, cams, n, R.radiance.cpu().numpy(), args.steps, args.warmup,
                               args.train_steps)
        print(json.dumps({"proposal_fp16": out}))
        return
    # launch shape (march and stage blocks per CU, stage tile, queue chunk and
    # batch, packet segments) from the library's autotuner, cached per
    # architecture and workload; the search runs outside every timed region
    opts_default = opts
    key = M.autotune_key("mid", sc.field.resolutions.tobytes(), len(sc.mesh.indices), sc.n_samples, n,
                         sc.max_bounces, cams.tobytes(), sc.occupancy_res)
    cache = os.path.join(os.environ.get("XDG_CACHE_HOME", os.path.expanduser("~/.cache")), "meshrf_autotune.json")
    os.makedirs(os.path.dirname(cache), exist_ok=True)
    search = {}

    def tune():
        t_s = time.perf_counter()
        M.mr_rays_from_cameras(cams, o, d, None, n)
        shape, ms, ms0, nt = M.mr_autotune_search(F.handle, G.handle, n, o, d, sc.max_bounces, None, sc.lights,
                                                  opts_default, R.out, R.workspace, R.ws_bytes, reps=2, passes=2)
        search.update({"shapes_timed": nt, "search_s": round(time.perf_counter() - t_s, 2),
                       "default_ms_in_search": round(ms0, 3), "tuned_ms_in_search": round(ms, 3)})
        return shape, ms
    shape, _, hit = M.autotune_cached(cache, key, tune)
    opts = M.apply_launch(M.make_opts(sc, use_occupancy=True), shape)
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # the library's default shape, for comparison (before the timed and
    # profiled passes of the tuned shape)
    def step_default():
        M.mr_rays_from_cameras(cams, o, d, None, n)
        R.render(F, G, o, d, sc.lights, opts_default)
    ms_default = timed(step_default, args.steps, args.warmup)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(args.steps):
        step()
    t1.record()
    torch.cuda.synchronize()
    ms_total = t0.elapsed_time(t1)
    # per-stage times from a second pass of the same steps with event pairs
    # around every launch (on the stream each kernel runs on)
    stage_ms, stage_n, counters = profiled(M, step, args.steps, R)   # counters: samples, segments, shadow rays, scatters
    ms_step = ms_total / args.steps
    rays_s = n / (ms_step / 1e3)
    samples = int(counters[0])
    segments = int(counters[1])

    # dominant kernel: the march (field gathers + MLPs + compositing)
    # the march: stage 3 the camera segment (k_march_pc), stage 1 the later segments (k_march_mfma)
    march_ms_per_step = (stage_ms[1] + stage_ms[3]) / args.steps
    march_launch_ms = (stage_ms[1] + stage_ms[3]) / max(1, stage_n[1] + stage_n[3])
    launches_per_step = (stage_n[1] + stage_n[3]) / args.steps
    flops_per_step = 2.0 * field_macs(sc.field) * samples
    tflops = flops_per_step / (march_ms_per_step / 1e3) / 1e12
    bf16_tflops = 6 * 2.0 * split_macs(sc.field) * samples / (march_ms_per_step / 1e3) / 1e12
    gbs = gather_bytes(sc.field) * samples / (march_ms_per_step / 1e3) / 1e9
    # split: camera segment (k_march_pc) and bounce segments (k_march_mfma); samples of the
    # camera segment from the same render stopped at its first surface (the same samples)
    R0 = M.Renderer(n, 0, with_hits=False)
    M.mr_rays_from_cameras(cams, o, d, None, n)
    R0.render(F, G, o, d, sc.lights, opts)
    torch.cuda.synchronize()
    cam_ms = stage_ms[3] / args.steps
    cam_samples = int(R0.counters.cpu().numpy()[0])
    bnc_ms = stage_ms[1] / args.steps
    bnc_samples = samples - cam_samples

    # random single-entry loads from this table (every load a line lookup, eight
    # independent ones per lane): the rate at which the memory side serves
    # incoherent 128-byte lines, the ceiling of a march whose gathers share no line
    names = ("march_blocks_per_cu", "stage_blocks_per_cu", "stage_tile", "march_chunk", "march_batch",
             "march_packets")
    launch = {"shape": dict(zip(names, shape)), "autotuned": True, "cache_hit": hit, "key": key, **search,
              "default_shape": {"value": round(n / (ms_default / 1e3), 1), "unit": "rays/s",
                                "ms_per_step": round(ms_default, 3)}}
    probe = gather_probe(M, sg, F)
    line_ceiling = probe["mid_fp32_64MiB"]["Gloads_per_s"]

    def seg_roof(ms, ns, fabric):
        fl = 2.0 * field_macs(sc.field) * ns / (ms / 1e3) / 1e12
        bfl = 6 * 2.0 * split_macs(sc.field) * ns / (ms / 1e3) / 1e12
        out = {"ms_per_step": round(ms, 3), "samples": ns, "ns_per_sample": round(ms * 1e6 / max(1, ns), 4),
               "fp32_TFLOPs": round(fl, 2), "frac_of_fp32_mfma_peak": round(fl / FP32_MFMA_PEAK_TFLOPS, 4),
               "bf16_instruction_TFLOPs": round(bfl, 2), "frac_of_bf16_mfma_peak": round(bfl / BF16_MFMA_PEAK_TFLOPS, 4),
               "algorithmic_gather_GB_per_s": round(gather_bytes(sc.field) * ns / (ms / 1e3) / 1e9, 1)}
        if fabric is not None:
            out["fabric_GB_per_s"] = round(fabric / (ms / 1e3) / 1e9, 1)
            out["fabric_frac_of_hbm_peak"] = round(fabric / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
            out["fabric_bytes_per_sample"] = round(fabric / max(1, ns), 1)
            # the march's reads are 128-byte requests (profiles/): lines per second
            # against the random-line ceiling measured on the same table
            lines = fabric / 128.0 / (ms / 1e3) / 1e9
            out["fabric_lines_G_per_s"] = round(lines, 2)
            out["frac_of_random_line_ceiling"] = round(lines / line_ceiling, 4)
        return out

    line = {
        "metric": METRIC, "value": round(rays_s, 1), "unit": "rays/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded field, meshes, camera, light)",
        "config": {"workload": "mid scene, plain FP32 marcher: 800x800 camera, 16-level hash grid "
                               "2^19 x 2 FP32, MLPs 32-64-16 / 32-64-64-3, occupancy grid 128^3 at "
                               "density 0.01, 256 samples/segment, 20 494 triangles, 1 point light, "
                               "8 bounces",
                   "rays": n, "samples_per_step": samples, "segments_per_step": segments,
                   "sampler": "uniform",
                   "precision": "fp32 (MLP products on FP32 values split into three exact BF16 pieces, FP32 "
                                "accumulation; error against the FP64 oracle in error_vs_fp64_oracle)"},
        "segments_per_s": round(segments / (ms_step / 1e3), 1),
        "launch_shape": launch,
        "stage_ms_per_step": {"closest_hit": round(stage_ms[0] / args.steps, 3),
                              "march": round(march_ms_per_step, 3),
                              "shade": round(stage_ms[2] / args.steps, 3),
                              "note": "a second pass of the same steps with event pairs around each launch"},
        # the march's bound: the memory side serving the hash gathers (the 64 MiB
        # table sits in the Infinity Cache in front of HBM); achieved = the
        # algorithmic gather bytes (16 levels x 8 corners x 2 FP32) per second
        "roofline": {"kernel": "k_march_pc (camera segment) + k_march_mfma (later segments)", "bound": "hbm",
                     "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                     "traffic_unit": "bytes per launch (L2-to-memory reads by request size + writes)",
                     "launch_ms": round(march_launch_ms, 4),
                     "launches_per_step": launches_per_step,
                     "algorithmic_bytes_per_sample": gather_bytes(sc.field),
                     "matrix_cores": {
                         "instructions": "v_mfma_f32_16x16x32_bf16 / 16x16x16bf16 on FP32 operands split into "
                                         "three exact BF16 pieces, six piece products per multiply-add, FP32 "
                                         "accumulation",
                         "fp32_TFLOPs": round(tflops, 2),
                         "frac_of_fp32_mfma_peak": round(tflops / FP32_MFMA_PEAK_TFLOPS, 4),
                         "bf16_instruction_TFLOPs": round(bf16_tflops, 2),
                         "frac_of_bf16_mfma_peak": round(bf16_tflops / BF16_MFMA_PEAK_TFLOPS, 4)},
                     "camera_segment": dict(kernel="k_march_pc", **seg_roof(
                         cam_ms, cam_samples, measured_traffic("camera_segment_fabric_bytes"))),
                     "bounce_segments": dict(kernel="k_march_mfma", **seg_roof(
                         bnc_ms, bnc_samples, measured_traffic("bounce_segments_fabric_bytes")))},
        "gather": {"achieved": round(gbs, 1), "unit": "GB/s", "peak_hbm": HBM_PEAK_GBS,
                   "bytes_per_sample": gather_bytes(sc.field)},
    }
    line["gather"]["probe_random_gather"] = probe
    # the march's gathers are coherent (packets, consecutive samples); these are
    # its rates relative to fully random loads from the same table and from an
    # L2-resident one, not fractions of a ceiling
    line["gather"]["ratio_to_random_gather_same_table"] = round(gbs / probe["mid_fp32_64MiB"]["GB_per_s"], 2)
    line["gather"]["ratio_to_random_gather_l2_table"] = round(gbs / probe["tiny_fp32_1MiB"]["GB_per_s"], 2)
    plain_img = R.radiance.cpu().numpy()
    if not args.no_extras:
        line["proposal_fp16"] = proposal_variant(M, sg, sc, F, G, cams, n, plain_img, args.steps, 1,
                                                 args.train_steps)
        line["shell_field_proposal_vs_uniform"] = shell_proposal(M, sg, args.steps, args.train_steps)
        line["moving_field"] = moving_field(M, sg, sc, F, G, cams, n, args.steps, shape=shape)
        line["sample_shadows"] = sample_shadows(M, sg, sc, F, G, cams, n, args.steps, shape=shape)
        line["emitters"] = emitters(M, sg, args.steps, shape=shape)
        line["several_fields"] = several_fields(M, sg, args.steps, train_steps=args.train_steps)
        line["multicam_16_cameras"] = multicam(M, sg, 2)
        line["scaling_spheres"] = scaling(M, sg, 3)
        line["cloth_refit"] = cloth(M, sg, args.cloth_frames, args.train_steps)
    if not args.no_cpu_baseline:
        # the oracle leg: its time on the host cores, and the GPU's error against it per configuration
        oh = o.cpu().numpy()
        dh = d.cpu().numpy()
        line["cpu_baseline"] = cpu_baseline(sc, oh, dh, args.cpu_frac)
        if not args.no_extras:
            line["precision_tiny_vs_fp64_oracle"] = precision_report(M, sg)
            line["error_vs_fp64_oracle"] = error_vs_oracle(M, sg)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
