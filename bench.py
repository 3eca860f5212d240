#!/usr/bin/env python3
"""Throughput of the hybrid surface-volumetric marcher on one MI355X.

Workload (mid scene): 800x800 pinhole camera, 16-level hash grid (2^19
entries, 2 features, resolutions 16..2048, FP32), density MLP 32->64->16,
colour MLP (16 + 16 SH)->64->64->3, 256 uniform samples per segment on
[0.05, 4.0], glass icosphere (20 480 triangles) + mirror cube + diffuse floor
(20 494 triangles, SAH BVH), one point light with one shadow ray per diffuse
hit, up to 8 bounces.  Synthetic seeded inputs stand in for the paper's
captured scenes.

One step = camera ray generation + the whole bounce loop (closest hit, march,
shade/compaction per bounce) for all 640 000 primary rays, with field, mesh
and workspace resident in HBM.  Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rays/sec (full bounce paths) plain FP32 vs proposal+FP16 at >=40 dB PSNR"
HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK_TFLOPS = 78.6    # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz (no packed FP32)


def field_macs(f):
    """Real multiply-accumulates per field sample (density + colour MLPs),
    counting only the non-padded inputs."""
    nfeat = f.n_levels * f.feats
    macs = nfeat * f.d_hidden + f.d_hidden * f.d_out
    macs += (f.d_out + f.sh) * f.c_hidden + (f.c_layers - 1) * f.c_hidden * f.c_hidden + 3 * f.c_hidden
    return macs


def gather_bytes(f, bytes_per_value=4):
    return f.n_levels * 8 * f.feats * bytes_per_value


def cpu_baseline(sc, o, d, frac):
    from oracle import oracle as orc
    import numpy as np
    n = len(o)
    rng = np.random.default_rng(7)
    m = max(1, n // frac)
    idx = np.sort(rng.choice(n, m, replace=False))
    threads = orc.n_threads_default()
    t0 = time.perf_counter()
    orc.render(sc, o[idx], d[idx], ray_ids=idx, n_threads=threads)
    dt = time.perf_counter() - t0
    return {"value": m / dt, "unit": "rays/s", "cores": threads, "kind": "oracle",
            "sample": f"seeded uniform 1/{frac} ray subset ({m} of {n} rays), FP64 brute force, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-frac", type=int, default=64, help="oracle runs on 1/frac of the rays")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    o = torch.empty(n, 3, device="cuda")
    d = torch.empty(n, 3, device="cuda")
    R = M.Renderer(n, sc.max_bounces, with_hits=False)
    opts = M.make_opts(sc)

    def step():
        M.mr_rays_from_cameras(cams, o, d, None, n)
        R.render(F, G, o, d, sc.lights, opts)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    M.mr_profile_read()
    M.mr_profile_enable(True)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(args.steps):
        step()
    t1.record()
    torch.cuda.synchronize()
    M.mr_profile_enable(False)
    ms_total = t0.elapsed_time(t1)
    stage_ms, stage_n = M.mr_profile_read()
    counters = R.counters.cpu().numpy()          # last step: samples, segments, shadow rays, scatters
    ms_step = ms_total / args.steps
    rays_s = n / (ms_step / 1e3)
    samples = int(counters[0])
    segments = int(counters[1])

    # dominant kernel: the march (field gathers + MLPs + compositing)
    march_ms_per_step = stage_ms[1] / args.steps
    march_launch_ms = stage_ms[1] / max(1, stage_n[1])
    launches_per_step = stage_n[1] / args.steps
    flops_per_step = 2.0 * field_macs(sc.field) * samples
    tflops = flops_per_step / (march_ms_per_step / 1e3) / 1e12
    gbs = gather_bytes(sc.field) * samples / (march_ms_per_step / 1e3) / 1e9

    line = {
        "metric": METRIC, "value": round(rays_s, 1), "unit": "rays/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded field, meshes, camera, light)",
        "config": {"workload": "mid scene, plain FP32 marcher: 800x800 camera, 16-level hash grid "
                               "2^19 x 2 FP32, MLPs 32-64-16 / 32-64-64-3, 256 samples/segment, "
                               "20 494 triangles, 1 point light, 8 bounces",
                   "rays": n, "samples_per_step": samples, "segments_per_step": segments,
                   "sampler": "uniform", "precision": "fp32"},
        "segments_per_s": round(segments / (ms_step / 1e3), 1),
        "stage_ms_per_step": {"closest_hit": round(stage_ms[0] / args.steps, 3),
                              "march": round(march_ms_per_step, 3),
                              "shade": round(stage_ms[2] / args.steps, 3)},
        "roofline": {"kernel": "k_march", "bound": "alu", "achieved": round(tflops, 2),
                     "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tflops / FP32_VALU_PEAK_TFLOPS, 4), "traffic": None,
                     "launch_ms": round(march_launch_ms, 4),
                     "launches_per_step": launches_per_step},
        "gather": {"achieved": round(gbs, 1), "unit": "GB/s", "peak_hbm": HBM_PEAK_GBS,
                   "bytes_per_sample": gather_bytes(sc.field)},
    }
    if not args.no_cpu_baseline:
        oh = o.cpu().numpy()
        dh = d.cpu().numpy()
        line["cpu_baseline"] = cpu_baseline(sc, oh, dh, args.cpu_frac)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
