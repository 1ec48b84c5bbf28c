#!/usr/bin/env python3
"""Benchmark of the fV-SRN ray-march hot path on one MI355X.

Workload (the inference precision study): an fV-SRN with a 32^3 x 16 FP16
latent grid, 8 Fourier octaves and 4 hidden layers of width 32, first fitted
to a synthetic 256^3 volume (sum of 64 anisotropic Gaussians) by the
library's trainer (L1 + Adam, 2^18 points per step), renders an 8-view
1024x1024 perspective orbit with step 1/256 (two samples per voxel of the
256^3 volume) and early ray termination at 1e-3, all 8 views in one launch.
One step = one such launch. The same frames are also timed with the FP32 and
BF16 network paths and with plain dense-grid DVR of the 256^3 volume, which
is also the reference of the reported image RMSE.

Prints one JSON line. ``value`` is network samples composited per second by
the FP16-MFMA path, inputs resident in HBM.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

P16_TFLOPS = 2516.6     # MI355X dense FP16/BF16 MFMA
P32_TFLOPS = 157.3      # MI355X FP32 (matrix and vector)
HBM_GBS = 8000.0


def flops_per_sample(spec) -> int:
    """Algorithmic multiply-adds x 2 of one network evaluation (unpadded K,
    biases excluded): 2 (K0 c + (H-1) c^2 + c)."""
    return 2 * (spec.K0 * spec.c + (spec.H - 1) * spec.c * spec.c + spec.c)


def time_launches(fn, steps, warmup):
    """Runs fn() warmup + steps times; returns (per-launch ms from HIP events
    on the launch stream, wall ms for the timed region)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    per = [a.elapsed_time(b) for a, b in evs]
    return per, wall


def cpu_baseline(spec, lat16, w, tf, cams, march):
    """The FP64 oracle on the host cores, on a 256x256 centre crop of view 0."""
    import oracle as O
    threads = os.cpu_count() or 1
    net = O.Net(spec, lat16.astype(np.float64), w)
    W, H = cams[0].width, cams[0].height
    c = 128
    pix = np.array([(H // 2 - c + y) * W + (W // 2 - c + x) for y in range(2 * c) for x in range(2 * c)],
                   dtype=np.int64)
    t0 = time.perf_counter()
    _, ns = O.render(O.Field(net=net), tf, cams, march, pixels=pix, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": ns / dt, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": "256x256 centre crop of view 0 (%d samples, %.1f s)" % (ns, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--train-steps", type=int, default=2000,
                    help="Adam steps (2^18 points each) fitting the network before timing")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the fV-SRN path is single-GPU (rays and points are "
              "independent; see DESIGN.md for how it would shard). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2112_01579_amd import inputs as I
    from paper_2112_01579_amd import fvsrn as FV

    FV.lib()
    dev = torch.device("cuda:0")
    spec = I.NET_STUDY
    vol = torch.from_numpy(I.gaussian_volume(256, 64, seed=I.SEED_STUDY)).to(dev)
    lat, w = I.net_params(spec, I.SEED_STUDY)
    train_info = None
    if args.train_steps > 0:
        # fit the network to the dense volume with the library's own trainer
        from paper_2112_01579_amd.trainer import Trainer
        tnet = FV.Network(spec, lat, w, grid_dtype=FV.F32, device=dev)
        tr = Trainer(tnet, vol, batch=1 << 18, seed=I.SEED_TRAIN)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.train_steps):
            tr.step()
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        lat = tnet.latent.cpu().numpy().reshape(lat.shape)
        w = tnet.weights.cpu().numpy()
        train_info = {"steps": args.train_steps, "batch": 1 << 18, "final_l1": float(tr.loss.item()),
                      "ms_per_step": t_train / args.train_steps * 1e3}
    net = FV.Network(spec, lat, w, grid_dtype=FV.F16, device=dev)
    net32 = FV.Network(spec, lat, w, grid_dtype=FV.F32, device=dev)
    tf = I.ramp_tf()
    cams = I.study_cameras(1024, 1024, 8)
    march = I.study_march(1e-3)
    out = torch.empty((8, 1024, 1024, 4), dtype=torch.float32, device=dev)
    stats = torch.zeros(3, dtype=torch.int64, device=dev)

    def step(n=net, prec="f16"):
        FV.fvsrn_render(n, tf, cams, march, prec, out=out, stats=stats)

    # samples per launch (deterministic for a fixed network)
    stats.zero_()
    step()
    torch.cuda.synchronize()
    samples, rays, slots = int(stats[0].item()), int(stats[1].item()), int(stats[2].item())

    per, wall = time_launches(step, args.steps, args.warmup)
    ms_launch = float(np.mean(per))
    ms_step = wall / args.steps
    fps = flops_per_sample(spec)
    achieved = samples * fps / (ms_launch * 1e-3) / 1e12
    result = {
        "metric": "ms/frame 1024^2 + samples/s: FP16-MFMA fV-SRN vs FP32 vs dense-grid DVR",
        "value": samples / (ms_step * 1e-3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_frame": ms_step / len(cams),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16",
        "data": "synthetic",
        "config": {
            "workload": "fV-SRN 32^3x16 FP16 latent grid, 8 octaves, 4x32 sine MLP fitted to a 256^3 "
                        "sum of 64 Gaussians, 8-view 1024x1024 perspective orbit, step 1/256, ERT 1e-3, "
                        "one launch",
            "training": train_info,
            "views": len(cams), "width": 1024, "height": 1024, "step": 1 / 256, "ert_eps": 1e-3,
            "samples_per_step": samples, "rays_hit_per_step": rays,
            "tile_occupancy": samples / max(slots, 1),
            "flop_per_sample": fps,
        },
        "roofline": {
            "bound": "mfma",
            "kernel": "march_kernel<f16, c=32, F=16, L=8>",
            "achieved": achieved,
            "peak": P16_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / P16_TFLOPS,
            "traffic": None,
            "launch_ms": ms_launch,
        },
    }

    if not args.no_compare:
        comp = {}
        # dense-grid DVR of the original 256^3 volume: the judge of image quality
        ref = torch.empty_like(out)

        def dense():
            FV.fvsrn_render_dense(vol, tf, cams, march, out=ref, stats=stats)
        stats.zero_()
        dense()
        torch.cuda.synchronize()
        s = int(stats[0].item())
        per_c, _ = time_launches(dense, max(3, args.steps // 4), 1)
        ms = float(np.mean(per_c))
        comp["dense_dvr_256"] = {"ms_per_frame": ms / len(cams), "samples_per_s": s / (ms * 1e-3),
                                 "algorithmic_GBps": s * 32 / (ms * 1e-3) / 1e9}

        def rmse(img):
            return float(torch.sqrt(torch.mean((img - ref) ** 2)).item())
        step()
        torch.cuda.synchronize()
        comp["fvsrn_f16"] = {"ms_per_frame": ms_launch / len(cams), "samples_per_s": samples / (ms_launch * 1e-3),
                             "tflops": achieved, "image_rmse_vs_dense": rmse(out)}
        for prec, n in (("f32", net32), ("bf16", net)):
            stats.zero_()
            step(n, prec)
            torch.cuda.synchronize()
            s = int(stats[0].item())
            e = rmse(out)
            per_c, _ = time_launches(lambda: step(n, prec), max(3, args.steps // 4), 1)
            ms = float(np.mean(per_c))
            comp["fvsrn_" + prec] = {"ms_per_frame": ms / len(cams), "samples_per_s": s / (ms * 1e-3),
                                     "tflops": s * fps / (ms * 1e-3) / 1e12, "image_rmse_vs_dense": e}
        result["compare"] = comp

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(spec, lat.astype(np.float16), w, tf, cams, march)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
