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
# weight of the predicted gradient's L1 term next to the density's when the
# four-output network is fitted (gradients of the unit-range volume are O(1-10))
PRED_GRAD_WEIGHT = 0.1


def progress(msg: str):
    """One line per bench section on stderr (the JSON result goes to stdout)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


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


# mangled name of the study render kernel (FP16 network, c = 32, F = 16, L = 8,
# sine, FP16 latent grid, no time input or Fourier matrix, no shading)
STUDY_KERNEL = ("_ZN12fvsrn_detail12_GLOBAL__N_112march_kernelINS_3CfgILi1ELi32ELi16ELi8ELi0ELi1ELi0ELi0EEELi0ELi0EEEvNS_"
                "6NetDevENS_5TFDevENS_9ViewBatchENS_8MarchDevEPfPyPjii")


def kernel_isa_hash():
    """sha256 of the study render kernel's instructions, as recorded by the
    build next to the library (None when the record is missing)."""
    path = os.path.join(ROOT, "paper_2112_01579_amd", "libfvsrn_kernels.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        return json.load(fh).get(STUDY_KERNEL)


def counter_record(name):
    """A committed rocprofv3 counter record of the study render kernel, if it
    was taken on the kernel code that is built now (else None)."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    h = kernel_isa_hash()
    if h is None or rec.get("kernel_isa_sha256") != h:
        return None
    return rec


def measured_traffic():
    """HBM bytes per launch of the FP16 render (FETCH_SIZE + WRITE_SIZE,
    copy-calibrated)."""
    rec = counter_record("march_f16_study_traffic.json")
    return None if rec is None else rec.get("hbm_bytes_per_launch")


def measured_valu_busy():
    """Fraction of SIMD cycles the study render keeps the vector ALU issuing:
    4 x SQ_ACTIVE_INST_VALU (quad-cycles, summed over waves) over SIMDs x the
    kernel's cycles."""
    rec = counter_record("march_f16_study_sq.json")
    return None if rec is None else rec.get("valu_busy")


def cpu_cores():
    """Host cores the process may use: its CPU affinity, capped by the cgroup
    CPU quota and by OMP_NUM_THREADS when either is set (a GPU host gives
    each GPU's processes a share of its cores and says so there)."""
    n = len(os.sched_getaffinity(0))
    try:
        quota, period = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if quota != "max":
            n = min(n, max(1, int(int(quota) // int(period))))
    except (OSError, ValueError):
        pass
    omp = os.environ.get("OMP_NUM_THREADS", "")
    if omp.isdigit() and int(omp) > 0:
        n = min(n, int(omp))
    return max(1, n)


def torch_layerwise(spec, lat, w, xyz, dtype):
    """The same fV-SRN evaluated the way a framework would (the comparison of
    Sec. 5.1): grid_sample for the latent vector, elementwise Fourier
    features, one GEMM + activation per layer, every intermediate in HBM."""
    import torch
    import torch.nn.functional as Fn
    dev = xyz.device
    R, F = spec.R, spec.F
    grid = torch.as_tensor(lat, device=dev).reshape(R, R, R, F).permute(3, 0, 1, 2).unsqueeze(0).to(dtype)
    mats, off = [], 0
    wt = torch.as_tensor(w, device=dev)
    for o, i in spec.layer_shapes():
        mats.append((wt[off:off + o * i].reshape(o, i).to(dtype), wt[off + o * i:off + o * i + o].to(dtype)))
        off += o * i + o
    k = torch.pi * (2.0 ** torch.arange(spec.L, device=dev, dtype=torch.float32))

    def run():
        z = Fn.grid_sample(grid, xyz.to(dtype).view(1, 1, 1, -1, 3), mode="bilinear", padding_mode="border",
                           align_corners=True).view(F, -1).t()
        ph = (xyz.unsqueeze(1) * k.view(1, -1, 1)).reshape(-1, 3 * spec.L)
        h = torch.cat([xyz.to(dtype), z, torch.sin(ph).to(dtype), torch.cos(ph).to(dtype)], 1)
        for i, (W, b) in enumerate(mats):
            h = Fn.linear(h, W, b)
            h = torch.sin(h) if i < len(mats) - 1 else torch.sigmoid(h)
        return h
    return run


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(spec, lat16, w, tf, cams, march):
    """The FP64 oracle on every host core the process may use, on a 352x352
    centre crop of view 0."""
    import oracle as O
    threads = cpu_cores()
    net = O.Net(spec, lat16.astype(np.float64), w)
    W, H = cams[0].width, cams[0].height
    c = 176
    pix = np.array([(H // 2 - c + y) * W + (W // 2 - c + x) for y in range(2 * c) for x in range(2 * c)],
                   dtype=np.int64)
    t0 = time.perf_counter()
    _, ns = O.render(O.Field(net=net), tf, cams, march, pixels=pix, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": ns / dt, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": "%dx%d centre crop of view 0 (%d samples, %.1f s)" % (2 * c, 2 * c, ns, dt),
            "cpu_model": cpu_model(), "cpu_affinity": len(os.sched_getaffinity(0))}


def eval_points_only(args, spec, dev):
    """2^24 uniform points through fvsrn_eval_points, FP16 network on the FP16
    grid and FP32 network on the FP32 grid: one JSON line of points/s."""
    import torch
    from paper_2112_01579_amd import inputs as I
    from paper_2112_01579_amd import fvsrn as FV
    lat, w = I.net_params(spec, I.SEED_STUDY)
    npts = 1 << 24
    xyz = FV.fvsrn_sample_points(I.SEED_STUDY, 1 << 43, npts, device=dev)
    dens = torch.empty(npts, device=dev)
    res = {"metric": "fused point evaluation, 2^24 uniform points", "unit": "points/s"}
    for prec, gd in (("f16", FV.F16), ("f32", FV.F32)):
        net = FV.Network(spec, lat, w, grid_dtype=gd, device=dev)
        per, _ = time_launches(lambda: FV.fvsrn_eval_points(net, xyz, 0.0, prec, out=dens), args.steps, args.warmup)
        res[prec] = {"points_per_s": npts / (float(np.median(per)) * 1e-3), "ms": float(np.median(per))}
    print(json.dumps(res))


def train_only(args, dev):
    """2^18-point gradient steps (no sampling, targets or Adam) of the three
    network shapes in FP32 and FP16: one JSON line of ms per step."""
    import torch
    from paper_2112_01579_amd import inputs as I
    from paper_2112_01579_amd import fvsrn as FV
    n = 1 << 18
    xyz = FV.fvsrn_sample_points(I.SEED_TRAIN, 1 << 42, n, device=dev)
    target = torch.rand(n, device=dev)
    res = {"metric": "training gradient step, 2^18 uniform points", "unit": "ms"}
    for sname in ("NET_SMALL", "NET_STUDY", "NET_SHADED"):
        spec = getattr(I, sname)
        lat, w = I.net_params(spec, 3)
        net = FV.Network(spec, lat, w, grid_dtype=FV.F32, device=dev)
        d_lat, d_w = torch.empty_like(net.latent), torch.empty_like(net.weights)
        ws = torch.empty(max(FV.fvsrn_train_workspace_size(spec, n), 16), dtype=torch.uint8, device=dev)
        for prec in ("f32", "f16"):
            per, _ = time_launches(lambda: FV.fvsrn_train_step(net, d_lat, d_w, xyz, target=target, workspace=ws,
                                                               precision=prec), args.steps, args.warmup)
            res["%s_%s_ms" % (sname.lower(), prec)] = float(np.median(per))
    print(json.dumps(res))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device-to-device copy (reference for rocprofv3 byte counters)")
    ap.add_argument("--train-steps", type=int, default=2000,
                    help="Adam steps (2^18 points each) fitting the network before timing")
    ap.add_argument("--eval-points-only", action="store_true",
                    help="time only the fused point evaluation of 2^24 uniform points (FP16 and FP32 networks, "
                         "the study network with its initial weights); for profiling that kernel")
    ap.add_argument("--train-only", action="store_true",
                    help="time only 2^18-point training gradient steps of the three network shapes in FP32 and FP16; "
                         "for profiling the training kernels")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the fV-SRN path is single-GPU (rays and points are "
              "independent). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2112_01579_amd import inputs as I
    from paper_2112_01579_amd import fvsrn as FV

    FV.lib()
    dev = torch.device("cuda:0")
    spec = I.NET_STUDY
    if args.eval_points_only:
        eval_points_only(args, spec, dev)
        return
    if args.train_only:
        train_only(args, dev)
        return
    vol = torch.from_numpy(I.gaussian_volume(256, 64, seed=I.SEED_STUDY)).to(dev)
    lat, w = I.net_params(spec, I.SEED_STUDY)
    train_info = None
    if args.train_steps > 0:
        progress("training the study network")
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

    progress("timing the study render")
    per, wall = time_launches(step, args.steps, args.warmup)
    # the median launch (8 frames each) sets the kernel's rate
    ms_launch = float(np.median(per))
    ms_step = wall / args.steps
    fps = flops_per_sample(spec)
    achieved = samples * fps / (ms_launch * 1e-3) / 1e12
    # unique bytes a launch must move: FP16 latent grid + FP32 weights in, RGBA image out
    algo_bytes = net.latent.numel() * 2 + net.weights.numel() * 4 + out.numel() * 4
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
            "traffic": measured_traffic(),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "algorithmic_bytes": algo_bytes,
            "launch_ms": ms_launch,
            "launch_ms_mean": float(np.mean(per)),
            "launches_timed": len(per),
            # the unit that binds the kernel: the vector ALU issues the
            # activations, gathers and features; the matrix cores wait on it
            "binding_unit": "valu",
            "valu_busy": measured_valu_busy(),
        },
    }

    progress("comparisons")
    if not args.no_compare:
        comp = {}
        # dense-grid DVR of the original 256^3 volume: the reference for image quality
        ref = torch.empty_like(out)

        def dense():
            FV.fvsrn_render_dense(vol, tf, cams, march, out=ref, stats=stats)
        stats.zero_()
        dense()
        torch.cuda.synchronize()
        s = int(stats[0].item())
        per_c, _ = time_launches(dense, max(3, args.steps // 4), 1)
        ms = float(np.median(per_c))
        # eight FP32 corners per sample come from the caches (L1/L2/MALL); the
        # volume itself and the image cross HBM once
        comp["dense_dvr_256"] = {"ms_per_frame": ms / len(cams), "samples_per_s": s / (ms * 1e-3),
                                 "cache_gather_GBps": s * 32 / (ms * 1e-3) / 1e9,
                                 "hbm_unique_GBps": (vol.numel() * 4 + ref.numel() * 4) / (ms * 1e-3) / 1e9}

        def rmse(img):
            return float(torch.sqrt(torch.mean((img - ref) ** 2)).item())

        def ssim(img):
            return FV.fvsrn_ssim(img, ref)
        step()
        torch.cuda.synchronize()
        comp["fvsrn_f16"] = {"ms_per_frame": ms_launch / len(cams), "samples_per_s": samples / (ms_launch * 1e-3),
                             "tflops": achieved, "image_rmse_vs_dense": rmse(out), "image_ssim_vs_dense": ssim(out)}
        net_u8 = FV.Network(spec, lat, w, grid_dtype=FV.U8, device=dev)
        for prec, n, name in (("f32", net32, "fvsrn_f32"), ("bf16", net, "fvsrn_bf16"),
                              ("f16", net_u8, "fvsrn_f16_uint8_grid")):
            stats.zero_()
            step(n, prec)
            torch.cuda.synchronize()
            s = int(stats[0].item())
            e, q = rmse(out), ssim(out)
            per_c, _ = time_launches(lambda: step(n, prec), max(3, args.steps // 4), 1)
            ms = float(np.median(per_c))
            comp[name] = {"ms_per_frame": ms / len(cams), "samples_per_s": s / (ms * 1e-3),
                          "tflops": s * fps / (ms * 1e-3) / 1e12, "image_rmse_vs_dense": e,
                          "image_ssim_vs_dense": q}
        progress("shading strategies")
        # gradient strategies for Phong shading (Sec. 6): no shading, forward
        # mode, central differences with a one-voxel step of the 256^3 volume;
        # image error against dense DVR shaded with one-voxel central differences
        import dataclasses
        shade = {}
        m_dense = dataclasses.replace(march, phong=True)
        FV.fvsrn_render_dense(vol, tf, cams, m_dense, out=ref)
        for name, m in (("none", march), ("forward", m_dense),
                        ("central", dataclasses.replace(m_dense, grad_mode=1, fd_step=2.0 / 255)),
                        ("adjoint", dataclasses.replace(m_dense, grad_mode=3))):
            FV.fvsrn_render(net, tf, cams, m, "f16", out=out, stats=stats.zero_())
            torch.cuda.synchronize()
            ns = int(stats[0].item())
            e, q = rmse(out), ssim(out)
            per_c, _ = time_launches(lambda: FV.fvsrn_render(net, tf, cams, m, "f16", out=out), 3, 1)
            shade[name] = {"ms_per_frame": float(np.median(per_c)) / len(cams),
                           "samples_per_s": ns / (float(np.median(per_c)) * 1e-3)}
            if m.phong:
                shade[name]["image_rmse_vs_dense_phong"] = e
                shade[name]["image_ssim_vs_dense_phong"] = q
        shade["central_over_forward"] = shade["central"]["ms_per_frame"] / shade["forward"]["ms_per_frame"]
        shade["forward_over_adjoint"] = shade["forward"]["ms_per_frame"] / shade["adjoint"]["ms_per_frame"]
        if args.train_steps > 0:
            # the network predicts its own gradient (four outputs, Sec. 6):
            # the same architecture fitted to densities and to one-voxel
            # central differences of the volume, shaded from outputs 1..3
            from paper_2112_01579_amd.trainer import Trainer
            spec4 = dataclasses.replace(spec, outputs=4)
            lat4, w4 = I.net_params(spec4, I.SEED_STUDY)
            p32 = FV.Network(spec4, lat4, w4, grid_dtype=FV.F32, device=dev)
            ptr = Trainer(p32, vol, batch=1 << 18, seed=I.SEED_TRAIN, grad_weight=PRED_GRAD_WEIGHT)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.train_steps):
                ptr.step()
            torch.cuda.synchronize()
            t_train = time.perf_counter() - t0
            pnet = FV.Network(spec4, p32.latent.cpu().numpy(), p32.weights.cpu().numpy(), grid_dtype=FV.F16,
                              device=dev)
            m_pred = dataclasses.replace(m_dense, grad_mode=2)
            FV.fvsrn_render(pnet, tf, cams, m_pred, "f16", out=out, stats=stats.zero_())
            torch.cuda.synchronize()
            ns = int(stats[0].item())
            e, q = rmse(out), ssim(out)
            per_c, _ = time_launches(lambda: FV.fvsrn_render(pnet, tf, cams, m_pred, "f16", out=out), 3, 1)
            shade["predicted"] = {"ms_per_frame": float(np.median(per_c)) / len(cams),
                                  "samples_per_s": ns / (float(np.median(per_c)) * 1e-3),
                                  "image_rmse_vs_dense_phong": e, "image_ssim_vs_dense_phong": q,
                                  "training": {"steps": args.train_steps, "batch": 1 << 18,
                                               "grad_weight": PRED_GRAD_WEIGHT, "final_loss": float(ptr.loss.item()),
                                               "ms_per_step": t_train / args.train_steps * 1e3}}
            for k in ("forward", "central", "adjoint"):
                shade[k + "_over_predicted"] = shade[k]["ms_per_frame"] / shade["predicted"]["ms_per_frame"]
            del ptr, p32, pnet
        comp["shading_f16"] = shade
        progress("time-varying workload")
        # time-varying workload (Sec. 8): keyframe latent grids every 4 timesteps
        # trained on all 16 timesteps of the 256^3 advected-blob field, then 8
        # views at fractional times in one launch; compared with dense DVR of
        # the field at each view's time
        if args.train_steps > 0:
            from paper_2112_01579_amd.trainer import Trainer
            prm = I.blob_sequence_params(seed=I.SEED_TIME)
            raw = [I.blob_volume_torch(256, float(t), prm, device=dev) for t in range(16)]
            norm = max(float(v.max().item()) for v in raw)
            frames = [(float(t), v / norm) for t, v in enumerate(raw)]
            del raw
            tspec = I.NET_TIME
            tlat, tw = I.net_params(tspec, I.SEED_TIME)
            tnet32 = FV.Network(tspec, tlat, tw, key_times=I.TIME_KEYS, grid_dtype=FV.F32, device=dev)
            ttr = Trainer(tnet32, frames, batch=1 << 18, seed=I.SEED_TIME)
            tsteps = max(1, args.train_steps // 2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(tsteps):
                ttr.step()
            torch.cuda.synchronize()
            t_train = time.perf_counter() - t0
            tnet = FV.Network(tspec, tnet32.latent.cpu().numpy(), tnet32.weights.cpu().numpy(),
                              key_times=I.TIME_KEYS, grid_dtype=FV.F16, device=dev)
            tcams = I.time_cameras(1024, 1024)
            stats.zero_()
            FV.fvsrn_render(tnet, tf, tcams, march, "f16", out=out, stats=stats)
            torch.cuda.synchronize()
            ts = int(stats[0].item())
            per_c, _ = time_launches(lambda: FV.fvsrn_render(tnet, tf, tcams, march, "f16", out=out), 3, 1)
            ms = float(np.median(per_c))
            for v, cam in enumerate(tcams):
                vt = I.blob_volume_torch(256, cam.time, prm, norm, device=dev)
                FV.fvsrn_render_dense(vt, tf, [cam], march, out=ref[v:v + 1])
            comp["time_varying_f16"] = {
                "ms_per_frame": ms / len(tcams), "samples_per_s": ts / (ms * 1e-3),
                "tflops": ts * fps / (ms * 1e-3) / 1e12, "image_rmse_vs_dense": rmse(out),
                "image_ssim_vs_dense": ssim(out),
                "view_times": [c.time for c in tcams],
                "training": {"steps": tsteps, "batch": 1 << 18, "timesteps": 16, "final_l1": float(ttr.loss.item()),
                             "ms_per_step": t_train / tsteps * 1e3}}
            # time encodings (Sec. 8): the same keyframe network with no time
            # input, the normalised time as an input, its Fourier features, or
            # both, trained on the even timesteps only and evaluated on the odd
            # ones it never saw (mean |density error| over 2^18 points each)
            enc = {}
            train_frames = [f for f in frames if int(f[0]) % 2 == 0]
            held_out = [f for f in frames if int(f[0]) % 2 == 1]
            xe = FV.fvsrn_sample_points(I.SEED_TIME, 1 << 40, 1 << 18, device=dev)
            esteps = max(1, args.train_steps // 4)
            for te, name in ((0, "latent_only"), (1, "direct"), (2, "fourier"), (3, "both")):
                espec = dataclasses.replace(tspec, time_enc=te)
                elat, ew = I.net_params(espec, I.SEED_TIME)
                enet = FV.Network(espec, elat, ew, key_times=I.TIME_KEYS, grid_dtype=FV.F32, device=dev)
                etr = Trainer(enet, train_frames, batch=1 << 18, seed=I.SEED_TIME)
                for _ in range(esteps):
                    etr.step()

                def mean_err(fr):
                    return float(np.mean([torch.mean(torch.abs(FV.fvsrn_eval_points(enet, xe, t, "f32") -
                                                               FV.fvsrn_dense_eval_points(v, xe))).item()
                                          for t, v in fr]))
                e16 = FV.Network(espec, enet.latent.cpu().numpy(), enet.weights.cpu().numpy(), key_times=I.TIME_KEYS,
                                 grid_dtype=FV.F16, device=dev)
                per_c, _ = time_launches(lambda: FV.fvsrn_render(e16, tf, tcams, march, "f16", out=out), 3, 1)
                enc[name] = {"l1_trained_timesteps": mean_err(train_frames), "l1_unseen_timesteps": mean_err(held_out),
                             "render_ms_per_frame_f16": float(np.median(per_c)) / len(tcams)}
                del etr, enet, e16
            comp["time_encodings"] = {"train": "even timesteps 0..14, %d steps of 2^18 points" % esteps,
                                      "evaluated_on": "odd timesteps 1..15", **enc}
            # adaptive resampling of the time-varying network (Sec. 5.4 with
            # Sec. 8): uniform positions against one error grid per timestep
            # (64^3 voxels x 8 positions, refreshed every 50 steps), the same
            # steps each; mean |density error| over all 16 timesteps
            tvr = {}
            for name, every in (("uniform", 0), ("resampled_every_50", 50)):
                rlat, rw = I.net_params(tspec, I.SEED_TIME)
                rnet = FV.Network(tspec, rlat, rw, key_times=I.TIME_KEYS, grid_dtype=FV.F32, device=dev)
                rtr = Trainer(rnet, frames, batch=1 << 18, seed=I.SEED_TIME, resample_every=every, error_grid=64,
                              per_voxel=8)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(esteps):
                    rtr.step()
                torch.cuda.synchronize()
                t_r = time.perf_counter() - t0
                l1 = float(np.mean([torch.mean(torch.abs(FV.fvsrn_eval_points(rnet, xe, t, "f32") -
                                                         FV.fvsrn_dense_eval_points(v, xe))).item() for t, v in frames]))
                tvr[name] = {"l1_all_timesteps": l1, "train_ms_per_step": t_r / esteps * 1e3}
                del rtr, rnet
            comp["time_varying_adaptive_resampling"] = {
                "train": "16 timesteps, %d steps of 2^18 points, error grids 64^3 x 8 per timestep" % esteps, **tvr}
            del frames, ttr, tnet32
        progress("Fourier features")
        # Fourier features (Sec. 3, Sec. 5.3): the octave construction against
        # random Fourier features (entries ~ N(0, (2 pi sigma)^2)), the study
        # network trained the same number of steps on the 256^3 volume; mean
        # |density error| over 2^18 random points and the FP16 render time
        if args.train_steps > 0:
            from paper_2112_01579_amd.trainer import Trainer
            ff = {}
            fsteps = max(1, args.train_steps // 4)
            xf = FV.fvsrn_sample_points(I.SEED_STUDY, 1 << 41, 1 << 18, device=dev)
            dref = FV.fvsrn_dense_eval_points(vol, xf)
            for name, sigma in (("octaves", None), ("random_sigma_2", 2.0), ("random_sigma_8", 8.0)):
                fmx = None if sigma is None else I.random_fourier_matrix(spec.L, sigma, I.SEED_STUDY)
                flat, fw = I.net_params(spec, I.SEED_STUDY)
                fnet = FV.Network(spec, flat, fw, grid_dtype=FV.F32, device=dev, fourier_matrix=fmx)
                ftr = Trainer(fnet, vol, batch=1 << 18, seed=I.SEED_TRAIN)
                for _ in range(fsteps):
                    ftr.step()
                l1 = torch.mean(torch.abs(FV.fvsrn_eval_points(fnet, xf, 0.0, "f32") - dref)).item()
                f16 = FV.Network(spec, fnet.latent.cpu().numpy(), fnet.weights.cpu().numpy(), grid_dtype=FV.F16,
                                 device=dev, fourier_matrix=fmx)
                per_c, _ = time_launches(lambda: FV.fvsrn_render(f16, tf, cams, march, "f16", out=out), 3, 1)
                ff[name] = {"l1": l1, "render_ms_per_frame_f16": float(np.median(per_c)) / len(cams)}
                del ftr, fnet, f16
            comp["fourier_features"] = {"train": "%d steps of 2^18 points on the 256^3 volume" % fsteps, **ff}
        progress("point evaluation")
        # adaptive resampling (Sec. 5.4): the study network trained with
        # uniform positions and with positions drawn from a 128^3 error grid
        # refreshed every 50 steps, the same number of steps each; density
        # error at uniform points and the FP16 image against dense DVR
        if args.train_steps > 0:
            progress("adaptive resampling")
            ar = {}
            rsteps = max(1, args.train_steps // 4)
            FV.fvsrn_render_dense(vol, tf, cams, march, out=ref)
            for name, every in (("uniform", 0), ("resampled_every_50", 50)):
                rlat, rw = I.net_params(spec, I.SEED_STUDY)
                rnet = FV.Network(spec, rlat, rw, grid_dtype=FV.F32, device=dev)
                rtr = Trainer(rnet, vol, batch=1 << 18, seed=I.SEED_TRAIN, resample_every=every, error_grid=128,
                              per_voxel=8)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(rsteps):
                    rtr.step()
                torch.cuda.synchronize()
                t_r = time.perf_counter() - t0
                l1 = torch.mean(torch.abs(FV.fvsrn_eval_points(rnet, xf, 0.0, "f32") - dref)).item()
                r16 = FV.Network(spec, rnet.latent.cpu().numpy(), rnet.weights.cpu().numpy(), grid_dtype=FV.F16,
                                 device=dev)
                FV.fvsrn_render(r16, tf, cams, march, "f16", out=out)
                ar[name] = {"l1_uniform_points": l1, "image_rmse_vs_dense": rmse(out), "image_ssim_vs_dense": ssim(out),
                            "train_ms_per_step": t_r / rsteps * 1e3}
                del rtr, rnet, r16
            comp["adaptive_resampling"] = {"train": "%d steps of 2^18 points, error grid 128^3 x 8" % rsteps, **ar}
        # the training workload: the small network (16^3 x 8 grid, 3 x 32)
        # fitted to the 256^3 power-law field, 2000 Adam steps of 2^18 points
        if args.train_steps > 0:
            progress("training workload")
            pvol = I.power_law_volume_torch(256, 512, seed=I.SEED_TRAIN, device=dev)
            slat, sw = I.net_params(I.NET_SMALL, I.SEED_SMALL)
            snet = FV.Network(I.NET_SMALL, slat, sw, grid_dtype=FV.F32, device=dev)
            xs = FV.fvsrn_sample_points(I.SEED_TRAIN, 1 << 42, 1 << 18, device=dev)
            ps = FV.fvsrn_dense_eval_points(pvol, xs)
            l1_0 = torch.mean(torch.abs(FV.fvsrn_eval_points(snet, xs, 0.0, "f32") - ps)).item()
            str_ = Trainer(snet, pvol, batch=1 << 18, seed=I.SEED_TRAIN)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.train_steps):
                str_.step()
            torch.cuda.synchronize()
            t_s = time.perf_counter() - t0
            l1_1 = torch.mean(torch.abs(FV.fvsrn_eval_points(snet, xs, 0.0, "f32") - ps)).item()
            comp["training_small_power_law"] = {"steps": args.train_steps, "batch": 1 << 18,
                                                "ms_per_step": t_s / args.train_steps * 1e3,
                                                "l1_untrained": l1_0, "l1_trained": l1_1}
            # the same fit with the network's forward and backward on FP16 MFMA
            snet16 = FV.Network(I.NET_SMALL, slat, sw, grid_dtype=FV.F32, device=dev)
            str16 = Trainer(snet16, pvol, batch=1 << 18, seed=I.SEED_TRAIN, precision="f16")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.train_steps):
                str16.step()
            torch.cuda.synchronize()
            t_16 = time.perf_counter() - t0
            comp["training_small_power_law"]["fp16"] = {
                "ms_per_step": t_16 / args.train_steps * 1e3,
                "l1_trained": torch.mean(torch.abs(FV.fvsrn_eval_points(snet16, xs, 0.0, "f32") - ps)).item()}
            # gradient steps alone (no sampling, targets or Adam), FP32 and FP16
            # networks, the three network shapes, 2^18 points
            gsteps = {}
            for sname in ("NET_SMALL", "NET_STUDY", "NET_SHADED"):
                gspec = getattr(I, sname)
                glat, gw = I.net_params(gspec, 3)
                gnet = FV.Network(gspec, glat, gw, grid_dtype=FV.F32, device=dev)
                gdl, gdw = torch.empty_like(gnet.latent), torch.empty_like(gnet.weights)
                gws = torch.empty(max(FV.fvsrn_train_workspace_size(gspec, 1 << 18), 16), dtype=torch.uint8,
                                  device=dev)
                row = {}
                for gp in ("f32", "f16"):
                    per, _ = time_launches(lambda: FV.fvsrn_train_step(gnet, gdl, gdw, xs, target=ps, workspace=gws,
                                                                       precision=gp), 20, 3)
                    row[gp + "_ms"] = float(np.median(per))
                row["fp16_speedup"] = row["f32_ms"] / row["f16_ms"]
                gsteps[sname.lower()] = row
            comp["training_gradient_step_2e18"] = gsteps
            del pvol, str_, snet, str16, snet16
            # the shaded workload: the 64^3 x 16, 4 x 48 network fitted to the
            # 512^3 Marschner-Lobb field, one 1920 x 1080 view at step 1/512
            # with Phong shading, FP16 MFMA; gradients by forward mode (the
            # configured strategy) and by the adjoint; dense DVR of the 512^3
            # field with one-voxel central differences as the image reference
            progress("shaded workload")
            mvol = torch.from_numpy(I.marschner_lobb_volume(512)).to(dev)
            mlat, mw = I.net_params(I.NET_SHADED, I.SEED_SHADED)
            mnet32 = FV.Network(I.NET_SHADED, mlat, mw, grid_dtype=FV.F32, device=dev)
            mtr = Trainer(mnet32, mvol, batch=1 << 18, seed=I.SEED_SHADED)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.train_steps):
                mtr.step()
            torch.cuda.synchronize()
            t_m = time.perf_counter() - t0
            mnet = FV.Network(I.NET_SHADED, mnet32.latent.cpu().numpy(), mnet32.weights.cpu().numpy(),
                              grid_dtype=FV.F16, device=dev)
            scam = [I.shaded_camera()]
            smarch = I.shaded_march(1e-3)
            sout = torch.empty((1, 1080, 1920, 4), dtype=torch.float32, device=dev)
            sref = torch.empty_like(sout)
            FV.fvsrn_render_dense(mvol, tf, scam, smarch, out=sref)
            per_d, _ = time_launches(lambda: FV.fvsrn_render_dense(mvol, tf, scam, smarch, out=sref), 3, 1)
            shaded = {"training": {"steps": args.train_steps, "ms_per_step": t_m / args.train_steps * 1e3,
                                   "final_l1": float(mtr.loss.item())},
                      "dense_dvr_512_ms_per_frame": float(np.median(per_d))}
            for name, gm in (("forward", 0), ("adjoint", 3)):
                mm = dataclasses.replace(smarch, grad_mode=gm)
                FV.fvsrn_render(mnet, tf, scam, mm, "f16", out=sout, stats=stats.zero_())
                torch.cuda.synchronize()
                ns = int(stats[0].item())
                per_c, _ = time_launches(lambda: FV.fvsrn_render(mnet, tf, scam, mm, "f16", out=sout), 3, 1)
                ms = float(np.median(per_c))
                shaded[name] = {"ms_per_frame": ms, "samples_per_s": ns / (ms * 1e-3),
                                "image_rmse_vs_dense": float(torch.sqrt(torch.mean((sout - sref) ** 2)).item()),
                                "image_ssim_vs_dense": FV.fvsrn_ssim(sout, sref)}
            comp["shaded_1920x1080_marschner_lobb"] = shaded
            del mvol, mtr, mnet32, mnet, sout, sref
        # where the MFMA ceiling lies: the same render with networks of more
        # matrix work per activation (c = 48) and without transcendental
        # activations (identity), random weights, the same cameras and grid
        progress("MFMA fraction by network")
        mf = {}
        for name, sp in (("c32_sine", spec), ("c48_sine", dataclasses.replace(spec, c=48)),
                         ("c32_identity", dataclasses.replace(spec, act="identity")),
                         ("c48_identity", dataclasses.replace(spec, c=48, act="identity"))):
            qlat, qw = I.net_params(sp, I.SEED_STUDY)
            if sp.act == "identity":
                qw = qw * 0.5   # keep the linear network's densities away from saturation
            qnet = FV.Network(sp, qlat, qw, grid_dtype=FV.F16, device=dev)
            stats.zero_()
            FV.fvsrn_render(qnet, tf, cams, march, "f16", out=out, stats=stats)
            torch.cuda.synchronize()
            qs = int(stats[0].item())
            per_c, _ = time_launches(lambda: FV.fvsrn_render(qnet, tf, cams, march, "f16", out=out), 3, 1)
            ms = float(np.median(per_c))
            tfl = qs * flops_per_sample(sp) / (ms * 1e-3) / 1e12
            mf[name] = {"samples_per_s": qs / (ms * 1e-3), "tflops": tfl, "frac_of_fp16_peak": tfl / P16_TFLOPS}
            del qnet
        comp["mfma_fraction_by_network"] = mf
        # fused point evaluation vs the framework-style layer-by-layer network (2^24 points)
        npts = 1 << 24
        xyz = torch.rand((npts, 3), device=dev) * 2 - 1
        dens = torch.empty(npts, device=dev)
        for prec, n in (("f32", net32), ("f16", net)):
            per_c, _ = time_launches(lambda: FV.fvsrn_eval_points(n, xyz, 0.0, prec, out=dens), 5, 1)
            comp["eval_points_fused_" + prec] = {"points_per_s": npts / (float(np.median(per_c)) * 1e-3)}
            # the paper's protocol: 10^6 random reconstructions per call
            m6 = 1000000
            per_m, _ = time_launches(lambda: FV.fvsrn_eval_points(n, xyz[:m6], 0.0, prec, out=dens[:m6]), 20, 3)
            comp["eval_points_fused_" + prec]["ms_per_1e6_points"] = float(np.median(per_m))
        for name, dt in (("f32", torch.float32), ("f16", torch.float16)):
            run = torch_layerwise(spec, lat, w, xyz, dt)
            per_c, _ = time_launches(run, 3, 1)
            pts = npts / (float(np.median(per_c)) * 1e-3)
            comp["eval_points_torch_layerwise_" + name] = {
                "points_per_s": pts,
                "fused_speedup": comp["eval_points_fused_" + name]["points_per_s"] / pts}
        result["compare"] = comp

    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_calibration_bytes"] = {"read": src.numel() * 4, "write": dst.numel() * 4}
    progress("CPU oracle baseline")
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(spec, lat.astype(np.float16), w, tf, cams, march)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
