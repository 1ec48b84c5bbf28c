"""World-space fitting of an fV-SRN on the GPU (Sec. 3, Sec. 5): uniform
random positions, targets sampled trilinearly from the original dense grid,
L1 loss and Adam with separate learning rates for the latent grid and the
network. Every step runs in the HIP library: point sampling, target lookup,
the fused forward/backward kernel, the gradient reduction and Adam.

Also provides ``FvsrnPoints``, a torch.autograd.Function whose forward is
fvsrn_eval_points and whose backward is fvsrn_train_step in VJP mode (latent
grid and weights) and fvsrn_grad_points (positions), so the fV-SRN can sit
inside any torch loss.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from . import fvsrn as FV
from . import inputs as I


class Trainer:
    """Adam training of ``net`` (FP32 latent grids) on a dense volume ``vol``
    [nz][ny][nx] (device FP32), or, for a time-varying network (K keyframe
    grids, Sec. 8), on a sequence ``vol`` = [(time, volume), ...]: every step
    splits the batch evenly over the timesteps, each part drawing its targets
    from its own volume at its own time, so the keyframe grids around each
    time and the shared network learn together.

    A 4-output network (density and predicted gradient, Sec. 6) trained with
    ``grad_weight`` > 0 also fits its gradient outputs to one-voxel central
    differences of the volume (the gradients the dense renderer shades with),
    weighted L1 next to the density's L1.

    ``resample_every`` = N > 0 turns on adaptive resampling (Sec. 5.4): after
    every N steps the mean absolute error of the network is measured on an
    ``error_grid``^3 voxel grid (``per_voxel`` positions per voxel), and the
    next N steps draw their positions in proportion to it. A time-varying
    network keeps one error grid per timestep (the network at that time
    against that timestep's volume), and each timestep's part of the batch
    is drawn from its own grid.
    ``precision`` "f16" runs the network's forward and backward passes on
    FP16 MFMA (FP32 master parameters, gradients and Adam)."""

    def __init__(self, net: FV.Network, vol, batch: int = 1 << 18, lr_grid: float = 1e-2,
                 lr_mlp: float = 1e-3, betas=(0.9, 0.999), eps: float = 1e-8, seed: int = 0,
                 grad_weight: float = 0.0, resample_every: int = 0, error_grid: int = 128, per_voxel: int = 8,
                 precision: str = "f32"):
        assert net.grid_dtype == FV.F32
        assert grad_weight == 0.0 or net.spec.outputs == 4
        if isinstance(vol, torch.Tensor):
            vol = [(0.0, vol)]
        self.frames = list(vol)
        assert len(self.frames) >= 1 and (net.spec.K > 1 or len(self.frames) == 1)
        self.net, self.vol, self.batch, self.seed = net, self.frames[0][1], batch, seed
        self.precision = precision
        dev = net.weights.device
        # points of timestep j occupy rows [bounds[j], bounds[j + 1]) of the
        # batch (multiples of 4 rows keep every slice 16-byte aligned)
        T = len(self.frames)
        self.bounds = [(batch * j // T) // 4 * 4 for j in range(T)] + [batch]
        self.times = None
        if net.spec.K > 1:
            tt = np.concatenate([np.full(self.bounds[j + 1] - self.bounds[j], self.frames[j][0], np.float32)
                                 for j in range(T)])
            self.times = torch.from_numpy(tt).to(dev)
        self.opt = dict(lr_grid=lr_grid, lr_mlp=lr_mlp, beta1=betas[0], beta2=betas[1], eps=eps, step=0,
                        m_latent=torch.zeros_like(net.latent), v_latent=torch.zeros_like(net.latent),
                        m_weights=torch.zeros_like(net.weights), v_weights=torch.zeros_like(net.weights))
        self.d_latent = torch.empty_like(net.latent)
        self.d_weights = torch.empty_like(net.weights)
        self.xyz = torch.empty((batch, 3), dtype=torch.float32, device=dev)
        self.target = torch.empty(batch, dtype=torch.float32, device=dev)
        self.grad_weight = float(grad_weight)
        self.target_grad = torch.empty((batch, 3), dtype=torch.float32, device=dev) if grad_weight else None
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        ws = FV.fvsrn_train_workspace_size(net.spec, batch)
        self.workspace = torch.empty(max(ws, 16), dtype=torch.uint8, device=dev)
        self.resample_every, self.G, self.per_voxel = int(resample_every), int(error_grid), int(per_voxel)
        self.E = None
        if self.resample_every:
            n_err = self.G ** 3 * self.per_voxel
            self.err_xyz = torch.empty((n_err, 3), dtype=torch.float32, device=dev)
            self.err_scratch = torch.empty(n_err, dtype=torch.float32, device=dev)
            # one error grid per timestep ([T][G^3]); E is the first one
            self.E_all = torch.empty((len(self.frames), self.G ** 3), dtype=torch.float32, device=dev)
            self.E = self.E_all[0]
            self.E_ready = False
            # one sampling workspace per timestep: its prefix sums are built
            # from the error grid once per refresh and reused until the next
            self.sample_ws = torch.empty((len(self.frames), FV.weighted_points_stride(self.G)), dtype=torch.uint8,
                                         device=dev)
            self.cdf_fresh = False

    def update_error_grid(self):
        """Measure the error grid of the current network at every timestep
        (Sec. 5.4), all on the same voxel positions."""
        FV.fvsrn_voxel_points(self.seed ^ 0x5DEECE66D, self.opt["step"], self.G, self.per_voxel, out=self.err_xyz)
        for j, (t, v) in enumerate(self.frames):
            FV.fvsrn_error_grid(self.net, v, self.err_xyz, self.per_voxel, t, out=self.E_all[j],
                                scratch=self.err_scratch)
        self.E_ready = True
        self.cdf_fresh = False

    def step(self) -> torch.Tensor:
        """One training step; returns the L1 loss of the batch (device scalar)."""
        self.opt["step"] += 1
        if self.resample_every and self.opt["step"] > 1 and (self.opt["step"] - 1) % self.resample_every == 0:
            self.update_error_grid()
        if self.E is not None and self.E_ready:
            # timestep j's rows from its own error grid; counters step * T + j
            T = len(self.frames)
            if not self.cdf_fresh:
                for j in range(T):
                    a, b = self.bounds[j], self.bounds[j + 1]
                    FV.fvsrn_sample_points_weighted(self.seed, self.opt["step"] * T + j, self.E_all[j], self.G,
                                                    b - a, out=self.xyz[a:b], workspace=self.sample_ws[j])
                self.cdf_fresh = True
            else:
                # the same draws from the kept prefix sums, in one launch
                FV.fvsrn_sample_points_weighted_multi(
                    self.seed, self.opt["step"] * T, self.G,
                    [self.bounds[j + 1] - self.bounds[j] for j in range(T)], self.sample_ws, out=self.xyz)
        else:
            FV.fvsrn_sample_points(self.seed, self.opt["step"], self.batch, out=self.xyz)
        for j, (_, v) in enumerate(self.frames):
            a, b = self.bounds[j], self.bounds[j + 1]
            if self.target_grad is None:
                FV.fvsrn_dense_eval_points(v, self.xyz[a:b], out=self.target[a:b])
            else:
                FV.fvsrn_dense_grad_points(v, self.xyz[a:b], out=self.target[a:b], out_grad=self.target_grad[a:b])
        FV.fvsrn_train_step(self.net, self.d_latent, self.d_weights, self.xyz, target=self.target, adam=self.opt,
                            out_loss=self.loss, workspace=self.workspace, times=self.times,
                            target_grad=self.target_grad, grad_weight=self.grad_weight, precision=self.precision)
        return self.loss

    def state_dict(self) -> dict:
        o = self.opt
        return {"latent": self.net.latent.cpu().numpy(), "weights": self.net.weights.cpu().numpy(),
                "m_latent": o["m_latent"].cpu().numpy(), "v_latent": o["v_latent"].cpu().numpy(),
                "m_weights": o["m_weights"].cpu().numpy(), "v_weights": o["v_weights"].cpu().numpy(),
                "step": np.int64(o["step"]), "seed": np.int64(self.seed)}

    def save(self, path: str):
        np.savez(path, **self.state_dict())

    def load(self, path: str):
        d = np.load(path)
        self.net.latent.copy_(torch.from_numpy(d["latent"]))
        self.net.weights.copy_(torch.from_numpy(d["weights"]))
        for k in ("m_latent", "v_latent", "m_weights", "v_weights"):
            self.opt[k].copy_(torch.from_numpy(d[k]))
        self.opt["step"] = int(d["step"])
        self.seed = int(d["seed"])


class FvsrnPoints(torch.autograd.Function):
    """density = fV-SRN(xyz, time), differentiable in xyz, the latent grid and
    the weights.

    ``latent`` and ``weights`` must be the network's own tensors (passed so
    that autograd tracks them and torch's version counters catch an in-place
    update between forward and backward). Forward runs fvsrn_eval_points in
    ``precision``; the parameter gradients come from fvsrn_train_step in VJP
    mode (the FP32 network, each point at ``time``), the position gradient
    from fvsrn_grad_points in reverse mode (adjoint) at ``precision``, scaled
    by the upstream gradient."""

    @staticmethod
    def forward(ctx, xyz: torch.Tensor, latent: torch.Tensor, weights: torch.Tensor, net: FV.Network,
                time: float = 0.0, precision: str = "f32"):
        if latent.data_ptr() != net.latent.data_ptr() or weights.data_ptr() != net.weights.data_ptr():
            raise FV.FvsrnArgumentError("latent and weights must be the network's own tensors")
        ctx.net, ctx.time, ctx.precision = net, float(time), precision
        xyz = xyz.contiguous()
        ctx.save_for_backward(xyz, latent, weights)
        return FV.fvsrn_eval_points(net, xyz, ctx.time, precision)

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        xyz, latent, weights = ctx.saved_tensors  # raises if modified in place since forward
        net = ctx.net
        g = grad_out.contiguous().float()
        d_xyz = d_lat = d_w = None
        if ctx.needs_input_grad[1] or ctx.needs_input_grad[2]:
            d_lat = torch.empty_like(latent)
            d_w = torch.empty_like(weights)
            times = None
            if net.spec.K > 1 or net.spec.time_enc:
                times = torch.full((xyz.shape[0],), ctx.time, dtype=torch.float32, device=xyz.device)
            FV.fvsrn_train_step(net, d_lat, d_w, xyz, dloss_dy=g, times=times)
        if ctx.needs_input_grad[0]:
            _, grad = FV.fvsrn_grad_points(net, xyz, ctx.time, ctx.precision, mode="adjoint")
            d_xyz = grad * g[:, None]
        return d_xyz, d_lat, d_w, None, None, None


def fvsrn_points(net: FV.Network, xyz: torch.Tensor, time: float = 0.0, precision: str = "f32") -> torch.Tensor:
    return FvsrnPoints.apply(xyz, net.latent, net.weights, net, time, precision)
