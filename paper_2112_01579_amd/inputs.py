"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the
CPU oracle.

This module holds plain data only: network shapes, random parameters drawn
from a seed, transfer-function control points, camera placements, march
settings and synthetic density volumes. It contains none of the method's own
arithmetic (no interpolation, encoding, network, shading or compositing), so
that both sides can consume the same inputs without sharing any of the code
under test. Transfer functions, cameras and march settings hold FP32 values
(the precision of the library's interface), so the oracle receives exactly
what the library receives.

Workloads (stand-ins for the paper's datasets, which are not available):
  * small ortho  -- 16^3 x 8 latent grid, 4 octaves, 35->32->32->32->1 sine
                    MLP (NET_SMALL), orthographic 64x64 view, 128 segments.
  * study        -- 256^3 sum of 64 anisotropic Gaussians (the 256^3
                    performance study of Sec. 5.1 / protocol of Sec. 7),
                    32^3 x 16 latent grid, 8 octaves, 4 hidden layers of 32
                    (NET_STUDY), 8-view 1024^2 orbit, step 1/256 (two samples
                    per voxel).
  * training     -- 256^3 power-law (k^-5/3) random-phase Fourier field fitted
                    by NET_SMALL on 2^18 uniform points per step.
  * shaded       -- 512^3 Marschner-Lobb signal (f_M = 6, alpha = 0.25),
                    64^3 x 16 grid, 4 hidden layers of 48 (NET_SHADED),
                    1920x1080, step 1/512, Phong.
  * time         -- 16 timesteps of 32 advected Gaussian blobs, keyframe
                    latent grids every 4 steps (NET_TIME), 8 views at
                    fractional times.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np


# --------------------------------------------------------------- plain data

def _f32(x: float) -> float:
    """The FP32 value nearest to x, as a Python float. The library receives
    transfer functions, cameras and march settings as FP32; rounding them
    here gives the oracle the very values the library sees (a camera eye
    rounded on one side only moves a grazing ray's entry point by up to
    1/|d_axis| times the rounding, which is visible in the image)."""
    return float(np.float32(x))


def _round_fields(obj, names):
    for n in names:
        v = getattr(obj, n)
        object.__setattr__(obj, n, tuple(_f32(x) for x in v) if isinstance(v, tuple) else _f32(v))

@dataclasses.dataclass(frozen=True)
class NetSpec:
    R: int            # latent vertices per axis
    F: int            # latent channels
    L: int            # Fourier octaves
    c: int            # hidden width
    H: int            # activated (hidden) layers; one c->outputs output layer follows
    K: int = 1        # latent keyframes
    act: str = "sine"
    outputs: int = 1  # 1 (density) or 4 (density and its predicted gradient)
    time_enc: int = 0  # time input (Sec. 8): 0 latent only, 1 direct, 2 Fourier, 3 both

    @property
    def K0(self) -> int:
        return 3 + self.F + 6 * self.L + (0, 1, 8, 9)[self.time_enc]

    def layer_shapes(self) -> List[Tuple[int, int]]:
        """(out, in) of every weight matrix, input layer first."""
        shapes = [(self.c, self.K0)] + [(self.c, self.c)] * (self.H - 1) + [(self.outputs, self.c)]
        return shapes

    @property
    def n_weights(self) -> int:
        return sum(o * i + o for o, i in self.layer_shapes())

    @property
    def n_latent(self) -> int:
        return self.K * self.R ** 3 * self.F


@dataclasses.dataclass(frozen=True)
class TF:
    """Control points (density, r, g, b, alpha), ascending in density, and the
    extinction per world unit at alpha = 1."""
    points: Tuple[Tuple[float, float, float, float, float], ...]
    opacity_scale: float = 20.0

    def __post_init__(self):
        object.__setattr__(self, "points", tuple(tuple(_f32(x) for x in p) for p in self.points))
        _round_fields(self, ("opacity_scale",))


@dataclasses.dataclass(frozen=True)
class Camera:
    ortho: bool
    eye: Tuple[float, float, float]
    target: Tuple[float, float, float]
    up: Tuple[float, float, float]
    width: int
    height: int
    fov_y_deg: float = 45.0
    ortho_half_extent: float = 1.0
    time: float = 0.0

    def __post_init__(self):
        _round_fields(self, ("eye", "target", "up", "fov_y_deg", "ortho_half_extent", "time"))


@dataclasses.dataclass(frozen=True)
class March:
    step: float = 1.0 / 256.0
    fixed_steps: int = 0
    ert_eps: float = 0.0
    phong: bool = False
    ka: float = 0.1
    kd: float = 0.7
    ks: float = 0.2
    shininess: float = 32.0
    grad_mode: int = 0      # Phong gradient: 0 forward mode, 1 central differences, 2 predicted, 3 adjoint
    fd_step: float = 0.0    # central-difference step (world units)

    def __post_init__(self):
        _round_fields(self, ("step", "ert_eps", "ka", "kd", "ks", "shininess", "fd_step"))


# ------------------------------------------------------- random parameters

def net_params(spec: NetSpec, seed: int, latent_std: float = 0.1):
    """Latent grid ~ N(0, latent_std) and Xavier-uniform weights (gain 1,
    bound sqrt(6/(fan_in+fan_out))), zero biases. Draw order: latent, then
    W of each layer. Returns float32 arrays (latent [K][R][R][R][F], packed
    weights: per layer W[out][in] row-major then b[out])."""
    rng = np.random.default_rng(seed)
    latent = rng.normal(0.0, latent_std, size=(spec.K, spec.R, spec.R, spec.R, spec.F))
    parts = []
    for o, i in spec.layer_shapes():
        bound = math.sqrt(6.0 / (i + o))
        parts.append(rng.uniform(-bound, bound, size=o * i))
        parts.append(np.zeros(o))
    weights = np.concatenate(parts)
    return latent.astype(np.float32), weights.astype(np.float32)


def random_fourier_matrix(L: int, sigma: float, seed: int) -> np.ndarray:
    """[3L][3] Fourier matrix with entries ~ N(0, (2 pi sigma)^2) (random
    Fourier features, Sec. 3), float32, rows in the sin/cos block order."""
    rng = np.random.default_rng(seed)
    return (2.0 * math.pi * sigma * rng.normal(size=(3 * L, 3))).astype(np.float32)


def octave_fourier_matrix(L: int, dtype=np.float32) -> np.ndarray:
    """The octave construction as a matrix: row 3k+a = pi 2^k e_a."""
    m = np.zeros((3 * L, 3), dtype=dtype)
    for k in range(L):
        for a in range(3):
            m[3 * k + a, a] = math.pi * 2 ** k
    return m


def uniform_points(n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(n, 3)).astype(np.float32)


# --------------------------------------------------------- TF and cameras

def ramp_tf() -> TF:
    """4-point piecewise-linear RGBA ramp used by every configuration."""
    return TF(points=((0.0, 0.0, 0.0, 0.0, 0.0),
                      (0.3, 0.1, 0.3, 1.0, 0.1),
                      (0.6, 1.0, 0.9, 0.3, 0.5),
                      (1.0, 1.0, 0.3, 0.1, 1.0)), opacity_scale=20.0)


def ortho_camera(width: int = 64, height: int = 64) -> Camera:
    """Looks down -z from z = +2 over the whole [-1,1]^2 face."""
    return Camera(ortho=True, eye=(0.0, 0.0, 2.0), target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0),
                  width=width, height=height, ortho_half_extent=1.0)


def orbit_cameras(n_views: int, width: int, height: int, radius: float = 3.0,
                  elevation_deg: float = 20.0, fov_y_deg: float = 45.0,
                  times: Optional[Sequence[float]] = None) -> List[Camera]:
    """Perspective cameras on a circle around the origin (azimuth 2*pi*v/n)."""
    cams = []
    el = math.radians(elevation_deg)
    for v in range(n_views):
        az = 2.0 * math.pi * v / n_views
        eye = (radius * math.cos(el) * math.sin(az), radius * math.sin(el),
               radius * math.cos(el) * math.cos(az))
        cams.append(Camera(ortho=False, eye=eye, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0),
                           width=width, height=height, fov_y_deg=fov_y_deg,
                           time=0.0 if times is None else float(times[v])))
    return cams


# ------------------------------------------------------- synthetic volumes

def _axis(n: int) -> np.ndarray:
    """Vertex positions of an n-vertex axis spanning [-1, 1]."""
    return np.linspace(-1.0, 1.0, n)


def gaussian_volume(D: int = 256, n: int = 64, seed: int = 1001, sigma=(0.02, 0.2),
                    amp=(0.2, 1.0), centre_extent: float = 0.7, cutoff: float = 5.0) -> np.ndarray:
    """Sum of n anisotropic, randomly rotated Gaussians, normalized by its
    maximum: rho(x) = sum_j a_j exp(-|S_j^-1 R_j^T (x - c_j)|^2 / 2). Each
    Gaussian is evaluated inside a box of cutoff * max(sigma_j) around its
    centre (beyond which it is below exp(-12.5)). Returns float32 [D][D][D]
    (z, y, x)."""
    rng = np.random.default_rng(seed)
    ax = _axis(D)
    vol = np.zeros((D, D, D), dtype=np.float32)
    for _ in range(n):
        cen = rng.uniform(-centre_extent, centre_extent, size=3)
        sig = rng.uniform(sigma[0], sigma[1], size=3)
        a = rng.uniform(amp[0], amp[1])
        q, r = np.linalg.qr(rng.normal(size=(3, 3)))
        rot = q * np.sign(np.diag(r))           # uniformly random orthogonal matrix
        reach = cutoff * sig.max()
        sl = []
        for k in range(3):   # k: 0 = x, 1 = y, 2 = z
            lo = np.searchsorted(ax, cen[k] - reach)
            hi = np.searchsorted(ax, cen[k] + reach, side="right")
            sl.append((lo, hi))
        (x0, x1), (y0, y1), (z0, z1) = sl
        if x1 <= x0 or y1 <= y0 or z1 <= z0:
            continue
        # quadratic form (x-c)^T M (x-c) with M = R S^-2 R^T, evaluated by broadcasting
        M = (rot / sig[None, :] ** 2) @ rot.T
        X = (ax[x0:x1] - cen[0]).astype(np.float32)[None, None, :]
        Y = (ax[y0:y1] - cen[1]).astype(np.float32)[None, :, None]
        Z = (ax[z0:z1] - cen[2]).astype(np.float32)[:, None, None]
        M = M.astype(np.float32)
        e = (M[0, 0] * X * X + M[1, 1] * Y * Y) + (M[2, 2] * Z * Z + 2 * M[0, 1] * X * Y)
        e = e + (2 * M[0, 2] * X * Z + 2 * M[1, 2] * Y * Z)
        vol[z0:z1, y0:y1, x0:x1] += np.float32(a) * np.exp(np.float32(-0.5) * e)
    vol /= vol.max()
    return vol.astype(np.float32)


def power_law_volume(D: int = 256, n_modes: int = 512, seed: int = 1003,
                     kmin: float = math.pi, kmax: float = 64 * math.pi) -> np.ndarray:
    """Random-phase Fourier field f(x) = sum_j A_j cos(k_j . x + phi_j) with
    directions uniform on the sphere, |k| log-uniform in [kmin, kmax] and
    A_j ~ |k_j|^(-1/3) (energy spectrum ~ k^(-5/3) under log-uniform
    sampling); min-max normalized to [0, 1]. float32 [D][D][D]."""
    rng = np.random.default_rng(seed)
    dirs = rng.normal(size=(n_modes, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    kmag = np.exp(rng.uniform(math.log(kmin), math.log(kmax), size=n_modes))
    kv = dirs * kmag[:, None]
    amp = kmag ** (-1.0 / 3.0)
    phase = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)
    ax = _axis(D).astype(np.float32)
    vol = np.zeros((D, D, D), dtype=np.float32)
    Y, X = np.meshgrid(ax, ax, indexing="ij")
    for z in range(D):
        acc = np.zeros((D, D), dtype=np.float64)
        for j0 in range(0, n_modes, 64):
            kk = kv[j0:j0 + 64]
            arg = (X[..., None] * kk[:, 0] + Y[..., None] * kk[:, 1] + ax[z] * kk[:, 2]
                   + phase[j0:j0 + 64])
            acc += (np.cos(arg) * amp[j0:j0 + 64]).sum(-1)
        vol[z] = acc
    vol -= vol.min()
    vol /= vol.max()
    return vol


def power_law_volume_torch(D: int = 256, n_modes: int = 512, seed: int = 1003, kmin: float = math.pi,
                           kmax: float = 64 * math.pi, device="cuda"):
    """``power_law_volume`` (the same modes, drawn in the same order)
    evaluated with torch in FP64 on ``device``; FP32 [D][D][D]."""
    import torch
    rng = np.random.default_rng(seed)
    dirs = rng.normal(size=(n_modes, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    kmag = np.exp(rng.uniform(math.log(kmin), math.log(kmax), size=n_modes))
    kv = torch.as_tensor(dirs * kmag[:, None], dtype=torch.float64, device=device)
    amp = torch.as_tensor(kmag ** (-1.0 / 3.0), dtype=torch.float64, device=device)
    phase = torch.as_tensor(rng.uniform(0.0, 2.0 * math.pi, size=n_modes), dtype=torch.float64, device=device)
    ax = torch.as_tensor(_axis(D).astype(np.float32), dtype=torch.float64, device=device)
    Y, X = torch.meshgrid(ax, ax, indexing="ij")
    vol = torch.empty((D, D, D), dtype=torch.float64, device=device)
    for z in range(D):
        acc = torch.zeros((D, D), dtype=torch.float64, device=device)
        for j0 in range(0, n_modes, 64):
            kk = kv[j0:j0 + 64]
            arg = X[..., None] * kk[:, 0] + Y[..., None] * kk[:, 1] + ax[z] * kk[:, 2] + phase[j0:j0 + 64]
            acc += (torch.cos(arg) * amp[j0:j0 + 64]).sum(-1)
        vol[z] = acc
    vol -= vol.min()
    vol /= vol.max()
    return vol.float().contiguous()


def marschner_lobb_volume(D: int, fm: float = 6.0, alpha: float = 0.25) -> np.ndarray:
    """Marschner-Lobb test signal sampled at the D^3 vertices of [-1,1]^3.
    float32 [D][D][D] in [0, 1]."""
    ax = _axis(D)
    out = np.empty((D, D, D), dtype=np.float32)
    Y, X = np.meshgrid(ax, ax, indexing="ij")
    r = np.sqrt(X * X + Y * Y)
    radial = np.cos(2.0 * math.pi * fm * np.cos(math.pi * r / 2.0))
    for z in range(D):
        out[z] = (1.0 - math.sin(math.pi * ax[z] / 2.0) + alpha * (1.0 + radial)) / (2.0 * (1.0 + alpha))
    return out


def blob_sequence_params(n_blobs: int = 32, seed: int = 1005):
    """Centres, per-step velocities, widths and amplitudes of the advected
    isotropic blobs of the time-varying workload."""
    rng = np.random.default_rng(seed)
    c0 = rng.uniform(-0.6, 0.6, size=(n_blobs, 3))
    vel = rng.uniform(-0.04, 0.04, size=(n_blobs, 3))
    sig = rng.uniform(0.05, 0.15, size=n_blobs)
    amp = rng.uniform(0.2, 1.0, size=n_blobs)
    return c0, vel, sig, amp


def blob_volume(D: int, t: float, params, norm: float = 1.0) -> np.ndarray:
    """Blob field at (possibly fractional) timestep t, divided by ``norm``."""
    c0, vel, sig, amp = params
    ax = _axis(D)
    vol = np.zeros((D, D, D), dtype=np.float64)
    for j in range(c0.shape[0]):
        c = c0[j] + vel[j] * t
        gz = np.exp(-0.5 * ((ax - c[2]) / sig[j]) ** 2)
        gy = np.exp(-0.5 * ((ax - c[1]) / sig[j]) ** 2)
        gx = np.exp(-0.5 * ((ax - c[0]) / sig[j]) ** 2)
        vol += amp[j] * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    return (vol / norm).astype(np.float32)


def blob_volume_torch(D: int, t: float, params, norm: float = 1.0, device="cuda"):
    """``blob_volume`` evaluated with torch on ``device`` (FP64, returned as
    FP32): the same separable sum of blobs, for volumes too large to build
    quickly on the host."""
    import torch
    c0, vel, sig, amp = (torch.as_tensor(a, dtype=torch.float64, device=device) for a in params)
    ax = torch.linspace(-1.0, 1.0, D, dtype=torch.float64, device=device)
    c = c0 + vel * t                                                  # [B, 3]
    g = torch.exp(-0.5 * ((ax[None, None, :] - c[:, :, None]) / sig[:, None, None]) ** 2)  # [B, 3, D]
    vol = torch.einsum("b,bz,by,bx->zyx", amp, g[:, 2], g[:, 1], g[:, 0])
    return (vol / norm).float().contiguous()


# ------------------------------------------------------------ presets

NET_SMALL = NetSpec(R=16, F=8, L=4, c=32, H=3)       # 16^3x8 grid, 4 octaves, 3 x 32
NET_STUDY = NetSpec(R=32, F=16, L=8, c=32, H=4)      # 32^3x16 grid, 8 octaves, 4 x 32
NET_SHADED = NetSpec(R=64, F=16, L=8, c=48, H=4)     # 64^3x16 grid, 8 octaves, 4 x 48
NET_TIME = NetSpec(R=32, F=16, L=8, c=32, H=4, K=4)  # 4 keyframe grids of 32^3x16
TIME_KEYS = (0.0, 4.0, 8.0, 12.0)

SEED_SMALL, SEED_STUDY, SEED_TRAIN, SEED_SHADED, SEED_TIME = 1001, 1002, 1003, 1004, 1005


def ortho_march() -> March:
    return March(step=0.0, fixed_steps=128, ert_eps=0.0)


def study_cameras(width: int = 1024, height: int = 1024, n_views: int = 8) -> List[Camera]:
    return orbit_cameras(n_views, width, height)


def study_march(ert_eps: float = 1e-3) -> March:
    return March(step=1.0 / 256.0, ert_eps=ert_eps)


def shaded_camera(width: int = 1920, height: int = 1080) -> Camera:
    return orbit_cameras(8, width, height)[0]


def shaded_march(ert_eps: float = 1e-3) -> March:
    return March(step=1.0 / 512.0, ert_eps=ert_eps, phong=True)


def time_cameras(width: int = 1024, height: int = 1024) -> List[Camera]:
    return orbit_cameras(8, width, height, times=[0.5 + 1.5 * v for v in range(8)])
