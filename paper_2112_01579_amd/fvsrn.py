"""ctypes binding of the C ABI in ``include/fvsrn.h``.

Argument marshalling only: every step of the path runs in the HIP library
``libfvsrn.so``. torch tensors provide device memory and streams. The library
must have been built (``paper_2112_01579_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional, Sequence

import numpy as np
import torch

from . import inputs as I

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfvsrn.so")

F32, F16, BF16, U8 = 0, 1, 2, 3
ACT = {"sine": 0, "snakealt": 1, "identity": 2}
PREC = {"f32": F32, "fp32": F32, "f16": F16, "fp16": F16, "bf16": BF16}

OK, ERR_INVALID_ARGUMENT, ERR_UNSUPPORTED, ERR_WORKSPACE, ERR_DEVICE = 0, 1, 2, 3, 4

EXPORTS = (
    "fvsrn_render", "fvsrn_eval_points", "fvsrn_grad_points", "fvsrn_train_step",
    "fvsrn_train_workspace_size", "fvsrn_render_dense", "fvsrn_dense_eval_points", "fvsrn_dense_grad_points",
    "fvsrn_sample_points", "fvsrn_cast_grid", "fvsrn_quantize_grid", "fvsrn_ssim_map", "fvsrn_num_weights",
    "fvsrn_voxel_points", "fvsrn_error_grid", "fvsrn_sample_points_weighted", "fvsrn_weighted_points_workspace_size",
    "fvsrn_status_str", "fvsrn_last_error", "fvsrn_build_id", "fvsrn_train_step_noalloc",
    "fvsrn_sample_points_weighted_multi",
)


class FvsrnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


class FvsrnArgumentError(FvsrnError, ValueError):
    """A tensor argument the binding refuses before anything reaches the library."""

    def __init__(self, msg: str):
        super().__init__(ERR_INVALID_ARGUMENT, msg)


class NetDesc(C.Structure):
    _fields_ = [("grid_res", C.c_int32), ("grid_channels", C.c_int32), ("grid_dtype", C.c_int32),
                ("num_keyframes", C.c_int32), ("num_freqs", C.c_int32), ("hidden_width", C.c_int32),
                ("hidden_layers", C.c_int32), ("activation", C.c_int32), ("precision", C.c_int32),
                ("num_outputs", C.c_int32), ("time_encoding", C.c_int32), ("time_lo", C.c_float),
                ("time_hi", C.c_float), ("fourier_matrix", C.POINTER(C.c_float))]


class Params(C.Structure):
    _fields_ = [("latent", C.c_void_p), ("weights", C.c_void_p), ("key_times", C.POINTER(C.c_float)),
                ("latent_dequant", C.c_void_p)]


class TFStruct(C.Structure):
    _fields_ = [("n", C.c_int32), ("density", C.c_float * 16), ("rgba", (C.c_float * 4) * 16),
                ("opacity_scale", C.c_float)]


class CameraStruct(C.Structure):
    _fields_ = [("ortho", C.c_int32), ("eye", C.c_float * 3), ("target", C.c_float * 3),
                ("up", C.c_float * 3), ("fov_y_deg", C.c_float), ("ortho_half_extent", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32), ("time", C.c_float)]


class MarchStruct(C.Structure):
    _fields_ = [("step", C.c_float), ("fixed_steps", C.c_int32), ("ert_eps", C.c_float),
                ("phong", C.c_int32), ("ka", C.c_float), ("kd", C.c_float), ("ks", C.c_float),
                ("shininess", C.c_float), ("grad_mode", C.c_int32), ("fd_step", C.c_float)]


class AdamStruct(C.Structure):
    _fields_ = [("lr_grid", C.c_float), ("lr_mlp", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("step", C.c_int32),
                ("m_latent", C.c_void_p), ("v_latent", C.c_void_p), ("m_weights", C.c_void_p),
                ("v_weights", C.c_void_p)]


_lib = None


def lib():
    """Load libfvsrn.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libfvsrn.so is not built; run paper_2112_01579_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        st = C.c_int
        sig = {
            "fvsrn_render": (st, [vp, vp, vp, vp, i32, vp, vp, vp, vp]),
            "fvsrn_eval_points": (st, [vp, vp, vp, i64, C.c_float, vp, vp]),
            "fvsrn_grad_points": (st, [vp, vp, vp, i64, C.c_float, i32, vp, vp, vp]),
            "fvsrn_train_step": (st, [vp, vp, vp, C.POINTER(C.c_float), vp, vp, vp, vp, i64, vp, vp, C.c_float,
                                      vp, vp, vp, vp, sz, vp]),
            "fvsrn_train_step_noalloc": (st, [vp, vp, vp, C.POINTER(C.c_float), vp, vp, vp, vp, i64, vp, vp,
                                              C.c_float, vp, vp, vp, vp]),
            "fvsrn_train_workspace_size": (sz, [vp, i64]),
            "fvsrn_render_dense": (st, [vp, i32, i32, i32, vp, vp, i32, vp, vp, vp, vp]),
            "fvsrn_dense_eval_points": (st, [vp, i32, i32, i32, vp, i64, vp, vp]),
            "fvsrn_dense_grad_points": (st, [vp, i32, i32, i32, vp, i64, vp, vp, vp]),
            "fvsrn_sample_points": (st, [C.c_uint64, C.c_uint64, i64, vp, vp]),
            "fvsrn_cast_grid": (st, [vp, vp, i64, i32, vp]),
            "fvsrn_quantize_grid": (st, [vp, i64, i32, vp, vp, vp]),
            "fvsrn_ssim_map": (st, [vp, vp, i32, i32, i32, vp, vp]),
            "fvsrn_num_weights": (i64, [vp]),
            "fvsrn_voxel_points": (st, [C.c_uint64, C.c_uint64, i32, i32, vp, vp]),
            "fvsrn_error_grid": (st, [vp, vp, vp, i32, i32, i32, vp, i64, i32, C.c_float, vp, vp, vp]),
            "fvsrn_sample_points_weighted": (st, [C.c_uint64, C.c_uint64, vp, i32, i64, vp, vp, sz, vp]),
            "fvsrn_sample_points_weighted_multi": (st, [C.c_uint64, C.c_uint64, i32, i32, C.POINTER(C.c_int64), vp,
                                                        vp, sz, vp]),
            "fvsrn_weighted_points_workspace_size": (sz, [i32]),
            "fvsrn_status_str": (C.c_char_p, [st]),
            "fvsrn_last_error": (C.c_char_p, []),
            "fvsrn_build_id": (C.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        from .build import source_hash
        built, here = L.fvsrn_build_id().decode(), source_hash()
        if built != here:
            raise RuntimeError("libfvsrn.so was built from other sources (build id %s..., sources %s...); "
                               "rebuild with paper_2112_01579_amd.build.build()" % (built[:12], here[:12]))
        _lib = L
    return _lib


def _check(status: int, what: str):
    if status != OK:
        L = lib()
        raise FvsrnError(status, "%s: %s (%s)" % (what, L.fvsrn_status_str(status).decode(),
                                                  L.fvsrn_last_error().decode()))


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def check_tensor(t, name: str, dtype=torch.float32, shape=None, numel=None, device=None):
    """Validates a tensor handed to the library: a torch tensor of ``dtype``,
    of the given shape (None entries match any size) or element count,
    contiguous, and on a GPU (``device`` when given). Raises
    FvsrnArgumentError before any library call."""
    if not isinstance(t, torch.Tensor):
        raise FvsrnArgumentError("%s must be a torch tensor, got %s" % (name, type(t).__name__))
    if t.dtype != dtype:
        raise FvsrnArgumentError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if shape is not None and (t.dim() != len(shape) or
                              any(w is not None and w != g for w, g in zip(shape, t.shape))):
        raise FvsrnArgumentError("%s must have shape %s, got %s" % (
            name, tuple("*" if w is None else w for w in shape), tuple(t.shape)))
    if numel is not None and t.numel() != numel:
        raise FvsrnArgumentError("%s must hold %d elements, got %d" % (name, numel, t.numel()))
    if not t.is_contiguous():
        raise FvsrnArgumentError("%s must be contiguous" % name)
    if t.device.type != "cuda":
        raise FvsrnArgumentError("%s must be on a GPU, got %s" % (name, t.device))
    if device is not None and t.device != torch.device(device):
        raise FvsrnArgumentError("%s must be on %s, got %s" % (name, device, t.device))
    return t


def _check_net(net: "Network"):
    check_tensor(net.weights, "net.weights", numel=net.spec.n_weights)
    dev = net.weights.device
    want = {F32: torch.float32, F16: torch.float16, U8: torch.uint8}[net.grid_dtype]
    check_tensor(net.latent, "net.latent", dtype=want, numel=net.spec.n_latent, device=dev)
    if net.dequant is not None:
        check_tensor(net.dequant, "net.dequant", numel=net.spec.K * net.spec.F * 2, device=dev)
    return dev


def _check_points(xyz, dev):
    return check_tensor(xyz, "xyz", shape=(None, 3), device=dev)


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


# ----------------------------------------------------------- structs

def net_desc(spec: I.NetSpec, precision="f32", grid_dtype=F32, time_range=(0.0, 1.0), fourier=None) -> NetDesc:
    """fourier: a ctypes float array [3L*3] (the Fourier matrix) or None."""
    return NetDesc(spec.R, spec.F, grid_dtype, spec.K, spec.L, spec.c, spec.H, ACT[spec.act],
                   PREC[precision] if isinstance(precision, str) else precision, spec.outputs, spec.time_enc,
                   float(time_range[0]), float(time_range[1]),
                   C.cast(fourier, C.POINTER(C.c_float)) if fourier is not None else None)


def tf_struct(tf: I.TF) -> TFStruct:
    s = TFStruct()
    s.n = len(tf.points)
    for i, (d, r, g, b, a) in enumerate(tf.points):
        s.density[i] = d
        s.rgba[i][0], s.rgba[i][1], s.rgba[i][2], s.rgba[i][3] = r, g, b, a
    s.opacity_scale = tf.opacity_scale
    return s


def camera_structs(cams: Sequence[I.Camera]):
    arr = (CameraStruct * len(cams))()
    for k, c in enumerate(cams):
        s = arr[k]
        s.ortho = 1 if c.ortho else 0
        for a in range(3):
            s.eye[a], s.target[a], s.up[a] = c.eye[a], c.target[a], c.up[a]
        s.fov_y_deg, s.ortho_half_extent = c.fov_y_deg, c.ortho_half_extent
        s.width, s.height, s.time = c.width, c.height, c.time
    return arr


def march_struct(m: I.March) -> MarchStruct:
    return MarchStruct(m.step, m.fixed_steps, m.ert_eps, 1 if m.phong else 0, m.ka, m.kd, m.ks,
                       m.shininess, m.grad_mode, m.fd_step)


class Network:
    """Device-resident fV-SRN: latent grid (FP32, FP16 or uint8 codes with a
    per-channel offset and scale), FP32 weights and (host) keyframe times."""

    def __init__(self, spec: I.NetSpec, latent, weights, key_times=None, device="cuda",
                 grid_dtype=F32, time_range=None, fourier_matrix=None):
        """time_range (lo, hi): normalisation of the time input of a network
        with a time encoding (default: the first and last key time).
        fourier_matrix: [3L][3] angular frequencies (random Fourier features);
        None keeps the octave construction."""
        self.spec = spec
        self._fm = None
        if fourier_matrix is not None:
            fm = np.asarray(fourier_matrix, dtype=np.float32).reshape(-1)
            assert fm.size == 9 * spec.L
            self._fm = (C.c_float * fm.size)(*fm.tolist())
        if time_range is None:
            time_range = (key_times[0], key_times[-1]) if (spec.time_enc and key_times is not None) else (0.0, 1.0)
        self.time_range = (float(time_range[0]), float(time_range[1]))
        lat = torch.as_tensor(latent, dtype=torch.float32).reshape(-1).contiguous().to(device)
        self.dequant = None
        if grid_dtype == F16:
            half = torch.empty(lat.numel(), dtype=torch.float16, device=device)
            fvsrn_cast_grid(lat, half, F16)
            lat = half
        elif grid_dtype == U8:
            per = lat.numel() // spec.K
            codes = torch.empty(lat.numel(), dtype=torch.uint8, device=device)
            self.dequant = torch.empty((spec.K, spec.F, 2), dtype=torch.float32, device=device)
            for k in range(spec.K):
                fvsrn_quantize_grid(lat[k * per:(k + 1) * per], spec.F, codes[k * per:(k + 1) * per],
                                    self.dequant[k])
            lat = codes
        self.latent = lat
        self.grid_dtype = grid_dtype
        self.weights = torch.as_tensor(weights, dtype=torch.float32).reshape(-1).contiguous().to(device)
        if spec.K > 1:
            kt = list(key_times)
            self._kt = (C.c_float * len(kt))(*kt)
        else:
            self._kt = None
        assert self.weights.numel() == spec.n_weights
        assert self.latent.numel() == spec.n_latent

    def desc(self, precision="f32") -> NetDesc:
        return net_desc(self.spec, precision, self.grid_dtype, self.time_range, self._fm)

    def params(self) -> Params:
        return Params(self.latent.data_ptr(), self.weights.data_ptr(),
                      C.cast(self._kt, C.POINTER(C.c_float)) if self._kt is not None else None,
                      self.dequant.data_ptr() if self.dequant is not None else None)


# ----------------------------------------------------------- calls

def fvsrn_render(net: Network, tf: I.TF, cams: Sequence[I.Camera], march: I.March,
                 precision="f32", out: Optional[torch.Tensor] = None,
                 stats: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    cams = list(cams)
    dev = _check_net(net)
    if out is None:
        out = torch.empty((len(cams), cams[0].height, cams[0].width, 4), dtype=torch.float32, device=dev)
    check_tensor(out, "out", shape=(len(cams), cams[0].height, cams[0].width, 4), device=dev)
    if stats is not None:
        check_tensor(stats, "stats", dtype=torch.int64, numel=3, device=dev)
    d, p, t, cs, m = net.desc(precision), net.params(), tf_struct(tf), camera_structs(cams), march_struct(march)
    _check(lib().fvsrn_render(C.byref(d), C.byref(p), C.byref(t), cs, len(cams), C.byref(m), _ptr(out),
                              _ptr(stats), _stream(stream)), "fvsrn_render")
    return out


def fvsrn_eval_points(net: Network, xyz: torch.Tensor, time: float = 0.0, precision="f32",
                      out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    dev = _check_net(net)
    _check_points(xyz, dev)
    n = xyz.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=xyz.device)
    check_tensor(out, "out", numel=n, device=dev)
    d, p = net.desc(precision), net.params()
    _check(lib().fvsrn_eval_points(C.byref(d), C.byref(p), _ptr(xyz), n, time, _ptr(out), _stream(stream)),
           "fvsrn_eval_points")
    return out


GRAD_MODES = {"forward": 0, "central": 1, "predicted": 2, "adjoint": 3}


def fvsrn_grad_points(net: Network, xyz: torch.Tensor, time: float = 0.0, precision="f32", mode="forward",
                      stream=None):
    """Density and d density / d p at points: forward mode, adjoint (reverse
    mode) or a 4-output network's predicted gradient (``mode``)."""
    dev = _check_net(net)
    _check_points(xyz, dev)
    if mode not in GRAD_MODES:
        raise FvsrnArgumentError("mode must be one of %s" % sorted(GRAD_MODES))
    n = xyz.shape[0]
    dens = torch.empty(n, dtype=torch.float32, device=xyz.device)
    grad = torch.empty((n, 3), dtype=torch.float32, device=xyz.device)
    d, p = net.desc(precision), net.params()
    _check(lib().fvsrn_grad_points(C.byref(d), C.byref(p), _ptr(xyz), n, time, GRAD_MODES[mode], _ptr(dens),
                                   _ptr(grad), _stream(stream)), "fvsrn_grad_points")
    return dens, grad


def fvsrn_pred_grad_points(net: Network, xyz: torch.Tensor, time: float = 0.0, precision="f32", stream=None):
    """Density and the predicted gradient (outputs 1..3) of a 4-output network."""
    return fvsrn_grad_points(net, xyz, time, precision, "predicted", stream)


def fvsrn_render_dense(vol: torch.Tensor, tf: I.TF, cams: Sequence[I.Camera], march: I.March,
                       out: Optional[torch.Tensor] = None, stats: Optional[torch.Tensor] = None,
                       stream=None) -> torch.Tensor:
    cams = list(cams)
    check_tensor(vol, "vol", shape=(None, None, None))
    nz, ny, nx = vol.shape
    if out is None:
        out = torch.empty((len(cams), cams[0].height, cams[0].width, 4), dtype=torch.float32,
                          device=vol.device)
    check_tensor(out, "out", shape=(len(cams), cams[0].height, cams[0].width, 4), device=vol.device)
    if stats is not None:
        check_tensor(stats, "stats", dtype=torch.int64, numel=3, device=vol.device)
    t, cs, m = tf_struct(tf), camera_structs(cams), march_struct(march)
    _check(lib().fvsrn_render_dense(_ptr(vol), nx, ny, nz, C.byref(t), cs, len(cams), C.byref(m), _ptr(out),
                                    _ptr(stats), _stream(stream)), "fvsrn_render_dense")
    return out


def fvsrn_dense_eval_points(vol: torch.Tensor, xyz: torch.Tensor, out=None, stream=None):
    check_tensor(vol, "vol", shape=(None, None, None))
    _check_points(xyz, vol.device)
    nz, ny, nx = vol.shape
    n = xyz.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=xyz.device)
    check_tensor(out, "out", numel=n, device=vol.device)
    _check(lib().fvsrn_dense_eval_points(_ptr(vol), nx, ny, nz, _ptr(xyz), n, _ptr(out), _stream(stream)),
           "fvsrn_dense_eval_points")
    return out


def fvsrn_dense_grad_points(vol: torch.Tensor, xyz: torch.Tensor, out=None, out_grad=None, stream=None):
    """Trilinear samples of a dense grid and their one-voxel central-difference gradients."""
    check_tensor(vol, "vol", shape=(None, None, None))
    _check_points(xyz, vol.device)
    nz, ny, nx = vol.shape
    n = xyz.shape[0]
    dens = out if out is not None else torch.empty(n, dtype=torch.float32, device=xyz.device)
    grad = out_grad if out_grad is not None else torch.empty((n, 3), dtype=torch.float32, device=xyz.device)
    check_tensor(dens, "out", numel=n, device=vol.device)
    check_tensor(grad, "out_grad", shape=(n, 3), device=vol.device)
    _check(lib().fvsrn_dense_grad_points(_ptr(vol), nx, ny, nz, _ptr(xyz), n, _ptr(dens), _ptr(grad),
                                         _stream(stream)), "fvsrn_dense_grad_points")
    return dens, grad


def fvsrn_sample_points(seed: int, counter: int, n: int, out=None, device="cuda", stream=None):
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float32, device=device)
    check_tensor(out, "out", shape=(n, 3))
    _check(lib().fvsrn_sample_points(seed, counter, n, _ptr(out), _stream(stream)), "fvsrn_sample_points")
    return out


def fvsrn_voxel_points(seed: int, counter: int, G: int, per_voxel: int, out=None, device="cuda", stream=None):
    """per_voxel positions in each of the G^3 voxels (error-grid samples, Sec. 5.4)."""
    if out is None:
        out = torch.empty((G ** 3 * per_voxel, 3), dtype=torch.float32, device=device)
    check_tensor(out, "out", shape=(G ** 3 * per_voxel, 3))
    _check(lib().fvsrn_voxel_points(seed, counter, G, per_voxel, _ptr(out), _stream(stream)), "fvsrn_voxel_points")
    return out


def fvsrn_error_grid(net: "Network", vol: torch.Tensor, xyz: torch.Tensor, per_voxel: int, time: float = 0.0,
                     out=None, scratch=None, stream=None):
    """Mean |density - trilinear target| per voxel (Sec. 5.4), FP32 network."""
    dev = _check_net(net)
    check_tensor(vol, "vol", shape=(None, None, None), device=dev)
    _check_points(xyz, dev)
    if per_voxel < 1 or xyz.shape[0] % per_voxel:
        raise FvsrnArgumentError("xyz must hold a whole number of voxels of per_voxel points")
    nz, ny, nx = vol.shape
    nvox = xyz.shape[0] // per_voxel
    if out is None:
        out = torch.empty(nvox, dtype=torch.float32, device=xyz.device)
    if scratch is None:
        scratch = torch.empty(nvox * per_voxel, dtype=torch.float32, device=xyz.device)
    check_tensor(out, "out", numel=nvox, device=dev)
    check_tensor(scratch, "scratch", numel=nvox * per_voxel, device=dev)
    d, p = net.desc("f32"), net.params()
    _check(lib().fvsrn_error_grid(C.byref(d), C.byref(p), _ptr(vol), nx, ny, nz, _ptr(xyz), nvox, per_voxel, time,
                                  _ptr(out), _ptr(scratch), _stream(stream)), "fvsrn_error_grid")
    return out


def fvsrn_sample_points_weighted(seed: int, counter: int, E: Optional[torch.Tensor], G: int, n: int, out=None,
                                 workspace=None, stream=None):
    """n positions drawn in proportion to the error grid E [G^3] (Sec. 5.4).
    E None draws from the prefix sums an earlier call left in ``workspace``
    (same G, the grid unchanged since)."""
    if E is None:
        if workspace is None:
            raise FvsrnArgumentError("E None needs the workspace of an earlier call")
        dev = workspace.device
    else:
        check_tensor(E, "E", numel=G ** 3)
        dev = E.device
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float32, device=dev)
    check_tensor(out, "out", shape=(n, 3), device=dev)
    if workspace is None:
        workspace = torch.empty(lib().fvsrn_weighted_points_workspace_size(G), dtype=torch.uint8, device=dev)
    check_tensor(workspace, "workspace", dtype=torch.uint8, device=dev)
    _check(lib().fvsrn_sample_points_weighted(seed, counter, _ptr(E), G, n, _ptr(out), _ptr(workspace),
                                              workspace.numel(), _stream(stream)), "fvsrn_sample_points_weighted")
    return out


def weighted_points_stride(G: int) -> int:
    """Bytes of one workspace slice for fvsrn_sample_points_weighted_multi."""
    return (lib().fvsrn_weighted_points_workspace_size(G) + 15) // 16 * 16


def fvsrn_sample_points_weighted_multi(seed: int, counter: int, G: int, n_per_grid: Sequence[int],
                                       workspace: torch.Tensor, out=None, stream=None):
    """The draws of len(n_per_grid) calls of fvsrn_sample_points_weighted
    with E None in one launch: grid k draws n_per_grid[k] points with
    counter + k from the prefix sums in workspace slice k (``workspace``
    [n_grids][weighted_points_stride(G)] bytes, each slice left by an earlier
    call with that grid), the grids' points one after the other in ``out``."""
    counts = [int(x) for x in n_per_grid]
    stride = weighted_points_stride(G)
    check_tensor(workspace, "workspace", dtype=torch.uint8, shape=(len(counts), stride))
    n = sum(counts)
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float32, device=workspace.device)
    check_tensor(out, "out", shape=(n, 3), device=workspace.device)
    arr = (C.c_int64 * max(len(counts), 1))(*counts)
    _check(lib().fvsrn_sample_points_weighted_multi(seed, counter, G, len(counts), arr, _ptr(out), _ptr(workspace),
                                                    stride, _stream(stream)), "fvsrn_sample_points_weighted_multi")
    return out


def fvsrn_cast_grid(src: torch.Tensor, dst: torch.Tensor, dtype: int = F16, stream=None):
    if dtype not in (F16, BF16):
        raise FvsrnArgumentError("dtype must be F16 or BF16")
    check_tensor(src, "src")
    check_tensor(dst, "dst", dtype=torch.float16 if dtype == F16 else torch.bfloat16, numel=src.numel(),
                 device=src.device)
    _check(lib().fvsrn_cast_grid(_ptr(src), _ptr(dst), src.numel(), dtype, _stream(stream)),
           "fvsrn_cast_grid")
    return dst


def fvsrn_ssim_map(a: torch.Tensor, b: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None):
    """SSIM maps of [n][H][W][4] (or [H][W][4]) image pairs: [n][H-10][W-10]."""
    if a.dim() < 3 or a.shape[-1] != 4:
        raise FvsrnArgumentError("images must be [..., H, W, 4] RGBA")
    check_tensor(a, "a")
    check_tensor(b, "b", shape=tuple(a.shape), device=a.device)
    a4 = a.reshape(-1, a.shape[-3], a.shape[-2], 4)
    n, H, W = a4.shape[0], a4.shape[1], a4.shape[2]
    if out is None:
        out = torch.empty((n, H - 10, W - 10), dtype=torch.float32, device=a.device)
    check_tensor(out, "out", numel=n * max(H - 10, 0) * max(W - 10, 0), device=a.device)
    _check(lib().fvsrn_ssim_map(_ptr(a), _ptr(b), W, H, n, _ptr(out), _stream(stream)), "fvsrn_ssim_map")
    return out


def fvsrn_ssim(a: torch.Tensor, b: torch.Tensor) -> float:
    """Mean SSIM of an image pair (or of a batch of views, pooled)."""
    return float(fvsrn_ssim_map(a, b).mean().item())


def fvsrn_quantize_grid(src: torch.Tensor, channels: int, codes: Optional[torch.Tensor] = None,
                        dequant: Optional[torch.Tensor] = None, stream=None):
    """uint8 codes and (offset, scale) per channel of one keyframe grid
    (src FP32 [..., channels] on the device)."""
    if channels < 1 or src.numel() % channels:
        raise FvsrnArgumentError("src must hold a whole number of %d-channel vertices" % channels)
    check_tensor(src, "src")
    n = src.numel() // channels
    if codes is None:
        codes = torch.empty(src.numel(), dtype=torch.uint8, device=src.device)
    if dequant is None:
        dequant = torch.empty((channels, 2), dtype=torch.float32, device=src.device)
    check_tensor(codes, "codes", dtype=torch.uint8, numel=src.numel(), device=src.device)
    check_tensor(dequant, "dequant", numel=channels * 2, device=src.device)
    _check(lib().fvsrn_quantize_grid(_ptr(src), n, channels, _ptr(codes), _ptr(dequant), _stream(stream)),
           "fvsrn_quantize_grid")
    return codes, dequant


def fvsrn_num_weights(spec: I.NetSpec) -> int:
    d = net_desc(spec)
    return lib().fvsrn_num_weights(C.byref(d))


def fvsrn_train_workspace_size(spec: I.NetSpec, n: int) -> int:
    d = net_desc(spec)
    return lib().fvsrn_train_workspace_size(C.byref(d), n)


def fvsrn_train_step(net: Network, d_latent: torch.Tensor, d_weights: torch.Tensor, xyz: torch.Tensor,
                     target: Optional[torch.Tensor] = None, dloss_dy: Optional[torch.Tensor] = None,
                     adam: Optional[dict] = None, out_loss: Optional[torch.Tensor] = None,
                     workspace: Optional[torch.Tensor] = None, times: Optional[torch.Tensor] = None,
                     target_grad: Optional[torch.Tensor] = None, grad_weight: float = 0.0, stream=None,
                     precision="f32"):
    """One training step on ``net`` (FP32 latent grids and master weights;
    ``precision`` "f16" runs the network's forward and backward passes on
    FP16 MFMA, L1 targets only). ``times`` (device
    [n], optional) holds each point's keyframe time; ``target_grad`` ([n][3],
    4-output networks, L1 mode) the gradient targets of the predicted
    gradient, weighted by ``grad_weight``. ``adam`` is a dict with
    lr_grid, lr_mlp, beta1, beta2, eps, step and the four moment tensors
    m_latent, v_latent, m_weights, v_weights; None computes gradients only.
    ``workspace`` (uint8, optional) is allocated here when None."""
    _train_step(net, d_latent, d_weights, xyz, target, dloss_dy, adam, out_loss, workspace, times, target_grad,
                grad_weight, stream, noalloc=False, precision=precision)


def fvsrn_train_step_noalloc(net: Network, d_latent: torch.Tensor, d_weights: torch.Tensor, xyz: torch.Tensor,
                             target: Optional[torch.Tensor] = None, dloss_dy: Optional[torch.Tensor] = None,
                             adam: Optional[dict] = None, out_loss: Optional[torch.Tensor] = None,
                             times: Optional[torch.Tensor] = None, target_grad: Optional[torch.Tensor] = None,
                             grad_weight: float = 0.0, stream=None, precision="f32"):
    """fvsrn_train_step on the library's static per-GPU workspace: nothing
    is allocated (by the library or here). Calls on one GPU share that
    workspace and must not overlap."""
    _train_step(net, d_latent, d_weights, xyz, target, dloss_dy, adam, out_loss, None, times, target_grad,
                grad_weight, stream, noalloc=True, precision=precision)


def _train_step(net, d_latent, d_weights, xyz, target, dloss_dy, adam, out_loss, workspace, times, target_grad,
                grad_weight, stream, noalloc, precision="f32"):
    dev = _check_net(net)
    if net.grid_dtype != F32:
        raise FvsrnArgumentError("training needs an FP32 latent grid")
    _check_points(xyz, dev)
    n = xyz.shape[0]
    check_tensor(d_latent, "d_latent", numel=net.spec.n_latent, device=dev)
    check_tensor(d_weights, "d_weights", numel=net.spec.n_weights, device=dev)
    for name, t, shp in (("target", target, (n,)), ("dloss_dy", dloss_dy, (n,)), ("times", times, (n,)),
                         ("target_grad", target_grad, (n, 3))):
        if t is not None:
            check_tensor(t, name, shape=shp, device=dev)
    if out_loss is not None:
        check_tensor(out_loss, "out_loss", numel=1, device=dev)
    if adam is not None:
        for k, cnt in (("m_latent", net.spec.n_latent), ("v_latent", net.spec.n_latent),
                       ("m_weights", net.spec.n_weights), ("v_weights", net.spec.n_weights)):
            check_tensor(adam[k], "adam[%s]" % k, numel=cnt, device=dev)
    if precision not in PREC:
        raise FvsrnArgumentError("precision must be one of %s" % sorted(PREC))
    d = net.desc(precision)
    if not noalloc:
        if workspace is None:
            ws = lib().fvsrn_train_workspace_size(C.byref(d), n)
            workspace = torch.empty(max(ws, 16), dtype=torch.uint8, device=xyz.device)
        check_tensor(workspace, "workspace", dtype=torch.uint8, device=dev)
    a = None
    if adam is not None:
        a = AdamStruct(adam["lr_grid"], adam["lr_mlp"], adam.get("beta1", 0.9), adam.get("beta2", 0.999),
                       adam.get("eps", 1e-8), adam["step"], adam["m_latent"].data_ptr(),
                       adam["v_latent"].data_ptr(), adam["m_weights"].data_ptr(), adam["v_weights"].data_ptr())
    kt = C.cast(net._kt, C.POINTER(C.c_float)) if net._kt is not None else None
    if noalloc:
        _check(lib().fvsrn_train_step_noalloc(C.byref(d), _ptr(net.latent), _ptr(net.weights), kt, _ptr(d_latent),
                                              _ptr(d_weights), _ptr(xyz), _ptr(times), n, _ptr(target),
                                              _ptr(target_grad), float(grad_weight), _ptr(dloss_dy),
                                              C.byref(a) if a is not None else None, _ptr(out_loss),
                                              _stream(stream)), "fvsrn_train_step_noalloc")
        return
    _check(lib().fvsrn_train_step(C.byref(d), _ptr(net.latent), _ptr(net.weights), kt, _ptr(d_latent),
                                  _ptr(d_weights), _ptr(xyz), _ptr(times), n, _ptr(target), _ptr(target_grad),
                                  float(grad_weight), _ptr(dloss_dy),
                                  C.byref(a) if a is not None else None, _ptr(out_loss), _ptr(workspace),
                                  workspace.numel(), _stream(stream)), "fvsrn_train_step")
