"""The C ABI without a GPU: the library loads, exports every function that
include/fvsrn.h declares, and rejects bad arguments on the host before any
launch (so these calls are safe on a machine without a GPU)."""
import ctypes as C
import os
import re

import pytest

from paper_2112_01579_amd import fvsrn as FV
from paper_2112_01579_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _built():
    return os.path.exists(FV.LIB_PATH)


pytestmark = pytest.mark.skipif(not _built(), reason="libfvsrn.so not built")


def declared_functions():
    src = open(os.path.join(ROOT, "include", "fvsrn.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(fvsrn_[a-z_]+)\s*\(", src)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 12
    L = FV.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(FV.EXPORTS) == set(names)


def test_num_weights_matches_layout():
    for spec in (I.NET_SMALL, I.NET_STUDY, I.NET_SHADED):
        assert FV.fvsrn_num_weights(spec) == spec.n_weights
    assert FV.fvsrn_num_weights(I.NET_SMALL) == 3297
    assert FV.fvsrn_num_weights(I.NET_STUDY) == 5377
    # time inputs widen layer 0 by 1, 8 or 9 columns
    for te, extra in ((1, 1), (2, 8), (3, 9)):
        spec_t = I.NetSpec(R=32, F=16, L=8, c=32, H=4, time_enc=te)
        assert FV.fvsrn_num_weights(spec_t) == spec_t.n_weights == 5377 + 32 * extra
    # four outputs add three output rows and three biases
    spec4 = I.NetSpec(R=32, F=16, L=8, c=32, H=4, outputs=4)
    assert FV.fvsrn_num_weights(spec4) == spec4.n_weights == 5377 + 3 * 33


def test_status_strings():
    L = FV.lib()
    for s in range(5):
        assert L.fvsrn_status_str(s)


def test_build_id_matches_sources():
    from paper_2112_01579_amd.build import source_hash
    assert FV.lib().fvsrn_build_id().decode() == source_hash()


FAKE = 0x10000  # aligned, never dereferenced: validation fails first


def _desc(**kw):
    d = FV.net_desc(I.NET_SMALL)
    for k, v in kw.items():
        setattr(d, k, v)
    return d


def _params(lat=FAKE, w=FAKE):
    return FV.Params(lat, w, None)


def _render(d, p=None, tf=None, cams=None, nv=1, m=None, out=FAKE):
    tf = tf or FV.tf_struct(I.ramp_tf())
    cams = cams if cams is not None else FV.camera_structs([I.ortho_camera(8, 8)])
    m = m or FV.march_struct(I.ortho_march())
    p = p or _params()
    return FV.lib().fvsrn_render(C.byref(d), C.byref(p), C.byref(tf), cams, nv, C.byref(m),
                                 C.c_void_p(out) if out else None, None, None)


def test_render_argument_errors():
    L = FV.lib()
    assert _render(_desc(grid_res=1)) == FV.ERR_INVALID_ARGUMENT
    assert _render(_desc(hidden_width=40)) == FV.ERR_UNSUPPORTED
    assert _render(_desc(grid_channels=12)) == FV.ERR_UNSUPPORTED      # F = 12 not compiled
    assert _render(_desc(num_freqs=6)) == FV.ERR_UNSUPPORTED           # L = 6 not compiled
    assert _render(_desc(hidden_width=96)) == FV.ERR_UNSUPPORTED
    # one keyframe grid must stay below 2^31 bytes (512^3 x 8 FP32 = 4 GiB)
    assert _render(_desc(grid_res=512)) == FV.ERR_UNSUPPORTED
    assert b"2^31" in L.fvsrn_last_error()
    assert _render(_desc(precision=7)) == FV.ERR_INVALID_ARGUMENT
    assert _render(_desc(activation=9)) == FV.ERR_INVALID_ARGUMENT
    assert _render(_desc(), p=_params(lat=0)) == FV.ERR_INVALID_ARGUMENT
    assert _render(_desc(), p=_params(w=FAKE + 4)) == FV.ERR_INVALID_ARGUMENT  # misaligned
    assert b"aligned" in L.fvsrn_last_error()
    assert _render(_desc(), nv=0) == FV.ERR_INVALID_ARGUMENT
    assert _render(_desc(), out=0) == FV.ERR_INVALID_ARGUMENT
    bad_tf = FV.tf_struct(I.TF(points=((0.5, 0, 0, 0, 0), (0.2, 1, 1, 1, 1))))
    assert _render(_desc(), tf=bad_tf) == FV.ERR_INVALID_ARGUMENT
    one_pt = FV.tf_struct(I.TF(points=((0.5, 0, 0, 0, 0),)))
    assert _render(_desc(), tf=one_pt) == FV.ERR_INVALID_ARGUMENT
    cams = FV.camera_structs([I.ortho_camera(8, 8), I.ortho_camera(8, 9)])
    assert _render(_desc(), cams=cams, nv=2) == FV.ERR_INVALID_ARGUMENT
    m = FV.march_struct(I.March(step=0.0, fixed_steps=0))
    assert _render(_desc(), m=m) == FV.ERR_INVALID_ARGUMENT
    m = FV.march_struct(I.March(step=0.1, ert_eps=-1.0))
    assert _render(_desc(), m=m) == FV.ERR_INVALID_ARGUMENT
    m = FV.march_struct(I.March(step=0.1, grad_mode=5))
    assert _render(_desc(), m=m) == FV.ERR_INVALID_ARGUMENT
    # time encodings: known values and a proper time range
    for te in (-1, 4):
        assert _render(_desc(time_encoding=te)) == FV.ERR_INVALID_ARGUMENT
    for lo, hi in ((1.0, 1.0), (2.0, 1.0), (0.0, float("nan")), (float("-inf"), 1.0)):
        assert _render(_desc(time_encoding=1, time_lo=lo, time_hi=hi)) == FV.ERR_INVALID_ARGUMENT
    assert b"time" in L.fvsrn_last_error()
    # a Fourier matrix: finite entries, no time encoding alongside
    fm = (C.c_float * 36)(*([1.0] * 35 + [float("inf")]))   # 3L x 3 entries for L = 4
    d = _desc()
    d.fourier_matrix = C.cast(fm, C.POINTER(C.c_float))
    assert _render(d) == FV.ERR_INVALID_ARGUMENT
    fm[35] = 2.0
    d.time_encoding, d.time_lo, d.time_hi = 1, 0.0, 1.0
    assert _render(d) == FV.ERR_UNSUPPORTED
    # network outputs: 1 or 4; predicted-gradient shading needs 4
    for no in (2, 3, 5, -1):
        assert _render(_desc(num_outputs=no)) == FV.ERR_INVALID_ARGUMENT
    m = FV.march_struct(I.March(step=0.1, phong=True, grad_mode=2))
    assert _render(_desc(), m=m) == FV.ERR_INVALID_ARGUMENT
    assert b"num_outputs" in L.fvsrn_last_error()
    for h in (0.0, -0.1, 1.5, float("nan")):
        m = FV.march_struct(I.March(step=0.1, phong=True, grad_mode=1, fd_step=h))
        assert _render(_desc(), m=m) == FV.ERR_INVALID_ARGUMENT
        assert b"fd_step" in L.fvsrn_last_error()
    # Phong coefficients: finite, non-negative, at most 1e6
    for field, bad in (("shininess", -1.0), ("shininess", float("inf")), ("ka", float("nan")), ("kd", -0.5),
                       ("ks", 2e6)):
        m = FV.march_struct(I.March(step=0.1, phong=True, grad_mode=0))
        setattr(m, field, bad)
        assert _render(_desc(), m=m) == FV.ERR_INVALID_ARGUMENT
        assert field.encode() in L.fvsrn_last_error()
    # unshaded renders ignore the Phong coefficients
    m = FV.march_struct(I.March(step=0.1, phong=False))
    m.shininess = -1.0
    assert _render(_desc(), m=m, out=0) == FV.ERR_INVALID_ARGUMENT   # fails on out, not on shininess
    assert b"out_rgba" in L.fvsrn_last_error()
    # time-varying needs ascending key times
    d = _desc(num_keyframes=2)
    kt = (C.c_float * 2)(1.0, 1.0)
    p = FV.Params(FAKE, FAKE, C.cast(kt, C.POINTER(C.c_float)))
    assert _render(d, p=p) == FV.ERR_INVALID_ARGUMENT
    p = FV.Params(FAKE, FAKE, None)
    assert _render(d, p=p) == FV.ERR_INVALID_ARGUMENT


def test_points_argument_errors_and_empty_noop():
    L = FV.lib()
    d, p = _desc(), _params()
    assert L.fvsrn_eval_points(C.byref(d), C.byref(p), C.c_void_p(FAKE), -1, 0.0, C.c_void_p(FAKE), None) \
        == FV.ERR_INVALID_ARGUMENT
    # n == 0 is a no-op that touches nothing
    assert L.fvsrn_eval_points(C.byref(d), C.byref(p), None, 0, 0.0, None, None) == FV.OK
    for gm in (0, 3):
        assert L.fvsrn_grad_points(C.byref(d), C.byref(p), None, 0, 0.0, gm, None, None, None) == FV.OK
    # central differences are not offered for points; unknown modes are rejected
    for gm in (1, 4, -1):
        assert L.fvsrn_grad_points(C.byref(d), C.byref(p), C.c_void_p(FAKE), 5, 0.0, gm, None, C.c_void_p(FAKE),
                                   None) == FV.ERR_INVALID_ARGUMENT
    assert L.fvsrn_eval_points(C.byref(d), C.byref(p), C.c_void_p(FAKE + 8), 5, 0.0, C.c_void_p(FAKE), None) \
        == FV.ERR_INVALID_ARGUMENT
    assert L.fvsrn_grad_points(C.byref(d), C.byref(p), C.c_void_p(FAKE), 5, 0.0, 0, None, None, None) \
        == FV.ERR_INVALID_ARGUMENT
    assert L.fvsrn_dense_eval_points(C.c_void_p(FAKE), 1, 4, 4, C.c_void_p(FAKE), 3, C.c_void_p(FAKE), None) \
        == FV.ERR_INVALID_ARGUMENT
    assert L.fvsrn_dense_eval_points(C.c_void_p(FAKE), 4, 4, 4, None, 0, None, None) == FV.OK
    assert L.fvsrn_dense_grad_points(C.c_void_p(FAKE), 4, 4, 4, None, 0, None, None, None) == FV.OK
    assert L.fvsrn_dense_grad_points(C.c_void_p(FAKE), 4, 4, 4, C.c_void_p(FAKE), 3, None, None, None) \
        == FV.ERR_INVALID_ARGUMENT
    assert L.fvsrn_dense_grad_points(C.c_void_p(FAKE), 4, 1, 4, C.c_void_p(FAKE), 3, None, C.c_void_p(FAKE),
                                     None) == FV.ERR_INVALID_ARGUMENT
    # predicted gradients need a 4-output network
    assert L.fvsrn_grad_points(C.byref(d), C.byref(p), C.c_void_p(FAKE), 5, 0.0, 2, None, C.c_void_p(FAKE),
                               None) == FV.ERR_INVALID_ARGUMENT
    assert b"num_outputs" in L.fvsrn_last_error()
    d4 = _desc(num_outputs=4)
    assert L.fvsrn_grad_points(C.byref(d4), C.byref(p), None, 0, 0.0, 2, None, None, None) == FV.OK
    assert L.fvsrn_grad_points(C.byref(d4), C.byref(p), C.c_void_p(FAKE), 5, 0.0, 2, None, None, None) \
        == FV.ERR_INVALID_ARGUMENT
    assert L.fvsrn_sample_points(1, 2, 0, None, None) == FV.OK
    assert L.fvsrn_sample_points(1, 2, -3, None, None) == FV.ERR_INVALID_ARGUMENT
    assert L.fvsrn_cast_grid(C.c_void_p(FAKE), C.c_void_p(FAKE), 4, 0, None) == FV.ERR_INVALID_ARGUMENT
    assert L.fvsrn_cast_grid(None, None, 0, 1, None) == FV.OK


def test_weighted_multi_draw_argument_errors():
    """The batched weighted draw checks its grid count, point counts and
    workspace slices on the host; all-zero counts launch nothing."""
    L = FV.lib()
    P = C.c_void_p
    stride = FV.weighted_points_stride(8)
    assert stride % 16 == 0 and stride >= L.fvsrn_weighted_points_workspace_size(8)

    def call(counts, G=8, n_grids=None, stride=stride, ws=FAKE, xyz=FAKE):
        arr = (C.c_int64 * max(len(counts), 1))(*counts)
        return L.fvsrn_sample_points_weighted_multi(1, 2, G, len(counts) if n_grids is None else n_grids, arr,
                                                    P(xyz) if xyz else None, P(ws) if ws else None, stride, None)
    assert call([0, 0, 0]) == FV.OK
    assert call([4], n_grids=0) == FV.ERR_INVALID_ARGUMENT
    assert call([4] * 65) == FV.ERR_INVALID_ARGUMENT
    assert call([4, -1]) == FV.ERR_INVALID_ARGUMENT
    assert call([4], G=0) == FV.ERR_INVALID_ARGUMENT
    assert call([4], xyz=None) == FV.ERR_INVALID_ARGUMENT
    assert call([4], stride=stride - 16) == FV.ERR_WORKSPACE
    assert call([4], stride=stride + 8) == FV.ERR_WORKSPACE
    assert call([4], ws=None) == FV.ERR_WORKSPACE
    assert L.fvsrn_sample_points_weighted_multi(1, 2, 8, 1, None, P(FAKE), P(FAKE), stride, None) \
        == FV.ERR_INVALID_ARGUMENT


def _train(d, key_times=None, xyz=FAKE, times=None, n=4, target=FAKE, dloss=None, adam=None, target_grad=None,
           grad_weight=0.0):
    L = FV.lib()
    P = C.c_void_p
    return L.fvsrn_train_step(C.byref(d), P(FAKE), P(FAKE), key_times, P(FAKE), P(FAKE),
                              P(xyz) if xyz else None, P(times) if times else None, n,
                              P(target) if target else None, P(target_grad) if target_grad else None,
                              grad_weight, P(dloss) if dloss else None,
                              C.byref(adam) if adam is not None else None, None, None, 0, None)


def test_train_argument_errors():
    L = FV.lib()
    d = _desc()
    # FP16 latent grids and BF16 are not trainable; FP16 trains in L1 mode only
    assert _train(_desc(grid_dtype=1)) == FV.ERR_UNSUPPORTED
    assert _train(_desc(precision=2)) == FV.ERR_UNSUPPORTED
    assert _train(_desc(precision=1), target=None, dloss=FAKE) == FV.ERR_UNSUPPORTED
    assert _train(_desc(precision=1)) == FV.ERR_WORKSPACE  # past the precision checks
    # keyframe grids need ascending key times
    dk = _desc(num_keyframes=2)
    assert _train(dk) == FV.ERR_INVALID_ARGUMENT
    kt = (C.c_float * 2)(1.0, 1.0)
    assert _train(dk, key_times=C.cast(kt, C.POINTER(C.c_float))) == FV.ERR_INVALID_ARGUMENT
    # ... and all K grids within 2^31 bytes (8 x 256^3 x 8 FP32 = 4 GiB)
    kt8 = (C.c_float * 8)(*range(8))
    assert _train(_desc(num_keyframes=8, grid_res=256), key_times=C.cast(kt8, C.POINTER(C.c_float))) \
        == FV.ERR_UNSUPPORTED
    assert b"2^31" in L.fvsrn_last_error()
    # misaligned times
    assert _train(d, times=FAKE + 2) == FV.ERR_INVALID_ARGUMENT
    # neither target nor upstream gradient
    assert _train(d, target=None) == FV.ERR_INVALID_ARGUMENT
    # missing Adam moments, Adam step 0
    a = FV.AdamStruct(1e-2, 1e-3, 0.9, 0.999, 1e-8, 1, FAKE, None, FAKE, FAKE)
    assert _train(d, adam=a) == FV.ERR_INVALID_ARGUMENT
    a = FV.AdamStruct(1e-2, 1e-3, 0.9, 0.999, 1e-8, 0, FAKE, FAKE, FAKE, FAKE)
    assert _train(d, adam=a) == FV.ERR_INVALID_ARGUMENT
    # a workspace is required once there are points
    assert _train(d) == FV.ERR_WORKSPACE
    # gradient targets: 4-output networks in L1 mode, finite non-negative weight
    assert _train(d, target_grad=FAKE, grad_weight=1.0) == FV.ERR_INVALID_ARGUMENT
    assert b"num_outputs" in L.fvsrn_last_error()
    d4 = _desc(num_outputs=4)
    assert _train(d4, target_grad=FAKE, grad_weight=1.0) == FV.ERR_WORKSPACE
    assert _train(d4, target=None, dloss=FAKE, target_grad=FAKE) == FV.ERR_INVALID_ARGUMENT
    for w in (-1.0, float("nan"), float("inf")):
        assert _train(d4, target_grad=FAKE, grad_weight=w) == FV.ERR_INVALID_ARGUMENT
    assert _train(d4, target_grad=FAKE + 2, grad_weight=1.0) == FV.ERR_INVALID_ARGUMENT