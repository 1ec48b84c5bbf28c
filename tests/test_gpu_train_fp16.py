"""FP16-MFMA training step (forward and backward passes on FP16 MFMA with
FP32 accumulation, FP32 master parameters, gradients and Adam) against the
FP64 oracle's gradients of the FP32 network.

Tolerances: the FP16 step rounds the weights, the input row, every
activation, act' and every delta to FP16 (unit roundoff 2^-11 = 4.9e-4);
summed over the points in FP32 the weight and latent gradients stay within
a few unit roundoffs of the largest entry (measured 3.8e-4 to 1.13e-3 over
every case here), bound 3e-3 of the largest |gradient|. The loss is the
mean of |d - t| over FP16-network densities, each within a few 1e-4 of
FP64, whose errors average out (measured <= 2e-6): bound 2e-5 absolute.
Targets sit 0.01 or more away from the FP64 density, so every sign(d - t)
agrees."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2112_01579_amd import inputs as I

pytestmark = pytest.mark.gpu

GRAD_TOL = 3e-3
LOSS_TOL = 2e-5


@pytest.fixture(scope="module")
def FV():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_01579_amd import fvsrn
    fvsrn.lib()
    return fvsrn


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)


def _targets(onet, xyz, seed):
    d = O.eval_points(onet, xyz)
    rng = np.random.default_rng(seed)
    return (d + rng.uniform(0.01, 0.3, len(xyz)) * rng.choice([-1, 1], len(xyz))).astype(np.float32)


def _step(FV, gnet, xyz, target, **kw):
    d_lat = torch.empty_like(gnet.latent)
    d_w = torch.empty_like(gnet.weights)
    loss = torch.zeros(1, device="cuda")
    FV.fvsrn_train_step(gnet, d_lat, d_w, torch.from_numpy(xyz).cuda(), target=torch.from_numpy(target).cuda(),
                        out_loss=loss, precision="f16", **kw)
    return d_lat.cpu().numpy(), d_w.cpu().numpy(), loss.item()


@pytest.mark.parametrize("spec", [I.NET_SMALL, I.NET_STUDY, I.NET_SHADED, I.NetSpec(R=12, F=8, L=4, c=48, H=2),
                                  I.NetSpec(R=12, F=16, L=8, c=32, H=6)],
                         ids=["small", "study", "shaded", "c48F8", "c32H6"])
def test_train_fp16_gradients_l1(FV, spec):
    """The four (c, F, L) shapes, one to six layers deep, a ragged point
    count (several chunks per wave group and a partial last chunk)."""
    n = 64 * 37 + 13
    lat, w = I.net_params(spec, 11)
    gnet, onet = FV.Network(spec, lat, w), O.Net(spec, lat, w)
    xyz = I.uniform_points(n, 12, -0.99, 0.99)
    target = _targets(onet, xyz, 2)
    dl_ref, dw_ref, loss_ref = O.train_grads(onet, xyz, target=target.astype(np.float64))
    d_lat, d_w, loss = _step(FV, gnet, xyz, target)
    e_w, e_l = _rel(d_w, dw_ref), _rel(d_lat, dl_ref)
    print("train fp16 c=%d F=%d L=%d H=%d: dW rel err %.3g, dG rel err %.3g, loss %.6g vs %.6g" %
          (spec.c, spec.F, spec.L, spec.H, e_w, e_l, loss, loss_ref), flush=True)
    assert e_w <= GRAD_TOL and e_l <= GRAD_TOL
    assert abs(loss - loss_ref) <= LOSS_TOL


def test_train_fp16_full_batch_and_fp32_agreement(FV):
    """The training workload's batch (2^18 points, the 16^3 x 8, 3 x 32
    network): FP16 gradients against the oracle and against the FP32 step
    on the same points; dW bitwise reproducible from call to call."""
    spec = I.NET_SMALL
    n = 1 << 18
    lat, w = I.net_params(spec, 17)
    gnet, onet = FV.Network(spec, lat, w), O.Net(spec, lat, w)
    xyz = I.uniform_points(n, 18, -0.99, 0.99)
    target = _targets(onet, xyz, 19)
    dl_ref, dw_ref, loss_ref = O.train_grads(onet, xyz, target=target.astype(np.float64))
    d_lat, d_w, loss = _step(FV, gnet, xyz, target)
    e_w, e_l = _rel(d_w, dw_ref), _rel(d_lat, dl_ref)
    print("train fp16 full batch: dW rel err %.3g, dG rel err %.3g, loss %.6g vs %.6g" % (e_w, e_l, loss, loss_ref),
          flush=True)
    assert e_w <= GRAD_TOL and e_l <= GRAD_TOL
    assert abs(loss - loss_ref) <= LOSS_TOL
    _, d_w2, _ = _step(FV, gnet, xyz, target)
    assert np.array_equal(d_w, d_w2)
    d_lat32, d_w32 = torch.empty_like(gnet.latent), torch.empty_like(gnet.weights)
    FV.fvsrn_train_step(gnet, d_lat32, d_w32, torch.from_numpy(xyz).cuda(), target=torch.from_numpy(target).cuda())
    assert _rel(d_w, d_w32.cpu().numpy()) <= GRAD_TOL and _rel(d_lat, d_lat32.cpu().numpy()) <= GRAD_TOL


@pytest.mark.parametrize("act", ["snakealt", "identity"])
def test_train_fp16_activations(FV, act):
    spec = I.NetSpec(R=16, F=8, L=4, c=32, H=3, act=act)
    n = 1000
    lat, w = I.net_params(spec, 4)
    if act == "identity":
        w = w * 0.5
    gnet, onet = FV.Network(spec, lat, w), O.Net(spec, lat, w)
    xyz = I.uniform_points(n, 6, -0.99, 0.99)
    target = _targets(onet, xyz, 3)
    dl_ref, dw_ref, loss_ref = O.train_grads(onet, xyz, target=target.astype(np.float64))
    d_lat, d_w, loss = _step(FV, gnet, xyz, target)
    e_w, e_l = _rel(d_w, dw_ref), _rel(d_lat, dl_ref)
    print("train fp16 act=%s: dW rel err %.3g, dG rel err %.3g" % (act, e_w, e_l), flush=True)
    assert e_w <= GRAD_TOL and e_l <= GRAD_TOL
    assert abs(loss - loss_ref) <= LOSS_TOL


def test_train_fp16_keyframes_and_predicted_gradient_targets(FV):
    """A four-output network on two keyframe grids, fitted to densities and
    gradient targets (Sec. 6, Sec. 8): every output row, the latent gradient
    split between the keyframes, and the loss."""
    spec = I.NetSpec(R=16, F=16, L=8, c=48, H=3, K=2, outputs=4)
    n = 64 * 21 + 9
    lat, w = I.net_params(spec, 8)
    kt = (0.0, 1.0)
    gnet, onet = FV.Network(spec, lat, w, key_times=kt), O.Net(spec, lat, w, kt)
    xyz = I.uniform_points(n, 9, -0.99, 0.99)
    times = np.random.default_rng(4).uniform(-0.2, 1.2, n).astype(np.float32)
    rng = np.random.default_rng(2)
    dref = np.empty(n)
    gref = np.empty((n, 3))
    for i in range(n):
        dref[i], gref[i] = O.density_grad(onet, xyz[i], float(times[i]), mode="pred")
    target = (dref + rng.uniform(0.01, 0.3, n) * rng.choice([-1, 1], n)).astype(np.float32)
    tgrad = (gref + rng.uniform(0.01, 0.5, (n, 3)) * rng.choice([-1, 1], (n, 3))).astype(np.float32)
    dl_ref, dw_ref, loss_ref = O.train_grads(onet, xyz, target=target.astype(np.float64), times=times,
                                             target_grad=tgrad, grad_weight=0.7)
    d_lat, d_w, loss = _step(FV, gnet, xyz, target, times=torch.from_numpy(times).cuda(),
                             target_grad=torch.from_numpy(tgrad).cuda(), grad_weight=0.7)
    e_w, e_l = _rel(d_w, dw_ref), _rel(d_lat, dl_ref)
    print("train fp16 4-output keyframes: dW rel err %.3g, dG rel err %.3g, loss %.6g vs %.6g" %
          (e_w, e_l, loss, loss_ref), flush=True)
    assert e_w <= GRAD_TOL and e_l <= GRAD_TOL
    assert abs(loss - loss_ref) <= LOSS_TOL


def test_train_fp16_unsupported(FV):
    """VJP mode, time inputs, Fourier matrices, the further (F, L) pairs and
    BF16 are not compiled for reduced-precision training."""
    xyz = torch.from_numpy(I.uniform_points(100, 1)).cuda()
    tgt = torch.zeros(100, device="cuda")
    cases = []
    spec = I.NET_SMALL
    lat, w = I.net_params(spec, 1)
    net = FV.Network(spec, lat, w)
    cases.append((net, dict(dloss_dy=torch.ones(100, device="cuda")), "f16"))
    cases.append((net, dict(target=tgt), "bf16"))
    tspec = I.NetSpec(R=8, F=8, L=4, c=32, H=2, K=2, time_enc=1)
    lat, w = I.net_params(tspec, 1)
    cases.append((FV.Network(tspec, lat, w, key_times=(0.0, 1.0)), dict(target=tgt), "f16"))
    lat, w = I.net_params(spec, 1)
    cases.append((FV.Network(spec, lat, w, fourier_matrix=I.random_fourier_matrix(spec.L, 1.0, 3)),
                  dict(target=tgt), "f16"))
    espec = I.NetSpec(R=8, F=16, L=4, c=32, H=2)
    lat, w = I.net_params(espec, 1)
    cases.append((FV.Network(espec, lat, w), dict(target=tgt), "f16"))
    for net, kw, prec in cases:
        with pytest.raises(FV.FvsrnError) as e:
            FV.fvsrn_train_step(net, torch.empty_like(net.latent), torch.empty_like(net.weights), xyz,
                                precision=prec, **kw)
        assert e.value.status == FV.ERR_UNSUPPORTED


def test_trainer_fp16_fits_like_fp32(FV):
    """The training workload (the 16^3 x 8, 3 x 32 network fitted to the
    256^3 power-law field, 2^18 points per step) for 400 Adam steps in FP16
    and in FP32 from the same start: the FP16 fit ends within 10% of the
    FP32 fit's L1 on held-out points, both far below the untrained error."""
    from paper_2112_01579_amd.trainer import Trainer
    vol = I.power_law_volume_torch(128, 256, seed=I.SEED_STUDY)
    lat, w = I.net_params(I.NET_SMALL, 7)
    xyz = torch.from_numpy(I.uniform_points(1 << 16, 99)).cuda()
    ref = FV.fvsrn_dense_eval_points(vol, xyz)
    res = {}
    for prec in ("f32", "f16"):
        net = FV.Network(I.NET_SMALL, lat, w)
        if prec == "f32":
            res["untrained"] = torch.mean(torch.abs(FV.fvsrn_eval_points(net, xyz) - ref)).item()
        tr = Trainer(net, vol, batch=1 << 18, seed=5, precision=prec)
        for _ in range(400):
            tr.step()
        res[prec] = torch.mean(torch.abs(FV.fvsrn_eval_points(net, xyz) - ref)).item()
    print("held-out L1: untrained %.4f, fp32 %.4f, fp16 %.4f" % (res["untrained"], res["f32"], res["f16"]),
          flush=True)
    assert res["f16"] <= 1.1 * res["f32"]
    assert res["f16"] < 0.5 * res["untrained"]
