"""GPU training step (fwd/bwd kernel, gradient reduction, Adam) against the
FP64 oracle. Tolerances: gradients within 1e-4 of the largest |gradient|
(FP32 sums over thousands of points); loss within 1e-5 relative; one Adam
update within 1e-6 of the oracle's update of the same gradients."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2112_01579_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def FV():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_01579_amd import fvsrn
    fvsrn.lib()
    return fvsrn


def _setup(FV, spec, seed, n):
    lat, w = I.net_params(spec, seed)
    gnet = FV.Network(spec, lat, w)
    onet = O.Net(spec, lat, w)
    xyz = I.uniform_points(n, seed + 1, -0.99, 0.99)
    return gnet, onet, xyz


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)


@pytest.mark.parametrize("spec_name", ["NET_SMALL", "NET_STUDY", "NET_SHADED"])
def test_train_gradients_l1(FV, spec_name):
    spec = getattr(I, spec_name)
    n = 64 * 37 + 13
    gnet, onet, xyz = _setup(FV, spec, 11, n)
    d = O.eval_points(onet, xyz)
    rng = np.random.default_rng(2)
    # targets away from the prediction so that sign(d - t) is the same in FP32 and FP64
    off = rng.uniform(0.01, 0.3, n) * rng.choice([-1, 1], n)
    target = (d + off).astype(np.float32)
    dl_ref, dw_ref, loss_ref = O.train_grads(onet, xyz, target=target.astype(np.float64))
    d_lat = torch.empty_like(gnet.latent)
    d_w = torch.empty_like(gnet.weights)
    loss = torch.zeros(1, device="cuda")
    FV.fvsrn_train_step(gnet, d_lat, d_w, torch.from_numpy(xyz).cuda(), target=torch.from_numpy(target).cuda(),
                        out_loss=loss)
    e_w, e_l = _rel(d_w.cpu().numpy(), dw_ref), _rel(d_lat.cpu().numpy(), dl_ref)
    print("train %s L1: dW rel err %.3g, dG rel err %.3g, loss %.6g vs %.6g" % (spec_name, e_w, e_l,
                                                                                  loss.item(), loss_ref), flush=True)
    assert e_w <= 1e-4 and e_l <= 1e-4
    # the mean of |d - t| inherits the FP32 rounding of each density (~2e-7)
    assert abs(loss.item() - loss_ref) <= 1e-5 * abs(loss_ref) + 1e-7


def test_train_gradients_full_batch(FV):
    """The training workload's launch configuration: the 16^3 x 8, 3 x 32
    network and a full batch of 2^18 points (2048 waves of eight 16-point
    chunks, eight reduction groups, the cell scan over 3,375 cells) against
    the oracle's gradients and loss for the same points and targets."""
    spec = I.NET_SMALL
    n = 1 << 18
    gnet, onet, xyz = _setup(FV, spec, 17, n)
    d = O.eval_points(onet, xyz)
    rng = np.random.default_rng(18)
    off = rng.uniform(0.01, 0.3, n) * rng.choice([-1, 1], n)
    target = (d + off).astype(np.float32)
    dl_ref, dw_ref, loss_ref = O.train_grads(onet, xyz, target=target.astype(np.float64))
    d_lat = torch.empty_like(gnet.latent)
    d_w = torch.empty_like(gnet.weights)
    loss = torch.zeros(1, device="cuda")
    FV.fvsrn_train_step(gnet, d_lat, d_w, torch.from_numpy(xyz).cuda(), target=torch.from_numpy(target).cuda(),
                        out_loss=loss)
    e_w, e_l = _rel(d_w.cpu().numpy(), dw_ref), _rel(d_lat.cpu().numpy(), dl_ref)
    print("train full batch: dW rel err %.3g, dG rel err %.3g" % (e_w, e_l), flush=True)
    assert e_w <= 1e-4 and e_l <= 1e-4
    assert abs(loss.item() - loss_ref) <= 1e-5 * abs(loss_ref) + 1e-7


@pytest.mark.parametrize("spec_name", ["NET_STUDY", "NET_SHADED"])
def test_train_gradients_full_batch_study_and_shaded(FV, spec_name):
    """A full 2^18-point batch on the 32^3 x 16 study grid (8.8 points per
    cell: the latent gradient's two-pass form, per-cell corner sums then per
    vertex) and on the 64^3 x 16 grid of the 4 x 48 network (about one point
    per cell: the one-pass gather; layer 0's first tile row in registers;
    1024 waves of sixteen 16-point chunks),
    FP32 and FP16 network passes, against the oracle."""
    spec = getattr(I, spec_name)
    n = 1 << 18
    gnet, onet, xyz = _setup(FV, spec, 23, n)
    d = O.eval_points(onet, xyz)
    rng = np.random.default_rng(24)
    target = (d + rng.uniform(0.01, 0.3, n) * rng.choice([-1, 1], n)).astype(np.float32)
    dl_ref, dw_ref, loss_ref = O.train_grads(onet, xyz, target=target.astype(np.float64))
    for prec, tol in (("f32", 1e-4), ("f16", 3e-3)):
        d_lat = torch.empty_like(gnet.latent)
        d_w = torch.empty_like(gnet.weights)
        loss = torch.zeros(1, device="cuda")
        FV.fvsrn_train_step(gnet, d_lat, d_w, torch.from_numpy(xyz).cuda(), target=torch.from_numpy(target).cuda(),
                            out_loss=loss, precision=prec)
        e_w, e_l = _rel(d_w.cpu().numpy(), dw_ref), _rel(d_lat.cpu().numpy(), dl_ref)
        print("train full batch %s %s: dW rel err %.3g, dG rel err %.3g" % (spec_name, prec, e_w, e_l), flush=True)
        assert e_w <= tol and e_l <= tol
        assert abs(loss.item() - loss_ref) <= 2e-5


def test_train_gradients_many_chunks_per_wave(FV):
    """More points than waves x chunk: waves walk several chunks and the
    reduction runs over every group of wave slices."""
    spec = I.NET_SMALL
    n = 16 * 2048 * 2 + 16 * 300 + 7
    gnet, onet, xyz = _setup(FV, spec, 21, n)
    d = O.eval_points(onet, xyz)
    rng = np.random.default_rng(5)
    target = (d + rng.uniform(0.01, 0.3, n) * rng.choice([-1, 1], n)).astype(np.float32)
    dl_ref, dw_ref, loss_ref = O.train_grads(onet, xyz, target=target.astype(np.float64))
    d_lat = torch.empty_like(gnet.latent)
    d_w = torch.empty_like(gnet.weights)
    loss = torch.zeros(1, device="cuda")
    FV.fvsrn_train_step(gnet, d_lat, d_w, torch.from_numpy(xyz).cuda(), target=torch.from_numpy(target).cuda(),
                        out_loss=loss)
    e_w, e_l = _rel(d_w.cpu().numpy(), dw_ref), _rel(d_lat.cpu().numpy(), dl_ref)
    print("train many chunks: dW rel err %.3g, dG rel err %.3g" % (e_w, e_l), flush=True)
    assert e_w <= 1e-4 and e_l <= 1e-4
    assert abs(loss.item() - loss_ref) <= 1e-5 * abs(loss_ref) + 1e-7


@pytest.mark.parametrize("act", ["sine", "snakealt", "identity"])
def test_train_gradients_vjp(FV, act):
    spec = I.NetSpec(R=16, F=8, L=4, c=32, H=3, act=act)
    n = 1000
    lat, w = I.net_params(spec, 4)
    if act == "identity":
        w = w * 0.5
    gnet, onet = FV.Network(spec, lat, w), O.Net(spec, lat, w)
    xyz = I.uniform_points(n, 6, -0.99, 0.99)
    up = np.random.default_rng(1).normal(size=n).astype(np.float32)
    dl_ref, dw_ref, loss_ref = O.train_grads(onet, xyz, dloss_dd=up.astype(np.float64))
    d_lat = torch.empty_like(gnet.latent)
    d_w = torch.empty_like(gnet.weights)
    loss = torch.zeros(1, device="cuda")
    FV.fvsrn_train_step(gnet, d_lat, d_w, torch.from_numpy(xyz).cuda(), dloss_dy=torch.from_numpy(up).cuda(),
                        out_loss=loss)
    e_w, e_l = _rel(d_w.cpu().numpy(), dw_ref), _rel(d_lat.cpu().numpy(), dl_ref)
    print("train act=%s VJP: dW rel err %.3g, dG rel err %.3g" % (act, e_w, e_l), flush=True)
    assert e_w <= 1e-4 and e_l <= 1e-4
    assert abs(loss.item() - loss_ref) <= 1e-5 * max(1.0, abs(loss_ref))


def test_train_gradients_deterministic_and_empty(FV):
    gnet, onet, xyz = _setup(FV, I.NET_SMALL, 3, 5000)
    up = torch.randn(5000, device="cuda")
    a = [torch.empty_like(gnet.weights) for _ in range(2)]
    for k in range(2):
        FV.fvsrn_train_step(gnet, torch.empty_like(gnet.latent), a[k], torch.from_numpy(xyz).cuda(), dloss_dy=up)
    assert torch.equal(a[0], a[1])
    d_lat = torch.full_like(gnet.latent, 7.0)
    d_w = torch.full_like(gnet.weights, 7.0)
    loss = torch.full((1,), 7.0, device="cuda")
    FV.fvsrn_train_step(gnet, d_lat, d_w, torch.empty((0, 3), device="cuda"), target=torch.empty(0, device="cuda"),
                        out_loss=loss)
    assert torch.count_nonzero(d_lat).item() == 0 and torch.count_nonzero(d_w).item() == 0 and loss.item() == 0.0


def test_adam_step_matches_oracle(FV):
    gnet, onet, xyz = _setup(FV, I.NET_SMALL, 5, 3000)
    target = np.random.default_rng(0).uniform(0, 1, 3000).astype(np.float32)
    opt = dict(lr_grid=1e-2, lr_mlp=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, step=0,
               m_latent=torch.zeros_like(gnet.latent), v_latent=torch.zeros_like(gnet.latent),
               m_weights=torch.zeros_like(gnet.weights), v_weights=torch.zeros_like(gnet.weights))
    lat0, w0 = gnet.latent.cpu().numpy().astype(np.float64), gnet.weights.cpu().numpy().astype(np.float64)
    d_lat, d_w = torch.empty_like(gnet.latent), torch.empty_like(gnet.weights)
    ml, vl, mw, vw = (np.zeros_like(lat0), np.zeros_like(lat0), np.zeros_like(w0), np.zeros_like(w0))
    for t in (1, 2):
        opt["step"] = t
        FV.fvsrn_train_step(gnet, d_lat, d_w, torch.from_numpy(xyz).cuda(), target=torch.from_numpy(target).cuda(),
                            adam=opt)
        # the oracle applies Adam to the gradients the GPU produced in this step,
        # with the hyperparameters as the FP32 values the C ABI receives
        f = lambda x: float(np.float32(x))
        O.adam(lat0, d_lat.cpu().numpy().astype(np.float64), ml, vl, f(1e-2), f(0.9), f(0.999), f(1e-8), t)
        O.adam(w0, d_w.cpu().numpy().astype(np.float64), mw, vw, f(1e-3), f(0.9), f(0.999), f(1e-8), t)
        assert np.abs(gnet.latent.cpu().numpy() - lat0).max() <= 1e-6
        assert np.abs(gnet.weights.cpu().numpy() - w0).max() <= 1e-6
        assert np.abs(opt["v_weights"].cpu().numpy() - vw).max() <= 1e-6 * max(1e-12, np.abs(vw).max()) + 1e-12


def test_training_reduces_loss_and_autograd(FV):
    from paper_2112_01579_amd.trainer import Trainer, fvsrn_points
    vol = torch.from_numpy(I.power_law_volume(48, 64, seed=3)).cuda()
    lat, w = I.net_params(I.NET_SMALL, 7)
    net = FV.Network(I.NET_SMALL, lat, w)
    tr = Trainer(net, vol, batch=1 << 14)
    losses = [tr.step().item() for _ in range(150)]
    print("loss first/last: %.4f %.4f" % (np.mean(losses[:10]), np.mean(losses[-10:])), flush=True)
    assert np.mean(losses[-10:]) < 0.6 * np.mean(losses[:10])
    # autograd: the gradient of sum(density * u) equals the VJP-mode train step
    xyz = torch.from_numpy(I.uniform_points(777, 1)).cuda()
    lat_p = net.latent.requires_grad_(True)
    w_p = net.weights.requires_grad_(True)
    u = torch.randn(777, device="cuda")
    dens = fvsrn_points(net, xyz)
    (dens * u).sum().backward()
    d_lat, d_w = torch.empty_like(net.latent), torch.empty_like(net.weights)
    FV.fvsrn_train_step(net, d_lat, d_w, xyz, dloss_dy=u)
    # dW is reduced in a fixed order (bitwise equal); the latent gradient sums
    # each cell's points in the order the counting sort placed them, which
    # varies between launches, so the two agree to FP32 rounding of the
    # largest entries
    assert torch.equal(w_p.grad, d_w)
    scale = d_lat.abs().max().item()
    assert torch.allclose(lat_p.grad, d_lat, rtol=0.0, atol=1e-6 * scale)
    net.latent.requires_grad_(False)
    net.weights.requires_grad_(False)


def test_autograd_position_gradient_and_time(FV):
    """fvsrn_points as a torch function of the positions, the latent grids
    and the weights at a time between two keyframes: d(sum u d)/dxyz is
    u * grad d (reverse mode through the network, the Fourier features and the
    trilinear weights, Sec. 6) and the parameter gradients are the VJP of the
    oracle, both against the FP64 oracle; an in-place update of the weights
    between forward and backward is refused."""
    from paper_2112_01579_amd.trainer import fvsrn_points
    spec = I.NetSpec(R=12, F=8, L=4, c=32, H=3, K=2)
    keys = [0.0, 4.0]
    lat, w = I.net_params(spec, 29)
    net = FV.Network(spec, lat, w, key_times=keys)
    onet = O.Net(spec, lat, w, key_times=keys)
    t = 1.3
    pts = I.uniform_points(901, 5)
    u = np.random.default_rng(2).normal(size=901).astype(np.float32)
    xyz = torch.from_numpy(pts).cuda().requires_grad_(True)
    uu = torch.from_numpy(u).cuda()
    net.latent.requires_grad_(True)
    net.weights.requires_grad_(True)
    try:
        dens = fvsrn_points(net, xyz, time=t)
        (dens * uu).sum().backward()
        d_ref, g_ref = O.grad_points(onet, pts, t)
        assert np.abs(dens.detach().cpu().numpy() - d_ref).max() <= 1e-5
        want = u[:, None] * g_ref
        err = np.abs(xyz.grad.cpu().numpy() - want).max() / np.abs(want).max()
        print("autograd d/dxyz error (relative to max) %.3g" % err, flush=True)
        assert err <= 1e-4
        dl, dw, _ = O.train_grads(onet, pts, dloss_dd=u, times=np.full(901, t))
        assert np.abs(net.weights.grad.cpu().numpy() - dw).max() <= 1e-4 * np.abs(dw).max()
        assert np.abs(net.latent.grad.cpu().numpy() - dl).max() <= 1e-4 * np.abs(dl).max()
        # an in-place change of a saved parameter is caught by torch's version check
        dens = fvsrn_points(net, xyz, time=t)
        with torch.no_grad():
            net.weights.mul_(1.0)
        with pytest.raises(RuntimeError, match="modified by an inplace operation"):
            dens.sum().backward()
        # only the positions: no parameter gradient is computed
        net.latent.requires_grad_(False)
        net.weights.requires_grad_(False)
        xyz.grad = None
        (fvsrn_points(net, xyz, time=t) * uu).sum().backward()
        assert np.abs(xyz.grad.cpu().numpy() - want).max() <= 1e-4 * np.abs(want).max()
    finally:
        net.latent.requires_grad_(False)
        net.weights.requires_grad_(False)


def test_keyframe_train_gradients(FV):
    """Keyframe latent grids (Sec. 8) with a time per point: the gradient of
    every keyframe grid and of the weights against the oracle; times below,
    inside and above the key range, and exactly at key times."""
    spec = I.NetSpec(R=12, F=8, L=4, c=32, H=3, K=4)
    keys = [0.0, 4.0, 8.0, 12.0]
    lat, w = I.net_params(spec, 17)
    gnet = FV.Network(spec, lat, w, key_times=keys)
    onet = O.Net(spec, lat, w, key_times=keys)
    n = 16 * 211 + 5
    xyz = I.uniform_points(n, 18, -0.99, 0.99)
    rng = np.random.default_rng(19)
    times = rng.uniform(-2.0, 14.0, n).astype(np.float32)
    times[:8] = [0.0, 4.0, 8.0, 12.0, -5.0, 20.0, 3.999, 8.001]
    u = rng.normal(size=n).astype(np.float32)
    dl_ref, dw_ref, _ = O.train_grads(onet, xyz, dloss_dd=u.astype(np.float64), times=times.astype(np.float64))
    d_lat = torch.empty_like(gnet.latent)
    d_w = torch.empty_like(gnet.weights)
    FV.fvsrn_train_step(gnet, d_lat, d_w, torch.from_numpy(xyz).cuda(), dloss_dy=torch.from_numpy(u).cuda(),
                        times=torch.from_numpy(times).cuda())
    e_w, e_l = _rel(d_w.cpu().numpy(), dw_ref), _rel(d_lat.cpu().numpy(), dl_ref)
    print("keyframe train VJP: dW rel err %.3g, dG rel err %.3g" % (e_w, e_l), flush=True)
    assert e_w <= 1e-4 and e_l <= 1e-4


def test_time_varying_training_gain(FV):
    """Training the keyframe grids on every timestep of the advected-blob
    sequence (Sec. 8) against training on the keyframe timesteps only: the
    network then reconstructs the timesteps between keyframes better."""
    from paper_2112_01579_amd.trainer import Trainer
    spec = I.NetSpec(R=16, F=8, L=4, c=32, H=3, K=4)
    keys = [0.0, 4.0, 8.0, 12.0]
    prm = I.blob_sequence_params(seed=I.SEED_TIME)
    D = 32
    vols = {t: I.blob_volume(D, float(t), prm) for t in range(13)}
    norm = max(v.max() for v in vols.values())
    frames_all = [(float(t), torch.from_numpy((vols[t] / norm).astype(np.float32)).cuda()) for t in range(13)]
    frames_key = [f for f in frames_all if f[0] in keys]
    between = [1.0, 2.0, 3.0, 5.0, 6.0, 7.0, 9.0, 10.0, 11.0]
    xyz = torch.from_numpy(I.uniform_points(1 << 15, 23, -0.99, 0.99)).cuda()

    def err(net):
        e = []
        for t, v in frames_all:
            if t in between:
                d = FV.fvsrn_eval_points(net, xyz, t, "f32")
                e.append(torch.mean(torch.abs(d - FV.fvsrn_dense_eval_points(v, xyz))).item())
        return float(np.mean(e))

    res = {}
    for name, frames in (("all", frames_all), ("keys", frames_key)):
        lat, w = I.net_params(spec, 29)
        net = FV.Network(spec, lat, w, key_times=keys)
        if name == "all":
            res["untrained"] = err(net)
        tr = Trainer(net, frames, batch=1 << 15, seed=31)
        for _ in range(300):
            tr.step()
        res[name] = err(net)
    print("time-varying L1 between keyframes: %s" % res, flush=True)
    assert res["all"] < 0.5 * res["untrained"]
    assert res["all"] < res["keys"]


@pytest.mark.parametrize("spec", [I.NetSpec(R=16, F=8, L=4, c=32, H=3, outputs=4),
                                  I.NetSpec(R=16, F=16, L=8, c=48, H=3, K=2, outputs=4)],
                         ids=["c32", "c48_keyframes"])
def test_train_gradients_predicted_gradient_targets(FV, spec):
    """Four-output network fitted to densities and gradient targets (Sec. 6):
    L1 on the density plus grad_weight/3 times the L1 of the predicted
    gradient; dW (all four output rows and biases), the latent gradient and
    the loss against the oracle. Then the same network in L1 mode without
    gradient targets and in VJP mode, where the gradient outputs get no
    gradient."""
    n = 64 * 21 + 9
    lat, w = I.net_params(spec, 8)
    kt = (0.0, 1.0) if spec.K > 1 else None
    gnet, onet = FV.Network(spec, lat, w, key_times=kt), O.Net(spec, lat, w, kt)
    xyz = I.uniform_points(n, 9, -0.99, 0.99)
    times = np.random.default_rng(4).uniform(-0.2, 1.2, n).astype(np.float32) if spec.K > 1 else None
    rng = np.random.default_rng(2)
    dref = np.empty(n)
    gref = np.empty((n, 3))
    for i in range(n):
        dref[i], gref[i] = O.density_grad(onet, xyz[i], 0.0 if times is None else float(times[i]), mode="pred")
    # targets away from the predictions so that every sign agrees in FP32 and FP64
    target = (dref + rng.uniform(0.01, 0.3, n) * rng.choice([-1, 1], n)).astype(np.float32)
    tgrad = (gref + rng.uniform(0.01, 0.5, (n, 3)) * rng.choice([-1, 1], (n, 3))).astype(np.float32)
    tt = None if times is None else torch.from_numpy(times).cuda()
    for tg, gw in ((tgrad, 0.7), (None, 0.0)):
        dl_ref, dw_ref, loss_ref = O.train_grads(onet, xyz, target=target.astype(np.float64), times=times,
                                                 target_grad=tg, grad_weight=gw)
        d_lat = torch.empty_like(gnet.latent)
        d_w = torch.empty_like(gnet.weights)
        loss = torch.zeros(1, device="cuda")
        FV.fvsrn_train_step(gnet, d_lat, d_w, torch.from_numpy(xyz).cuda(), target=torch.from_numpy(target).cuda(),
                            out_loss=loss, times=tt, target_grad=None if tg is None else torch.from_numpy(tg).cuda(),
                            grad_weight=gw)
        e_w, e_l = _rel(d_w.cpu().numpy(), dw_ref), _rel(d_lat.cpu().numpy(), dl_ref)
        print("train 4-output c=%d grad targets %s: dW rel err %.3g, dG rel err %.3g, loss %.6g vs %.6g" %
              (spec.c, tg is not None, e_w, e_l, loss.item(), loss_ref), flush=True)
        assert e_w <= 1e-4 and e_l <= 1e-4
        assert abs(loss.item() - loss_ref) <= 1e-5 * abs(loss_ref) + 1e-7
        if tg is None:
            # the gradient outputs' rows and biases receive nothing
            out_rows = d_w.cpu().numpy()[-4 * (spec.c + 1):]
            assert np.count_nonzero(out_rows[spec.c:4 * spec.c]) == 0
            assert np.count_nonzero(out_rows[4 * spec.c + 1:]) == 0
    up = rng.normal(size=n).astype(np.float32)
    dl_ref, dw_ref, loss_ref = O.train_grads(onet, xyz, dloss_dd=up.astype(np.float64), times=times)
    d_lat = torch.empty_like(gnet.latent)
    d_w = torch.empty_like(gnet.weights)
    FV.fvsrn_train_step(gnet, d_lat, d_w, torch.from_numpy(xyz).cuda(), dloss_dy=torch.from_numpy(up).cuda(),
                        times=tt)
    assert _rel(d_w.cpu().numpy(), dw_ref) <= 1e-4 and _rel(d_lat.cpu().numpy(), dl_ref) <= 1e-4


def test_trainer_learns_predicted_gradients(FV):
    """A four-output network trained with gradient targets on the blob field
    predicts gradients closer to the volume's central differences than at
    initialisation, and its density error still falls."""
    from paper_2112_01579_amd.trainer import Trainer
    spec = I.NetSpec(R=16, F=8, L=4, c=32, H=3, outputs=4)
    v = I.blob_volume(48, 0.0, I.blob_sequence_params(seed=I.SEED_TIME))
    vol = torch.from_numpy(v / v.max()).cuda()
    lat, w = I.net_params(spec, 1)
    net = FV.Network(spec, lat, w)
    xyz = FV.fvsrn_sample_points(99, 1, 1 << 14)
    dref, gref = FV.fvsrn_dense_grad_points(vol, xyz)

    def errs():
        d, g = FV.fvsrn_pred_grad_points(net, xyz)
        return torch.mean(torch.abs(d - dref)).item(), torch.mean(torch.abs(g - gref)).item()

    e0 = errs()
    tr = Trainer(net, vol, batch=1 << 14, lr_grid=1e-2, lr_mlp=2e-3, grad_weight=0.5)
    for _ in range(150):
        tr.step()
    e1 = errs()
    print("predicted-gradient training: density L1 %.4f, gradient L1 %.4f -> density %.4f, gradient %.4f" %
          (e0 + e1), flush=True)
    assert e1[0] < 0.5 * e0[0] and e1[1] < 0.7 * e0[1]


@pytest.mark.parametrize("te", [1, 2, 3], ids=["direct", "fourier", "both"])
def test_train_gradients_time_encodings(FV, te):
    """Training with a time input (Sec. 8): per-point times spanning and
    exceeding the time range; dW (including layer 0's time columns), the
    keyframe latent gradients and the loss against the oracle."""
    spec = I.NetSpec(R=12, F=16, L=8, c=32, H=3, K=3, time_enc=te)
    keys = (0.0, 2.0, 5.0)
    n = 64 * 19 + 7
    lat, w = I.net_params(spec, 50 + te)
    gnet, onet = FV.Network(spec, lat, w, key_times=keys), O.Net(spec, lat, w, keys)
    xyz = I.uniform_points(n, 3 + te, -0.99, 0.99)
    times = np.random.default_rng(te).uniform(-1.0, 6.0, n).astype(np.float32)
    up = np.random.default_rng(9).normal(size=n).astype(np.float32)
    dl_ref, dw_ref, loss_ref = O.train_grads(onet, xyz, dloss_dd=up.astype(np.float64), times=times)
    d_lat = torch.empty_like(gnet.latent)
    d_w = torch.empty_like(gnet.weights)
    loss = torch.zeros(1, device="cuda")
    FV.fvsrn_train_step(gnet, d_lat, d_w, torch.from_numpy(xyz).cuda(), dloss_dy=torch.from_numpy(up).cuda(),
                        times=torch.from_numpy(times).cuda(), out_loss=loss)
    e_w, e_l = _rel(d_w.cpu().numpy(), dw_ref), _rel(d_lat.cpu().numpy(), dl_ref)
    print("train time encoding %d: dW rel err %.3g, dG rel err %.3g" % (te, e_w, e_l), flush=True)
    assert e_w <= 1e-4 and e_l <= 1e-4
    assert abs(loss.item() - loss_ref) <= 1e-5 * max(1.0, abs(loss_ref))


def test_train_gradients_fourier_matrix(FV):
    """Training with random Fourier features: dW, latent gradient and loss
    against the oracle with the same matrix."""
    spec = I.NetSpec(R=12, F=16, L=8, c=48, H=3)
    n = 64 * 17 + 3
    lat, w = I.net_params(spec, 71)
    fm = I.random_fourier_matrix(spec.L, 0.8, 2)
    gnet = FV.Network(spec, lat, w, fourier_matrix=fm)
    onet = O.Net(spec, lat, w, fourier_matrix=fm.astype(np.float64))
    xyz = I.uniform_points(n, 13, -0.99, 0.99)
    up = np.random.default_rng(3).normal(size=n).astype(np.float32)
    dl_ref, dw_ref, loss_ref = O.train_grads(onet, xyz, dloss_dd=up.astype(np.float64))
    d_lat = torch.empty_like(gnet.latent)
    d_w = torch.empty_like(gnet.weights)
    loss = torch.zeros(1, device="cuda")
    FV.fvsrn_train_step(gnet, d_lat, d_w, torch.from_numpy(xyz).cuda(), dloss_dy=torch.from_numpy(up).cuda(),
                        out_loss=loss)
    e_w, e_l = _rel(d_w.cpu().numpy(), dw_ref), _rel(d_lat.cpu().numpy(), dl_ref)
    print("train fourier matrix: dW rel err %.3g, dG rel err %.3g" % (e_w, e_l), flush=True)
    assert e_w <= 1e-4 and e_l <= 1e-4
    assert abs(loss.item() - loss_ref) <= 1e-5 * max(1.0, abs(loss_ref))


def test_trainer_adaptive_resampling(FV):
    """Adaptive resampling (Sec. 5.4): after the first N steps the trainer
    measures the error grid and draws its positions from it; training still
    converges and ends below the error it started from, and the sampled
    positions concentrate where the error grid is large."""
    from paper_2112_01579_amd.trainer import Trainer
    vol = torch.from_numpy(I.gaussian_volume(48, 16, seed=4)).cuda()
    lat, w = I.net_params(I.NET_SMALL, 2)
    net = FV.Network(I.NET_SMALL, lat, w)
    tr = Trainer(net, vol, batch=1 << 14, resample_every=25, error_grid=16, per_voxel=8)
    losses = [tr.step().item() for _ in range(120)]
    assert tr.E_ready and torch.isfinite(tr.E).all()
    assert np.mean(losses[-10:]) < 0.7 * np.mean(losses[:10])
    E = tr.E.cpu().numpy()
    x = tr.xyz.cpu().numpy()
    idx = np.clip(((x + 1) * 8).astype(np.int64), 0, 15)
    ev = E[idx[:, 0] + 16 * idx[:, 1] + 256 * idx[:, 2]]
    print("adaptive resampling: mean E at sampled positions %.4g vs grid mean %.4g" % (ev.mean(), E.mean()),
          flush=True)
    assert ev.mean() > 1.5 * E.mean()


def test_trainer_adaptive_resampling_time_varying(FV):
    """Adaptive resampling of a time-varying network (Sec. 5.4 with Sec. 8):
    one error grid per timestep, each equal to fvsrn_error_grid of the
    network at that time against that timestep's volume on the same voxel
    positions, and each timestep's rows of the batch concentrated where its
    own grid is large."""
    from paper_2112_01579_amd.trainer import Trainer
    prm = I.blob_sequence_params(seed=3)
    frames = [(float(t), I.blob_volume_torch(40, float(t), prm, device="cuda")) for t in (0, 6)]
    norm = max(float(v.max().item()) for _, v in frames)
    frames = [(t, v / norm) for t, v in frames]
    spec = I.NetSpec(R=12, F=8, L=4, c=32, H=3, K=2)
    lat, w = I.net_params(spec, 5)
    net = FV.Network(spec, lat, w, key_times=(0.0, 6.0))
    tr = Trainer(net, frames, batch=1 << 14, resample_every=20, error_grid=16, per_voxel=8)
    losses = [tr.step().item() for _ in range(81)]
    assert np.mean(losses[-10:]) < 0.7 * np.mean(losses[:10])
    assert tr.E_all.shape == (2, 16 ** 3) and torch.isfinite(tr.E_all).all()
    # the grids the last batch was drawn from (measured after step 80)
    E_all = tr.E_all.clone()
    assert not torch.equal(E_all[0], E_all[1])
    # a fresh measurement: each timestep's grid is the error grid of the
    # network at that time against that timestep's volume
    tr.update_error_grid()
    for j, (t, v) in enumerate(frames):
        assert torch.equal(tr.E_all[j], FV.fvsrn_error_grid(net, v, tr.err_xyz, tr.per_voxel, t))
    x = tr.xyz.cpu().numpy()
    for j in range(2):
        a, b = tr.bounds[j], tr.bounds[j + 1]
        E = E_all[j].cpu().numpy()
        idx = np.clip(((x[a:b] + 1) * 8).astype(np.int64), 0, 15)
        ev = E[idx[:, 0] + 16 * idx[:, 1] + 256 * idx[:, 2]]
        print("timestep %d: mean E at sampled positions %.4g vs grid mean %.4g" % (j, ev.mean(), E.mean()), flush=True)
        assert ev.mean() > 1.5 * E.mean()


def test_train_gradients_against_central_differences(FV):
    """The training gradient of the small network against central finite
    differences (h = 1e-3) of the GPU's own FP32 densities on 64 points: for
    the VJP loss sum_i u_i d(x_i), the derivative with respect to weights of
    every layer and to latent entries of the cells the points touch."""
    spec = I.NET_SMALL
    lat, w = I.net_params(spec, 31)
    n = 64
    xyz = torch.from_numpy(I.uniform_points(n, 32, -0.9, 0.9)).cuda()
    u = torch.from_numpy(np.random.default_rng(4).normal(size=n).astype(np.float32)).cuda()
    net = FV.Network(spec, lat, w)
    d_lat, d_w = torch.empty_like(net.latent), torch.empty_like(net.weights)
    FV.fvsrn_train_step(net, d_lat, d_w, xyz, dloss_dy=u)
    h = 1e-3

    def loss(latent, weights):
        m = FV.Network(spec, latent, weights)
        return float(torch.sum(u.double() * FV.fvsrn_eval_points(m, xyz, 0.0, "f32").double()).item())

    K0 = spec.K0
    wi = [0, 5 * K0 + 7, 32 * K0 + 3, 32 * K0 + 32 + 100, spec.n_weights - 33, spec.n_weights - 1]
    for j in wi:
        wp, wm = w.copy(), w.copy()
        wp[j] += h
        wm[j] -= h
        fd = (loss(lat, wp) - loss(lat, wm)) / (2 * h)
        assert abs(fd - d_w[j].item()) <= 2e-3 * max(1.0, abs(fd)), (j, fd, d_w[j].item())
    g = d_lat.cpu().numpy()
    for j in np.argsort(-np.abs(g))[:6]:
        lp, lm = lat.reshape(-1).copy(), lat.reshape(-1).copy()
        lp[j] += h
        lm[j] -= h
        fd = (loss(lp, w) - loss(lm, w)) / (2 * h)
        assert abs(fd - g[j]) <= 2e-3 * max(1.0, abs(fd)), (j, fd, g[j])


@pytest.mark.parametrize("c,F,L", [(32, 16, 4), (48, 8, 8)])
def test_train_gradients_extended_shapes(FV, c, F, L):
    """One L1 training step of networks whose latent channels and Fourier
    octaves are chosen independently, against the oracle."""
    spec = I.NetSpec(R=12, F=F, L=L, c=c, H=3)
    n = 16 * 53 + 11
    gnet, onet, xyz = _setup(FV, spec, 17, n)
    d = O.eval_points(onet, xyz)
    rng = np.random.default_rng(5)
    target = (d + rng.uniform(0.01, 0.3, n) * rng.choice([-1, 1], n)).astype(np.float32)
    dl_ref, dw_ref, loss_ref = O.train_grads(onet, xyz, target=target.astype(np.float64))
    d_lat, d_w = torch.empty_like(gnet.latent), torch.empty_like(gnet.weights)
    loss = torch.zeros(1, device="cuda")
    FV.fvsrn_train_step(gnet, d_lat, d_w, torch.from_numpy(xyz).cuda(), target=torch.from_numpy(target).cuda(),
                        out_loss=loss)
    e_w, e_l = _rel(d_w.cpu().numpy(), dw_ref), _rel(d_lat.cpu().numpy(), dl_ref)
    print("train c=%d F=%d L=%d: dW %.3g, dG %.3g" % (c, F, L, e_w, e_l), flush=True)
    assert e_w <= 1e-4 and e_l <= 1e-4
    assert abs(loss.item() - loss_ref) <= 1e-5 * abs(loss_ref) + 1e-7
