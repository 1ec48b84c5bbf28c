"""fvsrn_train_step_noalloc (the training step on the library's static
per-GPU workspace, for callers that cannot allocate) against fvsrn_train_step
with a caller workspace: the same kernels and partition, so the weight
gradients and the loss agree bit for bit and the latent gradients to the
rounding of the per-cell summation order. Four calls in a row share the
static workspace, each on a smaller input than the one before it (the
study network at 2^18 points with Adam, the same network at ragged batches
in FP16 and FP32 network arithmetic, then the small network), so stale
workspace contents from a larger call must not leak into a smaller one."""
import numpy as np
import pytest
import torch

from paper_2112_01579_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def FV():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_01579_amd import fvsrn
    fvsrn.lib()
    return fvsrn


def _moments(net):
    z = lambda t: torch.zeros_like(t)  # noqa: E731
    return {"m_latent": z(net.latent), "v_latent": z(net.latent), "m_weights": z(net.weights),
            "v_weights": z(net.weights)}


def _pair(FV, spec, seed, n, adam, prec="f32"):
    """The same step through both entry points on two copies of one network;
    returns (reference, static) tuples of gradients, loss and parameters."""
    lat, w = I.net_params(spec, seed)
    xyz = FV.fvsrn_sample_points(seed, 77, n, device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(seed)
    target = torch.rand(n, device="cuda", generator=gen)
    out = []
    for noalloc in (False, True):
        net = FV.Network(spec, lat, w, device="cuda")
        d_lat, d_w = torch.full_like(net.latent, np.nan), torch.full_like(net.weights, np.nan)
        loss = torch.full((1,), np.nan, device="cuda")
        opt = None
        if adam:
            opt = dict(lr_grid=1e-2, lr_mlp=1e-3, step=1, **_moments(net))
        fn = FV.fvsrn_train_step_noalloc if noalloc else FV.fvsrn_train_step
        fn(net, d_lat, d_w, xyz, target=target, adam=opt, out_loss=loss, precision=prec)
        torch.cuda.synchronize()
        out.append((d_lat, d_w, loss, net.latent.clone(), net.weights.clone()))
    return out


@pytest.mark.parametrize("calls", [[("NET_STUDY", 1 << 18, True, "f32"), ("NET_STUDY", 50_001, False, "f16"),
                                    ("NET_STUDY", 20_001, False, "f32"), ("NET_SMALL", 4097, True, "f32")]])
def test_train_step_noalloc_matches_workspace_entry(FV, calls):
    for spec_name, n, adam, prec in calls:
        spec = getattr(I, spec_name)
        print("noalloc call: %s n=%d adam=%s %s" % (spec_name, n, adam, prec), flush=True)
        (dl_a, dw_a, l_a, lat_a, w_a), (dl_b, dw_b, l_b, lat_b, w_b) = _pair(FV, spec, 5, n, adam, prec)
        assert torch.isfinite(dl_b).all() and torch.isfinite(dw_b).all() and torch.isfinite(l_b).all()
        # the weight gradient and the loss are reduced in a fixed order
        assert torch.equal(dw_a, dw_b)
        assert torch.equal(l_a, l_b)
        # the latent gradient sums each cell's points in the order the
        # counting sort placed them, which varies between launches
        scale = dl_a.abs().max().item()
        err = (dl_a - dl_b).abs().max().item()
        print("  latent gradient max diff %.3g of max %.3g" % (err, scale), flush=True)
        assert err <= 1e-6 * scale
        assert torch.equal(w_a, w_b)
        if adam:
            # the first Adam step moves each latent entry by lr g / (|g| + eps)
            # of its own path's gradient (entries with |g| near eps are too
            # sensitive to compare across the two paths directly)
            lat0 = torch.from_numpy(I.net_params(spec, 5)[0].reshape(-1)).cuda()
            for lat, dl in ((lat_a, dl_a), (lat_b, dl_b)):
                want = lat0 - 1e-2 * dl / (dl.abs() + 1e-8)
                assert (lat.reshape(-1) - want.reshape(-1)).abs().max().item() <= 1e-6


def test_train_step_noalloc_refuses_a_step_above_its_workspace(FV):
    spec = I.NET_SHADED  # 3 x 2^18 points need 114 MiB of workspace
    n = 3 << 18
    assert FV.fvsrn_train_workspace_size(spec, n) > (96 << 20)
    lat, w = I.net_params(spec, 3)
    net = FV.Network(spec, lat, w, device="cuda")
    xyz = FV.fvsrn_sample_points(3, 1, n, device="cuda")
    d_lat, d_w = torch.empty_like(net.latent), torch.empty_like(net.weights)
    with pytest.raises(FV.FvsrnError) as e:
        FV.fvsrn_train_step_noalloc(net, d_lat, d_w, xyz, target=torch.zeros(n, device="cuda"))
    assert e.value.status == FV.ERR_WORKSPACE
    assert "static" in str(e.value)
