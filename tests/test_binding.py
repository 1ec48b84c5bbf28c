"""The Python binding refuses tensors the library cannot take (wrong dtype,
shape, layout or device) before any library call, so a host pointer or a
float64 buffer never reaches a kernel. Runs without a GPU: the library is
replaced by a stub that fails the test if it is called."""
import numpy as np
import pytest
import torch

from paper_2112_01579_amd import fvsrn as FV
from paper_2112_01579_amd import inputs as I


@pytest.fixture
def no_lib(monkeypatch):
    def fail():
        raise AssertionError("the library was called")
    monkeypatch.setattr(FV, "lib", fail)


def cpu_net():
    lat, w = I.net_params(I.NET_SMALL, 1)
    return FV.Network(I.NET_SMALL, lat, w, device="cpu")


def test_check_tensor_rules():
    t = torch.zeros((4, 3))
    with pytest.raises(FV.FvsrnArgumentError, match="float32"):
        FV.check_tensor(t.double(), "xyz", shape=(None, 3))
    with pytest.raises(FV.FvsrnArgumentError, match="shape"):
        FV.check_tensor(torch.zeros((4, 2)), "xyz", shape=(None, 3))
    with pytest.raises(FV.FvsrnArgumentError, match="contiguous"):
        FV.check_tensor(torch.zeros((3, 4)).t(), "xyz", shape=(None, 3))
    with pytest.raises(FV.FvsrnArgumentError, match="GPU"):
        FV.check_tensor(t, "xyz", shape=(None, 3))
    with pytest.raises(FV.FvsrnArgumentError, match="elements"):
        FV.check_tensor(torch.zeros(5), "out", numel=4)
    with pytest.raises(FV.FvsrnArgumentError, match="torch tensor"):
        FV.check_tensor(np.zeros((4, 3), np.float32), "xyz")
    # the error is both a library error (status INVALID_ARGUMENT) and a ValueError
    with pytest.raises(ValueError):
        FV.check_tensor(t.double(), "xyz")
    try:
        FV.check_tensor(t.double(), "xyz")
    except FV.FvsrnError as e:
        assert e.status == FV.ERR_INVALID_ARGUMENT


def test_wrappers_refuse_before_any_library_call(no_lib):
    net = cpu_net()
    xyz = torch.zeros((16, 3))
    # a CPU network is refused by every call that takes one
    with pytest.raises(FV.FvsrnArgumentError, match="net.weights must be on a GPU"):
        FV.fvsrn_eval_points(net, xyz)
    with pytest.raises(FV.FvsrnArgumentError, match="GPU"):
        FV.fvsrn_grad_points(net, xyz, mode="adjoint")
    with pytest.raises(FV.FvsrnArgumentError, match="GPU"):
        FV.fvsrn_render(net, I.ramp_tf(), [I.ortho_camera(8, 8)], I.ortho_march())
    with pytest.raises(FV.FvsrnArgumentError, match="GPU"):
        FV.fvsrn_train_step(net, torch.zeros(net.spec.n_latent), torch.zeros(net.spec.n_weights), xyz,
                            target=torch.zeros(16))
    vol = torch.zeros((8, 8, 8))
    with pytest.raises(FV.FvsrnArgumentError, match="vol must be on a GPU"):
        FV.fvsrn_dense_eval_points(vol, xyz)
    with pytest.raises(FV.FvsrnArgumentError, match="float32"):
        FV.fvsrn_dense_eval_points(vol.double(), xyz)
    with pytest.raises(FV.FvsrnArgumentError, match="shape"):
        FV.fvsrn_dense_grad_points(torch.zeros((8, 8)), xyz)
    with pytest.raises(FV.FvsrnArgumentError, match="src must be on a GPU"):
        FV.fvsrn_cast_grid(torch.zeros(8), torch.zeros(8, dtype=torch.float16))
    with pytest.raises(FV.FvsrnArgumentError, match="F16 or BF16"):
        FV.fvsrn_cast_grid(torch.zeros(8), torch.zeros(8), FV.F32)
    with pytest.raises(FV.FvsrnArgumentError, match="GPU"):
        FV.fvsrn_quantize_grid(torch.zeros(16), 8)
    with pytest.raises(FV.FvsrnArgumentError, match="whole number"):
        FV.fvsrn_quantize_grid(torch.zeros(15), 8)
    with pytest.raises(FV.FvsrnArgumentError, match="RGBA"):
        FV.fvsrn_ssim_map(torch.zeros((16, 16, 3)), torch.zeros((16, 16, 3)))
    with pytest.raises(FV.FvsrnArgumentError, match="shape"):
        FV.fvsrn_sample_points(1, 2, 16, out=torch.zeros((16, 2)))


def test_network_tensor_checks(no_lib):
    net = cpu_net()
    # a weight array of the wrong size is refused by its element count
    net.weights = net.weights[:-1]
    with pytest.raises(FV.FvsrnArgumentError, match="net.weights must hold"):
        FV.fvsrn_eval_points(net, torch.zeros((4, 3)))
    net = cpu_net()
    net.latent = net.latent.double()
    with pytest.raises(FV.FvsrnArgumentError, match="net.weights must be on a GPU|net.latent"):
        FV.fvsrn_eval_points(net, torch.zeros((4, 3)))


def test_autograd_function_refuses_foreign_parameters(no_lib):
    from paper_2112_01579_amd.trainer import FvsrnPoints
    net = cpu_net()
    with pytest.raises(FV.FvsrnArgumentError, match="own tensors"):
        FvsrnPoints.apply(torch.zeros((4, 3)), net.latent.clone(), net.weights, net, 0.0, "f32")
