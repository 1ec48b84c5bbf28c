"""Pins against figures printed in the paper (tests/golden/)."""
import os

import oracle as O
from paper_2112_01579_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))


def _read(name):
    vals = {}
    for line in open(os.path.join(HERE, "golden", name)):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            vals[k] = float(v)
    return vals


def test_network_and_grid_memory_of_default_configuration():
    """Sec. 4.2: the default fV-SRN (48-wide input, four layers of 32 read as
    three activated layers plus the output layer) holds about 7.3 kB of FP16
    weights, and its 32^3 x 16 grid 2 MB in FP32."""
    g = _read("paper_sizes.txt")
    # F = 15, L = 5 gives the 48-wide input 3 + 15 + 30
    spec = I.NetSpec(R=int(g["grid_res"]), F=15, L=5, c=int(g["network_hidden_width"]),
                     H=int(g["network_activated_layers"]))
    assert spec.K0 == g["network_input_width"]
    lat, w = I.net_params(spec, 0)
    net = O.Net(spec, lat, w)
    fp16_bytes = 2 * net.n_weights
    assert abs(fp16_bytes - g["network_fp16_bytes_approx"]) <= g["network_fp16_bytes_rel_tol"] * 7300
    # reading "four activated layers + output" would give 9.5 kB, outside the tolerance
    spec4 = I.NetSpec(R=32, F=15, L=5, c=32, H=4)
    assert abs(2 * spec4.n_weights - g["network_fp16_bytes_approx"]) > g["network_fp16_bytes_rel_tol"] * 7300
    grid_bytes = g["grid_res"] ** 3 * g["grid_channels"] * 4
    assert grid_bytes == g["grid_fp32_bytes"]
