"""GPU parity of spike-timing-dependent plasticity (Section 3.2,
"Plasticity") against the FP64 oracle through the C-ABI: the rasters, the
delivered inputs and V to the simulator's bars, and every weight after the
run equal to the oracle's (weights and their increments are multiples of
2^-20, so the sums are exact on both sides); plus the argument checks."""
import numpy as np
import pytest

import oracle
import synth
from tests import fixtures as fx
from tests.test_parity_gpu import check_parity, run_gpu

pytestmark = pytest.mark.gpu


def _weights(net):
    import torch
    import paper_0908_3934_amd as gn
    w = net.observe(gn.NET_OBS_WEIGHTS)
    torch.cuda.synchronize()
    return w.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("seed", range(6))
def test_tiny_plastic_networks(seed):
    n = 3 + seed % 6
    base = fx.random_tiny(n, 0.6, seed, w_scale=0.5, sigma=0.05 if seed % 2 else 0.0)
    spec = synth.plastic(base, alpha=0.02, beta=0.1)
    T = 3000
    g = run_gpu(spec, T)
    o = oracle.OracleNet(spec)
    out = o.step(T, v=True, inp=True)
    check_parity(g, out, exact_raster=True)
    wg = _weights(g["net"])
    wo = o.weights(spec.src, spec.dst)
    assert np.array_equal(wg, wo)
    assert (wo != spec.weight).sum() > 0
    g["net"].close()


@pytest.mark.parametrize("alpha,beta", [(0.005, 0.1), (0.02, 0.05)])
def test_config0_plastic(alpha, beta):
    """The 256-vertex config-0 geometry with recurrent weights and noise,
    10,000 steps with plasticity: parity, and every weight equal."""
    base = synth.config0_like(256, synth.config_seed(0), w0=0.36)
    base.noise_sigma = 0.05
    spec = synth.plastic(base, alpha=alpha, beta=beta)
    T = 10000
    g = run_gpu(spec, T)
    o = oracle.OracleNet(spec)
    out = o.step(T, v=True, inp=True)
    check_parity(g, out)
    wo = o.weights(spec.src, spec.dst)
    assert np.array_equal(_weights(g["net"]), wo)
    moved = np.abs(wo - spec.weight) > 0
    assert moved.mean() > 0.2
    g["net"].close()


def test_plastic_ignores_other_kernels():
    import paper_0908_3934_amd as gn
    base = synth.config0_like(256, synth.config_seed(0, 5), w0=0.36)
    base.noise_sigma = 0.05
    spec = synth.plastic(base)
    T = 2000
    a = run_gpu(spec, T)
    b = run_gpu(spec, T, flags=gn.NET_BUILD_FUSED_STEP | gn.NET_BUILD_AUTOTUNE)
    assert not (b["net"].info()["deliver_flags"] & gn.NET_BUILD_FUSED_STEP)
    for key in ("raster", "v", "input"):
        assert np.array_equal(a[key], b[key]), key
    assert np.array_equal(_weights(a["net"]), _weights(b["net"]))
    a["net"].close()
    b["net"].close()


def test_plastic_argument_errors():
    import paper_0908_3934_amd as gn
    base = synth.config0_like(64, 3, w0=0.36)
    bad = synth.plastic(base)
    bad.n_ref = 5                                            # too short for the spike-time history
    with pytest.raises(gn.GeonetError):
        gn.Net(bad)
    with pytest.raises(gn.GeonetError):
        gn.Net([synth.plastic(base), synth.plastic(base)])  # one network per handle
    plain = gn.Net(base)
    with pytest.raises(gn.GeonetError):
        plain.observe(gn.NET_OBS_WEIGHTS)                    # not plastic
    plain.close()
