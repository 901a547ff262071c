"""Spatial renumbering at build (NET_BUILD_REORDER): a network whose vertices
are numbered at random, built with the renumbering, gives the same records,
read-outs and observations, in the caller's numbering, as the same network
built without it (delivery is exact and the random streams follow the
caller's vertex index), and matches the oracle; for every kernel family."""
import numpy as np
import pytest

import oracle
import synth
from tests import fixtures as fx
from tests.test_parity_gpu import check_parity, run_gpu

pytestmark = pytest.mark.gpu


def _noisy(n, k):
    s = synth.config0_like(n, synth.config_seed(0, 900 + k), w0=0.36)
    s.noise_sigma = 0.05
    return fx.relabel(s, 77 + k)


def _same(a, b):
    for key in ("raster", "v", "input"):
        assert np.array_equal(a[key], b[key]), key


@pytest.mark.parametrize("variant", ["default", "FUSED_STEP", "DELIVER_PACKED"])
def test_reorder_equals_plain_and_oracle(variant):
    import paper_0908_3934_amd as gn
    spec = _noisy(300, 0)
    T = 3000
    flags = 0 if variant == "default" else getattr(gn, "NET_BUILD_" + variant)
    a = run_gpu(spec, T, flags=flags)
    b = run_gpu(spec, T, flags=flags | gn.NET_BUILD_REORDER)
    _same(a, b)
    o = oracle.OracleNet(spec).step(T, v=True, inp=True)
    check_parity(b, o)
    va = a["net"].observe(gn.NET_OBS_V).cpu().numpy()
    vb = b["net"].observe(gn.NET_OBS_V).cpu().numpy()
    assert np.array_equal(va, vb)
    a["net"].close()
    b["net"].close()


def test_reorder_larger_fused_network():
    import paper_0908_3934_amd as gn
    spec = fx.relabel(synth.config1(n=8192), 5)
    T = 600
    a = run_gpu(spec, T, flags=gn.NET_BUILD_FUSED_STEP)
    b = run_gpu(spec, T, flags=gn.NET_BUILD_FUSED_STEP | gn.NET_BUILD_REORDER)
    assert b["net"].info()["deliver_flags"] & gn.NET_BUILD_FUSED_STEP
    _same(a, b)
    a["net"].close()
    b["net"].close()


def test_reorder_ensemble_and_observation():
    import torch
    import paper_0908_3934_amd as gn
    specs = [_noisy(n, k) for k, n in enumerate([64, 257, 130])]
    T = 2000
    a = run_gpu(specs, T, frame_capacity=8)
    b = run_gpu(specs, T, frame_capacity=8, flags=gn.NET_BUILD_REORDER)
    _same(a, b)
    for what in (gn.NET_OBS_FRAMES, gn.NET_OBS_FLUOR, gn.NET_OBS_CALCIUM, gn.NET_OBS_REF):
        fa = a["net"].observe(what, frames=5, gamma=0.02)
        fb = b["net"].observe(what, frames=5, gamma=0.02)
        torch.cuda.synchronize()
        assert torch.equal(fa, fb), what
    a["net"].close()
    b["net"].close()


def test_reorder_izhikevich():
    import paper_0908_3934_amd as gn
    spec = fx.relabel(synth.izhikevich(synth.config0(), psc=2), 3)
    T = 2000
    a = run_gpu(spec, T)
    b = run_gpu(spec, T, flags=gn.NET_BUILD_REORDER)
    _same(a, b)
    a["net"].close()
    b["net"].close()


def test_reorder_noise_free_driven_ensemble():
    """Noise-free LIF networks draw their drive pulses for the driven
    vertices alone, keyed by the caller's vertex index: renumbered and plain
    builds of the same ensemble give the same records, and each network
    matches its oracle run."""
    import paper_0908_3934_amd as gn
    specs = []
    for k, n in enumerate([64, 1500, 257]):
        s = synth.config0_like(n, synth.config_seed(0, 930 + k), w0=0.36)
        s.drive_rate_hz = np.where(np.asarray(s.drive_rate_hz) > 0, 200.0, 0.0).astype(np.float32)
        specs.append(fx.relabel(s, 91 + k))
    T = 2000
    a = run_gpu(specs, T)
    b = run_gpu(specs, T, flags=gn.NET_BUILD_REORDER)
    assert a["net"].info()["ensemble_blocks"] > 0 and b["net"].info()["ensemble_blocks"] > 0
    _same(a, b)
    offs = a["net"].node_offsets()
    for k, s in enumerate(specs):
        lo, hi = offs[k], offs[k + 1]
        o = oracle.OracleNet(s).step(T, v=True, inp=True)
        check_parity({"raster": a["raster"][:, lo:hi], "v": a["v"][:, lo:hi], "input": a["input"][:, lo:hi]}, o)
        assert o["raster"].sum() > 100
    a["net"].close()
    b["net"].close()
