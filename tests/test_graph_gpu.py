"""Graph replays (NET_BUILD_GRAPH): calls without records run as replays of
a captured 256-step graph of the per-step kernels (or of the single-launch
ensemble kernel), the kernels reading the step from a device counter.  Every
replay must leave the same state as the plain launches: checked after each
call (several calls, eager work and synchronisations between them) through
V and, at the end, records of the steps that follow and the camera frames."""
import numpy as np
import pytest

import synth
from tests import fixtures as fx

pytestmark = pytest.mark.gpu


def _noisy(n, k, w0=0.36):
    s = synth.config0_like(n, synth.config_seed(0, 950 + k), w0=w0)
    s.noise_sigma = 0.05
    return s


def _pair(specs, flags=0, frame_capacity=0):
    import paper_0908_3934_amd as gn
    a = gn.Net(specs, flags=flags, frame_capacity=frame_capacity)
    b = gn.Net(specs, flags=flags | gn.NET_BUILD_GRAPH, frame_capacity=frame_capacity)
    return a, b


def _check_calls(a, b, calls):
    import torch
    import paper_0908_3934_amd as gn
    junk = torch.randn(1 << 20, device="cuda")
    for n in calls:
        a.step(n)
        b.step(n)
        junk = (junk * 1.0001).sin()                 # eager work between the replays
        torch.cuda.synchronize()
        va = a.observe(gn.NET_OBS_V)
        vb = b.observe(gn.NET_OBS_V)
        torch.cuda.synchronize()
        assert torch.equal(va, vb), n
    ra = a.step(300, raster=True, v=True, inp=True)
    rb = b.step(300, raster=True, v=True, inp=True)
    torch.cuda.synchronize()
    for key in ("raster", "v", "input"):
        assert torch.equal(ra[key], rb[key]), key
    assert a.t == b.t


@pytest.mark.parametrize("variant", ["default", "FUSED_STEP", "PUSH"])
def test_graph_per_step_kernels(variant):
    import paper_0908_3934_amd as gn
    flags = 0 if variant == "default" else getattr(gn, "NET_BUILD_" + variant)
    spec = synth.config1(n=8192) if variant == "FUSED_STEP" else _noisy(300, 0)
    a, b = _pair(spec, flags)
    if variant == "PUSH":
        assert b.info()["deliver_flags"] & gn.NET_BUILD_PUSH
    # from 0: three whole graphs then plain steps; then a call that starts mid-block
    _check_calls(a, b, [1000, 100, 1000, 256, 513])
    a.close()
    b.close()


def test_graph_ensemble_and_frames():
    import torch
    import paper_0908_3934_amd as gn
    specs = [_noisy(n, k) for k, n in enumerate([64, 257, 130])]
    a, b = _pair(specs, frame_capacity=12)
    assert b.info()["ensemble_blocks"] > 0
    _check_calls(a, b, [500, 500, 300, 1700])            # one graph per call length, reused
    assert a.info()["frames_done"] == b.info()["frames_done"] == 9      # 3,300 steps at 3 frames per 1,000
    fa = a.observe(gn.NET_OBS_FRAMES, frames=9)
    fb = b.observe(gn.NET_OBS_FRAMES, frames=9)
    torch.cuda.synchronize()
    assert torch.equal(fa, fb)
    a.close()
    b.close()


def test_graph_with_observation_per_step():
    import torch
    import paper_0908_3934_amd as gn
    spec = _noisy(300, 3)
    a, b = _pair(spec, frame_capacity=8)
    _check_calls(a, b, [768, 300, 1024])
    fa = a.observe(gn.NET_OBS_FLUOR, frames=7, gamma=0.02)
    fb = b.observe(gn.NET_OBS_FLUOR, frames=7, gamma=0.02)
    torch.cuda.synchronize()
    assert torch.equal(fa, fb)
    a.close()
    b.close()


def test_graph_falls_back_while_timing():
    import torch
    import paper_0908_3934_amd as gn
    spec = _noisy(300, 4)
    a, b = _pair(spec)
    b.timing_begin(64, every=1)
    a.step(600)
    b.step(600)
    tm = b.timing_end()
    assert tm["deliver_launches"] > 0                     # plain launches were timed
    torch.cuda.synchronize()
    assert torch.equal(a.observe(gn.NET_OBS_V), b.observe(gn.NET_OBS_V))
    a.close()
    b.close()
