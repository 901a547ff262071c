"""Push delivery (NET_BUILD_PUSH): the update kernel adds the out-edges of
each vertex that fires into an input ring indexed by arrival step.  The delivered
input of step t is still the sum over in-edges of w_ij s_i(t - d_ij)
(Section 2, the delayed signalling), only computed from the sources' side;
the sums are exact, so every bit must equal the oracle's and the pull
paths'."""
import numpy as np
import pytest

import oracle
import synth
from tests.test_parity_gpu import _gn, check_parity, run_gpu

pytestmark = pytest.mark.gpu


def _push(spec, T, **kw):
    gn, _ = _gn()
    flags = kw.pop("flags", 0) | gn.NET_BUILD_PUSH
    g = run_gpu(spec, T, flags=flags, **kw)
    info = g["net"].info()
    assert info["deliver_flags"] & gn.NET_BUILD_PUSH and info["ensemble_blocks"] == 0
    return g


def test_config0_full_run_push():
    spec = synth.config0()
    T = 10000
    g = _push(spec, T)
    o = oracle.OracleNet(spec).step(T, v=True, inp=True)
    check_parity(g, o)
    assert o["raster"].sum() > 100


def test_recurrent_noisy_push():
    spec = synth.config0_like(256, synth.config_seed(0), w0=0.36)
    spec.noise_sigma = 0.05
    T = 6000
    g = _push(spec, T)
    o = oracle.OracleNet(spec).step(T, v=True, inp=True)
    check_parity(g, o)
    assert o["raster"].sum() > 1000


def test_long_delays_push():
    """A source firing every ~23 steps with delays of 1..255 steps: several
    of its spikes are in flight on one edge, each in its own ring slot (256
    slots), and the 255-step arrivals land one slot behind the current one."""
    delays = np.array([1, 2, 43, 128, 200, 254, 255], dtype=np.uint8)
    k = delays.size
    spec = synth.NetSpec(name="fast", pos_um=np.zeros((k + 1, 2)), src=np.zeros(k, np.int32),
                         dst=np.arange(1, k + 1, dtype=np.int32), weight=synth.round_fp16(np.full(k, 0.25)),
                         delay_steps=delays, i_ext=np.r_[0.5, np.zeros(k)].astype(np.float32), seed=3)
    T = 1500
    g = _push(spec, T)
    o = oracle.OracleNet(spec).step(T, v=True, inp=True)
    assert np.array_equal(g["raster"], o["raster"])
    assert np.array_equal(g["input"], o["input"])
    assert (o["input"][:, k] != 0).sum() > 30


@pytest.mark.parametrize("n", [1, 100])
def test_no_edges_push(n):
    rng = np.random.default_rng(n)
    spec = synth.NetSpec(name="empty", pos_um=rng.random((n, 2)) * 100, src=np.zeros(0, np.int32),
                         dst=np.zeros(0, np.int32), weight=np.zeros(0, np.float32),
                         drive_rate_hz=np.full(n, 200.0, np.float32), noise_sigma=0.05, seed=17)
    T = 2000
    g = _push(spec, T)
    o = oracle.OracleNet(spec).step(T, v=True, inp=True)
    check_parity(g, o, exact_raster=True)
    assert not g["input"].any() and o["raster"].sum() > 0


@pytest.mark.parametrize("spread", [1, 16])
def test_synchronous_bursts_push(spread):
    """Every vertex fires in lockstep: all 2,048 vertices push in one step
    and each of their 256 out-edges lands in the slot of its delay."""
    gn, _ = _gn()
    rng = np.random.default_rng(spread)
    n, k = 2048, 256
    dst = np.repeat(np.arange(n, dtype=np.int32), k)
    src = np.argpartition(rng.random((n, n - 1)), k, axis=1)[:, :k].reshape(-1)
    src = np.where(src >= dst, src + 1, src).astype(np.int32)
    delays = (5 + rng.integers(0, spread, size=n * k)).astype(np.uint8)
    w = synth.round_fp16(np.full(n * k, 0.001))
    spec = synth.NetSpec(name="lockstep", pos_um=np.zeros((n, 2)), src=src, dst=dst, weight=w,
                         delay_steps=delays, i_ext=np.full(n, 0.5, np.float32), seed=11)
    T = 400
    a = run_gpu(spec, T)
    b = _push(spec, T)
    for key in ("raster", "v", "input"):
        assert np.array_equal(a[key], b[key]), key
    o = oracle.OracleNet(spec).step(T, v=True, inp=True)
    check_parity(b, o, v_steps=T)
    assert (o["input"] != 0).sum(1).max() == n


def test_ensemble_per_step_push():
    """A union of uneven networks through the per-step kernels with push
    delivery, against each network's own oracle run."""
    gn, _ = _gn()
    sizes = [64, 300, 1500, 97]
    specs = []
    for k, n in enumerate(sizes):
        s = synth.config0_like(n, synth.config_seed(3, 60 + k), w0=0.36)
        s.noise_sigma = 0.05
        specs.append(s)
    T = 2000
    g = _push(specs, T)
    offs = g["net"].node_offsets()
    for k, s in enumerate(specs):
        a, b = offs[k], offs[k + 1]
        o = oracle.OracleNet(s).step(T, v=True, inp=True)
        check_parity({"raster": g["raster"][:, a:b], "v": g["v"][:, a:b], "input": g["input"][:, a:b]}, o)


@pytest.mark.parametrize("psc", [0, 2])
def test_izhikevich_push(psc):
    spec = synth.izhikevich(synth.config0(), psc=psc, w_scale=60.0 if psc else None)
    spec.noise_sigma = 0.0
    T = 4000
    g = _push(spec, T)
    o = oracle.OracleNet(spec).step(T, v=True, inp=True)
    check_parity(g, o, v_steps=T, exact_raster=True)
    assert (o["input"] != 0).sum() > 100


def test_push_equals_fused_config1():
    """Config-1 density at N = 8,192 with state noise: push delivery and the
    fused step give the same bits for every step, and the observation frames
    agree too."""
    gn, _ = _gn()
    spec = synth.config1(n=8192)
    T = 1500
    a = run_gpu(spec, T, flags=gn.NET_BUILD_FUSED_STEP, frame_capacity=8)
    b = _push(spec, T, frame_capacity=8)
    for key in ("raster", "v", "input"):
        assert np.array_equal(a[key], b[key]), key
    fa = a["net"].observe(gn.NET_OBS_FRAMES, frames=4).cpu().numpy()
    fb = b["net"].observe(gn.NET_OBS_FRAMES, frames=4).cpu().numpy()
    assert np.array_equal(fa, fb)


@pytest.mark.timeout(600)
def test_full_size_push_equals_fused():
    """The benchmarked network (N = 2^20, 1.03e8 edges): push delivery and
    the fused step, bit for bit, over 400 steps (rasters every step; V and
    delivered inputs of the last 100 steps)."""
    gn, torch = _gn()
    spec = synth.config2()
    out = []
    for flags in (gn.NET_BUILD_FUSED_STEP, gn.NET_BUILD_PUSH):
        net = gn.Net(spec, flags=flags)
        r1 = net.step(300, raster=True)
        r2 = net.step(100, raster=True, v=True, inp=True)
        torch.cuda.synchronize()
        out.append((torch.cat([r1["raster"], r2["raster"]]).cpu().numpy(), r2["v"].cpu().numpy(),
                    r2["input"].cpu().numpy(), net.info()))
        del r1, r2
        net.close()
    (ra, va, ia, _), (rb, vb, ib, inf) = out
    assert inf["deliver_flags"] & gn.NET_BUILD_PUSH
    assert np.array_equal(ra, rb)
    assert np.array_equal(va, vb)
    assert np.array_equal(ia, ib)
    assert np.count_nonzero(ia) > 10000


def test_push_renumbered_equals_fused():
    """A network numbered at random, renumbered in Morton order at build:
    push delivery (out-edges in the internal numbering) and the fused step
    give the same records in the caller's numbering."""
    gn, _ = _gn()
    spec = synth.relabel(synth.config1(n=8192), 5)
    T = 800
    a = run_gpu(spec, T, flags=gn.NET_BUILD_FUSED_STEP | gn.NET_BUILD_REORDER)
    b = _push(spec, T, flags=gn.NET_BUILD_REORDER)
    for key in ("raster", "v", "input"):
        assert np.array_equal(a[key], b[key]), key
    assert np.count_nonzero(b["input"]) > 1000
