"""GPU parity of the Hodgkin-Huxley vertex (Section 3.1's four-state model,
dt = 0.03 ms) with every PSC kind against the FP64 oracle through the C-ABI:
delivered inputs bit-exact up to the first raster difference, V within 1e-4
over the first 1000 steps, raster Jaccard >= 0.995 over the run; single
vertices reproduce the oracle's firing exactly."""
import numpy as np
import pytest

import oracle
import synth
from tests import fixtures as fx
from tests.test_parity_gpu import check_parity, run_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("I", [0.0, 6.0, 10.0])
def test_single_vertex_hh(I):
    spec = synth.NetSpec(name="one", pos_um=np.zeros((1, 2)), src=np.zeros(0, np.int32), dst=np.zeros(0, np.int32),
                         weight=np.zeros(0, np.float32))
    spec = synth.hodgkin_huxley(spec, psc=0)
    spec.noise_sigma = 0.0
    spec.i_ext = np.array([I], np.float32)
    spec.v0 = np.array([-65.0], np.float32)
    T = 20000
    g = run_gpu(spec, T)
    o = oracle.OracleNet(spec).step(T, v=True, inp=True)
    check_parity(g, o, v_steps=T, exact_raster=True)
    if I >= 10.0:
        assert o["raster"].sum() >= 30
    g["net"].close()


@pytest.mark.parametrize("psc", [0, 1, 2])
@pytest.mark.parametrize("seed", range(3))
def test_tiny_hh(psc, seed):
    n = 3 + (seed + psc) % 6
    spec = fx.hodgkin_huxley_tiny(n, psc, seed)
    T = 6000
    g = run_gpu(spec, T)
    o = oracle.OracleNet(spec).step(T, v=True, inp=True)
    check_parity(g, o, v_steps=1000)
    assert o["raster"].sum() > 5
    g["net"].close()


@pytest.mark.parametrize("psc", [1, 2])
def test_config0_hh(psc):
    """The 256-vertex config-0 geometry as a Hodgkin-Huxley network for 1 s
    (33,334 steps at dt = 0.03 ms)."""
    spec = synth.hodgkin_huxley(synth.config0(), psc=psc)
    T = 33334
    g = run_gpu(spec, T)
    o = oracle.OracleNet(spec).step(T, v=True, inp=True)
    check_parity(g, o)
    assert o["raster"].sum() > 100
    g["net"].close()


def test_hh_in_mixed_ensemble():
    """HH, Izhikevich-free: HH and LIF networks sharing dt = 0.03 ms in the
    single-launch ensemble kernel, each against its own oracle run and the
    whole against the per-step kernels bit for bit."""
    import paper_0908_3934_amd as gn
    sizes = [64, 100, 257, 130]
    specs = []
    for k, n in enumerate(sizes):
        base = synth.config0_like(n, synth.config_seed(3, 60 + k), w0=0.36)
        if k == 0:
            base.noise_sigma = 0.05
            base.dt_ms = synth.HH_DT_MS
            base.frame_den = synth.FRAME_DEN * 10 // 3
            specs.append(base)
        else:
            specs.append(synth.hodgkin_huxley(base, psc=k % 3))
    T = 6000
    g = run_gpu(specs, T)
    assert g["net"].info()["ensemble_blocks"] > 0
    h = run_gpu(specs, T, flags=gn.NET_BUILD_PER_STEP)
    for key in ("raster", "v", "input"):
        assert np.array_equal(g[key], h[key]), key
    offs = g["net"].node_offsets()
    for k, s in enumerate(specs):
        a, b = offs[k], offs[k + 1]
        o = oracle.OracleNet(s).step(T, v=True, inp=True)
        check_parity({"raster": g["raster"][:, a:b], "v": g["v"][:, a:b], "input": g["input"][:, a:b]}, o)
    g["net"].close()
    h["net"].close()
