"""GPU parity of the Izhikevich vertex with every PSC kind (Section 3.1
Eq. izsimple; Section 3.2 Eqs. simplepsc, alphapsc, izpsc) against the FP64
oracle, through the C-ABI.  Both sides keep the vertex state in FP64, so the
bars are the simulator's own: delivered inputs bit-exact (up to the first
raster difference), V within 1e-4 (the FP32 record of an FP64 state) over the
first 1000 steps, raster Jaccard >= 0.995 over the run."""
import numpy as np
import pytest

import oracle
import synth
from tests import fixtures as fx
from tests.test_parity_gpu import check_parity, run_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("psc", [0, 1, 2])
@pytest.mark.parametrize("seed", range(4))
def test_tiny_izhikevich(psc, seed):
    n = 3 + (seed + psc) % 6
    spec = fx.izhikevich_tiny(n, psc, seed)
    T = 1500
    g = run_gpu(spec, T)
    o = oracle.OracleNet(spec).step(T, v=True, inp=True)
    check_parity(g, o, v_steps=T, exact_raster=True)
    assert o["raster"].sum() > 10
    g["net"].close()


@pytest.mark.parametrize("psc,scale", [(0, None), (1, None), (2, None), (1, 300.0), (2, 60.0)])
def test_config0_izhikevich(psc, scale):
    """The 256-vertex config-0 geometry as an Izhikevich network at dt = 1 ms,
    10 s: the quiet regime with state noise (arrivals trigger spikes now and
    then), and, with the larger weights, network-wide bursts.  The bursting
    network is chaotic: a one-ulp difference between two libraries' log or cos
    in the noise grows until a spike moves, so the bursting cases run without
    state noise (drive pulses only; every operation is then a basic IEEE one
    in the same order on both sides) and must agree exactly."""
    spec = synth.izhikevich(synth.config0(), psc=psc, w_scale=scale)
    bursting = scale is not None
    if bursting:
        spec.noise_sigma = 0.0
    T = 10000
    g = run_gpu(spec, T)
    o = oracle.OracleNet(spec).step(T, v=True, inp=True)
    J, dv = check_parity(g, o, v_steps=T if bursting else 1000, exact_raster=bursting)
    assert (o["input"] != 0).sum() > 1000
    if bursting:
        assert o["raster"].sum() > 50 * spec.n            # tens of Hz over the network
    g["net"].close()


def test_izhikevich_ensemble_kernel():
    """Mixed ensemble (LIF and Izhikevich networks of every PSC kind, uneven
    sizes) in the single-launch ensemble kernel against independent oracle
    runs, and against the per-step kernels bit for bit."""
    import paper_0908_3934_amd as gn
    sizes = [64, 100, 257, 300, 130, 97]
    psc_of = {1: 0, 2: 1, 4: 2, 5: 1}
    specs = []
    for k, n in enumerate(sizes):
        base = synth.config0_like(n, synth.config_seed(3, 40 + k), w0=0.36)
        if k % 3 == 0:
            base.noise_sigma = 0.05
            base.dt_ms = synth.IZ_DT_MS           # an ensemble shares dt and the frame rule
            base.frame_den = synth.FRAME_DEN // 10
            specs.append(base)
        else:
            specs.append(synth.izhikevich(base, psc=psc_of[k]))
    T = 2000
    g = run_gpu(specs, T)
    assert g["net"].info()["ensemble_blocks"] > 0
    h = run_gpu(specs, T, flags=gn.NET_BUILD_PER_STEP)
    for key in ("raster", "v", "input"):
        assert np.array_equal(g[key], h[key]), key
    offs = g["net"].node_offsets()
    for k, s in enumerate(specs):
        a, b = offs[k], offs[k + 1]
        o = oracle.OracleNet(s).step(T, v=True, inp=True)
        sub = {"raster": g["raster"][:, a:b], "v": g["v"][:, a:b], "input": g["input"][:, a:b]}
        check_parity(sub, o)
    g["net"].close()
    h["net"].close()


def test_fused_flag_falls_back_for_izhikevich():
    import paper_0908_3934_amd as gn
    spec = synth.izhikevich(synth.config0(), psc=2)
    T = 500
    a = run_gpu(spec, T, flags=gn.NET_BUILD_FUSED_STEP)
    assert not (a["net"].info()["deliver_flags"] & gn.NET_BUILD_FUSED_STEP)
    b = run_gpu(spec, T)
    for key in ("raster", "v", "input"):
        assert np.array_equal(a[key], b[key]), key
    a["net"].close()
    b["net"].close()


def test_izhikevich_rejects_bad_parameters():
    import paper_0908_3934_amd as gn
    spec = synth.izhikevich(synth.config0(), psc=1)
    spec.n_ref = 3
    with pytest.raises(gn.GeonetError):
        gn.Net(spec)
    spec = synth.izhikevich(synth.config0(), psc=1)
    spec.psc = 5
    with pytest.raises(gn.GeonetError):
        gn.Net(spec)
