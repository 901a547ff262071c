"""Pins of the oracle's Hodgkin-Huxley vertex (Section 3.1's four-state
model; the paper steps it at dt = 0.03 ms) against the model's published
behaviour and the mathematics rather than the code:

* the gates at rest take the textbook steady-state values of the standard
  squid-axon rate functions (m = 0.0529, h = 0.5961, n = 0.3177 at -65 mV);
* with no input the membrane rests at -65 mV, where the steady-state ionic
  current vanishes (root of the closed-form current, found by bisection);
* a constant current of 10 uA/cm^2 gives repetitive firing at about 68 Hz
  with action potentials peaking near +40 mV, and the onset of repetitive
  firing lies between 6 and 6.5 uA/cm^2 (one or two spikes below it);
* a spike is signalled once per action potential (upward crossing);
* the brute-force dense formulation for N <= 8 with every PSC kind.
"""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
import synth
from oracle import dense
from tests import fixtures as fx

STEPS_PER_S = int(round(1000.0 / synth.HH_DT_MS))


def _single(I, v0=-65.0):
    spec = synth.NetSpec(name="one", pos_um=np.zeros((1, 2)), src=np.zeros(0, np.int32), dst=np.zeros(0, np.int32),
                         weight=np.zeros(0, np.float32))
    spec = synth.hodgkin_huxley(spec, psc=0)
    spec.noise_sigma = 0.0
    spec.i_ext = np.array([I], np.float32)
    spec.v0 = np.array([v0], np.float32)
    return spec


def test_gates_at_rest_textbook_values():
    m, n, h = oracle.OracleNet(_single(0.0)).gates()
    assert m[0] == pytest.approx(0.0529, abs=5e-5)
    assert h[0] == pytest.approx(0.5961, abs=5e-5)
    assert n[0] == pytest.approx(0.3177, abs=5e-5)


def _steady_current(V, s):
    (am, bm), (ah, bh), (an, bn) = dense._rates(V)
    m, h, n = am / (am + bm), ah / (ah + bh), an / (an + bn)
    return s.hh_gna * m ** 3 * h * (V - s.hh_ena) + s.hh_gk * n ** 4 * (V - s.hh_ek) + s.hh_gl * (V - s.hh_el)


def test_resting_potential():
    s = _single(0.0, v0=-60.0)
    vstar = brentq(lambda v: _steady_current(v, s), -80.0, -55.0, xtol=1e-12)
    assert vstar == pytest.approx(-65.0, abs=0.02)            # E_L is chosen to rest at -65 mV
    o = oracle.OracleNet(s)
    r = o.step(2 * STEPS_PER_S)
    assert r["raster"].sum() == 0
    assert abs(o.v()[0] - vstar) < 1e-6


@pytest.mark.parametrize("I,lo,hi", [(10.0, 64.0, 72.0), (20.0, 80.0, 92.0)])
def test_repetitive_firing_rate_and_peak(I, lo, hi):
    o = oracle.OracleNet(_single(I))
    r = o.step(STEPS_PER_S, v=True)
    sp = np.nonzero(r["raster"][:, 0])[0]
    late = sp[sp > STEPS_PER_S // 5]
    rate = len(late) / 0.8
    assert lo <= rate <= hi, rate
    assert 38.0 <= r["v"].max() <= 45.0
    # once per action potential: every event is an upward crossing of 0 mV
    v = r["v"][:, 0]
    ups = np.nonzero((v[1:] >= 0.0) & (v[:-1] < 0.0))[0] + 1
    assert np.array_equal(ups, sp)


def test_onset_of_repetitive_firing():
    below = oracle.OracleNet(_single(6.0)).step(STEPS_PER_S)["raster"].sum()
    above = oracle.OracleNet(_single(6.5)).step(STEPS_PER_S)["raster"].sum()
    assert 1 <= below <= 3                                  # a transient spike or two, then rest
    assert above >= 40                                      # sustained firing


@pytest.mark.parametrize("psc", [0, 1, 2])
@pytest.mark.parametrize("seed", range(3))
def test_dense_bruteforce_hodgkin_huxley(psc, seed):
    n = 3 + (seed + psc) % 6
    spec = fx.hodgkin_huxley_tiny(n, psc, seed)
    T = 3000
    ref = dense.simulate(
        n, list(zip(spec.src.tolist(), spec.dst.tolist(), spec.weight.tolist(), spec.delay_steps.tolist())), T,
        dt=spec.dt_ms, v_th=spec.v_th,
        drive_thr=[oracle.drive_threshold(float(x), spec.dt_ms) for x in spec.drive_rate_hz],
        drive_amp=spec.drive_amp, i_ext=spec.i_ext.tolist(), sigma=spec.noise_sigma, seed=spec.seed,
        v0=spec.v0.tolist(), hodgkin_huxley=fx.hh_params(spec))
    out = oracle.OracleNet(spec).step(T, v=True, inp=True)
    assert out["raster"].tolist() == ref["raster"]
    assert out["input"].tolist() == ref["input"]
    assert out["v"].tolist() == ref["v"]
    assert out["raster"].sum() > 5
    assert (out["input"] != 0).sum() > 3
