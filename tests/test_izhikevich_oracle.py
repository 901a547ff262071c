"""Pins of the oracle's Izhikevich vertex and post-synaptic currents
(Section 3.1, Eq. izsimple; Section 3.2, Eqs. simplepsc, alphapsc, izpsc)
against facts fixed by the mathematics rather than by the code:

* one arrival into an exponential PSC: r decays as w (1 - a dt)^k, the
  exact solution of the Euler recurrence;
* one arrival into an alpha PSC: the recurrence matrix has the double
  eigenvalue lambda = 1 - a dt, so r(k) = (k-1) dt w lambda^(k-2) and
  p(k) = w lambda^(k-2) (lambda - (k-1) a dt) (the discrete t e^(-at));
* the rheobase of the quadratic model: with W at its nullcline the fixed
  points solve k x^2 - (k (Vt - Vr) + b) x + U = 0 (x = V - Vr), so a vertex
  below U* = (k (Vt - Vr) + b)^2 / (4k) settles at the smaller root and
  never fires, and one above it fires;
* the reset: after a spike V is exactly c and W exactly W + d; a vertex
  exactly at V_peak fires (Eq. spd uses >=);
* the brute-force dense formulation (full spike history, pure Python) for
  networks of N <= 8 with every PSC kind.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import dense
from tests import fixtures as fx


def _chain(psc, w, d, a_psc=0.2):
    """Source 0 -> target 1 with delay d; the target is far from firing."""
    spec = synth.NetSpec(name="chain", pos_um=np.array([[0.0, 0.0], [10.0, 0.0]]), src=np.array([0], np.int32),
                         dst=np.array([1], np.int32), weight=np.array([w], np.float32),
                         delay_steps=np.array([d], np.uint8))
    spec = synth.izhikevich(spec, psc=psc)
    spec.weight = np.array([w], np.float32)
    spec.noise_sigma = 0.0
    spec.v0 = np.array([-60.0, -60.0], np.float32)
    spec.psc_rate = float(np.float32(a_psc))          # the library takes FP32 constants
    spec.iz_C = 1e9                      # V of the target barely moves: it never fires
    return spec


def _trace(spec, T, force=None):
    o = oracle.OracleNet(spec)
    r, p, inp = [], [], []
    for t in range(T):
        W, rr, pp = o.izhikevich_state()            # state at the start of step t
        r.append(rr.copy())
        p.append(pp.copy())
        fr = None if force is None else force[t:t + 1]
        out = o.step(1, inp=True, force_raster=fr)
        inp.append(out["input"][0].copy())
    return np.array(r), np.array(p), np.array(inp)


@pytest.mark.parametrize("d", [1, 7])
def test_exp_psc_single_arrival(d):
    w = 80.0
    spec = _chain(1, w, d, 0.2)
    a = spec.psc_rate
    T = 120
    force = np.zeros((T, 2), np.uint8)
    force[0, 0] = 1
    r, p, inp = _trace(spec, T, force)
    assert np.nonzero(inp[:, 1])[0].tolist() == [d] and inp[d, 1] == w
    # r(t) is the state at the start of step t: zero up to d, w at d + 1
    assert not r[:d + 1, 1].any()
    k = np.arange(T - d - 1)
    expect = w * (1.0 - a * spec.dt_ms) ** k
    assert np.allclose(r[d + 1:, 1], expect, rtol=1e-12, atol=0)
    assert not p.any()


@pytest.mark.parametrize("a", [0.2, 0.05])
def test_alpha_psc_closed_form(a):
    w, d = 50.0, 3
    spec = _chain(2, w, d, a)
    a = spec.psc_rate
    T = 300
    force = np.zeros((T, 2), np.uint8)
    force[0, 0] = 1
    r, p, inp = _trace(spec, T, force)
    dt = spec.dt_ms
    lam = 1.0 - a * dt
    m = np.arange(1, T - d)                     # state at step d + m
    r_exp = (m - 1) * dt * w * lam ** (m - 2.0)
    p_exp = w * lam ** (m - 2.0) * (lam - (m - 1) * a * dt)
    assert not r[:d + 1, 1].any() and not p[:d + 1, 1].any()
    assert np.allclose(r[d + 1:, 1], r_exp, rtol=1e-10, atol=1e-12 * w)
    assert np.allclose(p[d + 1:, 1], p_exp, rtol=1e-10, atol=1e-12 * w)
    # the continuous alpha function peaks at t = 1/a; the discrete one at m - 1 = -1/ln(lam)
    peak = int(np.argmax(r[:, 1])) - d - 1
    assert abs(peak - (-1.0 / math.log(lam))) <= 1.0


def _single(i_ext, T, v0=-60.0, w0=0.0):
    spec = synth.NetSpec(name="one", pos_um=np.zeros((1, 2)), src=np.zeros(0, np.int32), dst=np.zeros(0, np.int32),
                         weight=np.zeros(0, np.float32))
    spec = synth.izhikevich(spec, psc=0)
    spec.noise_sigma = 0.0
    spec.i_ext = np.array([i_ext], np.float32)
    spec.v0 = np.array([v0], np.float32)
    spec.w0_iz = np.array([w0], np.float32)
    return spec


def _rheobase(spec):
    B = spec.iz_k * (spec.iz_vt - spec.iz_vr) + spec.iz_b
    return B, B * B / (4.0 * spec.iz_k)


def test_rheobase_and_rest_fixed_point():
    spec = _single(0.0, 1)
    B, ustar = _rheobase(spec)
    assert ustar == pytest.approx(144.0 / 2.8)
    u = float(np.float32(0.97 * ustar))
    spec = _single(u, 1)
    o = oracle.OracleNet(spec)
    out = o.step(20000)
    assert out["raster"].sum() == 0
    x = (B - math.sqrt(B * B - 4.0 * spec.iz_k * u)) / (2.0 * spec.iz_k)
    W, _, _ = o.izhikevich_state()
    assert abs(o.v()[0] - (spec.iz_vr + x)) < 1e-9
    assert abs(W[0] - spec.iz_b * x) < 1e-9
    # just above the rheobase the vertex fires repetitively
    above = oracle.OracleNet(_single(float(np.float32(1.03 * ustar)), 1)).step(20000)
    assert above["raster"].sum() >= 3


def test_reset_rule_and_tie():
    spec = _single(300.0, 1, v0=synth.IZ_V_PEAK, w0=5.0)
    o = oracle.OracleNet(spec)
    V, W, S = [], [], []
    for t in range(400):
        V.append(o.v()[0])
        W.append(o.izhikevich_state()[0][0])
        S.append(int(o.step(1)["raster"][0, 0]))
    V.append(o.v()[0])
    W.append(o.izhikevich_state()[0][0])
    assert S[0] == 1 and V[0] == synth.IZ_V_PEAK            # the tie fires
    spikes = [t for t, s in enumerate(S) if s]
    assert len(spikes) >= 3
    for t in spikes:
        assert V[t] >= synth.IZ_V_PEAK
        assert V[t + 1] == synth.IZ_C_RESET
        assert W[t + 1] == W[t] + spec.iz_d
    for t in range(400):
        if not S[t]:
            assert V[t] < synth.IZ_V_PEAK


@pytest.mark.parametrize("psc", [0, 1, 2])
@pytest.mark.parametrize("seed", range(4))
def test_dense_bruteforce_izhikevich(psc, seed):
    n = 3 + (seed + psc) % 6
    spec = fx.izhikevich_tiny(n, psc, seed)
    T = 800
    ref = dense.simulate(
        n, list(zip(spec.src.tolist(), spec.dst.tolist(), spec.weight.tolist(), spec.delay_steps.tolist())), T,
        dt=spec.dt_ms, v_reset=spec.v_reset, v_th=spec.v_th,
        drive_thr=[oracle.drive_threshold(float(x), spec.dt_ms) for x in spec.drive_rate_hz],
        drive_amp=spec.drive_amp, i_ext=spec.i_ext.tolist(), sigma=spec.noise_sigma, seed=spec.seed,
        v0=spec.v0.tolist(), izhikevich=fx.iz_params(spec))
    out = oracle.OracleNet(spec).step(T, v=True, inp=True)
    assert out["raster"].tolist() == ref["raster"]
    assert out["input"].tolist() == ref["input"]
    assert out["v"].tolist() == ref["v"]
    assert out["raster"].sum() > 10
    assert (out["input"] != 0).sum() > 10                 # arrivals do happen
