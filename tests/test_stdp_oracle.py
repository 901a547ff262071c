"""Pins of the oracle's spike-timing-dependent plasticity (Section 3.2,
"Plasticity": the time since the last spike s_j, the timing difference q_ij
and the weight transition G_ij) on cases worked out by hand from those
definitions, plus invariants and the brute-force dense formulation.

Hand cases use a two-vertex chain 0 -> 1 with delay d and spikes forced at
chosen steps; with s(u) = (u - t_last - 1) dt (u dt before any spike):
  pre spike at a, post spike at b (b > a + d):
    step a + d (arrival): q = s_0(a) - s_1(a + d) = a dt - (a + d) dt = -d dt
    step b (post):        q = s_0(b - d) - s_1(b) = (b - d - a - 1) dt - b dt
  each increment dt alpha sign(q) exp(-beta |q|), rounded to 2^-20.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import dense
from tests import fixtures as fx

Q = 2.0 ** -20


def _rounded(dw):
    return round(dw / Q) * Q


def _chain(d, w=0.25, alpha=0.005, beta=0.1):
    spec = synth.NetSpec(name="pair", pos_um=np.array([[0.0, 0.0], [10.0, 0.0]]), src=np.array([0], np.int32),
                         dst=np.array([1], np.int32), weight=np.array([w], np.float32),
                         delay_steps=np.array([d], np.uint8))
    return synth.plastic(spec, alpha, beta)


def _run_forced(spec, T, spikes):
    force = np.zeros((T, spec.n), np.uint8)
    for (j, t) in spikes:
        force[t, j] = 1
    o = oracle.OracleNet(spec)
    ws, ins = [], []
    for t in range(T):
        ws.append(o.weights(spec.src, spec.dst)[0])
        ins.append(o.step(1, inp=True, force_raster=force[t:t + 1])["input"][0].copy())
    ws.append(o.weights(spec.src, spec.dst)[0])
    return np.array(ws), np.array(ins)


@pytest.mark.parametrize("a,b,d", [(10, 40, 5), (3, 9, 2), (50, 60, 6)])
def test_pre_then_post_hand_values(a, b, d):
    spec = _chain(d)
    dt, al, be = spec.dt_ms, spec.stdp_alpha, spec.stdp_beta
    T = b + 5
    ws, ins = _run_forced(spec, T, [(0, a), (1, b)])
    w0 = 0.25
    q1 = -d * dt                                   # arrival step a + d
    w1 = w0 + _rounded(dt * al * math.copysign(1.0, q1) * math.exp(-be * abs(q1)))
    q2 = (b - d - a - 1) * dt - b * dt             # post step b
    dw2 = 0.0 if q2 == 0 else _rounded(dt * al * math.copysign(1.0, q2) * math.exp(-be * abs(q2)))
    assert ws[a + d] == w0 and ws[a + d + 1] == pytest.approx(w1, abs=0)       # changes right after the arrival
    assert ws[b + 1] == w1 + dw2
    assert (np.diff(ws) != 0).sum() <= 2                     # nothing changes on other steps
    # the spike is delivered with the weight it finds on arrival
    assert ins[a + d, 1] == w0 and np.count_nonzero(ins[:, 1]) == 1


def test_post_then_pre_sign_and_second_spike():
    """Post spike first (at 20), then a pre spike (at 30) arriving at 34,
    then a second post spike (at 60): three updates with their own s values."""
    d = 4
    spec = _chain(d)
    dt, al, be = spec.dt_ms, spec.stdp_alpha, spec.stdp_beta
    ws, ins = _run_forced(spec, 70, [(1, 20), (0, 30), (1, 60)])
    f = lambda q: 0.0 if q == 0 else _rounded(dt * al * math.copysign(1.0, q) * math.exp(-be * abs(q)))
    w = 0.25
    q_a = 16 * dt - 20 * dt                         # post at 20: s_0(16) = 16 dt, s_1(20) = 20 dt
    w += f(q_a)
    assert ws[21] == w
    q_b = 30 * dt - (34 - 20 - 1) * dt          # arrival at 34: s_0(30) = 30 dt, s_1(34) = 13 dt
    w += f(q_b)
    assert ws[35] == w and ins[34, 1] == ws[34]
    q_c = (56 - 30 - 1) * dt - (60 - 20 - 1) * dt   # post at 60: s_0(56) = 25 dt, s_1(60) = 39 dt
    w += f(q_c)
    assert ws[61] == w
    assert q_a < 0 and q_b > 0 and q_c < 0


def test_no_spikes_no_change_and_zero_q():
    spec = _chain(3)
    ws, _ = _run_forced(spec, 50, [])
    assert (ws == 0.25).all()
    # pre spike at 0 (arrives at 3), post spike at 2: the post spike gives
    # q = s_0(-1) - s_1(2) = 0 - 2 dt < 0; at the arrival s_0(0) = 0 and
    # s_1(3) = (3 - 2 - 1) dt = 0, so q = 0 and sign(q) = 0: no change
    ws, _ = _run_forced(spec, 10, [(0, 0), (1, 2)])
    assert ws[3] < ws[2]
    assert ws[4] == ws[3]


@pytest.mark.parametrize("seed", range(6))
def test_dense_bruteforce_stdp(seed):
    n = 3 + seed % 6
    base = fx.random_tiny(n, 0.6, seed, w_scale=0.5)
    base.n_ref = 20
    spec = synth.plastic(base, alpha=0.02, beta=0.1)
    T = 1500
    edges = list(zip(spec.src.tolist(), spec.dst.tolist(), spec.weight.tolist(), spec.delay_steps.tolist()))
    ref = dense.simulate(n, edges, T, drive_thr=[oracle.drive_threshold(float(x), spec.dt_ms) for x in spec.drive_rate_hz],
                         drive_amp=spec.drive_amp, sigma=spec.noise_sigma, seed=spec.seed, v0=spec.v0.tolist(),
                         stdp={"alpha": spec.stdp_alpha, "beta": spec.stdp_beta})
    o = oracle.OracleNet(spec)
    out = o.step(T, v=True, inp=True)
    assert out["raster"].tolist() == ref["raster"]
    assert out["input"].tolist() == ref["input"]
    assert out["v"].tolist() == ref["v"]
    w = o.weights(spec.src, spec.dst)
    assert w.tolist() == [ref["w_final"][a][b] for a, b in zip(spec.src.tolist(), spec.dst.tolist())]
    assert (w != spec.weight).sum() > 0                      # the weights did move
