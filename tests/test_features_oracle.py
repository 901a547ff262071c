"""CPU pins of the feature reference: the vectorised Philox against the
published known-answer vectors, the control-pulse schedule against the
simulation oracle's own spikes, the activity transform against a single
spike's calcium transient, and the lagged products against shifted copies."""
import numpy as np
import pytest

import oracle
import synth
from oracle import features as FE
from tests.test_oracle_pins import KAT


@pytest.mark.parametrize("ctr,key,expect", KAT)
def test_vectorised_philox_known_answers(ctr, key, expect):
    r = FE.philox_np(*[np.array([c], dtype=np.uint64) for c in ctr], key[0], key[1])
    assert tuple(int(a[0]) for a in r) == expect


def test_pulses_match_isolated_driven_vertex_spikes():
    """An isolated vertex driven with amplitude 1.5 fires at the step after
    each pulse that does not fall inside its 20-step hold; the pulse steps
    from the vectorised Philox must reproduce the oracle's spikes exactly."""
    n = 6
    spec = synth.NetSpec(name="iso", pos_um=np.zeros((n, 2)), src=np.zeros(0, np.int32), dst=np.zeros(0, np.int32),
                         weight=np.zeros(0, np.float32), drive_rate_hz=np.full(n, 20.0, np.float32), seed=1234)
    T = 3400
    r = oracle.OracleNet(spec).step(T)["raster"]
    thr = oracle.drive_threshold(20.0, spec.dt_ms)
    t = np.arange(T, dtype=np.uint64)
    nf = 10
    dc = FE.pulses_per_frame(n, nf, [thr] * n, spec.seed, spec.frame_num, spec.frame_den)
    for j in range(n):
        x0 = FE.philox_np(np.uint64(j), t, np.uint64(0), np.uint64(0), spec.seed & 0xFFFFFFFF, spec.seed >> 32)[0]
        pulse_steps = np.nonzero(x0 < np.uint64(thr))[0]
        expect, held_until = [], -1
        for ps in pulse_steps:
            if ps <= held_until or ps + 1 >= T:
                continue
            expect.append(ps + 1)                # fires at the next step
            held_until = ps + 1 + spec.n_ref     # held after that spike
        assert np.nonzero(r[:, j])[0].tolist() == expect
        per_frame = np.bincount(pulse_steps * spec.frame_num // spec.frame_den, minlength=nf)[:nf]
        assert np.array_equal(dc[j], per_frame)
    assert dc.sum() > 30


def test_activity_concentrates_at_a_single_spike():
    spec = synth.NetSpec(name="one", pos_um=np.zeros((1, 2)), src=np.zeros(0, np.int32), dst=np.zeros(0, np.int32),
                         weight=np.zeros(0, np.float32), v0=np.array([1.0], np.float32), seed=3)
    net = oracle.OracleNet(spec, frames_cap=12)
    net.step(4000)
    cbar = net.frames()                       # [nf][1], spike at step 0 (frame 0)
    rho = (1 - spec.dt_ms / spec.tau_c_ms) ** (spec.frame_den / spec.frame_num)
    e = FE.activity(cbar.T, rho, 0.0)[0]
    # frames alternate 334/333/333 steps, so later frames keep small residues
    assert e[0] > 0.9 * e.sum() and e[:2].sum() > 0.95 * e.sum()


def test_lagged_products_on_shifted_copies():
    rng = np.random.default_rng(0)
    a = FE.standardise(rng.normal(0, 1, 600))
    b = np.roll(a, 3)
    assert FE.lagcorr(a, b, 3) == pytest.approx(1.0, abs=2e-2)
    assert abs(FE.lagcorr(a, b, 0)) < 0.15
    assert FE.lagcorr(b, a, -3) == pytest.approx(FE.lagcorr(a, b, 3))
