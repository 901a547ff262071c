"""CPU pins of the simulation-based fit reference: its inner forward model
against the simulation oracle (same vertex, same control pulses, exact), the
likelihood of a silent vertex against its closed form, and the toggle search
against brute force over all subsets for a single small target."""
import itertools
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import features as FE
from oracle import simfit as SF


def _model(spec):
    return dict(frame_num=spec.frame_num, frame_den=spec.frame_den, dt=spec.dt_ms, tau=spec.tau_ms,
                v_rest=spec.v_rest, v_reset=spec.v_reset, v_th=spec.v_th, n_ref=spec.n_ref,
                drive_amp=spec.drive_amp, tau_c=spec.tau_c_ms)


def test_forward_model_matches_simulation_oracle():
    """No input, no noise: a driven vertex in the fit must reproduce the
    simulation oracle's calcium frames of the same isolated vertex."""
    spec = synth.NetSpec(name="iso", pos_um=np.zeros((1, 2)), src=np.zeros(0, np.int32), dst=np.zeros(0, np.int32),
                         weight=np.zeros(0, np.float32), drive_rate_hz=np.array([30.0], np.float32), seed=77)
    nf = 12
    steps = (nf * spec.frame_den + spec.frame_num - 1) // spec.frame_num
    o = oracle.OracleNet(spec, frames_cap=nf)
    o.step(steps)
    ref = o.frames()[:, 0]
    thr = oracle.drive_threshold(30.0, spec.dt_ms)
    t = np.arange(steps, dtype=np.uint64)
    pulses = (FE.philox_np(np.uint64(0), t, np.uint64(0), np.uint64(0), spec.seed & 0xFFFFFFFF, spec.seed >> 32)[0]
              < np.uint64(thr))[None, :]
    cb = SF.simulate_hypotheses([0], np.zeros((1, nf)), pulses, K=2, nf=nf, sigma=0.0, fit_seed=1, **_model(spec))
    assert ref.max() > 0
    assert np.allclose(cb[0, 0], ref, rtol=0, atol=1e-15) and np.allclose(cb[0, 1], ref, rtol=0, atol=1e-15)


def test_silent_vertex_likelihood_closed_form():
    spec = synth.NetSpec(name="s", pos_um=np.zeros((1, 2)), src=np.zeros(0, np.int32), dst=np.zeros(0, np.int32),
                         weight=np.zeros(0, np.float32))
    nf = 9
    pulses = np.zeros((1, 4000), dtype=bool)
    cb = SF.simulate_hypotheses([0], np.zeros((1, nf)), pulses, K=4, nf=nf, sigma=0.0, fit_seed=1, **_model(spec))
    F = np.linspace(-0.1, 0.2, nf)[None, :]
    g, b = 1.0, 0.05
    ll = SF.loglik(cb, F, g, b, 0.02)[0]
    assert ll == pytest.approx(-0.5 * np.sum((F - b) ** 2 / 0.02 ** 2 + math.log(0.02 ** 2)), rel=1e-12)


def test_search_reaches_the_best_subset_on_a_small_target():
    """Target 0 with four candidates: after enough sweeps the toggle search
    sits at a local optimum; check it against all 16 subsets."""
    n = 5
    rng = np.random.default_rng(0)
    pos = rng.random((n, 2)) * 60
    src = np.array([1, 2], np.int32)
    dst = np.array([0, 0], np.int32)
    spec = synth.NetSpec(name="t", pos_um=pos, src=src, dst=dst, weight=synth.round_fp16(np.array([0.45, 0.45])),
                         drive_rate_hz=np.array([0, 40, 40, 40, 40], np.float32), noise_sigma=0.05, seed=21)
    nf = 30
    steps = (nf * spec.frame_den + spec.frame_num - 1) // spec.frame_num
    o = oracle.OracleNet(spec, frames_cap=nf)
    o.step(steps)
    gamma = spec.dt_ms / 5
    F = oracle.fluorescence(o.frames(), 1.0, 0.0, gamma, spec.seed)
    pairs = np.array([[1, 0], [2, 0], [3, 0], [4, 0]])
    thr = [oracle.drive_threshold(float(r), spec.dt_ms) for r in spec.drive_rate_hz]
    common = dict(drive_thr=thr, control_seed=spec.seed, gain=1.0, offset=0.0, gamma=gamma, sigma=0.05, w=0.45,
                  K=4, fit_seed=5, **{k: v for k, v in _model(spec).items()})
    common = {k: v for k, v in common.items()}
    scores, member, ll = SF.fit(F, pairs, sweeps=6, **common)
    # likelihood of every subset, evaluated with the same machinery
    rho = (1 - spec.dt_ms / spec.tau_c_ms) ** (spec.frame_den / spec.frame_num)
    e = SF.activity_spikes(F, rho, 0.0, 1.0, spec.dt_ms)
    first = (np.arange(nf + 1) * spec.frame_den + spec.frame_num - 1) // spec.frame_num
    steps_f = np.diff(first).astype(float)
    subsets = list(itertools.product([0, 1], repeat=4))
    U = np.array([0.45 * sum(e[pairs[k, 0]] * m for k, m in enumerate(sub)) / steps_f for sub in subsets])
    t = np.arange(first[-1], dtype=np.uint64)
    pulses = np.zeros((n, first[-1]), dtype=bool)
    for j in range(n):
        if thr[j]:
            pulses[j] = FE.philox_np(np.uint64(j), t, np.uint64(0), np.uint64(0), spec.seed & 0xFFFFFFFF,
                                     spec.seed >> 32)[0] < np.uint64(thr[j])
    cb = SF.simulate_hypotheses([0] * len(subsets), U, pulses, K=4, nf=nf, sigma=0.05, fit_seed=5, **_model(spec))
    lls = SF.loglik(cb, np.repeat(F.T[[0]], len(subsets), 0), 1.0, 0.0, gamma)
    final = ll[len(pairs) + 0]
    k_final = subsets.index(tuple(int(m) for m in member))
    assert lls[k_final] == pytest.approx(final, rel=1e-12)
    # a local optimum under single toggles
    for k in range(4):
        flip = list(subsets[k_final])
        flip[k] ^= 1
        assert lls[subsets.index(tuple(flip))] <= final + 1e-9


@pytest.mark.parametrize("frac", [0.3, float(np.float32(0.3))])
def test_initial_member_count(frac):
    """ceil(f n) initial members per target, also for f given in FP32."""
    rng = np.random.default_rng(1)
    en = FE.standardise(rng.random((12, 40)))
    pairs = np.array([[i, 0] for i in range(1, 11)] + [[i, 11] for i in range(1, 8)])
    m = SF.initial_members(en, pairs, frac)
    assert m[:10].sum() == 3 and m[10:].sum() == 3        # ceil(3.0) and ceil(2.1)
