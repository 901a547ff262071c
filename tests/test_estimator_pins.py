"""CPU pins of the estimator-side references against hand-derived values.

* the control-pulse response of the pair features on pulse and activity
  trains whose products are counted by hand;
* the layout of the assembled 64-vector, one designed input per block whose
  value follows in closed form (a trace delayed by a whole number of frames,
  single-frame activity bursts, the two-vertex residual that is exactly
  antisymmetric);
* the BF16 rounding points of the scorer's backward pass (dH2, dH1) on a
  network whose only nonzero path is one unit wide, with every gradient
  entry worked out by hand in binary fractions;
* noise-free identifiability of the simulation-based fit: with no state
  noise and a small observation noise, the true in-set of a target has the
  highest likelihood among all subsets of its candidates, and the toggle
  search ends there.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import features as FE
from oracle import mlp as M
from oracle import simfit as SF

DT, TAU_C, NUM, DEN = 0.1, 500.0, 3, 1000
RHO = (1.0 - DT / TAU_C) ** (DEN / NUM)


# --------------------------------------------------------------------------
# pulse response
# --------------------------------------------------------------------------
def test_pulse_response_hand_values():
    """Pulses at frames 3 and 10, activity 1 at frames 5 and 12: the mean
    activity two frames after a pulse is 1, and 0 at every other lag."""
    nf = 20
    pa = np.zeros(nf)
    pa[[3, 10]] = 1.0
    b = np.zeros(nf)
    b[[5, 12]] = 1.0
    for L in range(6):
        assert FE.pulse_resp(pa, 2.0, b, L) == (1.0 if L == 2 else 0.0)
    # a frame with two pulses counts twice; no pulses divides by one
    pa2 = np.zeros(nf)
    pa2[3] = 2.0
    assert FE.pulse_resp(pa2, 2.0, b, 2) == 1.0
    assert FE.pulse_resp(np.zeros(nf), 0.0, b, 2) == 0.0
    # the lag reaches past the end: products stop at the last frame
    pa3 = np.zeros(nf)
    pa3[nf - 1] = 1.0
    assert FE.pulse_resp(pa3, 1.0, np.ones(nf), 1) == 0.0


# --------------------------------------------------------------------------
# 64-feature layout
# --------------------------------------------------------------------------
def _trace_from_activity(x, tail_zero=0):
    """Fluorescence (offset 0) whose frame-to-frame deconvolution is x: the
    frame-sampled calcium recursion F(f+1) = rho F(f) + x(f), F(0) = 0; the
    last `tail_zero` frames are forced to 0 (the max(0, .) clips that drop)."""
    nf = len(x)
    F = np.zeros(nf)
    for f in range(nf - 1):
        F[f + 1] = RHO * F[f] + x[f]
    if tail_zero:
        F[nf - tail_zero:] = 0.0
    return F


def _zscore(a):
    return (a - np.mean(a)) / np.std(a)


def test_feature_layout_delayed_copies():
    """Vertex 1 is vertex 0 delayed by 3 frames and vertex 2 by 2 frames; the
    traces start with a zero frame and end with three, so each copy is a
    cyclic shift of the original and keeps its mean and spread.  Then the
    lag-s product of the standardised activities is the mean square of the
    original over its first nf - s frames, in closed form from the s frames
    at its end (all equal to -m/sd)."""
    nf = 64
    rng = np.random.default_rng(5)
    x = np.zeros(nf)
    hits = rng.choice(np.arange(2, nf - 6), 14, replace=False)
    x[hits] = rng.integers(1, 4, hits.size)
    F0 = _trace_from_activity(x, tail_zero=3)
    F1 = np.concatenate([np.zeros(3), F0[:-3]])
    F2 = np.concatenate([np.zeros(2), F0[:-2]])
    F = np.stack([F0, F1, F2], axis=1)                      # [nf][n]
    pairs = np.array([[0, 1], [1, 0], [0, 2]])
    dist = np.array([30.0, 30.0, 75.0])
    feat = FE.features(F, pairs, dist, dt_ms=DT, tau_c_ms=TAU_C, num=NUM, den=DEN, offset=0.0,
                       thr=[0, 0, 0], seed=1)
    e = x.copy()                                             # the designed activity of vertex 0
    m, sd = e.mean(), e.std()
    mF, sF = F0.mean(), F0.std()
    ms3 = (nf - 3 * (m / sd) ** 2) / (nf - 3)                # activity, lag 3
    ms2 = (nf - 2 * (m / sd) ** 2) / (nf - 2)                # activity, lag 2
    zs2 = (nf - 2 * (mF / sF) ** 2) / (nf - 2)               # trace, lag 2
    tol = 1e-9
    # block 0..16: activity lags -8..8 (index 8 + L), source first
    assert feat[0, 8 + 3] == pytest.approx(ms3, abs=tol)
    assert feat[1, 8 - 3] == pytest.approx(ms3, abs=tol)     # reversed pair: the same product at lag -3
    assert feat[0, 8 + 3] > feat[0, 8 - 3] + 0.5
    assert feat[2, 8 + 2] == pytest.approx(ms2, abs=tol)
    assert int(np.argmax(feat[0, 0:17])) == 11 and int(np.argmax(feat[1, 0:17])) == 5
    # block 17..21: trace lags -2..2 (index 19 + L)
    assert feat[2, 19 + 2] == pytest.approx(zs2, abs=tol)
    assert int(np.argmax(feat[2, 17:22])) == 4
    # scalars: pulse counts (no control), mean activity, trace spread, distance
    assert np.all(feat[:, 32:34] == 0.0)
    assert feat[0, 34] == pytest.approx(m, abs=tol) and feat[0, 35] == pytest.approx(m, abs=tol)
    assert feat[0, 36] == pytest.approx(sF, abs=tol) and feat[0, 37] == pytest.approx(sF, abs=tol)
    assert feat[0, 38] == 30.0 / 150.0 and feat[2, 38] == 0.5
    # zero pads
    assert np.all(feat[:, 59:] == 0.0)


def test_feature_layout_single_bursts():
    """Two vertices, each active in exactly one frame (vertex 0 at f0,
    vertex 1 at g0), with control pulses from a fixed key.  Every product of
    a standardised one-frame burst a = (delta - m)/sd with another series z
    reduces to z at the burst frame minus m times a partial sum of z, which
    gives the mixed activity/trace blocks and both pulse-response blocks in
    closed form; with two vertices the population residuals are exact
    negatives of each other, so their lag-0 product is -1."""
    nf, f0, g0 = 48, 12, 30
    x0 = np.zeros(nf)
    x0[f0] = 1.0
    x1 = np.zeros(nf)
    x1[g0] = 1.0
    F = np.stack([_trace_from_activity(x0), _trace_from_activity(x1)], axis=1)
    thr = [0x30000000, 0x28000000]            # about 19 % and 16 % of steps carry a pulse
    seed = 0x1234ABCD5678
    feat = FE.features(F, np.array([[0, 1]]), np.array([99.0]), dt_ms=DT, tau_c_ms=TAU_C, num=NUM, den=DEN,
                       offset=0.0, thr=thr, seed=seed)[0]
    dc = FE.pulses_per_frame(2, nf, thr, seed, NUM, DEN)
    npul = dc.sum(1)
    m = 1.0 / nf
    sd = math.sqrt(m - m * m)
    z0, z1 = _zscore(F[:, 0]), _zscore(F[:, 1])

    def burst_dot(b, z, L, lead):
        """mean over f < nf - L of a(f) z(f + L) (lead: the burst is first)
        or z(f) a(f + L), a the standardised burst at frame b."""
        if lead:
            val = (z[b + L] if b + L < nf else 0.0) / sd - (m / sd) * z[L:].sum()
        else:
            val = (z[b - L] if b - L >= 0 else 0.0) / sd - (m / sd) * z[:nf - L].sum()
        return val / (nf - L)

    tol = 1e-9
    for L in range(8):
        assert feat[43 + L] == pytest.approx(burst_dot(f0, z1, L, True), abs=tol)      # activity i, trace j
        assert feat[51 + L] == pytest.approx(burst_dot(g0, z0, L, False), abs=tol)     # trace i, activity j
    for L in range(6):                                                                  # i's pulses, j's activity
        exp = (dc[0][g0 - L] / sd - (m / sd) * dc[0][:nf - L].sum()) / max(1.0, npul[0])
        assert feat[22 + L] == pytest.approx(exp, abs=tol)
    for L in range(4):                                                                  # j's pulses, i's activity
        exp = (dc[1][f0 - L] / sd - (m / sd) * dc[1][:nf - L].sum()) / max(1.0, npul[1])
        assert feat[28 + L] == pytest.approx(exp, abs=tol)
    assert npul[0] > 100 and npul[1] > 100
    assert feat[32] == pytest.approx(math.log1p(npul[0]), abs=tol)
    assert feat[33] == pytest.approx(math.log1p(npul[1]), abs=tol)
    assert feat[34] == pytest.approx(m, abs=tol) and feat[35] == pytest.approx(m, abs=tol)
    assert feat[39] == pytest.approx(-1.0, abs=tol)
    # single bursts at different frames: lag-0 activity product is -m/sd^2 * ... < 0
    assert feat[8] == pytest.approx((-2 * m / sd / sd + nf * m * m / sd / sd) / nf, abs=tol)
    assert feat[38] == 99.0 / 150.0


# --------------------------------------------------------------------------
# BF16 rounding points of the backward pass
# --------------------------------------------------------------------------
def test_bf16_backward_rounding_points():
    """One input unit feeds one hidden unit of each layer.  x = e0,
    W1[0][0] = 1, W2[0][0] = c = 1 + 2^-7 (both BF16), w3[0] = 1 + 3*2^-9 (not
    BF16, unrounded by the path), b3 = -c*w3[0] so the logit is exactly 0
    and dz = sigmoid(0) - 0 = 1/2.  Then
      dH2 = bf16(dz w3)  = bf16(1/2 + 3*2^-10)         = 1/2 + 2^-8
      dH1 = bf16(dH2 c)  = bf16(1/2 + 2^-7 + 2^-15)    = 1/2 + 2^-7
    and the gradient is H1 * dH2 for W2, dH2 for b2, x * dH1 for W1, dH1 for
    b1, H2 * dz for w3, dz for b3; zero elsewhere.  Without the two
    roundings W1's entry would be 0.50685882... instead of 0.5078125."""
    c = 1.0 + 2.0 ** -7
    w3 = 1.0 + 3 * 2.0 ** -9
    p = np.zeros(M.N_PARAMS)
    p[M.W1.start + 0] = 1.0                          # W1[0][0]
    p[M.W2.start + 0] = c                            # W2[0][0]
    p[M.W3.start + 0] = w3
    p[M.B3.start] = -c * w3
    X = np.zeros((1, M.IN))
    X[0, 0] = 1.0
    y = np.zeros(1)
    g, loss = M.grad(p, X, y, bf=True)
    dz = 0.5
    dh2 = 0.5 + 2.0 ** -8
    dh1 = 0.5 + 2.0 ** -7
    expect = np.zeros(M.N_PARAMS)
    expect[M.W3.start] = c * dz
    expect[M.B3.start] = dz
    expect[M.W2.start] = 1.0 * dh2
    expect[M.B2.start] = dh2
    expect[M.W1.start] = 1.0 * dh1
    expect[M.B1.start] = dh1
    assert np.array_equal(g, expect)
    assert loss == pytest.approx(math.log(2.0), rel=1e-15)
    # the unrounded network differs exactly where the rounding points are
    g64, _ = M.grad(p, X, y, bf=False)
    assert g64[M.W1.start] == pytest.approx(0.5 * w3 * c, rel=1e-15)
    assert g64[M.W2.start] == pytest.approx(0.5 * w3, rel=1e-15)
    assert g64[M.W1.start] != g[M.W1.start] and g64[M.W2.start] != g[M.W2.start]


def test_bf16_backward_ties_to_even():
    """A product exactly halfway between two BF16 values rounds to the one
    with the even mantissa: w3 = 1 + 3*2^-8 gives dz w3 = 1/2 + 1.5 ulp
    (ulp 2^-8 at 1/2), which goes to 1/2 + 2 ulp = 1/2 + 2^-7."""
    w3 = 1.0 + 3 * 2.0 ** -8
    p = np.zeros(M.N_PARAMS)
    p[M.W1.start] = 1.0
    p[M.W2.start] = 1.0
    p[M.W3.start] = w3
    p[M.B3.start] = -w3
    X = np.zeros((1, M.IN))
    X[0, 0] = 1.0
    g, _ = M.grad(p, X, np.zeros(1), bf=True)
    assert g[M.B2.start] == 0.5 + 2.0 ** -7
    assert g[M.B1.start] == 0.5 + 2.0 ** -7


# --------------------------------------------------------------------------
# noise-free identifiability of the simulation-based fit
# --------------------------------------------------------------------------
def test_fit_identifies_true_in_set_without_noise():
    """Ten candidate sources, each active in three frames that no other
    source uses, drive target 0 through its true in-set {2, 5, 7, 9} under
    the fit's own forward model (no state noise, a small observation noise).
    Over all 2^10 subsets the true one must have the highest likelihood, and
    the toggle search started from the empty set must end on it, with its
    likelihood equal to the one evaluated for that subset here.  (From the
    correlation start the search can stop one swap away from the truth, a
    wrong source whose calcium stands in for a missing one; that end must
    still be a local optimum under single toggles.)"""
    n, nf, C = 11, 36, 10
    gain, offset, gamma, w = 1.0, 0.02, 0.002, 4.0
    model = dict(frame_num=NUM, frame_den=DEN, dt=DT, tau=20.0, v_rest=0.0, v_reset=0.0, v_th=1.0, n_ref=20,
                 drive_amp=1.5, tau_c=TAU_C)
    rng = np.random.default_rng(11)
    x = np.zeros((n, nf))
    frames = rng.permutation(np.arange(1, nf - 2))[:3 * C].reshape(C, 3)   # no frame shared by two sources
    for i in range(1, n):
        x[i, frames[i - 1]] = 1.0
    # sources' fluorescence: the frame calcium recursion with jumps n*dt per spike
    F = np.zeros((nf, n))
    for i in range(1, n):
        Fi = offset + _trace_from_activity(x[i] * gain * DT)
        F[:, i] = Fi
    first = (np.arange(nf + 1) * DEN + NUM - 1) // NUM
    steps_f = np.diff(first).astype(float)
    e = SF.activity_spikes(F, RHO, offset, gain, DT)          # the fit's view of the sources
    assert np.allclose(e[1:, :nf - 1], x[1:, :nf - 1], atol=1e-9)
    true = (2, 5, 7, 9)
    pulses = np.zeros((n, first[-1]), dtype=bool)
    u_true = w * sum(e[i] for i in true) / steps_f
    cb = SF.simulate_hypotheses([0], u_true[None, :], pulses, K=1, nf=nf, sigma=0.0, fit_seed=3, **model)
    F[:, 0] = gain * cb[0, 0] + offset + gamma * rng.standard_normal(nf)
    assert cb[0, 0].max() > 0.01                              # the target fires
    cands = list(range(1, n))
    subsets = list(itertools.product([0, 1], repeat=C))
    U = np.array([w * sum((e[cands[k]] for k in range(C) if s[k]), np.zeros(nf)) / steps_f for s in subsets])
    cbs = SF.simulate_hypotheses([0] * len(subsets), U, pulses, K=1, nf=nf, sigma=0.0, fit_seed=3, **model)
    lls = SF.loglik(cbs, np.repeat(F.T[[0]], len(subsets), 0), gain, offset, gamma)
    k_true = subsets.index(tuple(1 if c in true else 0 for c in cands))
    order = np.argsort(-lls)
    assert order[0] == k_true
    assert lls[k_true] - lls[order[1]] > 1.0                  # identified by a clear margin
    pairs = np.array([[c, 0] for c in cands])
    common = dict(drive_thr=[0] * n, control_seed=1, gain=gain, offset=offset, gamma=gamma, sigma=0.0, w=w, K=1,
                  sweeps=8, fit_seed=3, **model)
    # from the empty set the toggle search adds one true source per sweep and stops at the truth
    scores, member, ll = SF.fit(F, pairs, init_fraction=0.0, **common)
    assert tuple(int(v) for v in member) == subsets[k_true]
    assert ll[C + 0] == pytest.approx(lls[k_true], rel=1e-12)
    # at the optimum every member scores positive and every non-member negative
    assert np.all(scores[member] > 0) and np.all(scores[~member] < 0)
    # from the correlation start it ends at a local optimum under single toggles,
    # whose likelihood is the one evaluated for that subset here
    _, member, ll = SF.fit(F, pairs, **common)
    k_end = subsets.index(tuple(int(v) for v in member))
    assert ll[C + 0] == pytest.approx(lls[k_end], rel=1e-12)
    for k in range(C):
        flip = list(subsets[k_end])
        flip[k] ^= 1
        assert lls[subsets.index(tuple(flip))] <= lls[k_end]


def test_fit_per_source_weights():
    """Per-source weights enter the fit's input as w_i * e_i(f).  Pinned by
    a scaling identity and the brute force of the identifiability case:
    halving a true source's calcium deviation (so its activity e halves
    exactly) while doubling its weight leaves every likelihood bit-identical;
    the target's own weight entry is never read; and with one false source
    given a negative (inhibitory) weight, the true in-set still has the
    highest likelihood over all 2^10 subsets and the search from the empty
    set ends on it."""
    n, nf, C = 11, 36, 10
    gain, offset, gamma, w = 1.0, 0.0, 0.002, 4.0       # offset 0: halving a trace is exact
    model = dict(frame_num=NUM, frame_den=DEN, dt=DT, tau=20.0, v_rest=0.0, v_reset=0.0, v_th=1.0, n_ref=20,
                 drive_amp=1.5, tau_c=TAU_C)
    rng = np.random.default_rng(11)
    x = np.zeros((n, nf))
    frames = rng.permutation(np.arange(1, nf - 2))[:3 * C].reshape(C, 3)
    for i in range(1, n):
        x[i, frames[i - 1]] = 1.0
    F = np.zeros((nf, n))
    for i in range(1, n):
        F[:, i] = offset + _trace_from_activity(x[i] * gain * DT)
    first = (np.arange(nf + 1) * DEN + NUM - 1) // NUM
    steps_f = np.diff(first).astype(float)
    e = SF.activity_spikes(F, RHO, offset, gain, DT)
    true = (2, 5, 7, 9)
    pulses = np.zeros((n, first[-1]), dtype=bool)
    cb = SF.simulate_hypotheses([0], (w * sum(e[i] for i in true) / steps_f)[None, :], pulses, K=1, nf=nf,
                                sigma=0.0, fit_seed=3, **model)
    F[:, 0] = gain * cb[0, 0] + offset + gamma * rng.standard_normal(nf)
    pairs = np.array([[c, 0] for c in range(1, n)])
    common = dict(drive_thr=[0] * n, control_seed=1, gain=gain, offset=offset, gamma=gamma, sigma=0.0, K=1,
                  sweeps=8, fit_seed=3, **model)
    s0, m0, ll0 = SF.fit(F, pairs, init_fraction=0.0, w=w, **common)
    # scaling identity on source 5, and a wild weight on the target itself
    F2 = F.copy()
    F2[:, 5] = F[:, 5] / 2.0
    assert np.array_equal(SF.activity_spikes(F2, RHO, offset, gain, DT)[5], e[5] / 2.0)
    ws = np.full(n, w)
    ws[5] = 2.0 * w
    ws[0] = -100.0
    s1, m1, ll1 = SF.fit(F2, pairs, init_fraction=0.0, w=ws, **common)
    # (ll[C + j] scores vertex j as a target: only target 0 is the case here)
    assert np.array_equal(m0, m1) and np.array_equal(ll0[:C + 1], ll1[:C + 1]) and np.array_equal(s0, s1)
    # an inhibitory false source: brute force over all subsets with the signed weights
    ws = np.full(n, w)
    ws[3] = -w
    subsets = list(itertools.product([0, 1], repeat=C))
    U = np.array([sum((ws[k + 1] * e[k + 1] for k in range(C) if s[k]), np.zeros(nf)) / steps_f for s in subsets])
    cbs = SF.simulate_hypotheses([0] * len(subsets), U, pulses, K=1, nf=nf, sigma=0.0, fit_seed=3, **model)
    lls = SF.loglik(cbs, np.repeat(F.T[[0]], len(subsets), 0), gain, offset, gamma)
    k_true = subsets.index(tuple(1 if c in true else 0 for c in range(1, n)))
    assert np.argmax(lls) == k_true
    _, member, ll = SF.fit(F, pairs, init_fraction=0.0, w=ws, **common)
    assert tuple(int(v) for v in member) == subsets[k_true]
    assert ll[C] == pytest.approx(lls[k_true], rel=1e-12)
