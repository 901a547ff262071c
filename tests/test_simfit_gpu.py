"""GPU simulation-based fit against the FP64 fit reference on the same
observation (simulated and observed by the CPU oracle), plus its argument
checks.  Both sides run the fit's vertex model and its Box-Muller noise in
FP64, so they follow the same toggle path and every score agrees to 1e-6
relative (the two sum the log-likelihood over frames and realisations in
different orders)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import simfit as SF
from oracle import metrics

pytestmark = pytest.mark.gpu

NF = 20


def _f32(x):
    return float(np.float32(x))


def _case(n_targets=16, seed=3, signed=False):
    spec = synth.config0_like(256, synth.config_seed(4, 700 + seed), w0=synth.W0)
    spec.noise_sigma = synth.NOISE_SIGMA
    if signed:
        # 20 % inhibitory sources at three times the excitatory magnitude
        inh = np.zeros(spec.n, dtype=bool)
        inh[np.random.default_rng(seed).permutation(spec.n)[: spec.n // 5]] = True
        spec.weight = np.where(inh[spec.src], synth.round_fp16(-3.0 * spec.weight), spec.weight).astype(np.float32)
        spec.inhibitory = inh
    steps = (NF * spec.frame_den + spec.frame_num - 1) // spec.frame_num
    o = oracle.OracleNet(spec, frames_cap=NF)
    o.step(steps)
    gamma = _f32(spec.dt_ms / 5.0)
    F = oracle.fluorescence(o.frames(), 1.0, 0.0, gamma, spec.seed).astype(np.float32)
    from paper_0908_3934_amd import estimate as est
    pairs, dist, labels = est.candidate_pairs(spec)
    targets = np.unique(pairs[:, 1])[:n_targets]
    sel = np.nonzero(np.isin(pairs[:, 1], targets))[0]
    sel = np.random.default_rng(seed).permutation(sel)        # library sorts by target internally
    return spec, F, gamma, pairs[sel], dist[sel], labels[sel]


def _gpu(spec, F, gamma, pairs, dist, labels, **kw):
    import torch
    from paper_0908_3934_amd import estimate as est
    ob = est.Observed(spec=spec, F=torch.tensor(F, device="cuda"), pairs=torch.tensor(pairs, device="cuda"),
                      dist=torch.tensor(dist, device="cuda"), labels=labels, gain=1.0, offset=0.0, gamma=gamma)
    return est.simfit(ob, **kw).cpu().numpy().astype(np.float64)


def _ref(spec, F, gamma, pairs, *, w, K, sweeps, fit_seed):
    w = np.asarray(w, dtype=np.float32).astype(np.float64) if np.ndim(w) else _f32(w)
    thr = [oracle.drive_threshold(float(r), spec.dt_ms) for r in spec.drive_rate_hz]
    return SF.fit(F.astype(np.float64), pairs, drive_thr=thr, control_seed=spec.seed, gain=1.0, offset=0.0,
                  gamma=gamma, dt=spec.dt_ms, tau=spec.tau_ms, v_rest=spec.v_rest, v_reset=spec.v_reset,
                  v_th=spec.v_th, n_ref=spec.n_ref, sigma=_f32(spec.noise_sigma), drive_amp=spec.drive_amp,
                  tau_c=spec.tau_c_ms, frame_num=spec.frame_num, frame_den=spec.frame_den, w=w, K=K,
                  sweeps=sweeps, init_fraction=0.3, fit_seed=fit_seed)


@pytest.mark.parametrize("sweeps", [0, 2])
def test_simfit_matches_reference(sweeps):
    spec, F, gamma, pairs, dist, labels = _case()
    w, K, fs = synth.W0, 4, 0x5EEDF17
    print("simfit parity: P=%d sweeps=%d K=%d" % (len(pairs), sweeps, K), flush=True)
    g = _gpu(spec, F, gamma, pairs, dist, labels, w_assumed=w, realisations=K, sweeps=sweeps, fit_seed=fs)
    ref, member, _ = _ref(spec, F, gamma, pairs, w=w, K=K, sweeps=sweeps, fit_seed=fs)
    assert np.isfinite(g).all()
    close = np.abs(g - ref) <= 1e-6 * np.maximum(1.0, np.abs(ref))
    bad_targets = sorted(set(pairs[~close, 1].tolist()))
    assert close.all(), (close.mean(), np.abs(g - ref).max(), bad_targets)
    assert abs(metrics.auc(g, labels) - metrics.auc(ref, labels)) <= 1e-9
    assert np.abs(ref).max() > 1e-3                     # the toggles do change the likelihood


def test_simfit_per_source_weights_match_reference():
    """Per-source assumed weights (inhibitory sources negative): the same
    fit as the reference, and a uniform w_source equals w_assumed exactly."""
    from paper_0908_3934_amd import estimate as est
    spec, F, gamma, pairs, dist, labels = _case(seed=5, signed=True)
    w0 = synth.W0
    ws = est.source_weights(spec, w0, g_inh=3.0)
    assert (ws < 0).sum() == spec.n // 5
    K, fs = 4, 0x5EEDF17
    print("simfit per-source weights: P=%d" % len(pairs), flush=True)
    g = _gpu(spec, F, gamma, pairs, dist, labels, w_assumed=w0, w_source=ws, realisations=K, sweeps=2, fit_seed=fs)
    ref, _, _ = _ref(spec, F, gamma, pairs, w=ws, K=K, sweeps=2, fit_seed=fs)
    close = np.abs(g - ref) <= 1e-6 * np.maximum(1.0, np.abs(ref))
    assert close.all(), (close.mean(), np.abs(g - ref).max())
    a = _gpu(spec, F, gamma, pairs, dist, labels, w_assumed=w0, realisations=K, sweeps=1, fit_seed=fs)
    b = _gpu(spec, F, gamma, pairs, dist, labels, w_assumed=0.0, w_source=np.full(spec.n, _f32(w0), np.float32),
             realisations=K, sweeps=1, fit_seed=fs)
    assert np.array_equal(a, b)
    with pytest.raises(ValueError):
        _gpu(spec, F, gamma, pairs, dist, labels, w_assumed=w0, w_source=ws[:-1])


def test_simfit_same_seed_same_scores():
    spec, F, gamma, pairs, dist, labels = _case(n_targets=3, seed=4)
    a = _gpu(spec, F, gamma, pairs, dist, labels, w_assumed=synth.W0, realisations=8, sweeps=1)
    b = _gpu(spec, F, gamma, pairs, dist, labels, w_assumed=synth.W0, realisations=8, sweeps=1)
    assert np.array_equal(a, b)


def test_simfit_argument_errors():
    import paper_0908_3934_amd as gn
    spec, F, gamma, pairs, dist, labels = _case(n_targets=2, seed=5)
    with pytest.raises(gn.GeonetError):
        _gpu(spec, F, gamma, pairs, dist, labels, w_assumed=synth.W0, realisations=3)   # must divide 64
    with pytest.raises(gn.GeonetError):
        _gpu(spec, F, gamma, pairs, dist, labels, w_assumed=synth.W0, sweeps=65)
    bad = pairs.copy()
    bad[0, 0] = bad[0, 1]
    with pytest.raises(gn.GeonetError):
        _gpu(spec, F, gamma, bad, dist, labels, w_assumed=synth.W0)                      # self pair


def test_auto_method_dispatch():
    """NET_EST_AUTO: the scorer's scores when a scorer is given, the fit's otherwise."""
    import torch
    from paper_0908_3934_amd import estimate as est
    spec, F, gamma, pairs, dist, labels = _case(n_targets=3, seed=6)
    ob = est.Observed(spec=spec, F=torch.tensor(F, device="cuda"), pairs=torch.tensor(pairs, device="cuda"),
                      dist=torch.tensor(dist, device="cuda"), labels=labels, gain=1.0, offset=0.0, gamma=gamma)
    sc = est.EdgeScorer(seed=1)
    assert torch.equal(est.estimate(ob, scorer=sc), est.scorer_scores(ob, sc))
    fit = dict(realisations=4, sweeps=1)
    assert torch.equal(est.estimate(ob, w_assumed=synth.W0, **fit), est.simfit(ob, synth.W0, **fit))
