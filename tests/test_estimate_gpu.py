"""GPU pair features against the FP64 feature reference on the same
observations (produced by the CPU oracle), and the estimation pipeline's
pieces end to end on a small scale."""
import numpy as np
import pytest

import oracle
import synth
from oracle import features as FE
from oracle import metrics

pytestmark = pytest.mark.gpu


def _oracle_observation(n=256, steps=68000, seed_net=0):
    spec = synth.config0_like(n, synth.config_seed(4, 500 + seed_net), w0=synth.W0)
    spec.noise_sigma = synth.NOISE_SIGMA
    nf = steps * spec.frame_num // spec.frame_den
    o = oracle.OracleNet(spec, frames_cap=nf)
    o.step(steps)
    cbar = o.frames()
    gamma = spec.dt_ms / 5.0
    F = oracle.fluorescence(cbar, 1.0, 0.0, gamma, spec.seed).astype(np.float32)
    return spec, F, gamma


def test_features_match_reference():
    import torch
    import paper_0908_3934_amd as gn
    from paper_0908_3934_amd import estimate as est
    spec, F, gamma = _oracle_observation()
    pairs, dist, labels = est.candidate_pairs(spec)
    sel = np.arange(0, len(pairs), max(1, len(pairs) // 400))     # a sample of pairs
    pairs, dist, labels = pairs[sel], dist[sel], labels[sel]
    o = est.Observed(spec=spec, F=torch.tensor(F, device="cuda"), pairs=torch.tensor(pairs, device="cuda"),
                     dist=torch.tensor(dist, device="cuda"), labels=labels, gain=1.0, offset=0.0, gamma=gamma)
    g = est.features(o).cpu().numpy().astype(np.float64)
    thr = [oracle.drive_threshold(float(r), spec.dt_ms) for r in spec.drive_rate_hz]
    ref = FE.features(F.astype(np.float64), pairs, dist.astype(np.float64), dt_ms=spec.dt_ms, tau_c_ms=spec.tau_c_ms,
                      num=spec.frame_num, den=spec.frame_den, offset=0.0, thr=thr, seed=spec.seed)
    err = np.abs(g - ref)
    assert err.max() <= 1e-4 * max(1.0, np.abs(ref).max()), (np.unravel_index(err.argmax(), err.shape), err.max())
    assert np.abs(ref[:, 22:28]).sum() > 0          # driven sources give pulse responses


def test_auc_binding_matches_metrics():
    from paper_0908_3934_amd import estimate as est
    rng = np.random.default_rng(0)
    s = np.round(rng.normal(0, 1, 5000), 2)
    y = rng.random(5000) < 0.3
    assert est.auc(s, y) == pytest.approx(metrics.auc(s, y), abs=1e-12)


def test_scorer_learns_on_simulated_networks():
    """Small-scale end-to-end: simulate, observe, train on 24 networks, score
    4 held-out ones; the learned scores must beat chance clearly."""
    from paper_0908_3934_amd import estimate as est
    specs = [synth.config4_net(m) for m in range(28)]
    obs = est.observe(specs, 100000)
    sc = est.EdgeScorer(seed=0).fit(obs[:24], epochs=3, batch=8192)
    s = np.concatenate([sc.score(o).cpu().numpy() for o in obs[24:]])
    y = np.concatenate([o.labels for o in obs[24:]])
    assert est.auc(s, y) > 0.54


def test_trained_scorer_gains_over_activity_correlation():
    """What training adds: on held-out networks the learned scorer ranks the
    candidate pairs better than the lag-0 + lag-1 correlation of the
    deconvolved activity (features 8 and 9, the statistic the fit starts
    from).  64 training networks of 1,024 vertices, 600 frames each."""
    from paper_0908_3934_amd import estimate as est
    specs = [synth.config4_net(m) for m in range(64)] + [synth.config4_net(9000 + m) for m in range(4)]
    obs = est.observe(specs, 200000)
    train, test = obs[:64], obs[64:]
    sc = est.EdgeScorer(seed=0).fit(train, epochs=4, batch=16384, feats=[est.features(o) for o in train])
    S, C, Y = [], [], []
    for o in test:
        f = est.features(o)
        S.append(sc.score(o, f).cpu().numpy())
        fc = f.cpu().numpy()
        C.append(fc[:, 8] + fc[:, 9])
        Y.append(o.labels)
    S, C, Y = map(np.concatenate, (S, C, Y))
    a_s, a_c = est.auc(S, Y), est.auc(C, Y)
    print("held-out AUC: scorer %.4f, activity correlation %.4f" % (a_s, a_c), flush=True)
    assert a_s > a_c + 0.015
