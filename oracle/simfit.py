"""FP64 reference of the simulation-based fit -- TEST INFRASTRUCTURE.

The paper leaves its estimator to later work (Sections 1 and 4), so the fit
is defined here, in the steps the GPU path follows:

1. activity e_i(f) = max(0, (F_i(f+1) - b) - rho (F_i(f) - b)) / (n dt), in
   spikes (calcium jumps by dt per spike, Section 3.3), last frame 0;
2. initial in-neighbours of target j: the top fraction of its candidates
   by the lag-0 plus lag-1 correlation of standardised activity;
3. a hypothesis (j, G) is scored by simulating vertex j (LIF Euler step with
   refractory hold, its control pulses, K realisations of state noise from
   the fit's own Philox key, calcium transition), teacher-forced by the input
   sum_{i in G} w_i e_i(f) / S(f) in every step of frame f (w_i the weight
   assumed on the edges out of i: one value for all, or negative for the
   inhibitory cells of a network whose cell types are known), and taking the
   Gaussian log-likelihood of the observed trace with the realisations'
   frame-mean calcium mean and variance;
4. each sweep evaluates every single toggle and, per target, applies the
   one that raises its likelihood most, if by more than min_gain nats; the
   score of a candidate is LL(G + e) - LL(G - e) at the final G.

Everything is float64 and vectorised over all hypotheses and realisations.
"""
from __future__ import annotations

import math

import numpy as np

from . import features as FE


def activity_spikes(F, rho, offset, gain, dt):
    """F: [nf][n] -> e: [n][nf] in spikes."""
    return FE.activity(np.asarray(F, dtype=np.float64).T, rho, offset) / (gain * dt)


def initial_members(en, pairs, frac):
    """Top `frac` of each target's candidates (candidates of a target taken in
    pair order, stable sort by the lag-0 + lag-1 activity correlation)."""
    P = len(pairs)
    score = np.array([FE.lagcorr(en[i], en[j], 0) + FE.lagcorr(en[i], en[j], 1) for i, j in pairs])
    member = np.zeros(P, dtype=bool)
    targets = pairs[:, 1]
    for j in np.unique(targets):
        idx = np.nonzero(targets == j)[0]
        order = idx[np.argsort(-score[idx], kind="stable")]
        member[order[:math.ceil(frac * idx.size - 1e-6)]] = True     # ceil(f n), f n integral counts exactly
    return member


def simulate_hypotheses(j_of, u_frames, pulses, *, K, frame_num, frame_den, nf, dt, tau, v_rest, v_reset, v_th,
                        n_ref, sigma, drive_amp, tau_c, fit_seed):
    """Vertex j_of[h] under per-frame input u_frames[h][f] (per step), K
    realisations each.  Returns cbar [H][K][nf] (frame-mean calcium)."""
    H = len(j_of)
    R = H * K
    jr = np.repeat(np.asarray(j_of, dtype=np.int64), K)
    kr = np.tile(np.arange(K, dtype=np.uint64), H)
    V = np.full(R, v_rest)
    age = np.full(R, 255, dtype=np.int64)
    c = np.zeros(R)
    acc = np.zeros(R)
    cbar = np.zeros((R, nf))
    decay = dt / tau
    lo, hi = fit_seed & 0xFFFFFFFF, fit_seed >> 32
    t = 0
    for f in range(nf):
        t1 = (((f + 1) * frame_den + frame_num - 1) // frame_num)
        u = np.repeat(u_frames[:, f], K)
        while t < t1:
            acc += c
            spike = V >= v_th
            c = c + dt * (-c / tau_c + spike.astype(np.float64))
            held = (age >= 1) & (age <= n_ref)
            age_n = np.where(spike, 1, np.minimum(age + 1, 255))
            q = FE.philox_np(jr.astype(np.uint64), np.uint64(t & 0xFFFFFFFF), np.uint64(t >> 32),
                             np.uint64(2) + kr, lo, hi)
            u1 = ((q[1] >> np.uint64(8)).astype(np.float64) + 0.5) / 16777216.0
            u2 = ((q[2] >> np.uint64(8)).astype(np.float64) + 0.5) / 16777216.0
            xi = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
            inp = u + np.where(pulses[jr, t], drive_amp, 0.0) + (sigma * xi if sigma != 0.0 else 0.0)
            integ = V + decay * (v_rest - V) + inp
            V = np.where(spike | held, v_reset, integ)
            age = age_n
            t += 1
        steps = t1 - (((f * frame_den) + frame_num - 1) // frame_num)
        cbar[:, f] = acc / steps
        acc[:] = 0.0
    return cbar.reshape(H, K, nf)


def loglik(cbar, Fj, gain, offset, gamma):
    """cbar: [H][K][nf]; Fj: [H][nf] observed trace of each hypothesis' target."""
    mean = cbar.mean(1)
    var = np.maximum((cbar * cbar).mean(1) - mean * mean, 0.0)
    mu = gain * mean + offset
    s2 = gamma * gamma + gain * gain * var
    return -0.5 * np.sum((Fj - mu) ** 2 / s2 + np.log(s2), axis=1)


def fit(F, pairs, *, drive_thr, control_seed, gain, offset, gamma, dt, tau, v_rest, v_reset, v_th, n_ref, sigma,
        drive_amp, tau_c, frame_num, frame_den, w, K=8, sweeps=2, init_fraction=0.3, fit_seed=0x5EEDF17,
        min_gain=1e-3):
    """Scores LL(G + e) - LL(G - e) per pair (in the given order); w is one
    weight for every source or a length-n array of per-source weights."""
    F = np.asarray(F, dtype=np.float64)
    nf, n = F.shape
    pairs = np.asarray(pairs, dtype=np.int64)
    P = len(pairs)
    rho = (1.0 - dt / tau_c) ** (frame_den / frame_num)
    e = activity_spikes(F, rho, offset, gain, dt)
    en = FE.standardise(FE.activity(F.T, rho, offset))
    member = initial_members(en, pairs, init_fraction)
    t_end = (nf * frame_den + frame_num - 1) // frame_num
    pulses = np.zeros((n, t_end), dtype=bool)
    tt = np.arange(t_end, dtype=np.uint64)
    for j in range(n):
        if drive_thr[j]:
            x0 = FE.philox_np(np.uint64(j), tt & np.uint64(0xFFFFFFFF), tt >> np.uint64(32), np.uint64(0),
                              control_seed & 0xFFFFFFFF, control_seed >> 32)[0]
            pulses[j] = x0 < np.uint64(drive_thr[j])
    wv = np.broadcast_to(np.asarray(w, dtype=np.float64), (n,))
    first = (np.arange(nf + 1) * frame_den + frame_num - 1) // frame_num
    steps = np.diff(first).astype(np.float64)
    targets = pairs[:, 1]
    j_of = np.concatenate([targets, np.arange(n)])
    ll = None
    for sw in range(sweeps + 1):
        base = np.zeros((n, nf))
        for p in np.nonzero(member)[0]:
            base[targets[p]] += wv[pairs[p, 0]] * e[pairs[p, 0]]
        base = base / steps
        toggle = np.where(member, -1.0, 1.0) * wv[pairs[:, 0]]
        u = np.concatenate([base[targets] + toggle[:, None] * e[pairs[:, 0]] / steps, base])
        cb = simulate_hypotheses(j_of, u, pulses, K=K, frame_num=frame_num, frame_den=frame_den, nf=nf, dt=dt,
                                 tau=tau, v_rest=v_rest, v_reset=v_reset, v_th=v_th, n_ref=n_ref, sigma=sigma,
                                 drive_amp=drive_amp, tau_c=tau_c, fit_seed=fit_seed)
        ll = loglik(cb, F.T[j_of], gain, offset, gamma)
        if sw == sweeps:
            break
        delta = ll[:P] - ll[P + targets]
        for j in np.unique(targets):
            idx = np.nonzero(targets == j)[0]          # candidates of j in pair order
            k = idx[np.argmax(delta[idx])]             # first maximum, as the library's scan
            if delta[k] > min_gain:
                member[k] = ~member[k]
    cur, tog = ll[P + targets], ll[:P]
    return np.where(member, cur - tog, tog - cur), member, ll
