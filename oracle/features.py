"""FP64 reference of the pair features -- TEST INFRASTRUCTURE.

Written from the definitions (activity from the frame-sampled calcium model
of Section 3.3, standardisation, lagged products, control-pulse-triggered
responses); it shares no code with the GPU feature kernels.
"""
from __future__ import annotations

import numpy as np

M32 = np.uint64(0xFFFFFFFF)


def philox_np(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 (Salmon et al., SC'11) over uint64 arrays."""
    x = [np.asarray(c, dtype=np.uint64) & M32 for c in (c0, c1, c2, c3)]
    x = np.broadcast_arrays(*x)
    x = [a.copy() for a in x]
    k0, k1 = np.uint64(k0) & M32, np.uint64(k1) & M32
    for r in range(10):
        if r:
            k0 = (k0 + np.uint64(0x9E3779B9)) & M32
            k1 = (k1 + np.uint64(0xBB67AE85)) & M32
        p0 = np.uint64(0xD2511F53) * x[0]
        p1 = np.uint64(0xCD9E8D57) * x[2]
        x = [((p1 >> np.uint64(32)) ^ x[1] ^ k0) & M32, p1 & M32, ((p0 >> np.uint64(32)) ^ x[3] ^ k1) & M32,
             p0 & M32]
    return x


def frame_first_step(f, num, den):
    """First step t of frame f under frame(t) = floor(t*num/den)."""
    return (np.asarray(f, dtype=np.int64) * den + num - 1) // num


def pulses_per_frame(n, n_frames, thr, seed, num, den):
    """Control pulses of each vertex per frame: [n][n_frames]."""
    out = np.zeros((n, n_frames))
    t_end = int(frame_first_step(n_frames, num, den))
    t = np.arange(t_end, dtype=np.uint64)
    fr = (np.arange(t_end, dtype=np.int64) * num) // den
    for j in range(n):
        if thr[j] == 0:
            continue
        r = philox_np(np.uint64(j), t & M32, t >> np.uint64(32), np.uint64(0), seed & 0xFFFFFFFF, seed >> 32)
        hit = r[0] < np.uint64(thr[j])
        out[j] = np.bincount(fr[hit], minlength=n_frames)[:n_frames]
    return out


def standardise(x):
    m = x.mean(axis=-1, keepdims=True)
    v = np.maximum((x * x).mean(axis=-1, keepdims=True) - m * m, 0.0)
    inv = np.where(v > 1e-12, 1.0 / np.sqrt(np.where(v > 1e-12, v, 1.0)), 0.0)
    return (x - m) * inv


def activity(F, rho, offset):
    """e(f) = max(0, (F(f+1)-b) - rho (F(f)-b)), last frame 0; F: [n][nf]."""
    e = np.zeros_like(F)
    e[:, :-1] = np.maximum(0.0, (F[:, 1:] - offset) - rho * (F[:, :-1] - offset))
    return e


def lagcorr(a, b, L):
    nf = a.shape[-1]
    if L >= 0:
        return float(np.mean(a[:nf - L] * b[L:])) if nf - L > 0 else 0.0
    return float(np.mean(a[-L:] * b[:nf + L]))


def pulse_resp(pa, npulse, b, L):
    nf = b.shape[-1]
    return float(np.sum(pa[:nf - L] * b[L:]) / max(1.0, npulse))


def features(F_frames, pairs, dist, *, dt_ms, tau_c_ms, num, den, offset, thr, seed):
    """F_frames: [nf][n] fluorescence; pairs: [P][2]; returns [P][64]."""
    F = np.asarray(F_frames, dtype=np.float64).T          # [n][nf]
    n, nf = F.shape
    rho = (1.0 - dt_ms / tau_c_ms) ** (den / num)
    e_raw = activity(F, rho, offset)
    en, zn = standardise(e_raw), standardise(F)
    rn = standardise(en - en.mean(axis=0, keepdims=True))
    dc = pulses_per_frame(n, nf, thr, seed, num, den)
    npulse = dc.sum(1)
    mean_e = e_raw.mean(1)
    std_f = np.sqrt(np.maximum((F * F).mean(1) - F.mean(1) ** 2, 0.0))
    out = np.zeros((len(pairs), 64))
    for p, (i, j) in enumerate(pairs):
        v = out[p]
        for L in range(-8, 9):
            v[L + 8] = lagcorr(en[i], en[j], L)
        for L in range(-2, 3):
            v[19 + L] = lagcorr(zn[i], zn[j], L)
        for L in range(6):
            v[22 + L] = pulse_resp(dc[i], npulse[i], en[j], L)
        for L in range(4):
            v[28 + L] = pulse_resp(dc[j], npulse[j], en[i], L)
        v[32], v[33] = np.log1p(npulse[i]), np.log1p(npulse[j])
        v[34], v[35] = mean_e[i], mean_e[j]
        v[36], v[37] = std_f[i], std_f[j]
        v[38] = dist[p] / 150.0
        for L in range(4):
            v[39 + L] = lagcorr(rn[i], rn[j], L)
        for L in range(8):
            v[43 + L] = lagcorr(en[i], zn[j], L)
            v[51 + L] = lagcorr(zn[i], en[j], L)
    return out
