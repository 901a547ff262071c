"""Brute-force dense formulation for tiny networks (N <= 8) -- TEST INFRASTRUCTURE.

A second, deliberately different way to evaluate the same model as
``oracle.c``, used to pin it:

* the delayed input of vertex j at step t is evaluated straight from the
  definition, sum over k != j of w_kj * spd(V_k(t - tau_kj)) (Section 3.2,
  Eq. izpsc, last term), reading a full spike-history matrix instead of an
  event-driven inbox;
* the refractory hold is expressed through the time since the last spike
  (held while 1 <= t - t_last <= n_ref) rather than a countdown;
* everything is pure-Python floats and ints, one loop per vertex.

Philox4x32-10 (Salmon et al., SC'11) is re-implemented here in Python
integers so the formulation is self-contained; both implementations are
pinned by the published known-answer vectors.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence

M32 = 0xFFFFFFFF


def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> List[int]:
    x0, x1, x2, x3 = (int(c) & M32 for c in ctr)
    k0, k1 = int(key[0]) & M32, int(key[1]) & M32
    for r in range(10):
        if r:
            k0 = (k0 + 0x9E3779B9) & M32
            k1 = (k1 + 0xBB67AE85) & M32
        p0 = 0xD2511F53 * x0
        p1 = 0xCD9E8D57 * x2
        x0, x1, x2, x3 = ((p1 >> 32) ^ x1 ^ k0) & M32, p1 & M32, ((p0 >> 32) ^ x3 ^ k1) & M32, p0 & M32
    return [x0, x1, x2, x3]


def gauss(a: int, b: int) -> float:
    u1 = ((a >> 8) + 0.5) / 16777216.0
    u2 = ((b >> 8) + 0.5) / 16777216.0
    return math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)


def simulate(n: int, edges: Sequence, steps: int, *, dt: float = 0.1, tau: float = 20.0,
             v_rest: float = 0.0, v_reset: float = 0.0, v_th: float = 1.0, n_ref: int = 20,
             drive_thr: Optional[Sequence[int]] = None, drive_amp: float = 1.5,
             i_ext: Optional[Sequence[float]] = None, sigma: float = 0.0, seed: int = 0,
             v0: Optional[Sequence[float]] = None, izhikevich: Optional[dict] = None,
             hodgkin_huxley: Optional[dict] = None, stdp: Optional[dict] = None) -> Dict[str, list]:
    """edges: iterable of (src, dst, weight, delay_steps).

    izhikevich: None for the LIF vertex, else a dict with C, k, vr, vt, a,
    b, d, psc (0 none, 1 exponential, 2 alpha), psc_a and optionally w0: the
    simple model of Section 3.1 (V_peak = v_th, c = v_reset) whose synaptic
    states follow Section 3.2; the records then also hold W, r and p.

    hodgkin_huxley: None, or a dict with C, gna, gk, gl, ena, ek, el, psc,
    psc_a: the four-state vertex of Section 3.1 with the standard rate
    functions (written below independently of oracle.c), spikes signalled on
    the upward crossing of v_th, gates starting at their steady state.

    stdp: None, or a dict with alpha, beta: the weights evolve by the
    plasticity rule of Section 3.2, evaluated from the full spike history
    (the time since the last spike read off the history matrix), each
    increment rounded to a multiple of 2^-20; the records then also hold the
    weight matrix after the run ("w_final")."""
    assert n <= 8, "brute force is for tiny networks"
    W = [[0.0] * n for _ in range(n)]
    A = [[False] * n for _ in range(n)]
    D = [[0] * n for _ in range(n)]
    for (i, j, w, d) in edges:
        assert i != j and not A[i][j]
        A[i][j] = True
        W[i][j] = float(w)
        D[i][j] = int(d)
    key = (seed & M32, (seed >> 32) & M32)
    V = [float(v) for v in v0] if v0 is not None else [v_rest] * n
    last = [None] * n
    hist: List[List[int]] = []
    rec_s, rec_v, rec_i = [], [], []
    hh = hodgkin_huxley
    if hh is not None:
        return _simulate_hh(n, A, W, D, steps, dt, v_th, drive_thr, drive_amp, i_ext, sigma, key,
                            [float(v) for v in v0] if v0 is not None else [v_rest] * n, hh)
    iz = izhikevich
    if iz is not None:
        Wr = [float(x) for x in iz["w0"]] if iz.get("w0") is not None else [0.0] * n
        R = [0.0] * n
        P = [0.0] * n
        rec_w, rec_r, rec_p = [], [], []
    for t in range(steps):
        s = [1 if V[j] >= v_th else 0 for j in range(n)]
        hist.append(s)
        rec_s.append(s)
        rec_v.append(list(V))
        I = []
        for j in range(n):
            tot = 0.0
            for k in range(n):
                if k == j or not A[k][j]:
                    continue
                tk = t - D[k][j]
                if tk >= 0 and hist[tk][k]:
                    tot += W[k][j]
            I.append(tot)
        rec_i.append(I)
        if stdp is not None:
            def since(k, u):
                # time since k's last spike strictly before step u
                if u <= 0:
                    return 0.0
                for v in range(u - 1, -1, -1):
                    if hist[v][k]:
                        return (u - v - 1) * dt
                return u * dt
            for k in range(n):
                for j in range(n):
                    if k == j or not A[k][j]:
                        continue
                    u = t - D[k][j]
                    pre = u >= 0 and hist[u][k]
                    if not (pre or s[j]):
                        continue
                    q = since(k, u) - since(j, t)
                    sg = 1.0 if q > 0 else (-1.0 if q < 0 else 0.0)
                    dw = dt * stdp["alpha"] * sg * math.exp(-stdp["beta"] * abs(q))
                    W[k][j] = (round(W[k][j] * 1048576.0) + int(round(dw * 1048576.0))) / 1048576.0
        newV = list(V)
        if iz is not None:
            rec_w.append(list(Wr))
            rec_r.append(list(R))
            rec_p.append(list(P))
            a = iz["psc_a"]
            newW, newR, newP = list(Wr), list(R), list(P)
            for j in range(n):
                # synaptic current: an arrival is an impulse into r (exp) or p (alpha)
                if iz["psc"] == 1:
                    newR[j] = R[j] - dt * a * R[j] + I[j]
                elif iz["psc"] == 2:
                    newR[j] = R[j] + dt * P[j]
                    newP[j] = P[j] + dt * (-a * a * R[j] - 2.0 * a * P[j]) + I[j]
                if s[j]:
                    newV[j] = v_reset
                    newW[j] = Wr[j] + iz["d"]
                    continue
                r = philox4x32_10((j, t & M32, t >> 32, 0), key)
                u = (float(i_ext[j]) if i_ext is not None else 0.0) + \
                    (drive_amp if (drive_thr is not None and r[0] < drive_thr[j]) else 0.0)
                xi = gauss(r[1], r[2])
                syn = 0.0 if iz["psc"] == 0 else R[j]
                cur = iz["k"] * (V[j] - iz["vr"]) * (V[j] - iz["vt"]) - Wr[j] + syn + u
                vn = V[j] + dt * (1.0 / iz["C"]) * cur
                if iz["psc"] == 0:
                    vn = vn + I[j]
                newV[j] = vn + sigma * xi
                newW[j] = Wr[j] + dt * iz["a"] * (iz["b"] * (V[j] - iz["vr"]) - Wr[j])
            V, Wr, R, P = newV, newW, newR, newP
            continue
        for j in range(n):
            if s[j]:
                newV[j] = v_reset
                last[j] = t
                continue
            if last[j] is not None and 1 <= t - last[j] <= n_ref:
                newV[j] = v_reset
                continue
            r = philox4x32_10((j, t & M32, t >> 32, 0), key)
            u = (float(i_ext[j]) if i_ext is not None else 0.0) + \
                (drive_amp if (drive_thr is not None and r[0] < drive_thr[j]) else 0.0)
            xi = gauss(r[1], r[2])
            newV[j] = V[j] + (dt / tau) * (v_rest - V[j]) + I[j] + u + sigma * xi
        V = newV
    out = {"raster": rec_s, "v": rec_v, "input": rec_i, "v_final": V, "w_final": W}
    if iz is not None:
        out.update(w=rec_w, r=rec_r, p=rec_p)
    return out


def _rates(V: float):
    """(alpha, beta) of m, h, n at V (mV, ms), the standard squid-axon set."""
    x = V + 40.0
    am = 1.0 if x == 0.0 else 0.1 * x / (1.0 - math.exp(-x / 10.0))
    bm = 4.0 * math.exp(-(V + 65.0) / 18.0)
    ah = 0.07 * math.exp(-(V + 65.0) / 20.0)
    bh = 1.0 / (1.0 + math.exp(-(V + 35.0) / 10.0))
    y = V + 55.0
    an = 0.1 if y == 0.0 else 0.01 * y / (1.0 - math.exp(-y / 10.0))
    bn = 0.125 * math.exp(-(V + 65.0) / 80.0)
    return (am, bm), (ah, bh), (an, bn)


def _simulate_hh(n, A, W, D, steps, dt, v_th, drive_thr, drive_amp, i_ext, sigma, key, V, hh):
    gates = []
    for j in range(n):
        (am, bm), (ah, bh), (an, bn) = _rates(V[j])
        gates.append([am / (am + bm), ah / (ah + bh), an / (an + bn)])   # m, h, n at rest
    Vprev = list(V)
    R = [0.0] * n
    P = [0.0] * n
    hist: List[List[int]] = []
    rec_s, rec_v, rec_i = [], [], []
    a = hh["psc_a"]
    for t in range(steps):
        s = [1 if (V[j] >= v_th and Vprev[j] < v_th) else 0 for j in range(n)]
        hist.append(s)
        rec_s.append(s)
        rec_v.append(list(V))
        I = []
        for j in range(n):
            tot = 0.0
            for k in range(n):
                if k != j and A[k][j] and t - D[k][j] >= 0 and hist[t - D[k][j]][k]:
                    tot += W[k][j]
            I.append(tot)
        rec_i.append(I)
        newV, newR, newP, newG = list(V), list(R), list(P), [list(g) for g in gates]
        for j in range(n):
            if hh["psc"] == 1:
                newR[j] = R[j] - dt * a * R[j] + I[j]
            elif hh["psc"] == 2:
                newR[j] = R[j] + dt * P[j]
                newP[j] = P[j] + dt * (-a * a * R[j] - 2.0 * a * P[j]) + I[j]
            r = philox4x32_10((j, t & M32, t >> 32, 0), key)
            u = (float(i_ext[j]) if i_ext is not None else 0.0) + \
                (drive_amp if (drive_thr is not None and r[0] < drive_thr[j]) else 0.0)
            xi = gauss(r[1], r[2])
            m, h, nn = gates[j]
            syn = 0.0 if hh["psc"] == 0 else R[j]
            i_na = hh["gna"] * m * m * m * h * (V[j] - hh["ena"])
            i_k = hh["gk"] * nn * nn * nn * nn * (V[j] - hh["ek"])
            i_l = hh["gl"] * (V[j] - hh["el"])
            vn = V[j] + dt * (1.0 / hh["C"]) * (-i_na - i_k - i_l + syn + u)
            if hh["psc"] == 0:
                vn = vn + I[j]
            newV[j] = vn + sigma * xi
            (am, bm), (ah, bh), (an, bn) = _rates(V[j])
            newG[j] = [m + dt * (am * (1.0 - m) - bm * m), h + dt * (ah * (1.0 - h) - bh * h),
                       nn + dt * (an * (1.0 - nn) - bn * nn)]
        Vprev = list(V)
        V, R, P, gates = newV, newR, newP, newG
    return {"raster": rec_s, "v": rec_v, "input": rec_i, "v_final": V}
