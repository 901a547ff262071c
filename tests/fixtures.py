"""Shared test inputs: parsers for tests/golden and small hand-made networks."""
from __future__ import annotations

import os
from typing import Dict, List

import numpy as np

import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_fig2() -> Dict:
    """Parse golden/fig2_network.txt into edges and scenarios."""
    edges, scen, cur = [], {}, None
    with open(os.path.join(GOLDEN, "fig2_network.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            if tok[0] == "edge":
                edges.append((int(tok[1]) - 1, int(tok[2]) - 1, float(tok[3]), float(tok[4])))
            elif tok[0] == "scenario":
                cur = {"start": {}, "spikes": [], "inputs": []}
                scen[tok[1]] = cur
            elif tok[0] == "start":
                cur["start"][int(tok[1]) - 1] = float(tok[2])
            elif tok[0] == "steps":
                cur["steps"] = int(tok[1])
            elif tok[0] == "spike":
                cur["spikes"].append((int(tok[1]) - 1, int(tok[2])))
            elif tok[0] == "input":
                cur["inputs"].append((int(tok[1]) - 1, int(tok[2]), float(tok[3])))
    return {"edges": edges, "scenarios": scen}


def fig2_spec(scenario: str = "A") -> synth.NetSpec:
    g = load_fig2()
    sc = g["scenarios"][scenario]
    # Figure 1 vertex placement (arbitrary units; delays are explicit)
    pos = np.array([[0, 3], [3, 3], [6, 4], [2, 0.5], [6, 1]], dtype=np.float64) * 100.0
    src = np.array([e[0] for e in g["edges"]], dtype=np.int32)
    dst = np.array([e[1] for e in g["edges"]], dtype=np.int32)
    dly = np.array([int(round(e[2] * 10)) for e in g["edges"]], dtype=np.uint8)
    w = synth.round_fp16(np.array([e[3] for e in g["edges"]]))
    v0 = np.zeros(5, dtype=np.float32)
    for k, v in sc["start"].items():
        v0[k] = v
    spec = synth.NetSpec(name="fig2_" + scenario, pos_um=pos, src=src, dst=dst, weight=w,
                         delay_steps=dly, v0=v0, noise_sigma=0.0, seed=1)
    spec.meta["steps"] = sc["steps"]
    spec.meta["spikes"] = sc["spikes"]
    spec.meta["inputs"] = sc["inputs"]
    return spec


def single_vertex(i0: float, tau_ms: float = 20.0, dt_ms: float = 0.1) -> synth.NetSpec:
    """One isolated vertex with constant control u = (dt/tau) * i0 per step,
    so that its membrane relaxes towards i0."""
    u = np.float32((dt_ms / tau_ms) * i0)
    return synth.NetSpec(name="single", pos_um=np.zeros((1, 2)), src=np.zeros(0, np.int32),
                         dst=np.zeros(0, np.int32), weight=np.zeros(0, np.float32),
                         i_ext=np.array([u], np.float32), tau_ms=tau_ms, dt_ms=dt_ms, seed=3)


def two_vertex_chain(dist_um: float, w: float, dims: int = 2) -> synth.NetSpec:
    """Vertex 0 fires at step 0 (V0 = threshold); edge 0 -> 1 at distance dist."""
    pos = np.zeros((2, dims))
    pos[1, 0] = dist_um
    return synth.NetSpec(name="chain", pos_um=pos, src=np.array([0], np.int32),
                         dst=np.array([1], np.int32), weight=synth.round_fp16(np.array([w])),
                         v0=np.array([1.0, 0.0], np.float32), seed=5)


def random_tiny(n: int, p: float, seed: int, max_delay: int = 12, w_scale: float = 0.6,
                drive: bool = True, sigma: float = 0.0) -> synth.NetSpec:
    """Tiny random graph with explicit delays (for brute-force checks)."""
    rng = np.random.default_rng(seed)
    pairs = [(i, j) for i in range(n) for j in range(n) if i != j and rng.random() < p]
    src = np.array([a for a, _ in pairs], dtype=np.int32)
    dst = np.array([b for _, b in pairs], dtype=np.int32)
    sign = np.where(rng.random(len(pairs)) < 0.25, -1.0, 1.0)
    w = synth.round_fp16(sign * (0.5 + rng.random(len(pairs))) * w_scale)
    dly = rng.integers(1, max_delay + 1, len(pairs)).astype(np.uint8)
    rate = None
    if drive:
        rate = (rng.random(n) < 0.5).astype(np.float32) * 150.0
        rate[0] = 150.0
    return synth.NetSpec(name="tiny", pos_um=rng.random((n, 2)) * 100, src=src, dst=dst, weight=w,
                         delay_steps=dly, drive_rate_hz=rate, noise_sigma=sigma, seed=seed + 11,
                         v0=(rng.random(n) * 1.2).astype(np.float32))


def raster_events(r: np.ndarray) -> List[tuple]:
    t, j = np.nonzero(r)
    return sorted(zip(j.tolist(), t.tolist()))


def izhikevich_tiny(n: int, psc: int, seed: int, sigma: float = 1.0) -> synth.NetSpec:
    """Tiny random Izhikevich network (dt = 1 ms) with explicit delays, some
    driven vertices and a constant current on the others."""
    base = random_tiny(n, 0.5, seed, drive=True)
    rng = np.random.default_rng(1000 + seed)
    scale = synth.IZ_W0[psc] * 2.0
    w = synth.round_fp16(np.sign(base.weight) * (0.5 + rng.random(base.n_edges)) * scale)
    spec = synth.izhikevich(base, psc=psc)
    spec.weight = w
    spec.noise_sigma = sigma
    spec.i_ext = (rng.random(n) * 60.0).astype(np.float32)
    if base.drive_rate_hz is not None:
        spec.drive_rate_hz = (base.drive_rate_hz / 150.0 * 40.0).astype(np.float32)   # 40 Hz at dt = 1 ms
    return spec


def iz_params(spec) -> dict:
    return {"C": spec.iz_C, "k": spec.iz_k, "vr": spec.iz_vr, "vt": spec.iz_vt, "a": spec.iz_a, "b": spec.iz_b,
            "d": spec.iz_d, "psc": spec.psc, "psc_a": spec.psc_rate,
            "w0": None if spec.w0_iz is None else spec.w0_iz.tolist()}


def hodgkin_huxley_tiny(n: int, psc: int, seed: int, sigma: float = 0.1) -> synth.NetSpec:
    """Tiny random Hodgkin-Huxley network (dt = 0.03 ms) with explicit
    delays, driven vertices and a constant current on the others."""
    base = random_tiny(n, 0.5, seed, drive=True)
    rng = np.random.default_rng(2000 + seed)
    scale = synth.HH_W0[psc] * 2.0
    w = synth.round_fp16(np.sign(base.weight) * (0.5 + rng.random(base.n_edges)) * scale)
    spec = synth.hodgkin_huxley(base, psc=psc)
    spec.weight = w
    spec.noise_sigma = sigma
    spec.i_ext = (rng.random(n) * 8.0).astype(np.float32)
    if base.drive_rate_hz is not None:
        spec.drive_rate_hz = (base.drive_rate_hz / 150.0 * 40.0).astype(np.float32)
    return spec


def hh_params(spec) -> dict:
    return {"C": spec.hh_C, "gna": spec.hh_gna, "gk": spec.hh_gk, "gl": spec.hh_gl, "ena": spec.hh_ena,
            "ek": spec.hh_ek, "el": spec.hh_el, "psc": spec.psc, "psc_a": spec.psc_rate}


relabel = synth.relabel
