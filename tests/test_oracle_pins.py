"""Pins of the FP64 oracle against things other than itself.

Every check here is fixed by the paper, by mathematics or by a published
reference value; none retypes the oracle's formula and compares it with
itself.  All run on the CPU.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import dense
from tests import fixtures as fx

pytestmark = pytest.mark.filterwarnings("ignore")


# --------------------------------------------------------------------------
# Philox4x32-10: published known-answer vectors (Salmon et al., SC'11,
# reference distribution), and two independent implementations agreeing.
# --------------------------------------------------------------------------
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,expect", KAT)
def test_philox_known_answers(ctr, key, expect):
    assert tuple(int(x) for x in oracle.philox4x32_10(ctr, key)) == expect
    assert tuple(dense.philox4x32_10(ctr, key)) == expect


def test_philox_two_implementations_agree():
    rng = np.random.default_rng(0)
    for _ in range(300):
        ctr = rng.integers(0, 2**32, 4, dtype=np.uint64).tolist()
        key = rng.integers(0, 2**32, 2, dtype=np.uint64).tolist()
        assert oracle.philox4x32_10(ctr, key).tolist() == dense.philox4x32_10(ctr, key)


def test_uniform_is_exact_24bit_midpoint():
    assert oracle.u01_24(0) == 0.5 / 2**24
    assert oracle.u01_24(0xFFFFFFFF) == (2**24 - 0.5) / 2**24
    assert oracle.u01_24(0x80000000) == 0.5 + 0.5 / 2**24


def test_box_muller_moments():
    key = (123, 456)
    xs = []
    for j in range(40000):
        r = dense.philox4x32_10((j, 7, 0, 0), key)
        xs.append(oracle.box_muller(r[1], r[2]))
    x = np.array(xs)
    n = x.size
    assert abs(x.mean()) < 5 / math.sqrt(n)
    assert abs(x.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    # fourth moment of a standard normal is 3
    assert abs((x**4).mean() - 3.0) < 0.15
    # special values: u2 -> cos(2 pi u2) with u1 = 1/2 gives sqrt(2 ln 2)
    a = 0x7FFFFF00  # u1 = 0.5 - ~1e-8 (not exactly 1/2), check against closed form
    u1 = ((a >> 8) + 0.5) / 2**24
    assert oracle.box_muller(a, 0) == pytest.approx(math.sqrt(-2 * math.log(u1)) * math.cos(2 * math.pi * 0.5 / 2**24),
                                                    rel=1e-15)


def test_drive_threshold_integer_rule():
    # 5 Hz at 0.1 ms: p = 5e-4, floor(p * 2^32) = 2147483
    assert oracle.drive_threshold(5.0, 0.1) == 2147483
    assert oracle.drive_threshold(0.0, 0.1) == 0
    assert oracle.drive_threshold(1e9, 0.1) == 0xFFFFFFFF


# --------------------------------------------------------------------------
# Delays: Eq. delaydist, tau = |x_i - x_j| / s, in steps ceil(tau/dt) >= 1.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("xi,xj,expect", [
    ((0.0, 0.0), (150.0, 0.0), 15),            # exact multiple of s*dt = 10 um
    ((0.0, 0.0), (150.000001, 0.0), 16),
    ((0.0, 0.0), (149.999, 0.0), 15),
    ((0.0, 0.0), (30.0, 40.0), 5),             # 3-4-5 triangle: 50 um
    ((5.0, 5.0), (5.0, 5.0), 1),               # coincident vertices: causal minimum 1
    ((0.0, 0.0, 0.0), (20.0, 20.0, 10.0), 3),  # 3D: 30 um
    ((0.0, 0.0), (2550.0, 0.0), 255),
    ((0.0, 0.0), (2550.5, 0.0), -1),           # above the 8-bit range
])
def test_delay_rule(xi, xj, expect):
    assert oracle.delay_steps(xi, xj, synth.V_UM_PER_MS, synth.DT_MS) == expect


# --------------------------------------------------------------------------
# LIF closed forms (Section 3.1: voltage decays to a target, threshold, reset
# at the next step; Euler integration).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("i0,n_star,period", [(1.5, 220, 241), (2.0, 139, 160), (1.2, 358, 379)])
def test_lif_discrete_period_closed_form(i0, n_star, period):
    spec = fx.single_vertex(i0)
    a = spec.dt_ms / spec.tau_ms
    u = float(spec.i_ext[0])
    # From V = 0, V_k = u * (1 - (1-a)^k) / a; first k with V_k >= 1.
    k_exact = math.log(1.0 - spec.v_th * a / u) / math.log(1.0 - a)
    assert math.ceil(k_exact) == n_star
    assert abs(k_exact - round(k_exact)) > 1e-3      # no threshold tie
    net = oracle.OracleNet(spec)
    r = net.step(n_star + 5 * period + 3)["raster"][:, 0]
    spikes = np.nonzero(r)[0].tolist()
    assert spikes == [n_star + m * period for m in range(len(spikes))]
    assert len(spikes) == 6
    assert period == spec.n_ref + 1 + n_star


@pytest.mark.parametrize("i0", [1.5, 2.0, 3.0])
def test_lif_period_continuous_limit(i0):
    spec = fx.single_vertex(i0)
    net = oracle.OracleNet(spec)
    r = net.step(4000)["raster"][:, 0]
    s = np.nonzero(r)[0]
    P = int(s[2] - s[1])
    t_cont = spec.tau_ms * math.log(i0 / (i0 - spec.v_th)) + spec.n_ref * spec.dt_ms
    assert abs(P * spec.dt_ms - t_cont) <= 2 * spec.dt_ms


def test_refractory_hold_discards_input():
    """Input arriving during the hold is lost; after it, input counts again."""
    # 0 fires at step 0 and again never; 1 -> 0 delivers +0.5 at steps 10 and 30
    pos = np.zeros((3, 2))
    spec = synth.NetSpec(name="hold", pos_um=pos, src=np.array([1, 2], np.int32), dst=np.array([0, 0], np.int32),
                         weight=synth.round_fp16(np.array([0.5, 0.5])), delay_steps=np.array([10, 30], np.uint8),
                         v0=np.array([1.0, 1.0, 1.0], np.float32), seed=9)
    out = oracle.OracleNet(spec).step(40, v=True, inp=True)
    assert out["input"][10, 0] == 0.5 and out["input"][30, 0] == 0.5
    assert out["v"][11, 0] == 0.0          # discarded (step 10 is inside 1..20)
    assert out["v"][31, 0] == 0.5          # accepted (step 30 > 20 from rest)


# --------------------------------------------------------------------------
# Signalling: two-vertex chain, threshold tie, the paper's Figure 1/2 fixture.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dist,dims", [(150.0, 2), (73.2, 2), (10.0, 3), (1234.5, 3)])
def test_two_vertex_chain_arrival_step(dist, dims):
    d = math.ceil(dist / (synth.V_UM_PER_MS * synth.DT_MS))
    spec = fx.two_vertex_chain(dist, 1.0, dims)
    out = oracle.OracleNet(spec).step(d + 5, inp=True)
    inp = out["input"][:, 1]
    assert np.nonzero(inp)[0].tolist() == [d]
    assert inp[d] == 1.0
    # w = 1.0 from rest lands exactly on the threshold: spd uses >=, so it fires
    assert np.nonzero(out["raster"][:, 1])[0].tolist() == [d + 1]


def test_two_vertex_chain_subthreshold():
    spec = fx.two_vertex_chain(150.0, 0.75)
    out = oracle.OracleNet(spec).step(60, v=True)
    assert out["raster"][:, 1].sum() == 0
    assert out["v"][16, 1] == pytest.approx(0.75)


@pytest.mark.parametrize("scenario", ["A", "B"])
def test_fig2_golden(scenario):
    spec = fx.fig2_spec(scenario)
    net = oracle.OracleNet(spec)
    T = spec.meta["steps"]
    out = net.step(T, inp=True)
    assert fx.raster_events(out["raster"]) == sorted(spec.meta["spikes"])
    nz = [(int(j), int(t), float(out["input"][t, j])) for t, j in zip(*np.nonzero(out["input"]))]
    assert sorted(nz) == sorted(spec.meta["inputs"])
    # delays as given (Figure 2, ms * 10)
    assert net.edge_delay(0, 2) == 74 and net.edge_delay(4, 1) == 44


# --------------------------------------------------------------------------
# Brute force: definition-form delayed sum over a full history (N <= 8).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(12))
def test_dense_bruteforce_matches_oracle(seed):
    n = 2 + seed % 7
    spec = fx.random_tiny(n, 0.5, seed, sigma=0.05 if seed % 3 == 0 else 0.0)
    T = 1500
    ref = dense.simulate(
        n, list(zip(spec.src.tolist(), spec.dst.tolist(), spec.weight.tolist(), spec.delay_steps.tolist())), T,
        drive_thr=[oracle.drive_threshold(float(x), spec.dt_ms) for x in spec.drive_rate_hz],
        drive_amp=spec.drive_amp, sigma=spec.noise_sigma, seed=spec.seed, v0=spec.v0.tolist())
    out = oracle.OracleNet(spec).step(T, v=True, inp=True)
    assert out["raster"].tolist() == ref["raster"]
    assert out["input"].tolist() == ref["input"]
    assert out["v"].tolist() == ref["v"]
    assert out["raster"].sum() > 5      # the case is not trivially silent


# --------------------------------------------------------------------------
# Conservation: every spike is delivered exactly out-degree times.
# --------------------------------------------------------------------------
def test_delivery_conservation():
    spec = synth.config0_like(256, 77, w0=0.36)
    spec.noise_sigma = 0.05
    T = 3000
    net = oracle.OracleNet(spec)
    out = net.step(T, inp=True)
    r = out["raster"]
    outdeg = np.bincount(spec.src, minlength=spec.n)
    spikes = r.sum(0)
    assert net.delivered == int((spikes * outdeg).sum())
    # push formulation in numpy: each edge adds w at (t_spike + d) if inside the run
    d = np.array([oracle.delay_steps(spec.pos_um[a], spec.pos_um[b], spec.v_um_per_ms, spec.dt_ms)
                  for a, b in zip(spec.src, spec.dst)])
    expect = np.zeros((T, spec.n))
    for e in range(spec.n_edges):
        ts = np.nonzero(r[:, spec.src[e]])[0] + d[e]
        ts = ts[ts < T]
        np.add.at(expect[:, spec.dst[e]], ts, float(spec.weight[e]))
    assert np.array_equal(expect, out["input"])
    assert r.sum() > 50


# --------------------------------------------------------------------------
# Observation (Section 3.3): calcium closed form, camera frames, noise.
# --------------------------------------------------------------------------
def test_calcium_single_spike_closed_form_and_frames():
    spec = fx.two_vertex_chain(150.0, 0.0)     # vertex 0 fires once at step 0
    net = oracle.OracleNet(spec, frames_cap=8)
    T = 1000
    net.step(T)
    dt, tc = spec.dt_ms, spec.tau_c_ms
    r = 1.0 - dt / tc
    # c(0) = 0, c(t) = dt * r^(t-1) for t >= 1
    assert net.calcium()[0] == pytest.approx(dt * r ** (T - 1), rel=1e-12)
    fr = net.frames()
    # frame(t) = floor(3t/1000): frames of 334, 333, 333 steps in [0, 1000)
    assert fr.shape[0] == 3
    c = lambda t: 0.0 if t == 0 else dt * r ** (t - 1)
    bounds = [(0, 334), (334, 667), (667, 1000)]
    for f, (a, b) in enumerate(bounds):
        expect = sum(c(t) for t in range(a, b)) / (b - a)
        assert fr[f, 0] == pytest.approx(expect, rel=1e-12)
    assert np.all(fr[:, 1] == 0.0)


def test_fluorescence_noise_moments():
    cbar = np.zeros((300, 400))
    F = oracle.fluorescence(cbar, 1.0, 2.0, 0.25, seed=42)
    assert abs(F.mean() - 2.0) < 5 * 0.25 / math.sqrt(F.size)
    assert abs(F.std() - 0.25) < 0.01
    cb2 = np.full((10, 20), 3.0)
    F2 = oracle.fluorescence(cb2, 2.0, 0.0, 0.0, seed=42)
    assert np.all(F2 == 6.0)


# --------------------------------------------------------------------------
# Control: Poisson drive events follow Binomial(steps, p).
# --------------------------------------------------------------------------
def test_drive_event_statistics():
    spec = synth.config0()
    T = 10000
    spec.weight = np.zeros_like(spec.weight)      # isolate the drive
    r = oracle.OracleNet(spec).step(T)["raster"]
    driven = spec.meta["driven"]
    assert r[:, ~driven].sum() == 0
    k = r[:, driven].sum()
    p = 2147483 / 2**32
    # a drive event fires a resting vertex; events inside the 21-step hold are lost
    mean = driven.sum() * T * p
    assert abs(k - mean) < 4.5 * math.sqrt(mean)


def test_oracle_deterministic():
    spec = fx.random_tiny(8, 0.4, 3, sigma=0.05)
    a = oracle.OracleNet(spec).step(500, v=True)
    b = oracle.OracleNet(spec).step(500, v=True)
    assert np.array_equal(a["v"], b["v"]) and np.array_equal(a["raster"], b["raster"])


def test_split_run_equals_single_run():
    spec = fx.random_tiny(6, 0.5, 4, sigma=0.05)
    a = oracle.OracleNet(spec)
    whole = a.step(600, v=True)
    b = oracle.OracleNet(spec)
    p1 = b.step(250, v=True)
    p2 = b.step(350, v=True)
    assert np.array_equal(whole["v"], np.concatenate([p1["v"], p2["v"]]))


def test_oracle_threads_bit_identical():
    """The oracle's per-vertex loops split over threads give the same bits as
    the serial run (the spike push stays serial, in vertex order)."""
    spec = synth.config1(n=8192)
    spec.drive_rate_hz = np.full(spec.n, 50.0, np.float32)
    out = []
    try:
        for th in (1, 4):
            oracle.set_threads(th)
            o = oracle.OracleNet(spec, frames_cap=4)
            r = o.step(400, raster=True, v=True, inp=True)
            r["c"] = o.calcium()
            r["frames"] = o.frames()
            out.append(r)
    finally:
        oracle.set_threads(1)
    assert out[0]["raster"].sum() > 100
    for k in out[0]:
        assert np.array_equal(out[0][k], out[1][k]), k
