"""Benchmark: HBM-bound step throughput of the geometric-network simulator.

Workload (one GPU): N = 1,048,576 LIF vertices in a 2.52 mm cube, about 100
in-edges per vertex by p = 0.0715*exp(-r/100 um) cut at 2 mm (~103M edges:
int32 source, FP16 weight, uint8 delay), 20 % inhibitory sources, Gaussian
state noise sigma = 0.05, dt = 0.1 ms.  One "step" is the whole hot path:
delayed-spike delivery over every edge, then the vertex update (drive,
noise, Euler LIF, refractory hold, spike test, history ring).  Inputs are
resident in HBM before timing starts.

By default a step is one fused kernel (each workgroup delivers into and
then updates its own range of vertices); --deliver-flags selects the
two-kernel variants.  Prints one JSON line: edge-steps/s over the timed
steps, the dominant kernel's roofline (algorithmic bytes / its measured
duration vs 8 TB/s) and the FP64 CPU oracle timed on a bounded sample of the
same workload.  --workload selects the other measured rows (ensemble,
estimate, mlp).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes of one step, per unit of work (the roofline's figure):
# every edge streams its int32 source and uint8 delay (5 B), an edge that
# delivers a spike also reads its FP16 weight (2 B), and every vertex update
# moves about 18 B (V read and written, refractory/age state, the history-ring
# bit and the delivered input).
BYTES_PER_EDGE = 5
BYTES_PER_ARRIVAL = 2
BYTES_PER_VERTEX = 18
# What the stream formats themselves move (reported beside the fraction):
BYTES_PER_EDGE_PACKED = 4   # packed two-kernel delivery: one word per edge, source | delay << 24
BYTES_PER_EDGE_NARROW = 3.5  # fused step: 16 + 4 source bits and the delay byte per edge
BYTES_PER_EDGE_STREAMED_W = 7   # delivery variant that streams every weight with its edge
# fused step's vertex update: V read + written (8), two-spike ages read +
# written (4), history-ring word read + written (8), one summary bit (1/8)
BYTES_PER_VERTEX_UPDATE = 20.125
# Push delivery (NET_BUILD_PUSH), one update kernel per step: per vertex V
# read and written (8), ages read and written (4), the drive threshold (4),
# its input-ring slot read and cleared (8); per arriving spike the out-edge
# record (8) and the atomic add's read and write of the ring word (8); per
# spike the source's two out-edge offsets (8).
PUSH_BYTES_PER_VERTEX = 24
PUSH_BYTES_PER_ARRIVAL = 16
PUSH_BYTES_PER_SPIKE = 8
TIMING_EVERY = 16       # kernel-bound events on one launch in 16 across long timed regions
MIN_TIMED_LAUNCHES = 64  # shorter timed regions bind events to more launches (every launch below 64 steps)


def measured_traffic(deliver_flags):
    """HBM bytes per launch of the dominant kernel from a committed rocprofv3
    counter summary under profiles/, if one was taken on the kernel source as
    it is now and on the same delivery variant (else None)."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_0908_3934_amd", "csrc", "kernels.hip")
    try:
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    for prof in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        try:
            fields = dict(line.split(": ", 1) for line in open(prof).read().splitlines()
                          if line.startswith(("traffic_bytes_per_launch:", "kernels_hip_sha256_16:",
                                              "deliver_flags:")))
            if (fields.get("kernels_hip_sha256_16", "").strip() == sha
                    and int(fields.get("deliver_flags", "-1")) == deliver_flags):
                return int(fields["traffic_bytes_per_launch"])
        except (OSError, KeyError, ValueError):
            continue
    return None


def stream_ceiling(torch, nbytes):
    """Achievable HBM streaming rate on this device, for the roofline's
    context: a read-only pass (FP32 sum) and a device copy over `nbytes`,
    timed with events on torch's stream (median of 5 after 2 warm-ups)."""
    n = int(nbytes) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)

    def timed(fn):
        ms = []
        for k in range(7):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            if k >= 2:
                ms.append(a.elapsed_time(b))
        return sorted(ms)[len(ms) // 2] / 1e3

    t_read = timed(lambda: x.sum())
    t_copy = timed(lambda: y.copy_(x))
    del x, y
    torch.cuda.empty_cache()
    return {"bytes": n * 4, "read_only_GBps": n * 4 / t_read / 1e9, "copy_GBps": 2 * n * 4 / t_copy / 1e9,
            "method": "torch FP32 sum (read only) and device copy over the same byte count, median of 5"}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def host_cpu():
    """Model name of the host CPU (lscpu) and the cores the OS shows."""
    model = None
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, ValueError, Exception):
        pass
    if model is None:
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    return {"model": model, "nproc": os.cpu_count()}


def cpu_baseline(spec, steps):
    import oracle
    t0 = time.perf_counter()
    net = oracle.OracleNet(spec)
    t1 = time.perf_counter()
    net.step(steps, raster=False)
    t2 = time.perf_counter()
    net.close()
    return {
        "value": spec.n_edges * steps / (t2 - t1),
        "unit": "edge-steps/s",
        "cores": 1,
        "kind": "oracle",
        "host_cpu": host_cpu(),
        "sample": "same network, first %d of the steps (single-threaded FP64 event-driven oracle; "
                  "%.1f s run after %.1f s set-up; its per-step cost is the vertex update of all N "
                  "vertices, so the start-up's lower spike rate barely changes it)" % (steps, t2 - t1, t1 - t0),
    }


def push_variant(args, torch, gn, spec, arrivals, spikes, fused_ms):
    """The same network, pre-roll, warm-up and timed steps with push delivery
    (each spiking wave adds its out-edges into an input ring; bit-equal to the
    fused step): whole-step rate and the update kernel against the bytes it
    must move."""
    t0 = time.perf_counter()
    net = gn.Net(spec, flags=gn.NET_BUILD_PUSH)
    info = net.info()
    if not info["deliver_flags"] & gn.NET_BUILD_PUSH:
        net.close()
        return None
    build_s = time.perf_counter() - t0
    net.step(args.preroll + args.warmup)
    torch.cuda.synchronize()
    every = TIMING_EVERY if args.steps >= MIN_TIMED_LAUNCHES * TIMING_EVERY \
        else max(1, args.steps // MIN_TIMED_LAUNCHES)
    net.timing_begin(2 * args.steps // every + 4, every=every)
    t0 = time.perf_counter()
    net.step(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = net.timing_end()
    net.close()
    avg = tm["update_ms"] / tm["update_launches"] / 1e3
    alg = PUSH_BYTES_PER_VERTEX * spec.n + PUSH_BYTES_PER_ARRIVAL * arrivals + PUSH_BYTES_PER_SPIKE * spikes
    log("push delivery: %.2f us per step (update kernel %.2f us, %d timed), built in %.1f s"
        % (wall / args.steps * 1e6, avg * 1e6, tm["update_launches"], build_s))
    return {
        "flags": "NET_BUILD_PUSH",
        "value": spec.n_edges * args.steps / wall,
        "unit": "edge-steps/s",
        "ms_per_step": wall / args.steps * 1e3,
        "speedup_vs_value": fused_ms / (wall / args.steps * 1e3),
        "real_time_factor": args.steps * spec.dt_ms * 1e-3 / wall,
        "kernel": "node_update_kernel (vertex update + push of its spikes)",
        "avg_launch_us": avg * 1e6,
        "timed_launches": tm["update_launches"],
        "algorithmic_bytes_per_launch": alg,
        "bytes_rule": "%d B per vertex + %d B per arriving spike + %d B per spike"
                      % (PUSH_BYTES_PER_VERTEX, PUSH_BYTES_PER_ARRIVAL, PUSH_BYTES_PER_SPIKE),
        "achieved_GBps": alg / avg / 1e9,
        "frac": alg / avg / 1e9 / HBM_PEAK_GBS,
        "note": "same spikes, V and inputs bit for bit as the fused step; the fused step stays the headline "
                "(the pull over every in-edge with the history ring)",
    }


def spikes_per_vertex(net, spec, steps):
    """Spike counts of every vertex over the next `steps` steps (recorded)."""
    import torch
    words = net.step(steps, raster=True)["raster"]
    torch.cuda.synchronize()
    counts = torch.zeros(words.shape[1], 64, dtype=torch.int64, device=words.device)
    for b in range(64):
        counts[:, b] = ((words >> b) & 1).sum(0)
    return counts.reshape(-1)[:spec.n].cpu().numpy()


def arrivals_per_step(net, spec, steps):
    """Mean number of edges that deliver a spike per step over the next
    `steps` steps, which are recorded: sum over sources of spikes x
    out-degree, divided by the steps."""
    import numpy as np
    per_vertex = spikes_per_vertex(net, spec, steps)
    outdeg = np.bincount(np.asarray(spec.src), minlength=spec.n)
    return float((per_vertex * outdeg).sum()) / steps


def bench_ensemble(args, torch, synth, gn):
    """512 networks of 64..4096 vertices (log-uniform), 10,000 steps: the
    whole ensemble in one autotuned launch against every network on its own
    handle with its best single-network setting (the same LDS-resident kernel,
    one launch per network, autotuned).  value = networks per second for
    10,000-step runs."""
    specs = synth.config3()
    steps = args.steps
    E = sum(s.n_edges for s in specs)
    N = sum(s.n for s in specs)
    t0 = time.perf_counter()
    net = gn.Net(specs, flags=gn.NET_BUILD_AUTOTUNE)
    info = net.info()
    log("ensemble built in %.1f s: %d nets, N=%d, E=%d, %d blocks x %d threads (autotuned %d)"
        % (time.perf_counter() - t0, len(specs), N, E, info["ensemble_blocks"], info["ensemble_threads"],
           info["autotuned"]))
    net.step(args.warmup)
    torch.cuda.synchronize()
    net.timing_begin(8)
    t0 = time.perf_counter()
    net.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = net.timing_end()
    net.close()
    log("ensemble: %d steps in %.3f s (kernel %.3f ms)" % (steps, wall, tm["ensemble_ms"]))
    # sequential: every k-th network alone with its best setting (the
    # single-launch LDS-resident kernel, autotuned; the two per-step kernels
    # over the whole GPU; the fused per-step kernel), scaled to all
    sample = specs[::args.seq_sample]
    seq = 0.0
    variants = [("single-launch", gn.NET_BUILD_SINGLE_LAUNCH | gn.NET_BUILD_AUTOTUNE), ("per-step", 0),
                ("fused step", gn.NET_BUILD_FUSED_STEP)]
    wins = {name: 0 for name, _ in variants}
    largest = max(specs, key=lambda s: s.n_edges)
    largest_alone = {}
    for s in sample + [largest]:
        best = None
        for name, flags in variants:
            one = gn.Net(s, flags=flags)
            one.step(args.warmup)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            one.step(steps)
            torch.cuda.synchronize()
            tv = time.perf_counter() - t1
            one.close()
            if s is largest:
                largest_alone[name] = tv
            if best is None or tv < best[0]:
                best = (tv, name)
        if s is not largest or largest in sample:
            seq += best[0]
            wins[best[1]] += 1
    seq_all = seq * len(specs) / len(sample)
    log("sequential: %d of %d networks alone in %.3f s -> %.3f s for all (best setting counts %s); largest network "
        "(N=%d, E=%d) alone: %s" % (len(sample), len(specs), seq, seq_all, wins, largest.n, largest.n_edges,
                                    {k: "%.3f s" % v for k, v in largest_alone.items()}))
    value = len(specs) / wall * (steps / 10000.0)
    return {
        "metric": "nets/s",
        "value": value,
        "unit": "networks per second (10,000-step runs)",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": wall / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "ensemble of %d LIF networks, 64..4096 vertices each (log-uniform), 1 mm square, "
                        "p = 0.3 within 150 um, %d vertices and %d edges in total, noise-free, 10 %% driven"
                        % (len(specs), N, E),
            "launch": "%d workgroups x %d threads, one launch per call" % (info["ensemble_blocks"],
                                                                          info["ensemble_threads"]),
        },
        "sequential": {
            "value": len(specs) / seq_all * (steps / 10000.0),
            "unit": "networks per second (10,000-step runs)",
            "method": "each network on its own handle with the fastest of three settings (single-launch "
                      "LDS-resident kernel autotuned, the two per-step kernels, the fused per-step kernel); "
                      "%d of %d networks timed and scaled" % (len(sample), len(specs)),
            "best_setting_counts": wins,
        },
        "largest_network_alone_s": largest_alone,
        "largest_network": {"n_vertices": largest.n, "n_edges": largest.n_edges},
        "speedup_vs_sequential": seq_all / wall,
        "edge_steps_per_s": E * steps / wall,
        # The kernel pushes each spike along its out-edges from an LDS spike
        # log (the in-edge stream is only the fallback of a step whose log
        # overflowed), so it moves far fewer bytes than the edge-steps it
        # covers: its bound is each workgroup's per-step latency (update,
        # two barriers, the dependent loads of a push).  Its ceiling is the
        # largest network alone on one workgroup with the same kernel.
        "roofline": {
            "bound": "latency", "kernel": "ensemble_kernel",
            "achieved": wall, "peak": largest_alone["single-launch"],
            "unit": "s per call of all steps (peak: the largest network alone, same kernel)",
            "frac": largest_alone["single-launch"] / wall,
            "traffic": None,
            "pull_equivalent_GBps": BYTES_PER_EDGE * E * steps / (tm["ensemble_ms"] / 1e3) / 1e9,
            "note": "frac = the largest network's own time over the whole ensemble's; pull_equivalent_GBps = "
                    "5 B per edge-step over the kernel time, what a pull over every in-edge would have to stream",
        },
        "cpu_baseline": None if args.no_cpu_baseline else ensemble_cpu_baseline(specs, len(specs)),
    }


def ensemble_cpu_baseline(specs, n_all, every=16, steps=2000):
    """The FP64 oracle on every 16th network for 2,000 steps, scaled to
    networks per second of 10,000-step runs."""
    import oracle
    sample = specs[::every]
    t = 0.0
    for s in sample:
        net = oracle.OracleNet(s)
        t0 = time.perf_counter()
        net.step(steps, raster=False)
        t += time.perf_counter() - t0
        net.close()
    per_net = t / len(sample) * (10000 / steps)
    return {"value": 1.0 / per_net, "unit": "networks per second (10,000-step runs)", "cores": 1, "kind": "oracle",
            "host_cpu": host_cpu(), "sample": "every %dth of the %d networks (%d), %d steps each, single-threaded FP64; %.1f s"
                      % (every, n_all, len(sample), steps, t)}


MFMA_BF16_PEAK_TFLOPS = 2500.0


def bench_mlp(args, torch, gn):
    """The edge scorer (64 -> 256 -> 256 -> 1, BF16 MFMA): training steps
    (forward, BCE backward, Adam) on batches of --mlp-rows pairs (default
    65,536), and the forward pass on 65,536 pairs (about one N = 1024
    network's candidates); the training step is also timed at 16,384 and
    262,144 rows.  FLOPs counted: 2 x (64*256 + 256*256 + 256) per pair
    forward, 3x that per training pair.  Timed with events on the stream of
    the calls, whole steps (all kernels)."""
    import numpy as np
    m = gn.Mlp(gn.Mlp.init_params(0))
    m.set_input_norm(np.zeros(64, np.float32), np.ones(64, np.float32))
    fw = 2 * (64 * 256 + 256 * 256 + 256)
    g = torch.Generator(device="cuda").manual_seed(0)
    Bt, Bf = args.mlp_rows, 65536
    rows_max = max(Bt, Bf, 262144)
    X = torch.randn(rows_max, 64, device="cuda", generator=g)
    y = (torch.rand(rows_max, device="cuda", generator=g) < 0.3).float()
    loss = torch.zeros(1, device="cuda")
    steps = args.steps

    def train_time(rows, n):
        Xt, yt = X[:rows].contiguous(), y[:rows].contiguous()
        for _ in range(args.warmup):
            m.train_step(Xt, yt, 1e-3, loss=loss)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            m.train_step(Xt, yt, 1e-3, loss=loss)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n

    train_s = train_time(Bt, steps)
    sweep = {}
    for rows in (16384, 65536, 262144):
        t = train_s if rows == Bt else train_time(rows, max(20, steps // 4))
        sweep[str(rows)] = {"ms_per_step": t * 1e3, "tflops": 3 * fw * rows / t / 1e12}
        log("training step on %d rows: %.3f ms (%.1f TFLOP/s)" % (rows, t * 1e3, sweep[str(rows)]["tflops"]))
    Xf = X[:Bf].contiguous()
    for _ in range(args.warmup):
        m.forward(Xf)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        m.forward(Xf)
    torch.cuda.synchronize()
    fwd_s = (time.perf_counter() - t0) / steps
    train_tflops = 3 * fw * Bt / train_s / 1e12
    return {
        "metric": "training pairs/s",
        "value": Bt / train_s,
        "unit": "pairs per second (one optimizer step per %d pairs)" % Bt,
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": train_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 (fp32 accumulation, fp32 Adam)",
        "data": "synthetic",
        "config": {"workload": "edge-scorer MLP 64 -> 256 -> 256 -> 1, batch %d (training), 65,536 (forward)" % Bt},
        "train_sweep": sweep,
        "forward_pairs_per_s": Bf / fwd_s,
        "forward_us": fwd_s * 1e6,
        "roofline": {"bound": "mfma", "achieved": train_tflops, "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": train_tflops / MFMA_BF16_PEAK_TFLOPS, "traffic": None,
                     "forward_achieved": fw * Bf / fwd_s / 1e12},
        "cpu_baseline": mlp_cpu_baseline(X[:16384].cpu().numpy(), y[:16384].cpu().numpy(), m.get_params()),
    }


def mlp_cpu_baseline(X, y, params, rows=16384):
    """The FP64 reference (same BF16 rounding points) for the gradient of one
    16,384-row training batch, in training pairs per second."""
    from threadpoolctl import threadpool_limits
    from oracle import mlp as M
    X, y = X[:rows].astype("float64"), y[:rows].astype("float64")
    with threadpool_limits(limits=1):                  # one core, like every oracle timing
        t0 = time.perf_counter()
        M.grad(params.astype("float64"), X, y, bf=True)
        t = time.perf_counter() - t0
    return {"value": rows / t, "unit": "training pairs per second (forward + gradient)", "cores": 1,
            "kind": "oracle", "host_cpu": host_cpu(), "sample": "one %d-row batch through the FP64 MLP reference (numpy); %.2f s" % (rows, t)}


TESTSET_CURRENT_PA = 60.0     # constant input above the regular-spiking rheobase (51.4 pA): tonic firing
TESTSET_W_PA = 25.0           # alpha-PSC weight scale at the in-degree of the k = 8 lattice


TESTSET_HH_CURRENT = 8.0      # uA/cm^2, above the HH model's onset of repetitive firing (~6.3)
TESTSET_HH_W = 6.0            # alpha-PSC weight scale (uA/cm^2) at the in-degree of the k = 8 lattice


def testset_specs(synth, dims=(2,), model="izhikevich"):
    """The standardized test networks as Izhikevich networks at dt = 1 ms or
    Hodgkin-Huxley networks at dt = 0.03 ms (the paper's two benchmark
    models and steps), with an alpha PSC, driven by a constant current as in
    its Figure 8; weights U[0.5,1.5] * scale, the scale multiplied by
    8 / mean in-degree so that denser classes are not driven harder."""
    from synth import testset as ts
    import numpy as np
    out = []
    for s in ts.test_set(dims_list=dims):
        indeg = max(1.0, s.n_edges / s.n)
        if model == "hh":
            z = synth.hodgkin_huxley(s, psc=2, w_scale=TESTSET_HH_W * min(1.0, 8.0 / indeg))
            z.i_ext = np.full(s.n, TESTSET_HH_CURRENT, np.float32)
            z.noise_sigma = synth.HH_NOISE_SIGMA
        else:
            z = synth.izhikevich(s, psc=2, w_scale=TESTSET_W_PA * min(1.0, 8.0 / indeg))
            z.i_ext = np.full(s.n, TESTSET_CURRENT_PA, np.float32)
            z.noise_sigma = synth.IZ_NOISE_SIGMA
        z.meta = dict(s.meta)
        out.append(z)
    return out


def bench_testset(args, torch, synth, gn):
    """The paper's benchmark (Section 3.4, Figure 4) on this GPU: its test
    networks (lattice, small-world, scale-free, random; low and high density;
    N = 10 .. 1000; here the 40 two-dimensional ones) with the Izhikevich
    vertex and an alpha PSC at dt = 1 ms for 10 s (10,000 steps).  Reported
    as the paper does, the real-time factor = simulated time / wall time:
    every network on its own handle (one launch per call, launch shape
    autotuned), and the 40 together as one ensemble launch.  value = the
    ensemble's real-time factor per network (40 x 10 s simulated / wall)."""
    import numpy as np
    specs = testset_specs(synth, model=args.model)
    hh = args.model == "hh"
    dt_ms = synth.HH_DT_MS if hh else synth.IZ_DT_MS
    # 10 s of Izhikevich time (10,000 steps) or 1 s of HH time (33,334 steps), as in the paper
    steps = args.steps if args.steps_given else (33334 if hh else 10000)
    sim_s = steps * dt_ms * 1e-3
    rows = []
    for s in specs:
        net = gn.Net(s, flags=gn.NET_BUILD_SINGLE_LAUNCH | gn.NET_BUILD_AUTOTUNE)
        net.step(args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = net.step(steps, raster=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        spikes = int(gn.unpack_raster(out["raster"], s.n).sum())
        net.close()
        rows.append({"name": s.name, "n": s.n, "edges": s.n_edges, "class": s.meta["class"],
                     "density": s.meta["density"], "rtf": sim_s / wall, "rate_hz": spikes / s.n / sim_s})
        log("%-28s N=%4d E=%6d  real-time factor %7.1f  (%.1f Hz)" % (s.name, s.n, s.n_edges, sim_s / wall,
                                                                      spikes / s.n / sim_s))
    ens = gn.Net(specs, flags=gn.NET_BUILD_AUTOTUNE)
    info = ens.info()
    ens.step(args.warmup)
    torch.cuda.synchronize()
    ens.timing_begin(8)
    t0 = time.perf_counter()
    ens.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = ens.timing_end()
    ens.close()
    E = sum(s.n_edges for s in specs)
    N = sum(s.n for s in specs)
    rtf = np.array([r["rtf"] for r in rows])
    worst = rows[int(np.argmin(rtf))]
    log("ensemble of %d: %.3f s for %d steps (kernel %.3f ms), %d blocks x %d threads"
        % (len(specs), wall, steps, tm["ensemble_ms"], info["ensemble_blocks"], info["ensemble_threads"]))
    cpu = None if args.no_cpu_baseline else testset_cpu_baseline(specs, steps, sample_steps=3334 if hh else 1000)
    return {
        "metric": "real-time factor",
        "value": len(specs) * sim_s / wall,
        "unit": "simulated seconds per wall second per network (40 test networks in one launch)",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": wall / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (vertex state), f32 (delivered sums)",
        "data": "synthetic",
        "config": {
            "workload": ("the paper's 40 two-dimensional test networks (4 classes x 2 densities x N = 10..1000), "
                         "Hodgkin-Huxley vertex with alpha PSC, dt 0.03 ms, 1 s, constant 8 uA/cm^2 input, "
                         "noise 0.1 mV") if hh else
                        ("the paper's 40 two-dimensional test networks (4 classes x 2 densities x N = 10..1000), "
                         "Izhikevich vertex with alpha PSC, dt 1 ms, 10 s, constant 60 pA input, noise 1 mV"),
            "model": args.model,
            "n_networks": len(specs), "n_vertices": N, "n_edges": E,
            "launch": "%d workgroups x %d threads, one launch per call" % (info["ensemble_blocks"],
                                                                          info["ensemble_threads"]),
        },
        "alone": {
            "method": "each network on its own handle, single-launch kernel, autotuned; real-time factor = "
                      "simulated time / wall",
            "min": float(rtf.min()), "median": float(np.median(rtf)), "max": float(rtf.max()),
            "slowest": worst,
            "by_network": [{k: (round(v, 2) if isinstance(v, float) else v) for k, v in r.items()} for r in rows],
        },
        "edge_steps_per_s": E * steps / wall,
        # The slowest network alone bounds the launch (one workgroup each, per-step
        # latency: FP64 vertex arithmetic, barriers, the push of its spikes).
        "roofline": {
            "bound": "latency", "kernel": "ensemble_kernel",
            "achieved": wall, "peak": sim_s / float(rtf.min()),
            "unit": "s per call of all steps (peak: the slowest network alone, same kernel)",
            "frac": sim_s / float(rtf.min()) / wall,
            "traffic": None,
            "pull_equivalent_GBps": BYTES_PER_EDGE * E * steps / (tm["ensemble_ms"] / 1e3) / 1e9,
            "note": "frac = the slowest network's own time over the whole launch's; the %.1f MB edge list is "
                    "not streamed (spikes are pushed from LDS logs)" % (BYTES_PER_EDGE * E / 1e6),
        },
        "paper_context": ("Section 3.4: on one Tesla C1060 its HH networks (dt 0.03 ms) ran in about real time "
                          "except the largest random ones (10-15x slower than real time); one 2.5 GHz Core2Duo "
                          "core was 15-800x slower than real time") if hh else
                         ("Section 3.4: on one Tesla C1060 its Izhikevich networks (dt 1 ms) ran 10-20x faster "
                          "than real time for most networks and about real time for the largest random ones; "
                          "one 2.5 GHz Core2Duo core ran them from just under real time (10 vertices) to ~15x "
                          "slower (largest random)"),
        "cpu_baseline": cpu,
    }


def bench_graph(args, torch, synth, gn):
    """Launch-bound single networks (N = 256, config 0; N = 8,192 and
    65,536, config-1 density) stepped without records: plain per-step
    launches, the same kernels replayed from a captured 256-step HIP graph
    (NET_BUILD_GRAPH), and the single-launch kernel (NET_BUILD_SINGLE_LAUNCH,
    one launch per call), for the two-kernel and the fused step.  value =
    steps/s of the N = 256 network with graph replays."""
    steps = args.graph_steps
    rows = []
    cases = [("config0 N=256", synth.config0(), [0, gn.NET_BUILD_GRAPH, gn.NET_BUILD_SINGLE_LAUNCH])]
    for n in (8192, 65536):
        cases.append(("config1-density N=%d" % n, synth.config1(n=n),
                      [0, gn.NET_BUILD_GRAPH, gn.NET_BUILD_FUSED_STEP, gn.NET_BUILD_FUSED_STEP | gn.NET_BUILD_GRAPH]))
    for name, spec, variants in cases:
        for flags in variants:
            net = gn.Net(spec, flags=flags)
            net.step(512)                                   # captures the graphs, past the start-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            net.step(steps)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            info = net.info()
            rows.append({"network": name, "n_vertices": spec.n, "n_edges": spec.n_edges, "flags": flags,
                         "deliver_flags": info["deliver_flags"], "us_per_step": wall / steps * 1e6,
                         "steps_per_s": steps / wall})
            log("%s flags %d: %.2f us per step" % (name, flags, wall / steps * 1e6))
            net.close()
    head = [r for r in rows if r["n_vertices"] == 256 and r["flags"] == gn.NET_BUILD_GRAPH][0]
    return {
        "metric": "steps/s",
        "value": head["steps_per_s"],
        "unit": "simulation steps per second (N = 256 network, graph replays)",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 512,
        "ms_per_step": head["us_per_step"] / 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single LIF networks stepped without records, plain launches vs graph replays"},
        "rows": rows,
    }


def bench_stdp(args, torch, synth, gn):
    """Spike-timing-dependent plasticity on a configuration-1-sized network
    (N = 65,536 in a 1 mm cube, ~6.7e6 edges, noise 0.05, dt 0.1 ms): every
    step delivers with the current weights and updates every edge whose spike
    arrives or whose target fires (per-step kernels: one wave per target row,
    then the vertex update).  value = edge-steps/s."""
    import numpy as np
    spec = synth.plastic(synth.config1(n=args.stdp_n))
    E = spec.n_edges
    net = gn.Net(spec)
    net.step(args.preroll)
    torch.cuda.synchronize()
    w0 = net.observe(gn.NET_OBS_WEIGHTS).cpu().numpy()
    net.timing_begin(2 * args.steps + 4, every=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net.step(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = net.timing_end()
    w1 = net.observe(gn.NET_OBS_WEIGHTS).cpu().numpy()
    # edges touched per step: arrivals (spikes x out-degree) and the in-edges
    # of targets that fire (spikes x in-degree)
    spk = spikes_per_vertex(net, spec, args.rate_steps)
    rate = float((spk * np.bincount(np.asarray(spec.src), minlength=spec.n)).sum()) / args.rate_steps
    post = float((spk * np.bincount(np.asarray(spec.dst), minlength=spec.n)).sum()) / args.rate_steps
    net.close()
    deliver_s = tm["deliver_ms"] / tm["deliver_launches"] / 1e3
    touched = rate + post
    alg = 5.0 * E + 8.0 * touched + 18.0 * spec.n
    log("stdp: %d steps in %.3f s; plastic delivery %.1f us, update %.1f us per step; %.0f arrivals per step"
        % (args.steps, wall, deliver_s * 1e6, tm["update_ms"] / tm["update_launches"] * 1e3, rate))
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        o = oracle.OracleNet(spec)
        t1 = time.perf_counter()
        o.step(args.cpu_steps, raster=False)
        dt = time.perf_counter() - t1
        o.close()
        cpu = {"value": E * args.cpu_steps / dt, "unit": "edge-steps/s", "cores": 1, "kind": "oracle",
               "host_cpu": host_cpu(), "sample": "the same plastic network, first %d steps, single-threaded FP64 "
               "oracle (event-driven delivery, updates on arrivals and post spikes); %.1f s" % (args.cpu_steps, dt)}
    return {
        "metric": "edge-steps/s",
        "value": E * args.steps / wall,
        "unit": "edge-steps/s (plastic weights)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.preroll, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (state), int32 x 2^-20 (plastic weights), f64 (plasticity increments)",
        "data": "synthetic",
        "config": {"workload": "LIF network with STDP, N=%d in a 1 mm cube, %d edges, alpha %.4g/ms, beta %.3g/ms, "
                               "noise 0.05, dt 0.1 ms" % (spec.n, E, spec.stdp_alpha, spec.stdp_beta),
                   "n_vertices": spec.n, "n_edges": E},
        "weights_moved_fraction": float(np.mean(w1 != w0)),
        "roofline": {"bound": "hbm", "kernel": "plastic_deliver_kernel",
                     "achieved": alg / deliver_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": alg / deliver_s / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "bytes_rule": "5 B per edge (source, delay) + 8 B per touched edge (its weight read and "
                                   "written: arrivals and the in-edges of firing targets) + 18 B per vertex",
                     "avg_launch_us": deliver_s * 1e6, "arrivals_per_step": rate,
                     "post_touches_per_step": post},
        "cpu_baseline": cpu,
    }


def testset_cpu_baseline(specs, steps, sample_steps=1000):
    """The FP64 oracle, single-threaded, on every test network for
    sample_steps steps: the real-time factor of each, as the paper's CPU
    panels report it."""
    import numpy as np
    import oracle
    rtf = []
    t_all = 0.0
    for s in specs:
        net = oracle.OracleNet(s)
        t0 = time.perf_counter()
        net.step(sample_steps, raster=False)
        dt = time.perf_counter() - t0
        net.close()
        t_all += dt
        rtf.append(sample_steps * s.dt_ms * 1e-3 / dt)
    rtf = np.array(rtf)
    return {"value": float(np.median(rtf)), "unit": "real-time factor (median over the 40 networks)",
            "cores": 1, "kind": "oracle", "host_cpu": host_cpu(), "min": float(rtf.min()), "max": float(rtf.max()),
            "sample": "every network for %d steps (%.2f s simulated), single-threaded FP64 oracle; %.1f s in all"
                      % (sample_steps, sample_steps * specs[0].dt_ms * 1e-3, t_all)}


def bench_estimate(args, torch, synth):
    """Functional-topology estimation on N = 1024 networks observed for
    obs-steps at 30 Hz with SNR 5: the learned scorer (64 pair features ->
    MLP, trained on the GPU on train-nets simulated networks) against the
    simulation-based fit, both scoring every candidate pair (< 150 um) of the
    same held-out networks.  value = the scorer's AUC; the fit's AUC and both
    wall times (features + MLP vs fit, per network, after observation) are
    reported beside it."""
    import numpy as np
    from paper_0908_3934_amd import estimate as est
    t0 = time.perf_counter()
    w0 = args.w0
    feats, labels = [], []
    n_train = 0
    batch = 256                                       # one ensemble launch fills the 256 CUs
    gsel = torch.Generator(device="cpu").manual_seed(12345)
    for b in range(0, args.train_nets, batch):
        obs = est.observe([synth.config4_net(m, w0=w0, inhibitory=args.inhibitory, g_inh=args.g_inh) for m in range(b, min(args.train_nets, b + batch))],
                          args.obs_steps)
        for o in obs:
            f = est.features(o)
            lab = o.labels
            if args.pairs_per_net and f.shape[0] > args.pairs_per_net:
                # a uniform sample of the network's candidate pairs (training data only)
                idx = torch.randperm(f.shape[0], generator=gsel)[:args.pairs_per_net]
                f = f[idx.to(f.device)].contiguous()
                lab = lab[idx.numpy()]
            feats.append(f)
            labels.append(lab)
        n_train += len(obs)
        del obs
        log("training data: %d networks simulated and featurised (%.1f s)" % (n_train, time.perf_counter() - t0))
    sim_train_s = time.perf_counter() - t0
    n_pairs = sum(len(l) for l in labels)
    t1 = time.perf_counter()
    sc = est.EdgeScorer(seed=0).fit([], epochs=args.epochs, batch=16384, lr=1e-3, feats=feats, labels=labels)
    torch.cuda.synchronize()
    fit_s = time.perf_counter() - t1
    log("scorer trained on %d pairs in %.2f s (loss history %s)" % (n_pairs, fit_s, ["%.3f" % h for h in sc.history]))
    del feats
    test = est.observe([synth.config4_net(90000 + m, w0=w0, inhibitory=args.inhibitory, g_inh=args.g_inh) for m in range(args.test_nets)], args.obs_steps)
    S, F, C, Y = [], [], [], []
    t_sc = t_sf = 0.0
    for k, o in enumerate(test):
        torch.cuda.synchronize()
        a = time.perf_counter()
        s_sc = est.scorer_scores(o, sc)
        torch.cuda.synchronize()
        b = time.perf_counter()
        # the fit assumes w0 out of every source, -g_inh * w0 out of the
        # inhibitory ones (cell types known) when the networks have them
        ws = est.source_weights(o.spec, w0, args.g_inh) if args.inhibitory > 0 else None
        s_sf = est.simfit(o, w_assumed=w0, w_source=ws, realisations=args.fit_realisations, sweeps=args.fit_sweeps)
        torch.cuda.synchronize()
        c = time.perf_counter()
        t_sc += b - a
        t_sf += c - b
        f = est.features(o).cpu().numpy()
        S.append(s_sc.cpu().numpy())
        F.append(s_sf.cpu().numpy())
        C.append(f[:, 8] + f[:, 9])                    # lag-0 + lag-1 activity correlation
        Y.append(o.labels)
        log("held-out net %d: %d pairs, scorer %.4f s AUC %.4f | fit %.2f s AUC %.4f"
            % (k, len(o.labels), b - a, est.auc(S[-1], o.labels), c - b, est.auc(F[-1], o.labels)))
    cpu = None if args.no_cpu_baseline else estimate_cpu_baseline(test[0], sc)
    S, F, C, Y = map(np.concatenate, (S, F, C, Y))
    auc_sc, auc_sf, auc_c = est.auc(S, Y), est.auc(F, Y), est.auc(C, Y)
    nf = args.obs_steps * 3 // 1000
    return {
        "metric": "AUC",
        "value": auc_sc,
        "unit": "area under the ROC curve over all candidate pairs of the held-out networks",
        "n_gpus": 1,
        "steps": args.obs_steps,
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 (MLP), f32/f64 (simulation and fit)",
        "data": "synthetic",
        "config": {
            "workload": "%d training and %d held-out LIF networks of 1024 vertices (1 mm square, p = 0.3 "
                        "within 150 um, weights U[0.5,1.5] x %.3g%s, 10 %% driven, noise 0.05), %d frames at 30 Hz, "
                        "SNR 5, candidates < 150 um%s" % (
                            args.train_nets, args.test_nets, w0,
                            (", %.0f %% inhibitory sources at -%.3g x" % (100 * args.inhibitory, args.g_inh))
                            if args.inhibitory > 0 else "", nf,
                            (", %d training pairs sampled per network" % args.pairs_per_net) if args.pairs_per_net else ""),
            "w0": w0, "inhibitory_fraction": args.inhibitory, "g_inh": args.g_inh,
            "simulate_and_featurise_training_s": sim_train_s,
            "train_pairs": n_pairs,
            "test_pairs": int(Y.size),
            "positive_fraction": float(Y.mean()),
        },
        "scorer": {"auc": auc_sc, "wall_s": t_sc, "train_s": fit_s, "epochs": args.epochs},
        "simfit": {"auc": auc_sf, "wall_s": t_sf, "realisations": args.fit_realisations, "sweeps": args.fit_sweeps},
        "correlation_baseline_auc": auc_c,
        "auc_gap": auc_sf - auc_sc,
        "wall_ratio_simfit_over_scorer": t_sf / max(t_sc, 1e-12),
        "scorer_pairs_per_s": float(Y.size) / max(t_sc, 1e-12),
        "cpu_baseline": cpu,
    }


def estimate_cpu_baseline(o, sc, pairs=32768):
    """The scorer's pipeline as the FP64 oracle computes it (pair features,
    then the MLP with the same BF16 rounding points and input
    standardisation), single-threaded, on the first `pairs` candidate pairs
    of one held-out network: pairs scored per second."""
    import numpy as np
    import oracle
    from oracle import features as FE
    from oracle import mlp as M
    from threadpoolctl import threadpool_limits
    spec = o.spec
    F = o.F.cpu().numpy().astype(np.float64)
    P = o.pairs.cpu().numpy()[:pairs]
    D = o.dist.cpu().numpy().astype(np.float64)[:pairs]
    thr = [oracle.drive_threshold(float(r), spec.dt_ms) for r in spec.drive_rate_hz] \
        if spec.drive_rate_hz is not None else [0] * spec.n
    p = sc.mlp.get_params().astype(np.float64)
    shift, scale = (a.astype(np.float64) for a in sc.input_norm)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        X = FE.features(F, P, D, dt_ms=spec.dt_ms, tau_c_ms=spec.tau_c_ms, num=spec.frame_num, den=spec.frame_den,
                        offset=o.offset, thr=thr, seed=spec.seed)
        M.forward(p, X, bf=True, shift=shift, scale=scale)
        wall = time.perf_counter() - t0
    return {"value": len(P) / wall, "unit": "candidate pairs scored per second (features + MLP)", "cores": 1,
            "kind": "oracle", "host_cpu": host_cpu(), "sample": "the first %d candidate pairs of one held-out network (FP64 oracle features "
            "and MLP, single-threaded); %.1f s" % (len(P), wall)}


def main():
    import numpy as np
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--cpu-steps", type=int, default=300)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-push-variant", action="store_true",
                    help="step workload: skip timing the same network with push delivery")
    ap.add_argument("--deliver-flags", type=int, default=1024,
                    help="NET_BUILD_* bits of the step variant (default 1024: one fused kernel per step, "
                         "the fastest measured; 16: delivery and update kernels, two chunks per wave "
                         "iteration; 2 streams every weight, 7 B per edge)")
    ap.add_argument("--autotune", action="store_true",
                    help="let the library time the delivery variants at build instead of --deliver-flags")
    ap.add_argument("--workload", choices=["step", "ensemble", "estimate", "mlp", "testset", "stdp", "graph"],
                    default="step",
                    help="step: the N = 2^20 network (default); ensemble: 512 uneven networks in one launch "
                         "against each network run alone; estimate: learned edge scorer against the "
                         "simulation-based fit on held-out N = 1024 networks; mlp: the edge scorer's training "
                         "step and forward pass; testset: the paper's test networks with the Izhikevich or "
                         "Hodgkin-Huxley vertex (real-time factors, Section 3.4); stdp: a 65,536-vertex network "
                         "with plastic weights")
    ap.add_argument("--train-nets", type=int, default=256, help="estimate workload: training networks")
    ap.add_argument("--test-nets", type=int, default=16, help="estimate workload: held-out networks")
    ap.add_argument("--obs-steps", type=int, default=200000, help="estimate workload: observed steps (20 s)")
    ap.add_argument("--epochs", type=int, default=4, help="estimate workload: scorer training epochs")
    ap.add_argument("--w0", type=float, default=None,
                    help="estimate workload: weight scale of the observed networks (default config 4's 0.065)")
    ap.add_argument("--graph-steps", type=int, default=25600, help="graph workload: timed steps per variant")
    ap.add_argument("--relabel", type=int, default=-1,
                    help="default workload: number the vertices in a random order (this seed) before the build")
    ap.add_argument("--reorder", action="store_true",
                    help="default workload: let net_build renumber the vertices in Morton order (NET_BUILD_REORDER)")
    ap.add_argument("--mlp-rows", type=int, default=65536,
                    help="mlp workload: training batch rows per optimizer step")
    ap.add_argument("--inhibitory", type=float, default=0.0,
                    help="estimate workload: fraction of inhibitory sources in the observed networks")
    ap.add_argument("--g-inh", type=float, default=1.0,
                    help="estimate workload: inhibitory weights are -g_inh times the sampled ones")
    ap.add_argument("--pairs-per-net", type=int, default=0,
                    help="estimate workload: training pairs sampled per network (0 = all of them)")
    ap.add_argument("--fit-realisations", type=int, default=8, help="estimate workload: noise realisations of the fit")
    ap.add_argument("--fit-sweeps", type=int, default=2, help="estimate workload: toggle sweeps of the fit")
    ap.add_argument("--seq-sample", type=int, default=8,
                    help="ensemble workload: time every k-th network alone and scale to all")
    ap.add_argument("--rate-steps", type=int, default=500,
                    help="steps recorded right before the warm-up and right after the timed region to count "
                         "arrivals per step")
    ap.add_argument("--preroll", type=int, default=2000,
                    help="untimed steps run first, whatever --warmup is, so that the timed steps see the "
                         "network's steady spike rate rather than the start from rest")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy three times (reference for HBM counters)")
    ap.add_argument("--stdp-n", type=int, default=65536, help="stdp workload: vertices (1 mm cube at 65,536)")
    ap.add_argument("--model", choices=["izhikevich", "hh"], default="izhikevich",
                    help="testset workload: the vertex model (Izhikevich at dt = 1 ms for 10 s, or "
                         "Hodgkin-Huxley at dt = 0.03 ms for 1 s)")
    args = ap.parse_args()
    args.steps_given = any(a == "--steps" or a.startswith("--steps=") for a in sys.argv[1:])
    if args.gpus != 1:
        print("bench.py measures one GPU only: the simulator is built and measured on a single "
              "MI355X; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_0908_3934_amd as gn
    if args.w0 is None:
        args.w0 = synth.CONFIG4_W0

    torch.cuda.set_device(0)
    if args.workload == "ensemble":
        print(json.dumps(bench_ensemble(args, torch, synth, gn)), flush=True)
        return
    if args.workload == "estimate":
        print(json.dumps(bench_estimate(args, torch, synth)), flush=True)
        return
    if args.workload == "graph":
        print(json.dumps(bench_graph(args, torch, synth, gn)), flush=True)
        return
    if args.workload == "stdp":
        print(json.dumps(bench_stdp(args, torch, synth, gn)), flush=True)
        return
    if args.workload == "testset":
        print(json.dumps(bench_testset(args, torch, synth, gn)), flush=True)
        return
    if args.workload == "mlp":
        print(json.dumps(bench_mlp(args, torch, gn)), flush=True)
        return
    if args.copy_calibration:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    t0 = time.perf_counter()
    spec = synth.config2(n=args.n)
    if args.relabel >= 0:
        # the same network with its vertices numbered in a random order
        spec = synth.relabel(spec, args.relabel)
    log("generated N=%d E=%d in %.1f s" % (spec.n, spec.n_edges, time.perf_counter() - t0))
    t0 = time.perf_counter()
    flags = gn.NET_BUILD_AUTOTUNE if args.autotune else args.deliver_flags
    if args.reorder:
        flags |= gn.NET_BUILD_REORDER
    net = gn.Net(spec, flags=flags)
    info = net.info()
    log("built in %.1f s: %s" % (time.perf_counter() - t0, info))

    # Untimed pre-roll past the start-up transient (V starts at rest and the
    # network needs a few hundred steps to reach its steady spike rate), then
    # a recorded window for the arrival count, the warm-up, the timed steps
    # and a second recorded window right after them.
    net.step(args.preroll)
    torch.cuda.synchronize()
    spk = spikes_per_vertex(net, spec, args.rate_steps)
    arr_before = float((spk * np.bincount(np.asarray(spec.src), minlength=spec.n)).sum()) / args.rate_steps
    spikes = float(spk.sum()) / args.rate_steps
    net.step(args.warmup)
    torch.cuda.synchronize()
    every = TIMING_EVERY if args.steps >= MIN_TIMED_LAUNCHES * TIMING_EVERY \
        else max(1, args.steps // MIN_TIMED_LAUNCHES)
    net.timing_begin(2 * args.steps // every + 4, every=every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net.step(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = net.timing_end()
    log("timed %d steps in %.3f s after %d pre-roll and %d warm-up steps; kernels: deliver %.3f ms, "
        "update %.3f ms, fused step %.3f ms" % (args.steps, wall, args.preroll, args.warmup, tm["deliver_ms"],
                                                tm["update_ms"], tm["step_ms"]))

    E = spec.n_edges
    value = E * args.steps / wall
    fused = tm["step_launches"] > 0
    pushed = bool(info["deliver_flags"] & gn.NET_BUILD_PUSH)
    kernel = "step_kernel" if fused else ("node_update_kernel" if pushed else "deliver_kernel")
    if fused:
        avg_deliver_s = tm["step_ms"] / tm["step_launches"] / 1e3
        timed_launches = tm["step_launches"]
    elif pushed:
        avg_deliver_s = tm["update_ms"] / tm["update_launches"] / 1e3
        timed_launches = tm["update_launches"]
    else:
        avg_deliver_s = tm["deliver_ms"] / tm["deliver_launches"] / 1e3
        timed_launches = tm["deliver_launches"]
    arr_after = arrivals_per_step(net, spec, args.rate_steps)
    arrivals = 0.5 * (arr_before + arr_after)
    streamed_w = bool(info["deliver_flags"] & gn.NET_BUILD_DELIVER_STREAM_WEIGHTS)
    packed = fused or bool(info["deliver_flags"] & gn.NET_BUILD_DELIVER_PACKED)
    # the roofline's algorithmic bytes (same for every variant: what the step must move)
    alg_bytes = BYTES_PER_EDGE * E + BYTES_PER_ARRIVAL * arrivals
    if fused:
        alg_bytes += BYTES_PER_VERTEX * spec.n
    # what this variant's stream format moves
    if streamed_w:
        fmt_bytes = BYTES_PER_EDGE_STREAMED_W * E
    else:
        per_edge = BYTES_PER_EDGE_NARROW if fused else (BYTES_PER_EDGE_PACKED if packed else BYTES_PER_EDGE)
        fmt_bytes = per_edge * E + BYTES_PER_ARRIVAL * arrivals
    if fused:
        fmt_bytes += BYTES_PER_VERTEX_UPDATE * spec.n
    if pushed:
        # the push path's own bytes: it reads no in-edge list
        alg_bytes = fmt_bytes = (PUSH_BYTES_PER_VERTEX * spec.n + PUSH_BYTES_PER_ARRIVAL * arrivals
                                 + PUSH_BYTES_PER_SPIKE * spikes)
    achieved = alg_bytes / avg_deliver_s / 1e9
    traffic = measured_traffic(info["deliver_flags"])
    log("arrivals per step %.0f before / %.0f after the timed steps (%.4f %% of edges); algorithmic bytes "
        "per launch %.0f, stream format %.0f; %s: %.2f us per timed launch (%d launches)"
        % (arr_before, arr_after, 100.0 * arrivals / E, alg_bytes, fmt_bytes, kernel, avg_deliver_s * 1e6,
           timed_launches))
    v_now = net.observe(gn.NET_OBS_V)
    torch.cuda.synchronize()
    sim_s = args.steps * spec.dt_ms * 1e-3
    result = {
        "metric": "edge-steps/s",
        "value": value,
        "unit": "edge-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "preroll_steps": args.preroll,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "LIF geometric network, N=%d vertices in a %.0f um cube, %d edges "
                        "(%s, fp16 w), 20%% inhibitory, noise 0.05, dt 0.1 ms"
                        % (spec.n, spec.meta["extent_um"][0], E,
                           "3.5 B per edge: 16 + 4 source bits and the u8 delay" if fused else
                           ("u32 source | u8 delay << 24" if packed else "int32 src, u8 delay")),
            "n_vertices": spec.n,
            "n_edges": E,
            "max_delay_steps": info["max_delay"],
            "deliver_flags": info["deliver_flags"],
            "numbering": ("random (seed %d)" % args.relabel if args.relabel >= 0 else "Morton order of the generator")
                         + (", renumbered in Morton order at build" if args.reorder else ""),
            "real_time_factor": sim_s / wall,
            "launch": "%d blocks x %d threads, summary in %s, variant flags %d%s" % (
                info["deliver_blocks"], info["deliver_threads"], "LDS" if info["lds_summary"] else "global",
                info["deliver_flags"], " (autotuned at build)" if info["autotuned"] else ""),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": kernel,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": alg_bytes,
            "bytes_rule": ("%d B per vertex + %d B per arriving spike + %d B per spike (push delivery)"
                           % (PUSH_BYTES_PER_VERTEX, PUSH_BYTES_PER_ARRIVAL, PUSH_BYTES_PER_SPIKE)) if pushed else
                          ("%d B per edge + %d B per arriving spike + %d B per vertex%s"
                           % (BYTES_PER_EDGE, BYTES_PER_ARRIVAL, BYTES_PER_VERTEX, "" if fused else
                              " (vertex bytes belong to the separate update kernel)")),
            "arrivals_per_step": arrivals,
            "arrivals_per_step_before_after": [arr_before, arr_after],
            "avg_launch_us": avg_deliver_s * 1e6,
            "timed_launches": timed_launches,
            "timing": "kernel-bound HIP events on one launch in %d across the timed region" % every,
            "stream_format_bytes_per_launch": fmt_bytes,
            "frac_stream_format": fmt_bytes / avg_deliver_s / 1e9 / HBM_PEAK_GBS,
            "frac_traffic": (traffic / avg_deliver_s / 1e9 / HBM_PEAK_GBS) if traffic else None,
            "target_frac": 0.60,
            "update_avg_launch_us": (tm["update_ms"] / tm["update_launches"] * 1e3) if tm["update_launches"] else None,
        },
    }
    net.close()
    if not (info["deliver_flags"] & gn.NET_BUILD_PUSH) and not args.no_push_variant:
        result["push_variant"] = push_variant(args, torch, gn, spec, arrivals, spikes, wall / args.steps * 1e3)
    ceil = stream_ceiling(torch, alg_bytes)
    ceil["frac_of_read_only"] = achieved / ceil["read_only_GBps"]
    result["roofline"]["measured_ceiling"] = ceil
    log("streaming ceiling over %.0f MB: read-only %.0f GB/s, copy %.0f GB/s"
        % (ceil["bytes"] / 1e6, ceil["read_only_GBps"], ceil["copy_GBps"]))
    del v_now
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on %d steps" % args.cpu_steps)
        result["cpu_baseline"] = cpu_baseline(spec, args.cpu_steps)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
