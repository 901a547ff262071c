"""Benchmark: HBM-bound step throughput of the geometric-network simulator.

Workload (one GPU): N = 1,048,576 LIF vertices in a 2.52 mm cube, about 100
in-edges per vertex by p = 0.0715*exp(-r/100 um) cut at 2 mm (~103M edges:
int32 source, FP16 weight, uint8 delay), 20 % inhibitory sources, Gaussian
state noise sigma = 0.05, dt = 0.1 ms.  One "step" is the whole hot path:
delayed-spike delivery over every edge, then the vertex update (drive,
noise, Euler LIF, refractory hold, spike test, history ring).  Inputs are
resident in HBM before timing starts.

Prints one JSON line: edge-steps/s over the timed steps, the delivery
kernel's roofline (algorithmic bytes / measured kernel time vs 8 TB/s) and
the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_EDGE = 5      # int32 source + uint8 delay, streamed every step
BYTES_PER_ARRIVAL = 2   # FP16 weight, loaded only when its edge delivers a spike
BYTES_PER_EDGE_STREAMED_W = 7   # with --stream-weights: the weight is streamed with its edge


def measured_traffic():
    """HBM bytes per delivery launch from the committed rocprofv3 counter
    summary, if it was taken on the kernel source as it is now (else None)."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "deliver_config2.md")
    src = os.path.join(ROOT, "paper_0908_3934_amd", "csrc", "kernels.hip")
    try:
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
        fields = dict(line.split(": ", 1) for line in open(prof).read().splitlines()
                      if line.startswith(("traffic_bytes_per_launch:", "kernels_hip_sha256_16:")))
        if fields.get("kernels_hip_sha256_16", "").strip() != sha:
            return None
        return int(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


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
        "sample": "same network, first %d of the steps (single-threaded FP64 event-driven oracle; "
                  "%.1f s run after %.1f s set-up)" % (steps, t2 - t1, t1 - t0),
    }


def arrivals_per_step(net, spec, steps):
    """Mean number of edges that deliver a spike per step, from a recorded
    stretch right after the timed region: sum over sources of spikes x
    out-degree, divided by the steps."""
    import numpy as np
    import torch
    words = net.step(steps, raster=True)["raster"]
    torch.cuda.synchronize()
    counts = torch.zeros(words.shape[1], 64, dtype=torch.int64, device=words.device)
    for b in range(64):
        counts[:, b] = ((words >> b) & 1).sum(0)
    per_vertex = counts.reshape(-1)[:spec.n].cpu().numpy()
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
    # sequential: every k-th network alone, scaled to all
    sample = specs[::args.seq_sample]
    seq = 0.0
    for s in sample:
        one = gn.Net(s, flags=gn.NET_BUILD_SINGLE_LAUNCH | gn.NET_BUILD_AUTOTUNE)
        one.step(args.warmup)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        one.step(steps)
        torch.cuda.synchronize()
        seq += time.perf_counter() - t1
        one.close()
    seq_all = seq * len(specs) / len(sample)
    log("sequential: %d of %d networks alone in %.3f s -> %.3f s for all" % (len(sample), len(specs), seq, seq_all))
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
            "method": "each network on its own handle, single-launch LDS-resident kernel, autotuned; "
                      "%d of %d networks timed and scaled" % (len(sample), len(specs)),
        },
        "speedup_vs_sequential": seq_all / wall,
        "edge_steps_per_s": E * steps / wall,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--cpu-steps", type=int, default=150)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stream-weights", action="store_true",
                    help="delivery variant that streams every weight (7 B per edge) instead of loading "
                         "weights only for arrivals")
    ap.add_argument("--workload", choices=["step", "ensemble"], default="step",
                    help="step: the N = 2^20 network (default); ensemble: 512 uneven networks in one launch "
                         "against each network run alone")
    ap.add_argument("--seq-sample", type=int, default=8,
                    help="ensemble workload: time every k-th network alone and scale to all")
    ap.add_argument("--rate-steps", type=int, default=500,
                    help="steps recorded after the timed region to count arrivals per step")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy three times (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the simulator is built and measured on a single "
              "MI355X; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_0908_3934_amd as gn

    torch.cuda.set_device(0)
    if args.workload == "ensemble":
        print(json.dumps(bench_ensemble(args, torch, synth, gn)), flush=True)
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
    log("generated N=%d E=%d in %.1f s" % (spec.n, spec.n_edges, time.perf_counter() - t0))
    t0 = time.perf_counter()
    net = gn.Net(spec, flags=gn.NET_BUILD_DELIVER_STREAM_WEIGHTS if args.stream_weights else 0)
    info = net.info()
    log("built in %.1f s: %s" % (time.perf_counter() - t0, info))

    net.step(args.warmup)
    torch.cuda.synchronize()
    net.timing_begin(2 * args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net.step(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = net.timing_end()
    log("timed %d steps in %.3f s; kernels: deliver %.3f ms, update %.3f ms"
        % (args.steps, wall, tm["deliver_ms"], tm["update_ms"]))

    E = spec.n_edges
    value = E * args.steps / wall
    avg_deliver_s = tm["deliver_ms"] / tm["deliver_launches"] / 1e3
    arrivals = arrivals_per_step(net, spec, args.rate_steps)
    if args.stream_weights:
        alg_bytes = BYTES_PER_EDGE_STREAMED_W * E
    else:
        alg_bytes = BYTES_PER_EDGE * E + BYTES_PER_ARRIVAL * arrivals
    achieved = alg_bytes / avg_deliver_s / 1e9
    log("arrivals per step %.0f (%.4f %% of edges); algorithmic bytes per launch %.0f"
        % (arrivals, 100.0 * arrivals / E, alg_bytes))
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
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "LIF geometric network, N=%d vertices in a %.0f um cube, %d edges "
                        "(int32 src, fp16 w, u8 delay), 20%% inhibitory, noise 0.05, dt 0.1 ms"
                        % (spec.n, spec.meta["extent_um"][0], E),
            "n_vertices": spec.n,
            "n_edges": E,
            "max_delay_steps": info["max_delay"],
            "real_time_factor": sim_s / wall,
            "deliver_launch": "%d blocks x %d threads, summary in %s" % (
                info["deliver_blocks"], info["deliver_threads"], "LDS" if info["lds_summary"] else "global"),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "deliver_kernel",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None if args.stream_weights else measured_traffic(),
            "algorithmic_bytes_per_launch": alg_bytes,
            "arrivals_per_step": arrivals,
            "avg_launch_us": avg_deliver_s * 1e6,
            "update_avg_launch_us": tm["update_ms"] / tm["update_launches"] * 1e3,
        },
    }
    net.close()
    del v_now
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on %d steps" % args.cpu_steps)
        result["cpu_baseline"] = cpu_baseline(spec, args.cpu_steps)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
