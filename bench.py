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
BYTES_PER_EDGE = 7      # int32 source + FP16 weight + uint8 delay, read once per step


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--cpu-steps", type=int, default=150)
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    net = gn.Net(spec)
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
    achieved = BYTES_PER_EDGE * E / avg_deliver_s / 1e9
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
            "traffic": measured_traffic(),
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
