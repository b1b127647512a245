"""Throughput of the VP-LBM time step on one MI355X.

Workload: the free vortex-induced-vibration run, 2048x1024 channel, disc D = 40 on a
transverse spring (mass ratio 10, reduced velocity 5, Re = 150), FP32 populations.
A step is one full fluid-structure step (pull-stream, penalization, MRT collision,
FP64 force/torque reduction, RK4 body update) over the whole grid, all on the GPU.

Prints one JSON line: MLUPS (million lattice-node updates per second) of the timed
region, the dominant kernel's achieved HBM bandwidth against the 8 TB/s peak, and the
FP64 CPU oracle timed on a bounded sample of the same workload on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_NODE = {"fp64": 144, "fp32": 72, "fp16": 36, "bf16": 36}  # 9 reads + 9 writes


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--storage", default="fp32")
    ap.add_argument("--graph-steps", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one device copy of 256 MiB first (scale for HBM byte counters)")
    ap.add_argument("--traffic", default=None,
                    help="JSON with measured HBM bytes per launch of the step kernel")
    return ap.parse_args()


def cpu_baseline(wl, target_seconds):
    """FP64 CPU oracle on the same grid for a bounded number of steps."""
    from oracle import oracle as orc
    cores = min(len(os.sched_getaffinity(0)), 16)
    orc.set_threads(cores)
    sim = orc.OracleSim(wl["spec"], wl["body"])
    sim.step(2)  # warm-up
    t0 = time.perf_counter()
    sim.step(3)
    per_step = (time.perf_counter() - t0) / 3
    n = max(3, min(400, int(target_seconds / per_step)))
    t0 = time.perf_counter()
    sim.step(n)
    dt = time.perf_counter() - t0
    nodes = wl["spec"]["nx"] * wl["spec"]["ny"]
    return {"value": nodes * n / dt / 1e6, "unit": "MLUPS", "cores": orc.max_threads(),
            "kind": "oracle",
            "sample": "%d steps of the %dx%d grid (FP64, %.1f s)" % (n, wl["spec"]["nx"],
                                                                     wl["spec"]["ny"], dt)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(sharding is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1905_05110_amd import workloads as W
    from paper_1905_05110_amd import vplbm

    wl = W.free_viv(storage=args.storage)
    spec, body = wl["spec"], wl["body"]
    nodes = spec["nx"] * spec["ny"]
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        sim = vplbm.Sim(spec, body, torch_memory=True, history_cap=1 << 17,
                        graph_steps=args.graph_steps)
        print("warmup %d steps" % args.warmup, file=sys.stderr, flush=True)
        sim.step(args.warmup)
        sim.sync()
        torch.cuda.synchronize()
        # timed region: K steps, one kernel launch each, with a HIP event pair around
        # every launch on the simulation's stream
        print("timed %d steps" % args.steps, file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        kernel_ms, region_ms = sim.step_timed(args.steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        sim.sync()
        recs = sim.forces(cap=16)
    ms_per_step = region_ms / args.steps
    mlups = nodes * args.steps / (region_ms * 1e-3) / 1e6
    avg_kernel_s = kernel_ms * 1e-3 / args.steps
    bytes_per_launch = BYTES_PER_NODE[args.storage] * nodes
    achieved = bytes_per_launch / avg_kernel_s / 1e9
    traffic = None
    if args.traffic and os.path.exists(args.traffic):
        traffic = json.load(open(args.traffic)).get("bytes_per_launch")
    out = {
        "metric": "MLUPS (D2Q9 MRT + volume penalization, full FSI step)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "fp32" else args.storage,
        "data": "synthetic (seeded lattice state, no dataset)",
        "config": {"workload": "free_viv_2048x1024", "nx": spec["nx"], "ny": spec["ny"],
                   "storage": args.storage, "body": "disc D=40, free in y, mass ratio 10, U_r 5",
                   "Re": 150, "graph_steps": args.graph_steps},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "k_step<%s>" % args.storage,
                     "avg_kernel_us": round(avg_kernel_s * 1e6, 3),
                     "algorithmic_bytes_per_launch": bytes_per_launch},
        "wall_s": round(wall, 3),
    }
    if not args.no_cpu_baseline:
        print("cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    sim.close()


if __name__ == "__main__":
    main()
