"""Throughput of the VP-LBM time step on one MI355X.

Workload: the free vortex-induced-vibration run, 2048x1024 channel, disc D = 40 on a
transverse spring (mass ratio 10, reduced velocity 5, Re = 150), FP32 populations.
A step is one full fluid-structure step (pull-stream, penalization, MRT collision,
FP64 force/torque reduction, RK4 body update) over the whole grid, all on the GPU.

Prints one JSON line: MLUPS (million lattice-node updates per second) of the timed
region, the step kernel's achieved HBM bandwidth against the 8 TB/s peak, and the FP64
CPU oracle timed on a bounded sample of the same workload on the host cores.  A step is
exactly one kernel launch (replayed from captured HIP graphs), so the kernel's average
duration is the timed region's event-measured time divided by the number of launches.

``--workload batch_sweep`` times the batched path instead: 64 free-VIV runs of uneven
size (ny drawn from U{128..512} with seed 0, nx = 2 ny, D = ny/12, U_r from 2 to 12),
all advanced by one launch per step.  ``--accuracy-steps N`` then also runs the sweep
for N steps in every storage precision and reports, per precision, the relative error
of each run's mean drag coefficient and RMS lift coefficient over the second half of
the run against the FP64 runs.

``--workload adjoint`` times the reverse-mode path: gradient of the time-averaged drag
coefficient of a fixed disc (D = 32, Re = 100, tanh indicator, 1024x512 channel) over
4000 steps with a checkpoint every 100, with respect to the indicator field and the
disc centre.  The value is the adjoint/forward time ratio (backward sweep including
the recomputation, over the forward run including the checkpoint copies).
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
    ap.add_argument("--workload", default="free_viv", choices=("free_viv", "batch_sweep", "adjoint"))
    ap.add_argument("--accuracy-steps", type=int, default=0,
                    help="batch_sweep: also compare storages over this many steps")
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--storage", default="fp32", choices=sorted(BYTES_PER_NODE))
    ap.add_argument("--graph-steps", type=int, default=64,
                    help="steps per captured HIP graph in the timed region (0: eager launches)")
    ap.add_argument("--rows", type=int, default=0, help="rows per tile (0: autotune)")
    ap.add_argument("--store", default="auto", choices=("auto", "plain", "nontemporal"))
    ap.add_argument("--tile-width", type=int, default=0, choices=(0, 256, 512),
                    help="columns per tile (0: autotune)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one device copy of 256 MiB first (scale for HBM byte counters)")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.txt"),
                    help="measured HBM bytes per launch of the step kernel (from rocprofv3)")
    return ap.parse_args()


def split_warmup(warmup, graph_steps):
    """Untimed steps before and after the launch configuration is chosen: the
    autotuner times its candidates from the developed flow, and the steps after it
    capture the graphs of the timed region.  Together they are the requested warm-up."""
    post = min(warmup // 2, max(2 * graph_steps, 128))
    return warmup - post, post


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
    return {"value": round(nodes * n / dt / 1e6, 2), "unit": "MLUPS", "cores": orc.max_threads(),
            "kind": "oracle",
            "sample": "%d steps of the %dx%d grid (FP64 oracle, %.1f s)" % (
                n, wl["spec"]["nx"], wl["spec"]["ny"], dt)}


def kernel_source_hash(storage):
    """Hash of the sources the step kernel of this storage is compiled from."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1905_05110_amd", "csrc")
    for name in ("vplbm_device.hpp", "vplbm_kernels.hpp", "kern_%s.hip" % storage):
        h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(path, storage, nx, ny, rows, nt, tile):
    """Measured HBM bytes per launch from the rocprofv3 counter summary, if one was
    recorded for this configuration and for the kernel sources as they are now."""
    if not path or not os.path.exists(path):
        return None
    want = "%s %d %d %d %d %d" % (storage, nx, ny, rows, int(bool(nt)), tile)
    src = kernel_source_hash(storage)
    for line in open(path):
        f = line.split()
        # traffic <storage> <nx> <ny> <rows> <nt> <tile> <source-hash> <bytes-per-launch>
        if len(f) == 9 and f[0] == "traffic" and " ".join(f[1:7]) == want and f[7] == src:
            return int(f[8])
    return None


def cpu_baseline_batch(sweep, target_seconds):
    """FP64 CPU oracle on the sweep's runs, smallest first, for a bounded time."""
    from oracle import oracle as orc
    cores = min(len(os.sched_getaffinity(0)), 16)
    orc.set_threads(cores)
    nodes_done, dt, used = 0, 0.0, []
    for w in sorted(sweep, key=lambda w: w["spec"]["nx"] * w["spec"]["ny"]):
        sim = orc.OracleSim(w["spec"], w["body"])
        sim.step(1)
        t0 = time.perf_counter()
        sim.step(20)
        dt += time.perf_counter() - t0
        nodes_done += w["spec"]["nx"] * w["spec"]["ny"] * 20
        used.append(w["name"])
        if dt > target_seconds:
            break
    return {"value": round(nodes_done / dt / 1e6, 2), "unit": "MLUPS", "cores": orc.max_threads(),
            "kind": "oracle",
            "sample": "20 steps of each of the %d smallest runs of the sweep (FP64 oracle, %.1f s)"
                      % (len(used), dt)}


def sweep_statistics(batch, sweep, steps):
    """Mean C_D and RMS C_L (from the hydrodynamic force) over the second half."""
    import numpy as np
    out = []
    for m, w in zip(batch.sims, sweep):
        r = m.forces(cap=steps)
        assert len(r) == steps, (w["name"], len(r))
        h = r[steps // 2:]
        scale = 0.5 * w["U0"] ** 2 * w["D"]
        cd = h["fh"][:, 0] / scale
        cl = h["fh"][:, 1] / scale
        out.append((float(cd.mean()), float(np.sqrt((cl ** 2).mean()))))
    return out


def batch_accuracy(args, vplbm, W):
    import numpy as np
    res = {}
    for storage in ("fp64", "fp32", "fp16", "bf16"):
        sweep = W.batch_sweep(storage=storage)
        members = [(w["spec"], w["body"]) for w in sweep]
        print("accuracy run %s, %d steps" % (storage, args.accuracy_steps), file=sys.stderr,
              flush=True)
        batch = vplbm.Batch(members, storage=storage, graph_steps=64,
                            history_cap=args.accuracy_steps)
        batch.step(args.accuracy_steps)
        batch.sync()
        res[storage] = sweep_statistics(batch, sweep, args.accuracy_steps)
        batch.close()
    ref = np.array(res["fp64"])
    out = {"steps": args.accuracy_steps, "fp64_mean_cd_range": [round(ref[:, 0].min(), 4),
                                                                  round(ref[:, 0].max(), 4)],
           "fp64_rms_cl_range": [round(ref[:, 1].min(), 4), round(ref[:, 1].max(), 4)]}
    for storage in ("fp32", "fp16", "bf16"):
        a = np.array(res[storage])
        ecd = np.abs(a[:, 0] - ref[:, 0]) / np.abs(ref[:, 0])
        ecl = np.abs(a[:, 1] - ref[:, 1]) / np.maximum(np.abs(ref[:, 1]), 1e-300)
        out[storage] = {"mean_cd_rel_err_max": float("%.3g" % ecd.max()),
                        "mean_cd_rel_err_median": float("%.3g" % np.median(ecd)),
                        "rms_cl_rel_err_max": float("%.3g" % ecl.max()),
                        "rms_cl_rel_err_median": float("%.3g" % np.median(ecl))}
    return out


def run_batch(args):
    import torch
    from paper_1905_05110_amd import workloads as W
    from paper_1905_05110_amd import vplbm

    sweep = W.batch_sweep(storage=args.storage)
    members = [(w["spec"], w["body"]) for w in sweep]
    nodes = sum(s["nx"] * s["ny"] for s, _ in members)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        rows = args.rows if args.rows else 0
        batch = vplbm.Batch(members, storage=args.storage, rows=rows, store=args.store,
                            history_cap=4096, stream=stream.cuda_stream,
                            tile_width=args.tile_width)
        tuned = None
        w_pre, w_post = split_warmup(args.warmup, args.graph_steps)
        print("warmup %d steps" % args.warmup, file=sys.stderr, flush=True)
        batch.step(w_pre)
        batch.sync()
        if not args.no_autotune and args.rows == 0 and args.store == "auto" and not args.tile_width:
            print("autotune", file=sys.stderr, flush=True)
            tuned = batch.autotune(trial_steps=20)
        b_rows, b_nt, b_tile = batch.sims[0].launch_config()
        if args.graph_steps:
            batch.set_graph_steps(args.graph_steps)
        batch.step(w_post)
        batch.sync()
        torch.cuda.synchronize()
        print("timed %d steps" % args.steps, file=sys.stderr, flush=True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        batch.step(args.steps)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        region_ms = e0.elapsed_time(e1)
        batch.sync()
        batch.close()
    ms_per_step = region_ms / args.steps
    mlups = nodes * args.steps / (region_ms * 1e-3) / 1e6
    avg_kernel_s = region_ms * 1e-3 / args.steps
    bytes_per_launch = BYTES_PER_NODE[args.storage] * nodes
    achieved = bytes_per_launch / avg_kernel_s / 1e9
    order_names = {0: "given", 1: "largest_first", 2: "interleaved"}
    out = {
        "metric": "MLUPS (D2Q9 MRT + volume penalization, full FSI step, batched runs)",
        "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "fp16": "f32 (fp16 storage)",
                  "bf16": "f32 (bf16 storage)"}[args.storage],
        "data": "synthetic (lattice flows from a uniform inflow state; no dataset)",
        "config": {"workload": "batch_sweep_64", "runs": len(members), "nodes": nodes,
                   "storage": args.storage, "graph_steps": args.graph_steps,
                   "rows_per_tile": b_rows, "nontemporal_stores": bool(b_nt),
                   "tile_width": b_tile,
                   "order": order_names[tuned[2]] if tuned else "largest_first"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None, "kernel": "k_step<%s> (batched)" % args.storage,
                     "avg_kernel_us": round(avg_kernel_s * 1e6, 3),
                     "algorithmic_bytes_per_launch": bytes_per_launch},
        "wall_s": round(wall, 3),
    }
    if args.accuracy_steps:
        out["accuracy_vs_fp64"] = batch_accuracy(args, vplbm, W)
    if not args.no_cpu_baseline:
        print("cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline_batch(sweep, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def cpu_baseline_adjoint(target_seconds):
    """Reverse-mode oracle (torch-CPU FP64) on the 128x64 copy of the workload."""
    import torch
    from oracle import adjoint_oracle as ado
    from paper_1905_05110_amd import workloads as W
    cores = min(len(os.sched_getaffinity(0)), 16)
    torch.set_num_threads(cores)
    wl = W.adjoint_drag(storage="fp64", nx=128, ny=64, D=8.0)
    m = ado.Mirror(wl["spec"], wl["body"])
    t0 = time.perf_counter()
    m.gradient(100, 50, (1.0, 0.0))
    per_step = (time.perf_counter() - t0) / 100
    n = max(100, min(2000, int(target_seconds / per_step) // 100 * 100))
    t0 = time.perf_counter()
    m.gradient(n, 100, (1.0, 0.0))
    dt = time.perf_counter() - t0
    return {"value": round(128 * 64 * n / dt / 1e6, 3), "unit": "MLUPS (forward + reverse)",
            "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": "reverse-mode oracle, 128x64 copy, %d steps (%.1f s)" % (n, dt)}


def run_adjoint(args):
    import statistics
    from paper_1905_05110_amd import workloads as W
    from paper_1905_05110_amd import vplbm

    wl = W.adjoint_drag(storage=args.storage)
    steps, every = wl["steps"], wl["checkpoint_every"]
    w = (1.0 / (steps * 0.5 * wl["U0"] ** 2 * wl["D"]), 0.0)
    nodes = wl["spec"]["nx"] * wl["spec"]["ny"]
    adj = vplbm.Adjoint(wl["spec"], wl["body"], steps, every, w, graphs=args.graph_steps != 0)
    print("adjoint warm-up", file=sys.stderr, flush=True)
    J = adj.forward()
    adj.backward()
    tf, tb = [], []
    for rep in range(3):
        t0 = time.perf_counter()
        adj.forward()
        t1 = time.perf_counter()
        adj.backward()
        t2 = time.perf_counter()
        tf.append(t1 - t0)
        tb.append(t2 - t1)
        print("rep %d forward %.4f s backward %.4f s" % (rep, tf[-1], tb[-1]), file=sys.stderr,
              flush=True)
    g = adj.gradient(chi=False)
    fwd, bwd = statistics.median(tf), statistics.median(tb)
    adj_us, step_us = adj.time_kernels(reps=400)
    esize = {"fp32": 4, "fp64": 8}[args.storage]
    # adjoint step per node: 9 state reads (re-pull), 9 adjoint reads, 9 adjoint writes,
    # dJ/dchi read and write
    adj_bytes = nodes * 29 * esize
    achieved = adj_bytes / (adj_us * 1e-6) / 1e9
    out = {
        "metric": "adjoint/forward time ratio (gradient of time-averaged drag)",
        "value": round(bwd / fwd, 3), "unit": "ratio", "n_gpus": 1, "steps": steps, "warmup": 1,
        "ms_per_step": round(1e3 * (fwd + bwd) / steps, 5), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64"}[args.storage],
        "data": "synthetic (channel flow from a uniform inflow state; no dataset)",
        "config": {"workload": "adjoint_drag_1024x512", "nx": wl["spec"]["nx"],
                   "ny": wl["spec"]["ny"], "storage": args.storage, "D": wl["D"], "Re": 100,
                   "steps": steps, "checkpoint_every": every, "indicator": "tanh, delta = 1",
                   "graphs": args.graph_steps != 0},
        "forward_s": round(fwd, 5), "backward_s": round(bwd, 5),
        "forward_mlups": round(nodes * steps / fwd / 1e6, 1),
        "backward_mlups": round(nodes * steps / bwd / 1e6, 1),
        "J": J, "dJ_dpos": [float(x) for x in g["pos"]],
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_adjoint<%s>" % args.storage, "avg_kernel_us": round(adj_us, 3),
                     "algorithmic_bytes_per_launch": adj_bytes,
                     "forward_step_kernel_us": round(step_us, 3)},
    }
    adj.close()
    if not args.no_cpu_baseline:
        print("cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline_adjoint(args.cpu_seconds)
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; it "
              "measures one GPU's share of the work", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch_sweep":
        return run_batch(args)
    if args.workload == "adjoint":
        if args.storage not in ("fp32", "fp64"):
            print("the adjoint runs in fp32 or fp64 storage", file=sys.stderr)
            sys.exit(2)
        return run_adjoint(args)
    import torch
    from paper_1905_05110_amd import workloads as W
    from paper_1905_05110_amd import vplbm

    wl = W.free_viv(storage=args.storage)
    spec = dict(wl["spec"], rows_per_tile=args.rows, store_mode=args.store,
                tile_width=args.tile_width)
    body = wl["body"]
    nodes = spec["nx"] * spec["ny"]
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        sim = vplbm.Sim(spec, body, torch_memory=True, history_cap=1 << 17)
        tuned = None
        w_pre, w_post = split_warmup(args.warmup, args.graph_steps)
        print("warmup %d steps" % args.warmup, file=sys.stderr, flush=True)
        sim.step(w_pre)
        sim.sync()
        if not args.no_autotune and args.rows == 0 and args.store == "auto" and not args.tile_width:
            print("autotune", file=sys.stderr, flush=True)
            tuned = sim.autotune(trial_steps=50)
        rows, nt, tile = sim.launch_config()
        if args.graph_steps:
            sim.set_graph_steps(args.graph_steps)
        sim.step(w_post)
        sim.sync()
        torch.cuda.synchronize()
        # timed region: K full steps on the simulation's stream, bracketed by events
        print("timed %d steps" % args.steps, file=sys.stderr, flush=True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        sim.step(args.steps)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        region_ms = e0.elapsed_time(e1)
        sim.sync()
    ms_per_step = region_ms / args.steps
    mlups = nodes * args.steps / (region_ms * 1e-3) / 1e6
    avg_kernel_s = region_ms * 1e-3 / args.steps  # one step-kernel launch per step
    bytes_per_launch = BYTES_PER_NODE[args.storage] * nodes
    achieved = bytes_per_launch / avg_kernel_s / 1e9
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
        "dtype": {"fp32": "f32", "fp64": "f64", "fp16": "f32 (fp16 storage)",
                  "bf16": "f32 (bf16 storage)"}[args.storage],
        "data": "synthetic (lattice flow from a uniform inflow state; no dataset)",
        "config": {"workload": "free_viv_2048x1024", "nx": spec["nx"], "ny": spec["ny"],
                   "storage": args.storage, "body": "disc D=40, free in y, mass ratio 10, U_r 5",
                   "Re": 150, "graph_steps": args.graph_steps,
                   "rows_per_tile": rows, "nontemporal_stores": bool(nt), "tile_width": tile},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_for(args.traffic, args.storage, spec["nx"], spec["ny"],
                                            rows, nt, tile),
                     "kernel": "k_step<%s>" % args.storage,
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
