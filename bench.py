"""Throughput of the VP-LBM time step on one MI355X.

Default workload (``--workload batch_sweep``): 64 independent free vortex-induced-
vibration runs of uneven size (ny drawn from U{128..512} with seed 0, nx = 2 ny,
D = ny/12, reduced velocity 2 to 12, mass ratio 10, Re = 150; 15.1 M nodes, 2.2 GB of
FP32 populations, far beyond the 256 MB Infinity Cache), all advanced by one kernel
launch per step.  A step is one full fluid-structure step of every run (pull-stream,
penalization, MRT collision, FP64 force/torque reduction, RK4 body update), all on the
GPU.

The timed region starts from a seeded random near-rest state, w_a (1 + 0.02 xi) with
xi ~ U(-1, 1) (the same generator as the parity tests), written into every run just
before it, whatever the warm-up was: no stored offset is then exactly zero (the memory
system moves lines of zeros faster than lines of data, so a state that still holds the
uniform inflow would overstate the rate).

Prints one JSON line: MLUPS (million lattice-node updates per second) of the timed
region (and the median rate of its five consecutive segments), the step kernel's achieved HBM bandwidth against the 8 TB/s peak, and the FP64
CPU oracle timed on a bounded sample of the same workload on the host cores (all the
cores of the GPU's share and one core).  A step is exactly one kernel launch (replayed
from captured HIP graphs), so the kernel's average duration is the timed region's
event-measured time divided by the number of launches.

Other workloads:
  ``free_viv``       2048x1024 channel, disc D = 40 on a transverse spring (151 MB in
                     FP32: largely resident in the Infinity Cache);
  ``sedimentation``  1024x4096 closed box, a disc D = 32 of density ratio 1.5 falling
                     free in x, y and theta (302 MB in FP32);
  ``roofline``       8192x8192 channel with a fixed disc D = 512 (4.8 GB in FP32);
  ``adjoint``        reverse-mode gradient of the time-averaged drag of a fixed disc
                     (1024x512, 4000 steps, a checkpoint every 100): the value is the
                     adjoint/forward time ratio.
``--accuracy-steps N`` (batch_sweep) also runs the sweep for N steps in every storage
precision and reports the relative error of each run's mean drag and RMS lift
coefficients over the second half of the run against the FP64 runs.
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
CPU_SHARE = 16  # host cores that go with one GPU of the box
STATE_SEED, STATE_AMP = 2024, 0.02
DTYPE = {"fp32": "f32", "fp64": "f64", "fp16": "f32 (fp16 storage)", "bf16": "f32 (bf16 storage)"}
DATA = ("synthetic: timed from a seeded random near-rest state w_a (1 + 0.02 xi), "
        "xi ~ U(-1, 1), seed %d, written into every run before the timed region; no dataset"
        % STATE_SEED)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="batch_sweep",
                    choices=("batch_sweep", "free_viv", "sedimentation", "roofline", "adjoint"))
    ap.add_argument("--accuracy-steps", type=int, default=0,
                    help="batch_sweep: also compare storages over this many steps")
    ap.add_argument("--steps", type=int, default=0, help="timed steps (0: the workload's default)")
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--storage", default="fp32", choices=sorted(BYTES_PER_NODE))
    ap.add_argument("--graph-steps", type=int, default=64,
                    help="steps per captured HIP graph in the timed region (0: eager launches)")
    ap.add_argument("--rows", type=int, default=0, help="rows per tile (0: autotune)")
    ap.add_argument("--store", default="auto", choices=("auto", "plain", "nontemporal"))
    ap.add_argument("--tile-width", type=int, default=0, choices=(0, 64, 256, 512),
                    help="columns per tile (0: autotune)")
    ap.add_argument("--order", default="auto",
                    choices=("auto", "given", "largest_first", "interleaved"),
                    help="batch_sweep: tile schedule order (auto: autotune)")
    ap.add_argument("--layout", default="auto", choices=("auto", "rows", "planes"))
    ap.add_argument("--offset-ref", default="auto", choices=("auto", "initial", "rest"),
                    help="reference of the stored offsets (auto: rest for 16-bit storage)")
    ap.add_argument("--finalize", default="auto", choices=("auto", "tiles", "kernel"),
                    help="how the body state is finalized (auto: autotune)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="CPU time of each oracle sample (all cores, then one core)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one device copy of 256 MiB first (scale for HBM byte counters)")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.txt"),
                    help="measured HBM bytes per launch of the step kernel (from rocprofv3)")
    return ap.parse_args()


DEFAULT_STEPS = {"batch_sweep": 4000, "free_viv": 20000, "sedimentation": 10000,
                 "roofline": 400, "adjoint": 0}


def pinned(args):
    return args.rows != 0 or args.store != "auto" or args.tile_width != 0 or \
        args.finalize != "auto" or (args.workload == "batch_sweep" and args.order != "auto")


def cpu_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def oracle_rate(members, target_seconds, threads):
    """FP64 CPU oracle over the given runs (smallest first, again from the first while
    time is left) for a bounded time: returns (MLUPS, steps per run, run-advances made,
    seconds, threads).  The first step of every run is not counted; that of the first
    run sizes the sample."""
    from oracle import oracle as orc
    orc.set_threads(threads)
    ordered = sorted(members, key=lambda w: w["spec"]["nx"] * w["spec"]["ny"])
    total_nodes = sum(w["spec"]["nx"] * w["spec"]["ny"] for w in ordered)
    steps, done, dt, used = None, 0, 0.0, 0
    sims = {}
    while dt <= target_seconds:
        for k, w in enumerate(ordered):
            nodes = w["spec"]["nx"] * w["spec"]["ny"]
            if k not in sims:
                sims[k] = orc.OracleSim(w["spec"], w["body"])
                t0 = time.perf_counter()
                sims[k].step(1)  # first touch of the arrays: not counted
                if steps is None:
                    per_node = (time.perf_counter() - t0) / nodes
                    steps = max(2, min(200, int(target_seconds / (per_node * total_nodes))))
            t0 = time.perf_counter()
            sims[k].step(steps)
            dt += time.perf_counter() - t0
            done += nodes * steps
            used += 1
            if dt > target_seconds:
                break
    sims.clear()
    return done / dt / 1e6, steps, used, dt, orc.max_threads()


def cpu_baseline(members, target_seconds, label):
    model, avail = cpu_info()
    cores = min(avail, CPU_SHARE)
    v_all, steps, used, dt, threads = oracle_rate(members, target_seconds, cores)
    v_one, steps1, used1, dt1, _ = oracle_rate(members, target_seconds, 1)
    return {"value": round(v_all, 2), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": "%d steps per run, %d run-advances over the %s, smallest run first "
                      "(FP64 oracle, %.1f s on %d threads)" % (steps, used, label, dt, threads),
            "single_core_value": round(v_one, 3),
            "single_core_sample": "%d steps per run, %d run-advances over the %s (%.1f s)" % (
                steps1, used1, label, dt1),
            "cpu_model": model, "cores_visible": avail, "cores_share": CPU_SHARE}


def kernel_source_hash(storage):
    """Hash of the sources the step kernel of this storage is compiled from."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1905_05110_amd", "csrc")
    for name in ("vplbm_device.hpp", "vplbm_kernels.hpp", "kern_%s.hip" % storage):
        h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(path, key):
    """Measured HBM bytes per launch from the rocprofv3 counter summary, if one was
    recorded for this workload and launch configuration and for the kernel sources as
    they are now.  Lines: traffic <key fields...> <source-hash> <bytes-per-launch>."""
    if not path or not os.path.exists(path):
        return None
    want = key.split()
    src = kernel_source_hash(want[1])
    for line in open(path):
        f = line.split()
        if len(f) == len(want) + 3 and f[0] == "traffic" and f[1:-2] == want and f[-2] == src:
            return int(f[-1])
    return None


def seeded_state(sim):
    """The timed region's start: w_a (1 + amp xi) on every node."""
    from paper_1905_05110_amd import workloads as W
    f = W.random_populations(sim.nx, sim.ny, seed=STATE_SEED, amp=STATE_AMP)
    sim.set_populations(f)


def roofline(args, bytes_per_launch, avg_kernel_s, kernel, traffic_key):
    achieved = bytes_per_launch / avg_kernel_s / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_for(args.traffic, traffic_key), "kernel": kernel,
            "avg_kernel_us": round(avg_kernel_s * 1e6, 3),
            "algorithmic_bytes_per_launch": bytes_per_launch, "traffic_key": traffic_key}


def keep_busy(stream, ms=60.0):
    """Read passes over a 512 MiB device buffer on `stream`, about `ms` of GPU time, that
    touch nothing of the simulation (returns what must live until the stream has passed
    them)."""
    import torch
    with torch.cuda.stream(stream):
        buf = torch.ones(128 << 20, dtype=torch.float32, device="cuda")
        acc = torch.zeros((), dtype=torch.float32, device="cuda")
        for _ in range(int(ms * 1e-3 / 80e-6)):  # one pass reads 512 MiB in about 80 us
            acc += buf.sum()
    return buf, acc


def timed(stream, run, steps, graph_steps=0, segments=5):
    """Time exactly `steps` steps on `stream` with HIP events: returns the region's ms, its
    wall-clock seconds and the ms per step of each of `segments` consecutive segments
    (lengths a multiple of the captured graph's steps where the count allows; the last
    takes the rest), whose median is reported beside the whole region's rate.

    The region's opening event is queued behind some 60 ms of unrelated device work
    (keep_busy), and the steps behind it, while that work runs: the timed steps then run
    back to back from the event on, as they do in a long run, instead of the region
    opening on an idle stream and waiting for the host to submit the first step (20-50
    us), and they start on a GPU that has been working rather than one that sat idle
    while the host wrote the seeded state (after seconds idle the step time rises by up
    to 8 % for some tens of steps while the power state settles).  A region of 20 steps
    would otherwise count both against the step's rate.  The wall-clock time runs from
    the moment the opening event has passed to the end."""
    import torch
    print("timed %d steps" % steps, file=sys.stderr, flush=True)
    g = max(1, graph_steps)
    seg = (steps // segments) // g * g or max(1, steps // segments)
    lens = [seg] * (segments - 1)
    lens.append(steps - sum(lens))
    if lens[-1] <= 0:
        lens = [steps]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(lens) + 1)]
    torch.cuda.synchronize()
    busy = keep_busy(stream)
    ev[0].record(stream)
    for k, n in enumerate(lens):
        run(n)
        ev[k + 1].record(stream)
    while not ev[0].query():
        pass
    t0 = time.perf_counter()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    del busy
    per = [ev[k].elapsed_time(ev[k + 1]) / n for k, n in enumerate(lens)]
    return ev[0].elapsed_time(ev[-1]), wall, per


def median_field(per):
    import statistics
    return {"median_ms_per_step_of_segments": round(statistics.median(per), 5),
            "segment_ms_per_step": [round(x, 5) for x in per]}


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
        members = [(dict(w["spec"], offset_ref=args.offset_ref), w["body"]) for w in sweep]
        print("accuracy run %s, %d steps" % (storage, args.accuracy_steps), file=sys.stderr,
              flush=True)
        batch = vplbm.Batch(members, storage=storage, graph_steps=64,
                            history_cap=args.accuracy_steps)
        batch.step(args.accuracy_steps)
        batch.sync()
        res[storage] = sweep_statistics(batch, sweep, args.accuracy_steps)
        batch.close()
    ref = np.array(res["fp64"])
    out = {"steps": args.accuracy_steps, "offset_ref": args.offset_ref,
           "fp64_mean_cd_range": [round(ref[:, 0].min(), 4),
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


def split_warmup(warmup, graph_steps):
    """Untimed steps before and after the launch configuration is chosen (the steps
    after it capture the graphs of the timed region); together the requested warm-up."""
    post = min(warmup // 2, max(2 * graph_steps, 64))
    return warmup - post, post


def copy_calibration():
    """One device copy of 256 MiB: the scale for the HBM byte counters."""
    import torch
    src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def run_batch(args):
    import torch
    from paper_1905_05110_amd import workloads as W
    from paper_1905_05110_amd import vplbm

    if args.copy_calibration:
        copy_calibration()

    steps = args.steps or DEFAULT_STEPS["batch_sweep"]
    sweep = W.batch_sweep(storage=args.storage)
    members = [(dict(w["spec"], offset_ref=args.offset_ref), w["body"]) for w in sweep]
    nodes = sum(s["nx"] * s["ny"] for s, _ in members)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        batch = vplbm.Batch(members, storage=args.storage, rows=args.rows, store=args.store,
                            history_cap=4096, stream=stream.cuda_stream,
                            tile_width=args.tile_width, layout=args.layout,
                            finalize=args.finalize,
                            order="largest_first" if args.order == "auto" else args.order)
        w_pre, w_post = split_warmup(args.warmup, args.graph_steps)
        print("warmup %d steps" % args.warmup, file=sys.stderr, flush=True)
        batch.step(w_pre)
        batch.sync()
        for m in batch.sims:
            seeded_state(m)
        tuned = None
        if not args.no_autotune and not pinned(args):
            print("autotune", file=sys.stderr, flush=True)
            tuned = batch.autotune(trial_steps=64)
        b_rows, b_nt, b_tile = batch.sims[0].launch_config()
        order = batch.order_name()
        if args.graph_steps:
            batch.set_graph_steps(args.graph_steps)
        batch.step(w_post)
        batch.sync()
        for m in batch.sims:
            seeded_state(m)
        region_ms, wall, per = timed(stream, batch.step, steps, args.graph_steps)
        batch.sync()
        layout = batch.sims[0].layout_name()
        nfin = sum(m.finalize_by_kernel() for m in batch.sims)
        batch.close()
    avg_kernel_s = region_ms * 1e-3 / steps  # one launch per step
    bytes_per_launch = BYTES_PER_NODE[args.storage] * nodes
    key = "batch_sweep_64 %s %s %d %d %d %s %d" % (args.storage, layout, b_rows, int(bool(b_nt)),
                                                  b_tile, order, int(nfin > 0))
    out = {
        "metric": "MLUPS (D2Q9 MRT + volume penalization, full FSI step, batched runs)",
        "value": round(nodes * steps / (region_ms * 1e-3) / 1e6, 1), "unit": "MLUPS",
        "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": round(region_ms / steps, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[args.storage], "data": DATA,
        "config": {"workload": "batch_sweep_64", "runs": len(members), "nodes": nodes,
                   "storage": args.storage, "layout": layout, "graph_steps": args.graph_steps,
                   "rows_per_tile": b_rows, "nontemporal_stores": bool(b_nt),
                   "tile_width": b_tile, "order": order,
                   "finalize_by_kernel": nfin, "launches_per_step": 1 + int(nfin > 0),
                   "autotuned": tuned is not None},
        "roofline": roofline(args, bytes_per_launch, avg_kernel_s,
                             "k_step<%s> (batched)" % args.storage, key),
        "wall_s": round(wall, 3),
    }
    out.update(median_field(per))
    if args.accuracy_steps:
        out["accuracy_vs_fp64"] = batch_accuracy(args, vplbm, W)
    if not args.no_cpu_baseline:
        print("cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(sweep, args.cpu_seconds, "64 runs of the sweep")
    print(json.dumps(out), flush=True)


SINGLE = {
    "free_viv": ("free_viv_2048x1024", "disc D=40, free in y, mass ratio 10, U_r 5, Re 150"),
    "sedimentation": ("sedimentation_1024x4096",
                      "disc D=32, density ratio 1.5, free in x, y, theta; closed box, Re_p 1"),
    "roofline": ("roofline_8192x8192", "fixed disc D=512, Re 100"),
}


def run_single(args):
    import torch
    from paper_1905_05110_amd import workloads as W
    from paper_1905_05110_amd import vplbm

    steps = args.steps or DEFAULT_STEPS[args.workload]
    wl = {"free_viv": W.free_viv, "sedimentation": W.sedimentation,
          "roofline": W.roofline_grid}[args.workload](storage=args.storage)
    spec = dict(wl["spec"], rows_per_tile=args.rows, store_mode=args.store,
                tile_width=args.tile_width, layout=args.layout, finalize=args.finalize,
                offset_ref=args.offset_ref)
    nodes = spec["nx"] * spec["ny"]
    if args.copy_calibration:
        copy_calibration()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        sim = vplbm.Sim(spec, wl["body"], torch_memory=True, history_cap=1 << 16)
        w_pre, w_post = split_warmup(args.warmup, args.graph_steps)
        print("warmup %d steps" % args.warmup, file=sys.stderr, flush=True)
        sim.step(w_pre)
        sim.sync()
        seeded_state(sim)
        tuned = None
        if not args.no_autotune and not pinned(args):
            print("autotune", file=sys.stderr, flush=True)
            tuned = sim.autotune(trial_steps=max(4, min(50, int(2e9 / nodes))))
        rows, nt, tile = sim.launch_config()
        if args.graph_steps:
            sim.set_graph_steps(args.graph_steps)
        sim.step(w_post)
        sim.sync()
        seeded_state(sim)
        region_ms, wall, per = timed(stream, sim.step, steps, args.graph_steps)
        sim.sync()
        layout = sim.layout_name()
        fin = sim.finalize_by_kernel()
    avg_kernel_s = region_ms * 1e-3 / steps  # one step-kernel launch per step
    bytes_per_launch = BYTES_PER_NODE[args.storage] * nodes
    name, body = SINGLE[args.workload]
    key = "%s %s %s %d %d %d - %d" % (name, args.storage, layout, rows, int(bool(nt)), tile,
                                      int(fin))
    out = {
        "metric": "MLUPS (D2Q9 MRT + volume penalization, full FSI step)",
        "value": round(nodes * steps / (region_ms * 1e-3) / 1e6, 1), "unit": "MLUPS",
        "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": round(region_ms / steps, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[args.storage], "data": DATA,
        "config": {"workload": name, "nx": spec["nx"], "ny": spec["ny"], "storage": args.storage,
                   "layout": layout, "body": body, "graph_steps": args.graph_steps,
                   "rows_per_tile": rows, "nontemporal_stores": bool(nt), "tile_width": tile,
                   "finalize_by_kernel": fin, "launches_per_step": 1 + int(fin),
                   "autotuned": tuned is not None},
        "roofline": roofline(args, bytes_per_launch, avg_kernel_s, "k_step<%s>" % args.storage,
                             key),
        "wall_s": round(wall, 3),
    }
    out.update(median_field(per))
    sim.close()
    if not args.no_cpu_baseline:
        print("cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline([wl], args.cpu_seconds, "%s grid" % name)
    print(json.dumps(out), flush=True)


def cpu_baseline_adjoint(target_seconds):
    """Reverse-mode oracle (torch-CPU FP64) on the 128x64 copy of the workload."""
    import torch
    from oracle import adjoint_oracle as ado
    from paper_1905_05110_amd import workloads as W
    model, avail = cpu_info()
    torch.set_num_threads(min(avail, CPU_SHARE))
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
            "sample": "reverse-mode oracle, 128x64 copy, %d steps (%.1f s)" % (n, dt),
            "cpu_model": model, "cores_visible": avail, "cores_share": CPU_SHARE}


def run_adjoint(args):
    import statistics
    from paper_1905_05110_amd import workloads as W
    from paper_1905_05110_amd import vplbm

    wl = W.adjoint_drag(storage=args.storage)
    steps, every = wl["steps"], wl["checkpoint_every"]
    w = (1.0 / (steps * 0.5 * wl["U0"] ** 2 * wl["D"]), 0.0)
    nodes = wl["spec"]["nx"] * wl["spec"]["ny"]
    spec = dict(wl["spec"], layout=args.layout)
    adj = vplbm.Adjoint(spec, wl["body"], steps, every, w, graphs=args.graph_steps != 0)
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
    # adjoint step per node: 9 state reads (re-pull), 9 adjoint reads, 9 adjoint writes in
    # the storage precision, and the FP64 dJ/dchi accumulator read and written
    adj_bytes = nodes * (27 * esize + 16)
    achieved = adj_bytes / (adj_us * 1e-6) / 1e9
    out = {
        "metric": "adjoint/forward time ratio (gradient of time-averaged drag)",
        "value": round(bwd / fwd, 3), "unit": "ratio", "n_gpus": 1, "steps": steps, "warmup": 1,
        "ms_per_step": round(1e3 * (fwd + bwd) / steps, 5), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[args.storage],
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
    return run_single(args)


if __name__ == "__main__":
    main()
