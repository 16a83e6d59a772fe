#!/usr/bin/env python3
"""Throughput of the coupled lattice-Boltzmann + finite-difference timestep on one MI355X.

Default workload: the 2048 x 2048 periodic dilute emulsion (64 active droplets, R = 20), FP64 -- the
configuration on which the HBM-roofline figure is quoted.  Variants in the same JSON line: the same
lattice in FP32, and the batched two-droplet sweep (32 lattices from 256 x 256 to 512 x 256, FP32) in one
launch sequence under hipGraph replay.

Timing: W warm-up steps, then exactly K steps bracketed by torch.cuda.synchronize() and hipEvents recorded
on the library's stream, replayed from hipGraphs of G steps (G the largest even divisor of K up to
--graph-steps), once and then five more times; MLUPS = lattice nodes x K / seconds / 1e6 from the median of
the five.  The roofline figure of the dominant kernel uses its algorithmic bytes per launch (one read and one
write of each value it must move) over its device time per launch: back-to-back launches replayed from a
graph between two hipEvents on the library's stream, divided by their number.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
METRIC = "MLUPS of coupled LB+FD step and % HBM roofline, FP64 vs FP32 vs batched"

# Algorithmic values moved per lattice node by each kernel of the timestep: (populations, field values).
#   k_step (fused): reads 9 populations + phi + c, writes the same          -> (18, 4)
#   k_wave (fused, one wavefront per strip): the same                      -> (18, 4)
#   k_lb (split):   reads 9 populations + phi + c, writes 9 populations + ux + uy -> (18, 4)
#   k_fd (split):   reads phi + c + ux + uy, writes phi + c                   -> (0, 6)
#   whole step, state only (9 populations + phi + c read and written)        -> (18, 4)
VALUES_PER_NODE = {"k_step": (18, 4), "k_wave": (18, 4), "k_lb": (18, 4), "k_fd": (0, 6), "step": (18, 4)}
# bytes of (a population, a field value) per precision code: FP64, FP32, FP16 population storage
ELEM_BYTES = {0: (8, 8), 1: (4, 4), 2: (2, 4)}
PREC_NAMES = {0: "fp64", 1: "fp32", 2: "fp16"}


def alg_bytes_per_node(kernel, precision):
    npop, nfield = VALUES_PER_NODE[kernel]
    pb, fb = ELEM_BYTES[precision]
    return npop * pb + nfield * fb
PATH_NAMES = {0: "fused", 1: "split", 2: "wave"}
PATH_NUMBERS = {v: k for k, v in PATH_NAMES.items()}


def note(msg: str) -> None:
    """A progress line on stderr (the JSON line goes to stdout)."""
    print(f"bench.py: {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("lbm_kernels_impl.h", "lbm_kernels_f64.hip", "lbm_kernels_f32.hip", "lbm_kernels_f16.hip",
              "lbm_internal.h"):
        with open(os.path.join(ROOT, "paper_1711_10984_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str, precision: str, strip_w, seg_rows):
    """HBM bytes per launch from the committed rocprofv3 counter summary (profiles/traffic.json), if it
    was taken on the current kernel source and the same strip height (null otherwise)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        return None
    if data.get("kernel_source_hash") != kernel_source_hash():
        return None
    ent = data.get("entries", {}).get(f"{kernel}:{workload}:{precision}:{strip_w}x{seg_rows}")
    return None if ent is None else ent.get("bytes_per_launch")


def emulsion_4096():
    """The 2048^2 emulsion's recipe on a 4096^2 lattice: 256 droplets (the same density), R = 20."""
    from paper_1711_10984_amd import workloads as W
    return W.c5_emulsion(seed=1015, n=4096, ndrop=256, R=20.0)


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """Plain device-to-device copy of nbytes (torch), best of reps: bytes read + written per second (GB/s).
    The practical ceiling that the kernels' algorithmic bandwidth is also compared with."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    best = 1e30
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    return 2.0 * nbytes / (best * 1e-3) / 1e9


def build_sim(workloads, precision, graph_steps, path):
    from paper_1711_10984_amd import lbm
    return lbm.Sim([w.param_dict() for w in workloads], [w.phi0 for w in workloads], [w.c0 for w in workloads],
                   [w.drop_dicts() for w in workloads], precision=precision, graph_steps=graph_steps, path=path)


def graph_size(steps, graph_steps):
    """Steps per hipGraph: the largest even divisor of `steps` not above `graph_steps` (0: no graphs), so that
    every timed step is graph-replayed."""
    if not graph_steps or steps < 2:
        return 0
    for g in range(min(graph_steps, steps), 1, -1):
        if g % 2 == 0 and steps % g == 0:
            return g
    return 0


def time_steps(sim, steps, warmup, repeats=0):
    """ms for exactly `steps` steps after `warmup` steps (hipEvents on the library's stream), the wall time,
    and the ms of `repeats` further timings of the same number of steps."""
    import torch
    sim.set_graph(graph_size(steps, sim.graph_steps))  # captured here, outside the timed region
    sim.step(warmup)
    sim.sync()
    torch.cuda.synchronize()

    def once():
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(sim.stream)
        sim.step(steps)
        e1.record(sim.stream)
        sim.sync()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), time.perf_counter() - t0

    ms, wall = once()
    more = [once()[0] for _ in range(repeats)]
    return ms, wall, more


def measure(workloads, precision, steps, warmup, graph_steps, label, prof_steps, path=-1, seg_rows=0, strip_w=0):
    """path -1: the autotuner picks the kernel path (fused or wave sweep with its strip width and height, or
    split).  seg_rows / strip_w 0: autotuned (with a given height, width 0 keeps the default)."""
    from paper_1711_10984_amd import lbm
    gsize = graph_size(steps, graph_steps)
    sim = build_sim(workloads, precision, gsize, 0 if path < 0 else path)
    tune_ms = {}
    if path != 1 and seg_rows == 0:
        # state-preserving: the trial launches write scratch only
        seg_rows, path, tune_ms = sim.autotune(30, both_paths=path < 0)
        if path == 1:
            seg_rows = None
    elif path != 1:
        if path < 0:
            path = 0
        sim.set_seg_rows(seg_rows)
        if strip_w:
            sim.set_strip_width(strip_w)
    else:
        seg_rows = None
    strip_w = sim.strip_width if seg_rows is not None else None
    nodes = sum(w.nodes for w in workloads)
    first_ms, wall, more = time_steps(sim, steps, warmup, repeats=5)
    ms = sorted(more)[len(more) // 2]  # the median of five timings of exactly `steps` steps
    obs = sim.observables(0)
    # device time per launch of each kernel: back-to-back launches replayed from a graph (state unchanged)
    device_ms = sim.time_launches(prof_steps)
    per_kernel = sim.time_kernels(prof_steps)  # hipEvents around each eager launch (gaps included)
    sim.close()
    mlups = nodes * steps / (ms * 1e-3) / 1e6
    dom = max((k for k in device_ms if k in VALUES_PER_NODE), key=lambda k: device_ms[k])
    alg_bytes = alg_bytes_per_node(dom, precision) * nodes
    # The dominant kernel's device time per launch: back-to-back launches replayed from a graph, divided by their
    # number.  They read the same input every time, so where a step reads what the step before wrote (partly
    # from the last-level cache) it runs up to a few per cent faster; the step time gives that bound
    # (step_roofline).
    dom_ms, dom_from = device_ms[dom], f"{prof_steps} back-to-back launches replayed from a graph"
    achieved = alg_bytes / (dom_ms * 1e-3) / 1e9
    step_bytes = alg_bytes_per_node("step", precision) * nodes
    step_gbs = step_bytes / (ms * 1e-3 / steps) / 1e9
    prec = PREC_NAMES[precision]
    traffic = measured_traffic(dom, label, prec, strip_w, seg_rows)
    note(f"{label} {prec}: {mlups:.0f} MLUPS, {PATH_NAMES[path]} kernel, height {seg_rows}")
    return {
        "mlups": mlups, "ms_per_step": ms / steps, "wall_s": wall, "nodes": nodes, "precision": prec,
        "median_of_5": {"ms_per_step": ms / steps, "mlups": mlups, "ms_per_step_each": [m / steps for m in more],
                        "first_timing_ms_per_step": first_ms / steps},
        "graph": {"steps_per_graph": gsize, "graph_replayed_steps": steps - steps % gsize if gsize else 0},
        "kernel_ms": per_kernel, "device_ms_per_launch": device_ms, "seg_rows": seg_rows, "strip_width": strip_w,
        "autotune_ms": tune_ms, "path": PATH_NAMES[path],
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "alg_bytes_per_launch": alg_bytes, "avg_launch_ms": dom_ms, "avg_launch_from": dom_from},
        "step_roofline": {"alg_bytes_per_step": step_bytes, "achieved": round(step_gbs, 1),
                          "frac": round(step_gbs / HBM_PEAK_GBS, 4)},
        "sanity": {"mass": obs["mass"], "sum_phi": obs["sum_phi"], "min_B": obs["min_B"], "max_u": obs["max_u"],
                   "unstable": obs["unstable"]},
    }


def sweep_heights(workloads, precision, prof_steps):
    """Both sweeping kernels at every strip height the autotuner tries, prof_steps eagerly launched steps each,
    in a fixed order (fused heights ascending, then wave heights ascending), so that a profiler's per-dispatch
    records can be attributed to (kernel, height) by their order.  Returns that order with the hipEvent
    times."""
    sim = build_sim(workloads, precision, None, 0)
    out = []
    for path in (0, 2):
        sim.set_path(path)
        for h in sim.tune_rows():
            sim.set_seg_rows(h)
            out.append({"path": PATH_NAMES[path], "seg_rows": h, "strip_width": sim.strip_width,
                        "kernel_ms": sim.time_kernels(prof_steps)})
    sim.close()
    return out


def _minimg(d, L):
    return (d + 0.5 * L) % L - 0.5 * L


def lowp_accuracy(workloads, steps, log_every, graph_steps, kernel, low):
    """A lower precision (`low`: LBM_FP32 or LBM_FP16) against FP64 on the GPU for the same inputs: largest
    centre-of-mass deviation over the run (trajectories logged every `log_every` steps), drift of the phi
    integral in both precisions, and the relative L2 difference of the velocity field at the end (first
    lattice).  `kernel` = (path, seg_rows, strip_width) of the throughput measurement whose accuracy this is:
    both runs use that kernel, height and width.  Every lattice's deviation is listed; a lattice is marked as
    merging when its droplets come within R_j + R_k of each other in the FP64 run (decided from the FP64
    trajectory alone, before comparing): two tracked centres then share one body, and which centre takes a node
    is a discrete decision that the two precisions may take differently."""
    import numpy as np
    from paper_1711_10984_amd import lbm
    path, seg_rows, strip_w = kernel
    traj = {}
    end = {}
    phi_sum = {}
    for prec in (lbm.LBM_FP64, low):
        sim = build_sim(workloads, prec, graph_steps, path)
        if path != 1:
            sim.set_seg_rows(seg_rows)
            sim.set_strip_width(strip_w)
        t = []
        s0 = [sim.observables(i)["sum_phi"] for i in range(len(workloads))]
        for k in range(steps // log_every):
            sim.step(log_every)
            t.append([[(d["x"], d["y"]) for d in sim.droplets(i)] for i in range(len(workloads))])
        traj[prec] = t
        end[prec] = sim.fields(0)
        phi_sum[prec] = [sim.observables(i)["sum_phi"] - s0[i] for i in range(len(workloads))]
        sim.close()
    per_lattice, merging = {}, []
    for i, w in enumerate(workloads):
        dev, close = 0.0, False
        for a in traj[lbm.LBM_FP64]:  # the merge criterion, from the FP64 run only
            for j in range(len(a[i])):
                for k in range(j + 1, len(a[i])):
                    sep = np.hypot(_minimg(a[i][j][0] - a[i][k][0], w.nx), _minimg(a[i][j][1] - a[i][k][1], w.ny))
                    close = close or sep < w.drops[j].R + w.drops[k].R
        for a, b in zip(traj[lbm.LBM_FP64], traj[low]):
            for (xa, ya), (xb, yb) in zip(a[i], b[i]):
                dev = max(dev, float(np.hypot(_minimg(xa - xb, w.nx), _minimg(ya - yb, w.ny))))
        per_lattice[w.name] = round(dev, 6)
        if close:
            merging.append(w.name)
    u64, u32 = end[lbm.LBM_FP64], end[low]
    num = np.sqrt(np.sum((u64["ux"] - u32["ux"]) ** 2 + (u64["uy"] - u32["uy"]) ** 2))
    den = np.sqrt(np.sum(u64["ux"] ** 2 + u64["uy"] ** 2))
    out = {"steps": steps, "lattices": len(workloads), "log_every": log_every,
           "kernel": {"path": PATH_NAMES[path], "seg_rows": seg_rows if path != 1 else None,
                      "strip_width": strip_w if path != 1 else None},
           "max_cm_deviation_lu": round(max(per_lattice.values()), 6),
           "phi_integral_drift_fp64": round(float(max(phi_sum[lbm.LBM_FP64], key=abs)), 6),
           f"phi_integral_drift_{PREC_NAMES[low]}": round(float(max(phi_sum[low], key=abs)), 6),
           "velocity_l2_rel_diff": float(num / den) if den > 0 else None}
    if len(workloads) > 1:
        apart = [v for k, v in per_lattice.items() if k not in merging]
        out["per_lattice_max_cm_deviation_lu"] = per_lattice
        out["merging_in_fp64_run"] = merging
        out["max_cm_deviation_lu_non_merging"] = round(max(apart), 6) if apart else None
    note(f"{PREC_NAMES[low]} accuracy over {steps} steps on {len(workloads)} lattice(s): "
         f"{out['max_cm_deviation_lu']} lu")
    return out

def adjoint_measure(precision, nsteps=2000, every=100, repeats=2, n=256):
    """Reverse mode on the n^2 single-active-droplet workload (256^2 by default; the droplet scales with n): wall
    time of the checkpointed forward pass and of the backward sweep (both synchronous library calls), best of
    `repeats`, on the autotuned kernel path."""
    from paper_1711_10984_amd import lbm, workloads as W
    w = W.c2_single_active(n=n)
    best_f, best_b = 1e300, 1e300
    for _ in range(repeats):
        sim = lbm.Sim([w.param_dict()], [w.phi0], [w.c0], [w.drop_dicts()], precision=precision, graph_steps=20)
        rows, path, _ = sim.autotune(10, both_paths=True)
        width = sim.strip_width
        sim.sync()
        t0 = time.perf_counter()
        sim.adjoint_forward(0, nsteps, every)
        t1 = time.perf_counter()
        sim.adjoint_backward()
        t2 = time.perf_counter()
        sim.close()
        best_f, best_b = min(best_f, t1 - t0), min(best_b, t2 - t1)
    note(f"reverse mode {PREC_NAMES[precision]}: backward {best_b / nsteps * 1e3:.3f} ms/step")
    return {"workload": f"{w.name}, {nsteps} steps, checkpoint every {every}", "nodes": w.nodes,
            "path": PATH_NAMES[path], "seg_rows": rows if path != 1 else None,
            "strip_width": width if path != 1 else None,
            "forward_ms_per_step": round(best_f / nsteps * 1e3, 5),
            "backward_ms_per_step": round(best_b / nsteps * 1e3, 5),
            "backward_mlups": round(w.nodes * nsteps / best_b / 1e6, 1),
            "backward_over_forward": round(best_b / best_f, 2)}


def oracle_rate(w, budget_s, max_steps=1000):
    """Full steps of the FP64 oracle on workload w for about budget_s seconds: (MLUPS, steps, seconds, threads)."""
    from oracle import OracleSim, Params, Drop, num_threads
    s = OracleSim(Params(nx=w.nx, ny=w.ny, **w.params), w.phi0, w.c0, [Drop(**d) for d in w.drop_dicts()])
    steps, t0 = 0, time.perf_counter()
    while True:
        s.run(1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= max_steps:
            break
    return w.nodes * steps / el / 1e6, steps, el, num_threads(w.nx, w.ny)


def host_cpu():
    """CPU model and the number of cores this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"model": model, "logical_cpus_available": avail, "os_cpu_count": os.cpu_count()}


def _oracle_instance(args):
    """Worker: `steps` single-threaded oracle steps of one lattice; returns node-steps and seconds."""
    from oracle import OracleSim, Params, Drop
    nx, ny, params, phi0, c0, drops, steps = args
    s = OracleSim(Params(nx=nx, ny=ny, **params), phi0, c0, [Drop(**d) for d in drops])
    t0 = time.perf_counter()
    s.run(steps)
    return nx * ny * steps, time.perf_counter() - t0


def oracle_parallel_instances(factory, steps, procs):
    """The lattices of workloads.<factory>() as independent single-threaded oracle runs, `procs` at a time
    (a process pool; run in a child started with OMP_NUM_THREADS=1): (MLUPS over the whole batch, lattices,
    steps, seconds)."""
    from multiprocessing import Pool
    from paper_1711_10984_amd import workloads as W
    ws = getattr(W, factory)()
    jobs = [(w.nx, w.ny, w.params, w.phi0, w.c0, w.drop_dicts(), steps) for w in ws]
    t0 = time.perf_counter()
    with Pool(procs) as pool:
        res = pool.map(_oracle_instance, jobs, chunksize=1)
    el = time.perf_counter() - t0
    return sum(r[0] for r in res) / el / 1e6, len(ws), steps, el


def _child_json(code, env_extra, timeout=600):
    import subprocess
    res = subprocess.run([sys.executable, "-c", code], env=dict(os.environ, **env_extra), capture_output=True,
                         text=True, timeout=timeout, cwd=ROOT)
    return json.loads(res.stdout.strip().splitlines()[-1])


def cpu_baseline(w, budget_s, single_budget_s=8.0, factory="c5_emulsion"):
    """The FP64 oracle as it stands on this host's cores, on bounded samples: the headline workload w (all
    threads, and one thread in a child process with OMP_NUM_THREADS=1, since OpenMP fixes its thread count at
    start-up, on workloads.<factory>(), the same lattice), the 64^2 and 256^2 single-lattice configurations, and
    the 32-lattice batch as independent single-threaded runs across the host's cores."""
    from paper_1711_10984_amd import workloads as W
    rate, steps, el, threads = oracle_rate(w, budget_s)
    note(f"CPU oracle, {w.name}: {rate:.1f} MLUPS on {threads} threads")
    host = host_cpu()
    out = {"value": round(rate, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
           "sample": f"{w.name}: {steps} FP64 steps of the full {w.nx}x{w.ny} lattice in {el:.1f} s",
           "host_cpu": host}
    code = ("import json, sys; sys.path.insert(0, %r); import bench; from paper_1711_10984_amd import workloads as W; "
            "w = W.%s(); r = bench.oracle_rate(w, %r); print(json.dumps(list(r) + [w.nx, w.ny]))"
            % (ROOT, factory, single_budget_s))
    try:
        r1, s1, e1, t1, nx1, ny1 = _child_json(code, {"OMP_NUM_THREADS": "1"})
        out["single_thread"] = {"value": round(r1, 3), "cores": t1,
                                "sample": f"{s1} FP64 steps of the full {nx1}x{ny1} lattice in {e1:.1f} s"}
    except Exception as e:  # noqa: BLE001 -- a failed child leaves a note, not a failed benchmark
        out["single_thread"] = {"error": str(e)[:200]}
    configs = {}
    for name, wl, budget in (("c1_64x64", W.c1_equilibrium(), 3.0), ("c2_256x256", W.c2_single_active(), 4.0)):
        r, st, e, t = oracle_rate(wl, budget, max_steps=5000)
        configs[name] = {"value": round(r, 3), "cores": t, "sample": f"{st} FP64 steps in {e:.1f} s"}
    procs = min(16, host["logical_cpus_available"] or 1)
    code = ("import json, sys; sys.path.insert(0, %r); import bench; "
            "print(json.dumps(bench.oracle_parallel_instances('c3_batch', 40, %d)))" % (ROOT, procs))
    try:
        r3, n3, s3, e3 = _child_json(code, {"OMP_NUM_THREADS": "1"})
        configs["c3_batch_32_lattices"] = {
            "value": round(r3, 3), "cores": procs,
            "sample": f"{n3} lattices as independent single-threaded runs, {procs} at a time, {s3} FP64 steps "
                      f"each, in {e3:.1f} s"}
    except Exception as e:  # noqa: BLE001
        configs["c3_batch_32_lattices"] = {"error": str(e)[:200]}
    out["configs"] = configs
    note("CPU oracle configurations done")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--graph-steps", type=int, default=100)
    ap.add_argument("--prof-steps", type=int, default=50, help="steps timed per kernel with hipEvents")
    ap.add_argument("--no-variants", action="store_true", help="FP64 2048^2 only")
    ap.add_argument("--path", type=int, default=-1, choices=[-1] + sorted(PATH_NAMES),
                    help="-1: autotuned choice of 0, 1 or 2; 0: fused sweep kernel; 1: split LB + FD kernels; "
                         "2: wavefront-per-strip sweep kernel")
    ap.add_argument("--seg-rows", type=int, default=0, help="sweeping-kernel strip height (0: autotune)")
    ap.add_argument("--strip-width", type=int, default=0,
                    help="sweeping-kernel strip width with --seg-rows (0: the library default)")
    ap.add_argument("--only", default=None,
                    choices=["fp64", "fp32", "fp16", "c3", "fp32_4096", "fp16_4096", "adjoint", "adjoint_1024"],
                    help="run one configuration (for profiling); the JSON line then reports that one")
    ap.add_argument("--sweep-heights", action="store_true",
                    help="with --only (default fp64): launch both sweeping kernels at every autotuner height, "
                         "--prof-steps steps each, and print the order (for per-height rocprofv3 counters)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle work for the CPU baseline")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the FP32/FP16-vs-FP64 accuracy runs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 512 MiB device copy (reference for rocprofv3 counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only (the timestep is a single-GPU kernel; the "
              "multi-GPU decomposition is a design note, not code) -- use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1711_10984_amd import lbm, workloads as W

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    lbm.load_library()
    if args.copy_calibration:
        a = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    copy_gbs = copy_bandwidth()
    c5 = W.c5_emulsion()
    if args.only == "adjoint":
        print(json.dumps({"only": "adjoint", "fp64": adjoint_measure(lbm.LBM_FP64, repeats=1)}), flush=True)
        return
    if args.only == "adjoint_1024":
        print(json.dumps({"only": "adjoint_1024", "fp64": adjoint_measure(lbm.LBM_FP64, 200, 20, 1, n=1024)}),
              flush=True)
        return
    if args.sweep_heights:
        only = args.only or "fp64"
        wl, prec, label = {"fp64": ([c5], lbm.LBM_FP64, "c5"), "fp32": ([c5], lbm.LBM_FP32, "c5"),
                           "fp16": ([c5], lbm.LBM_FP16, "c5"), "c3": (W.c3_batch(), lbm.LBM_FP32, "c3"),
                           "fp32_4096": ([emulsion_4096()], lbm.LBM_FP32, "c5_4096"),
                           "fp16_4096": ([emulsion_4096()], lbm.LBM_FP16, "c5_4096")}[only]
        print(json.dumps({"sweep": label, "precision": PREC_NAMES[prec], "prof_steps": args.prof_steps,
                          "kernel_source_hash": kernel_source_hash(),
                          "order": sweep_heights(wl, prec, args.prof_steps)}), flush=True)
        return
    if args.only in ("fp32", "fp16", "c3", "fp32_4096", "fp16_4096"):
        wl, prec, label = {"fp32": ([c5], lbm.LBM_FP32, "c5"), "fp16": ([c5], lbm.LBM_FP16, "c5"),
                           "c3": (W.c3_batch(), lbm.LBM_FP32, "c3"),
                           "fp32_4096": ([emulsion_4096()], lbm.LBM_FP32, "c5_4096"),
                           "fp16_4096": ([emulsion_4096()], lbm.LBM_FP16, "c5_4096")}[args.only]
        r = measure(wl, prec, args.steps, args.warmup, args.graph_steps, label, args.prof_steps, args.path,
                    args.seg_rows, args.strip_width)
        print(json.dumps({"only": args.only, "mlups": round(r["mlups"], 1), "ms_per_step": r["ms_per_step"],
                          "median_of_5": r["median_of_5"], "graph": r["graph"],
                          "device_ms_per_launch": r["device_ms_per_launch"],
                          "roofline": r["roofline"], "kernel_ms": r["kernel_ms"], "seg_rows": r["seg_rows"],
                          "strip_width": r["strip_width"], "path": r["path"]}),
              flush=True)
        return
    main_res = measure([c5], lbm.LBM_FP64, args.steps, args.warmup, args.graph_steps, "c5", args.prof_steps,
                       args.path, args.seg_rows, args.strip_width)
    variants = {}
    if not args.no_variants and args.only is None:
        variants["fp32_2048"] = measure([c5], lbm.LBM_FP32, args.steps, args.warmup, args.graph_steps, "c5",
                                        args.prof_steps, args.path, args.seg_rows, args.strip_width)
        variants["batched_c3_fp32"] = measure(W.c3_batch(), lbm.LBM_FP32, args.steps, args.warmup,
                                              args.graph_steps, "c3", args.prof_steps, args.path, args.seg_rows,
                                              args.strip_width)
        variants["fp16_storage_2048"] = measure([c5], lbm.LBM_FP16, args.steps, args.warmup, args.graph_steps,
                                                "c5", args.prof_steps, args.path, args.seg_rows, args.strip_width)
        # 4096^2: twice the 256 MB last-level cache per step even in FP16, so no step's state stays cached
        big = emulsion_4096()
        variants["fp32_4096"] = measure([big], lbm.LBM_FP32, args.steps, args.warmup, args.graph_steps, "c5_4096",
                                        args.prof_steps, args.path, args.seg_rows, args.strip_width)
        variants["fp16_storage_4096"] = measure([big], lbm.LBM_FP16, args.steps, args.warmup, args.graph_steps,
                                                "c5_4096", args.prof_steps, args.path, args.seg_rows,
                                                args.strip_width)
        del big
    for v in variants.values():
        v["gain_over_fp64"] = round(v["mlups"] / main_res["mlups"], 3)
    for res in [main_res] + list(variants.values()):
        res["roofline"]["copy_gbs"] = round(copy_gbs, 1)
        res["roofline"]["frac_of_copy"] = round(res["roofline"]["achieved"] / copy_gbs, 4)
    out = {
        "metric": METRIC,
        "value": round(main_res["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2048x2048 periodic dilute emulsion, 64 active droplets R=20 (seeded), FP64",
                   "nx": 2048, "ny": 2048, "droplets": 64,
                   "graph_steps": main_res["graph"]["steps_per_graph"],
                   "graph_replayed_steps": main_res["graph"]["graph_replayed_steps"],
                   "kernel_path": main_res["path"]},
        "median_of_5": main_res["median_of_5"],
        "roofline": main_res["roofline"],
        "step_roofline": main_res["step_roofline"],
        "kernel_ms": main_res["kernel_ms"],
        "device_ms_per_launch": main_res["device_ms_per_launch"],
        "autotune": {"seg_rows": main_res["seg_rows"], "strip_width": main_res["strip_width"],
                     "path": main_res["path"],
                     "ms_per_launch": main_res["autotune_ms"]},
        "variants": {k: {"mlups": round(v["mlups"], 1), "ms_per_step": round(v["ms_per_step"], 5),
                         "nodes": v["nodes"], "precision": v["precision"], "gain_over_fp64": v["gain_over_fp64"],
                         "roofline": v["roofline"], "step_roofline": v["step_roofline"],
                         "kernel_ms": v["kernel_ms"], "device_ms_per_launch": v["device_ms_per_launch"],
                         "median_of_5": v["median_of_5"], "graph": v["graph"],
                         "seg_rows": v["seg_rows"], "strip_width": v["strip_width"], "path": v["path"]}
                     for k, v in variants.items()},
        "kernel_source_hash": kernel_source_hash(),
    }
    if not args.no_accuracy and not args.no_variants and args.only is None:
        # each accuracy run uses the kernel, strip height and width of the throughput variant it qualifies
        kern = {k: (PATH_NUMBERS[v["path"]], v["seg_rows"], v["strip_width"]) for k, v in variants.items()}
        gs = args.graph_steps
        out["fp32_accuracy"] = {
            "single_droplet_256": lowp_accuracy([W.c2_single_active()], 100000, 1000, gs, kern["fp32_2048"],
                                                lbm.LBM_FP32),
            "batched_c3_config_length": lowp_accuracy(W.c3_batch(), 20000, 500, gs, kern["batched_c3_fp32"],
                                                      lbm.LBM_FP32),
            "batched_c3": lowp_accuracy(W.c3_batch(), 100000, 500, gs, kern["batched_c3_fp32"], lbm.LBM_FP32),
            "emulsion_2048_64_droplets": lowp_accuracy([c5], 100000, 1000, gs, kern["fp32_2048"], lbm.LBM_FP32),
        }
        out["fp16_accuracy"] = {
            "single_droplet_256": lowp_accuracy([W.c2_single_active()], 100000, 1000, gs, kern["fp16_storage_2048"],
                                                lbm.LBM_FP16),
            "emulsion_2048_64_droplets": lowp_accuracy([c5], 100000, 1000, gs, kern["fp16_storage_2048"],
                                                       lbm.LBM_FP16),
        }
    if not args.no_variants and args.only is None:
        out["adjoint"] = {"fp64": adjoint_measure(lbm.LBM_FP64), "fp32": adjoint_measure(lbm.LBM_FP32),
                          "fp64_1024": adjoint_measure(lbm.LBM_FP64, 200, 20, 1, n=1024)}
    if not args.no_cpu_baseline and args.only is None:
        out["cpu_baseline"] = cpu_baseline(c5, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
