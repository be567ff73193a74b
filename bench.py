"""Benchmark: bond updates per second of the explicit peridynamic step on one MI355X.

One step = the whole hot path through the C ABI (pd_step): contact-candidate
rebuild on its cadence, the fused bond-force / break / damage / contact / wall /
velocity-Verlet kernel, and the wall reduction.

The headline workload is the large aggregate: 999 tessellated grains with
log-normal sizes on one lattice (h = 41 um), 9,261,000 nodes and 967,622,492
directed bonds in a box of six walls, compressed by the platen at 10 m/s.  A
second object in the same line times the double-notched plate (720,000 nodes)
struck by a projectile face.  Inputs are seeded, synthetic, and resident in HBM
before timing starts.

The timed region launches every step directly with each step kernel
bracketed by HIP events on the library's stream, so the kernel's average
duration (the roofline's denominator) comes from the same region as the step
rate; the captured loop (HIP graphs of rebuild_every steps) is timed just
before it over as many steps and reported beside it.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix cores
KERNEL_SRC = os.path.join(ROOT, "paper_2506_05362_amd", "csrc", "pd_kernels.hip")
PROFILES = os.path.join(ROOT, "profiles")

# Algorithmic bytes of one step-kernel launch (CSR byte model):
#   per directed bond : 4 B column word + 1 bit of bond-broken mask = 4.125 B
#   per node          : 128 B (read u, X, v; write u, v; 8 B damage/intact)
BYTES_PER_BOND = 4.125
BYTES_PER_NODE = 128.0
# FP64 operations of the bond law per directed bond (eta 3, y 3, 2 xi + eta 3,
# |y|^2 - |xi|^2 3, x 1, series 8 + 1, break test 1, c V/|xi| g 1, force 3)
# against the FP64 vector issue rate: 256 CUs x 4 SIMDs x 16 FP64 lanes x 2.4 GHz
# (an FMA counted as one operation; 78.6 TFLOP/s counting it as two)
FP64_OPS_PER_BOND = 27
FP64_LANE_OPS_PEAK = 256 * 4 * 16 * 2.4e9


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def workload(name: str):
    from paper_2506_05362_amd import inputs as I
    if name == "large_aggregate":
        return I.large_aggregate()
    if name == "notched_plate":
        return I.notched_plate()
    if name == "two_spheres":
        return I.two_spheres()
    if name == "grain_aggregate":
        return I.grain_aggregate()
    raise SystemExit(f"unknown workload {name}")


def host_info():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"cpu_model": model, "logical_cpus": os.cpu_count() or 1, "usable_cpus": usable}


def cpu_baseline(wl, nnz_gpu: int, budget_s: float):
    """The oracle as it stands, timed on a bounded number of steps of the same
    workload after its bond build: with as many threads as the host gives this
    process (at most 16) and with one thread."""
    from oracle import pdref
    hi = host_info()
    threads = max(1, min(16, hi["usable_cpus"]))
    t0 = time.perf_counter()
    ora = pdref.Oracle(wl, flags=pdref.CELL_LIST, threads=threads)
    build_s = time.perf_counter() - t0
    assert ora.nnz == nnz_gpu, (ora.nnz, nnz_gpu)
    print(f"[bench] oracle built in {build_s:.1f} s", file=sys.stderr, flush=True)

    def timed(nthreads, share):
        pdref.lib().pdref_set_threads(nthreads)
        t = time.perf_counter()
        ora.step(1)
        one = time.perf_counter() - t
        if one >= share * budget_s:  # one step already fills the share
            return 1, one
        n = max(1, min(200, int(share * budget_s / max(one, 1e-6))))
        t = time.perf_counter()
        ora.step(n)
        return n, time.perf_counter() - t

    n_all, t_all = timed(threads, 0.6)
    n_one, t_one = timed(1, 0.4)
    nnz = ora.nnz
    return {"value": nnz * n_all / t_all, "unit": "bond-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_all} steps of the same {wl.n_nodes}-node workload after its bond build "
                      f"({t_all:.2f} s on {threads} OpenMP threads, plain C FP64, -O2 -ffp-contract=off); "
                      f"one thread: {n_one} steps in {t_one:.2f} s",
            "one_thread_value": nnz * n_one / t_one, "host": hi}


def traffic_record(workload_name: str, kernel: str):
    """HBM bytes per launch of the kernel from rocprofv3 counters, when the record
    was taken on the current kernel source."""
    path = os.path.join(PROFILES, f"traffic_{kernel}_{workload_name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        tr = json.load(f)
    if tr.get("kernel_src_sha256_16") != kernel_hash() or tr.get("workload") != workload_name:
        return None
    return tr.get("bytes_per_launch")


def time_workload(name: str, steps: int, warmup: int, bond_path_arg: str):
    """Build the workload, warm it up, align to the captured loop and time
    `steps` steps.  Returns the measurement and the workload."""
    import torch
    from paper_2506_05362_amd import pd

    wl = workload(name)
    t0 = time.perf_counter()
    sim = pd.Sim(wl)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    bond_path = pd.BONDS_SLICES
    if bond_path_arg in ("auto", "tiles"):
        try:
            sim.set_launch(bond_path=pd.BONDS_TILES)
            bond_path = pd.BONDS_TILES
        except pd.PDError:
            if bond_path_arg == "tiles":
                raise
    info = sim.info()
    nnz, N = info["nnz"], info["n_nodes"]
    print(f"[bench] {name}: {N} nodes, {nnz} bonds, padded {info['padded']}, build {build_s:.2f} s",
          file=sys.stderr, flush=True)
    sim.step(warmup)
    # the captured loop replays runs of graph_len steps that start on a multiple
    # of graph_len: step on (untimed) to the next such start
    graph_len = wl.params.rebuild_every if wl.params.rebuild_every % 2 == 0 else 2 * wl.params.rebuild_every
    align = (-(warmup)) % graph_len
    sim.step(align)
    torch.cuda.synchronize()
    print(f"[bench] {name}: warmup {warmup} + {align} alignment steps done", file=sys.stderr, flush=True)

    stream = sim.plumbing.stream  # the stream every kernel of the context runs on
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)

    # the captured loop: `steps` steps replayed as HIP graphs (not the headline,
    # since no per-kernel events can sit inside a replay)
    counts0 = sim.loop_counts()
    torch.cuda.synchronize()
    start.record(stream)
    sim.step(steps)
    stop.record(stream)
    torch.cuda.synchronize()
    graph_ms = start.elapsed_time(stop)
    counts1 = sim.loop_counts()
    replayed = counts1["graph_steps"] - counts0["graph_steps"]

    # the timed region: the next `steps` steps launched directly, every step
    # kernel bracketed by HIP events on the library's stream
    sim.set_timing(True)
    torch.cuda.synchronize()
    start.record(stream)
    sim.step(steps)
    stop.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    launches, kern_ms = sim.timing()
    sim.set_timing(False)
    counts2 = sim.loop_counts()
    direct = counts2["direct_steps"] - counts1["direct_steps"]
    avg_kernel_s = kern_ms / 1e3 / max(launches, 1)
    print(f"[bench] {name}: {steps} steps in graph replays ({replayed} replayed): {graph_ms:.2f} ms; "
          f"timed {steps} steps launched directly ({direct}): {total_ms:.2f} ms, step kernel "
          f"{avg_kernel_s * 1e6:.1f} us over {launches} launches", file=sys.stderr, flush=True)
    kernel = "k_step_tile" if bond_path == pd.BONDS_TILES else "k_step"
    bytes_launch = nnz * BYTES_PER_BOND + N * BYTES_PER_NODE
    achieved = bytes_launch / avg_kernel_s / 1e9
    traffic = traffic_record(name, kernel)
    out = {
        "value": nnz * steps / (total_ms / 1e3),
        "ms_per_step": total_ms / steps,
        "config": {"workload": name, "nodes": N, "bonds": nnz, "grains": wl.n_grains,
                   "step_loop": f"direct launches, every step kernel bracketed by HIP events ({direct} steps)",
                   "graph_replay_ms_per_step": graph_ms / steps, "graph_replayed_steps": replayed,
                   "bond_path": pd.BOND_PATH_NAMES[bond_path], "padded_slots": info["padded"],
                   "dt": wl.params.dt, "horizon_factor": wl.params.horizon_factor,
                   "rebuild_every": wl.params.rebuild_every, "walls": len(wl.walls),
                   "timed_steps": [warmup + align + steps + 1, warmup + align + 2 * steps],
                   "build_s": round(build_s, 3)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     # the counted HBM bytes over the same kernel time (null without a record
                     # taken on this kernel source): what the memory system actually carried
                     "traffic_GBps": traffic / avg_kernel_s / 1e9 if traffic else None,
                     "kernel": kernel, "avg_launch_us": avg_kernel_s * 1e6, "launches": launches,
                     "algorithmic_bytes_per_launch": bytes_launch,
                     "bytes_model": f"{BYTES_PER_BOND} B per directed bond + {BYTES_PER_NODE} B per node",
                     "kernel_bond_updates_per_s": nnz / avg_kernel_s},
        # the same kernel against the FP64 vector units, by the bond law's operation count
        "roofline_alu": {"bound": "alu", "achieved": nnz * FP64_OPS_PER_BOND / avg_kernel_s,
                         "peak": FP64_LANE_OPS_PEAK, "unit": "FP64 op/s",
                         "frac": nnz * FP64_OPS_PER_BOND / avg_kernel_s / FP64_LANE_OPS_PEAK,
                         "ops_model": f"{FP64_OPS_PER_BOND} FP64 operations per directed bond"},
    }
    sim.close()
    return out, wl


def copy_probe():
    """Attainable HBM bandwidth: a plain device copy of 4 GiB (reads 4 GiB, writes
    4 GiB) timed with events, best of 5."""
    import torch
    n = 1 << 29  # 4 GiB of float64
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    best = None
    for _ in range(6):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        y.copy_(x)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    del x, y
    torch.cuda.empty_cache()
    return {"bytes": 16 * n, "best_ms": best, "GB_per_s": 16 * n / (best / 1e3) / 1e9}


def surrogate_inference(n_paths: int = 100000, T: int = 100):
    """Throughput of the surrogate network's fused inference kernels (weights do
    not change the work: seeded random ones), on strain paths resident in HBM."""
    import numpy as np
    from paper_2506_05362_amd import surrogate as S
    rng = np.random.default_rng(0)
    sur = S.Surrogate()
    sur.xs = S.Scaler(np.zeros(6), np.ones(6))
    sur.ys = S.Scaler(np.zeros(7), np.ones(7))
    paths = rng.normal(size=(n_paths, T, 6)).astype(np.float32)
    r = S.time_inference(sur, paths)
    return {"metric": "surrogate inference samples/s", "value": r["samples"] / r["seconds"],
            "unit": "samples/s", "samples": r["samples"], "seconds": r["seconds"],
            "dims": list(sur.dims), "dtype": "bf16 matrix cores, fp32 accumulate",
            "roofline": {"bound": "mfma", "achieved": r["tflops"], "peak": BF16_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": r["tflops"] / BF16_PEAK_TFLOPS}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="large_aggregate")
    ap.add_argument("--secondary", default="notched_plate",
                    help="second workload timed in the same run ('' for none)")
    ap.add_argument("--cpu-budget", type=float, default=25.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-copy-probe", action="store_true")
    ap.add_argument("--bond-path", choices=["auto", "slices", "tiles"], default="auto",
                    help="bond loop: LDS tiles where the mesh allows (auto), or force one")
    ap.add_argument("--no-surrogate-inference", action="store_true",
                    help="skip the timing of the surrogate network's inference kernels")
    ap.add_argument("--surrogate", action="store_true",
                    help="also run the representative-volume surrogate pipeline (64 simulated "
                         "paths, training, held-out error, inference speed; many minutes)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library runs on a single device (a multi-GPU run "
              "would shard grains by spatial bisection and exchange surface-node halos)", file=sys.stderr)
        sys.exit(2)

    import torch  # noqa: F401

    probe = None if args.no_copy_probe else copy_probe()
    if probe:
        print(f"[bench] copy probe: {probe['GB_per_s']:.0f} GB/s", file=sys.stderr, flush=True)
    head, wl = time_workload(args.workload, args.steps, args.warmup, args.bond_path)
    out = {
        "metric": "bond updates/s",
        "value": head["value"],
        "unit": "bond-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": head["config"],
        "roofline": head["roofline"],
        "roofline_alu": head["roofline_alu"],
    }
    if probe:
        out["roofline"]["attainable_copy_GBps"] = probe["GB_per_s"]
        out["roofline"]["frac_of_attainable"] = out["roofline"]["achieved"] / probe["GB_per_s"]
    if args.secondary:
        sec, _ = time_workload(args.secondary, args.steps, args.warmup, args.bond_path)
        out["secondary"] = {"workload": args.secondary, "value": sec["value"], "ms_per_step": sec["ms_per_step"],
                            "config": sec["config"], "roofline": sec["roofline"],
                            "roofline_alu": sec["roofline_alu"]}
    if not args.no_surrogate_inference:
        out["surrogate_inference"] = surrogate_inference()
        print(f"[bench] surrogate inference: {out['surrogate_inference']['value']:.3g} samples/s, "
              f"{out['surrogate_inference']['roofline']['achieved']:.1f} TFLOP/s", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, head["config"]["bonds"], args.cpu_budget)
    if args.surrogate:
        from paper_2506_05362_amd import surrogate
        r = surrogate.run(log=lambda s: print(s, file=sys.stderr, flush=True))
        out["surrogate"] = {
            "metric": "RVE surrogate speedup per path at held-out axial stress error",
            "speedup_per_path": r["speedup_per_path"],
            "held_out_axial_rel_l2_mean": r["axial_rel_l2_mean"],
            "interpolation_axial_rel_l2_mean": r["interp_axial_rel_l2_mean"],
            "sim_seconds_per_path": r["sim_seconds_per_path"],
            "network_seconds_per_path": r["inference"]["seconds_per_path"],
            "paths": r["paths"], "held_out": r["held_out"], "dtype": "bf16 matrix cores, fp32 accumulate",
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
