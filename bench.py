"""Benchmark: bond updates per second of the explicit peridynamic step on one MI355X.

One step = the whole hot path through the C ABI (pd_step): contact-candidate
rebuild on its cadence, the fused bond-force / break / damage / contact / wall /
velocity-Verlet kernel, and the wall reduction.  The workload is the
double-notched plate (100 x 100 x 9 mm at h = 0.5 mm: 720,000 nodes, horizon 3h,
about 81 M directed bonds) struck on its edge by a rigid projectile face at
32 m/s; inputs are seeded, synthetic, and resident in HBM before timing starts.

Prints one JSON line with the metric, the roofline of the fused step kernel
(algorithmic bytes per launch over its event-timed average duration) and the
CPU oracle timed on the host cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
KERNEL_SRC = os.path.join(ROOT, "paper_2506_05362_amd", "csrc", "pd_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_step_tile_notched_plate.json")

# algorithmic bytes of the fused step kernel (per launch):
#   per directed bond : 4 B column word (it also carries the bond-broken state)
#   per node          : read u, v, a (72 B) + write u, v, a (72 B) + 4 B lattice/grain word
BYTES_PER_BOND = 4.0
BYTES_PER_NODE = 148.0


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def workload(name: str):
    from paper_2506_05362_amd import inputs as I
    if name == "notched_plate":
        return I.notched_plate()
    if name == "two_spheres":
        return I.two_spheres()
    if name == "grain_aggregate":
        return I.grain_aggregate()
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(wl, nnz_gpu: int, budget_s: float):
    """The oracle as it stands, on a bounded number of steps of the same workload."""
    from oracle import pdref
    threads = max(1, min(16, os.cpu_count() or 1))
    ora = pdref.Oracle(wl, flags=pdref.CELL_LIST, threads=threads)
    t0 = time.perf_counter()
    ora.step(1)
    t1 = time.perf_counter() - t0
    n = max(1, min(200, int(budget_s / max(t1, 1e-6))))
    t0 = time.perf_counter()
    ora.step(n)
    dt = time.perf_counter() - t0
    nnz = ora.nnz
    assert nnz == nnz_gpu, (nnz, nnz_gpu)
    return {"value": nnz * n / dt, "unit": "bond-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} steps of the same {wl.n_nodes}-node workload after its bond build "
                      f"({dt:.2f} s, {threads} OpenMP threads, plain C FP64)"}


def copy_probe():
    """Plain device kernels of known size, for scaling hardware byte counters:
    a fill (writes 1 GiB) and a scale (reads 1 GiB, writes 1 GiB)."""
    import torch
    n = 1 << 27  # 1 GiB of float64
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.mul(x, 2.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": 8 * n}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="notched_plate")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--bond-path", choices=["auto", "slices", "tiles"], default="auto",
                    help="bond loop: LDS tiles where the mesh allows (auto), or force one")
    ap.add_argument("--surrogate", action="store_true",
                    help="also run the representative-volume surrogate pipeline (64 simulated "
                         "paths, training, held-out error, inference speed; several minutes)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library runs on a single device (a multi-GPU run "
              "would shard grains by spatial bisection and exchange surface-node halos)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2506_05362_amd import pd

    if args.copy_probe:
        copy_probe()

    wl = workload(args.workload)
    t0 = time.perf_counter()
    sim = pd.Sim(wl)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    bond_path = pd.BONDS_SLICES
    if args.bond_path in ("auto", "tiles"):
        try:
            sim.set_launch(bond_path=pd.BONDS_TILES)
            bond_path = pd.BONDS_TILES
        except pd.PDError:
            if args.bond_path == "tiles":
                raise
    info = sim.info()
    nnz, N = info["nnz"], info["n_nodes"]
    print(f"[bench] {args.workload}: {N} nodes, {nnz} bonds, padded {info['padded']}, "
          f"build {build_s:.2f} s", file=sys.stderr, flush=True)

    sim.step(args.warmup)
    torch.cuda.synchronize()
    print(f"[bench] warmup {args.warmup} steps done", file=sys.stderr, flush=True)

    stream = sim.plumbing.stream  # the stream every kernel of the context runs on
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)

    # timed region 1: the production path (captured step loop replayed as HIP graphs)
    torch.cuda.synchronize()
    start.record(stream)
    sim.step(args.steps)
    stop.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    print(f"[bench] timed {args.steps} steps (graph replay): {total_ms:.1f} ms", file=sys.stderr,
          flush=True)

    # timed region 2: the same steps launched directly, every step kernel bracketed
    # by HIP events on the context stream (its average duration feeds the roofline)
    sim.set_timing(True)
    torch.cuda.synchronize()
    start.record(stream)
    sim.step(args.steps)
    stop.record(stream)
    torch.cuda.synchronize()
    direct_ms = start.elapsed_time(stop)
    launches, kern_ms = sim.timing()
    sim.set_timing(False)
    print(f"[bench] timed {args.steps} steps (direct launches): {direct_ms:.1f} ms, step kernel "
          f"{kern_ms / max(launches, 1) * 1e3:.1f} us", file=sys.stderr, flush=True)

    value = nnz * args.steps / (total_ms / 1e3)
    avg_kernel_s = kern_ms / 1e3 / max(launches, 1)
    bytes_launch = nnz * BYTES_PER_BOND + N * BYTES_PER_NODE
    achieved = bytes_launch / avg_kernel_s / 1e9

    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_src_sha256_16") == kernel_hash() and tr.get("workload") == args.workload:
            traffic = tr.get("bytes_per_launch")

    out = {
        "metric": "bond updates/s",
        "value": value,
        "unit": "bond-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "nodes": N, "bonds": nnz,
                   "step_loop": "hip graph replay", "bond_path": pd.BOND_PATH_NAMES[bond_path],
                   "direct_launch_ms_per_step": direct_ms / args.steps,
                   "padded_slots": info["padded"], "dt": wl.params.dt,
                   "horizon_factor": wl.params.horizon_factor,
                   "rebuild_every": wl.params.rebuild_every, "walls": len(wl.walls),
                   "build_s": round(build_s, 3)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_step_tile" if bond_path == pd.BONDS_TILES else "k_step<MODE_STEP>",
                     "avg_launch_us": avg_kernel_s * 1e6,
                     "launches": launches, "algorithmic_bytes_per_launch": bytes_launch,
                     "kernel_bond_updates_per_s": nnz / avg_kernel_s},
    }
    sim.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, nnz, args.cpu_budget)
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
