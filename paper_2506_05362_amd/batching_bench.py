"""Step-loop comparison on the uneven-grain aggregate (100 grains of 2e3 to 5e4
nodes between platens): the batched fused launch replayed as a HIP graph, the
same launches issued directly, the persistent cooperative kernel, and the
unbatched reference with one launch per grain per step; then the launch
autotuner's choice.  Prints one JSON object.

    python -m paper_2506_05362_amd.batching_bench [--steps 400] [--grains 100]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import inputs as I
from . import pd


def time_mode(sim, cfg, steps, warm):
    sim.set_launch(**cfg)
    sim.step(warm)  # pd_step returns once the GPU is done
    t0 = time.perf_counter()
    sim.step(steps)
    wall = (time.perf_counter() - t0) / steps
    u = sim.get("displacement")  # state after warm + steps, the same in every mode
    # kernel time of the step launches alone (events; direct or persistent launches)
    sim.set_timing(True)
    sim.step(steps if cfg["loop"] != pd.LOOP_GRAPH else min(steps, 100))
    n, ms = sim.timing()
    sim.set_timing(False)
    per_step = ms / max(n, 1) if cfg["loop"] != pd.LOOP_PERSISTENT else ms / steps
    return wall, per_step, u


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--grains", type=int, default=100)
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args(argv)
    wl = I.grain_aggregate(n_grains=a.grains, seed=a.seed, rebuild_every=20)
    sim = pd.Sim(wl)
    info = sim.info()
    sizes = np.diff(wl.grain_begin)
    start = sim.get_state()
    modes = {
        "graph": dict(loop=pd.LOOP_GRAPH, slices_per_block=4, xcd_remap=1),
        "direct": dict(loop=pd.LOOP_DIRECT, slices_per_block=4, xcd_remap=1),
        "persistent": dict(loop=pd.LOOP_PERSISTENT, slices_per_block=4, xcd_remap=1),
        "per_grain": dict(loop=pd.LOOP_PER_GRAIN, slices_per_block=4, xcd_remap=1),
    }
    res = {}
    ref = None
    for name, cfg in modes.items():
        sim.set_state(start)
        wall, kern, u = time_mode(sim, cfg, a.steps, 40)
        same = None if ref is None else bool(np.array_equal(u, ref))
        if ref is None:
            ref = u
        res[name] = {"ms_per_step": wall * 1e3, "step_kernels_ms_per_step": kern,
                     "bond_updates_per_s": info["nnz"] / wall, "bitwise_equal_to_graph": same}
        print(f"{name}: {wall * 1e3:.4f} ms/step (kernels {kern:.4f} ms)", flush=True)
    from . import autotune
    sim.set_state(start)
    tuned = autotune.tune(sim, use_cache=False)
    out = {"workload": "grain_aggregate", "grains": int(wl.n_grains), "nodes": info["n_nodes"],
           "bonds": info["nnz"], "padded_slots": info["padded"],
           "grain_nodes_min": int(sizes.min()), "grain_nodes_max": int(sizes.max()),
           "steps": a.steps, "modes": res,
           "speedup_batched_graph_vs_per_grain": res["per_grain"]["ms_per_step"] / res["graph"]["ms_per_step"],
           "autotune": {"config": tuned["config"],
                        "ms_per_step": {k: v * 1e3 for k, v in tuned["times"].items()}}}
    sim.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    from paper_2506_05362_amd.batching_bench import main as _main
    _main()
