"""Shape study: bulk strength of 125-grain aggregates of spheres, shells and jacks.

Each aggregate (inputs.shape_study: grains of radius 1 mm on a 5 x 5 x 5 grid
in a box of rigid walls, lid moving down at 10 m/s, Sec. 7.6) is first timed
with both bond paths from the same state (and checked to reach bitwise the
same state), then compressed from the start for the requested duration.  Every
500 steps (5 us, the time unit of the paper's plots) the script logs the
compressive reactions of the lid and of the floor, their sum (the two forces
point opposite ways along z, so the difference of the z components the paper
calls bulk strength is the sum of the magnitudes), the mean damage and the
kinetic energy.  Prints JSON lines.

    python -m paper_2506_05362_amd.shape_study [--shapes sphere,shell,jack] [--duration 5e-4]
        [--self-contact 1] [--wall-corners 1]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import inputs as I
from . import pd
from .scale_bench import time_path


def run_shape(shape, a):
    import torch

    t0 = time.perf_counter()
    wl = I.shape_study(shape, seed=a.seed, grid=a.grid, cavity=a.cavity, h=a.h, dt=a.dt, duration=a.duration,
                       rebuild_every=a.rebuild_every)
    wl.params.contact_damping = a.damping
    wl.params.skin = a.skin * wl.grain_h[0]
    wl.params.self_contact = bool(a.self_contact)
    wl.params.wall_corners = bool(a.wall_corners)
    sim = pd.Sim(wl, candidate_capacity_per_node=a.capacity)
    torch.cuda.synchronize()
    info = sim.info()
    out = {"workload": wl.name, "grains": int(wl.n_grains), "nodes": info["n_nodes"], "bonds": info["nnz"],
           "cavity": a.cavity if shape == "shell" else None,
           "setup_s": round(time.perf_counter() - t0, 2), "dt": wl.params.dt, "steps": wl.steps,
           "contact_damping": a.damping, "self_contact": bool(a.self_contact),
           "wall_corners": bool(a.wall_corners),
           "rebuild_every": a.rebuild_every, "skin_h": a.skin,
           "lid_speed": wl.walls[1].velocity}
    print(json.dumps(out), flush=True)

    start = sim.get_state()
    paths, ref = {}, None
    for name, bp in (("slices", pd.BONDS_SLICES), ("tiles", pd.BONDS_TILES)):
        wall, kern_ms, u = time_path(sim, bp, start, a.time_steps)
        same = None if ref is None else bool(np.array_equal(u, ref))
        ref = u if ref is None else ref
        paths[name] = {"ms_per_step": wall * 1e3, "step_kernel_ms": kern_ms,
                       "bond_updates_per_s": info["nnz"] / wall, "bitwise_equal_to_slices": same}
        print(shape, name, json.dumps(paths[name]), flush=True)
    out["paths"] = paths
    best = min(paths, key=lambda p: paths[p]["ms_per_step"])

    sim.set_state(start)
    sim.set_launch(bond_path=pd.BONDS_TILES if best == "tiles" else pd.BONDS_SLICES)
    unit = a.log_steps
    mass = wl.materials[0].density * wl.grain_h[0] ** 3
    log, done, status = [], 0, "complete"
    t0 = time.perf_counter()
    while done < wl.steps:
        n = min(unit, wl.steps - done)
        st = sim.step_status(n)
        if st != pd.PD_OK:
            status = "stopped: " + pd.lib().pd_last_error(sim.h).decode()
            break
        done += n
        f = sim.get("wall_force")
        top = float(-(f[1] @ np.array(wl.walls[1].normal)))
        floor = float(-(f[0] @ np.array(wl.walls[0].normal)))
        v = sim.get("velocity")
        log.append({"t_5us": round(done * wl.params.dt / 5e-6, 3), "lid_n": top, "floor_n": floor,
                    "bulk_strength_n": top + floor, "mean_damage": float(sim.get("damage").mean()),
                    "kinetic_energy_j": float(0.5 * mass * np.sum(v * v))})
        if len(log) % max(1, 5000 // unit) == 0 or done == wl.steps:
            print(shape, json.dumps(log[-1]), flush=True)
    out["compression"] = {"steps": done, "status": status, "seconds": time.perf_counter() - t0,
                          "ms_per_step": 1e3 * (time.perf_counter() - t0) / max(done, 1), "log": log}
    sim.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--shapes", default=",".join(I.SHAPES))
    ap.add_argument("--grid", default="5",
                    help="grains per side, or nx,ny,nz (1: one grain in the box; 1,1,2: two stacked)")
    ap.add_argument("--cavity", type=float, default=0.5, help="shell cavity radius over the outer radius")
    ap.add_argument("--h", type=float, default=1e-4, help="lattice spacing [m] (grain radius 1 mm)")
    ap.add_argument("--dt", type=float, default=1e-8, help="time step [s]")
    ap.add_argument("--log-steps", type=int, default=500, help="steps between log entries (500: 5 us at 10 ns)")
    ap.add_argument("--duration", type=float, default=5e-4, help="simulated seconds (the paper plots 500 us)")
    ap.add_argument("--time-steps", type=int, default=200, help="steps timed per bond path")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--damping", type=float, default=6.7e21,
                    help="normal contact damping beta_d (Sec. 3.4); the representative volume's "
                         "2.8e22 at h = 70 um scaled by h^-4 to h = 100 um")
    ap.add_argument("--rebuild-every", type=int, default=5)
    ap.add_argument("--skin", type=float, default=0.4,
                    help="Verlet skin in lattice spacings (below sqrt(2) - 0.95, so the own-grain "
                         "candidates of self-contact are the six face neighbours until a grain deforms)")
    ap.add_argument("--capacity", type=int, default=48,
                    help="contact candidates per node (own-grain neighbours count with self-contact)")
    ap.add_argument("--self-contact", type=int, default=1, choices=(0, 1),
                    help="contact between fragments of one grain (Sec. 5)")
    ap.add_argument("--wall-corners", type=int, default=1, choices=(0, 1),
                    help="inclusion-exclusion of the box's walls at its edges and corners (Sec. 4.1.1)")
    ap.add_argument("--out", default=None, help="write every shape's full log to this JSON file")
    a = ap.parse_args(argv)
    a.grid = int(a.grid) if "," not in a.grid else tuple(int(v) for v in a.grid.split(","))
    results = []
    for shape in a.shapes.split(","):
        results.append(run_shape(shape, a))
        if a.out:
            with open(a.out, "w") as fh:
                json.dump(results, fh)
    print(json.dumps({"shape_study": [{k: r[k] for k in r if k != "compression"} |
                                      {"compression": {k: v for k, v in r["compression"].items() if k != "log"},
                                       "peak_bulk_strength_n": max((e["bulk_strength_n"] for e in
                                                                    r["compression"]["log"]), default=0.0)}
                                      for r in results]}), flush=True)
    return results


if __name__ == "__main__":
    from paper_2506_05362_amd.shape_study import main as _main
    _main()
