"""Launch autotuner of the step loop (libpd_mi355x's pd_set_launch).

For one simulation context it times every candidate launch configuration -
step-loop mode (captured graph, persistent cooperative kernel at full
residency or one workgroup per compute unit), 64-node slices per workgroup,
the XCD-aware workgroup order and the bond path (sliced rows or LDS tiles) - on the context's own state, keeps the fastest and restores the
state it started from, so tuning changes nothing but speed (every candidate
computes bitwise the same node state; the tile path is left out when a wall is
servo-controlled, since its wall reactions, and through them the servo, agree
with the slice path only to rounding).

Results are cached in a JSON file keyed by the GPU architecture, the node and
bond counts and a histogram of grain sizes (log2 bins), so a later context of
the same shape skips the measurement.  The cache path is the PD_TUNE_CACHE
environment variable, else ~/.cache/paper_2506_05362_amd/launch.json.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, Iterable, List, Optional

import numpy as np

from . import inputs as I
from . import pd

PERSISTENT_ONE_PER_CU = 256  # MI355X compute units

DEFAULT = dict(loop=pd.LOOP_GRAPH, slices_per_block=4, xcd_remap=1, persistent_blocks=0,
               bond_path=pd.BONDS_SLICES)


def cache_path() -> str:
    p = os.environ.get("PD_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2506_05362_amd", "launch.json")


def shape_key(arch: str, n_nodes: int, nnz: int, grain_sizes: Iterable[int]) -> str:
    """Cache key: architecture, node and bond counts, grain-size histogram."""
    sizes = np.asarray(list(grain_sizes), dtype=np.int64)
    bins = np.bincount(np.floor(np.log2(np.maximum(sizes, 1))).astype(np.int64), minlength=1)
    hist = ",".join(str(int(b)) for b in bins)
    return f"{arch}|n={int(n_nodes)}|nnz={int(nnz)}|g={hist}"


def candidates(persistent: bool = True, tiles: bool = True) -> List[Dict[str, int]]:
    out = [dict(loop=pd.LOOP_GRAPH, slices_per_block=spb, xcd_remap=x, persistent_blocks=0,
                bond_path=pd.BONDS_SLICES) for spb in (1, 2, 4, 8) for x in (1, 0)]
    if persistent:
        # as many workgroups as fit at once (0), or one per compute unit
        out += [dict(loop=pd.LOOP_PERSISTENT, slices_per_block=4, xcd_remap=x, persistent_blocks=nb,
                     bond_path=pd.BONDS_SLICES) for nb in (0, PERSISTENT_ONE_PER_CU) for x in (1, 0)]
    if tiles:
        out += [dict(loop=pd.LOOP_GRAPH, slices_per_block=4, xcd_remap=x, persistent_blocks=0,
                     bond_path=pd.BONDS_TILES) for x in (1, 0)]
    return out


def name_of(cfg: Dict[str, int]) -> str:
    base = f"{pd.LOOP_NAMES[cfg['loop']]}/spb{cfg['slices_per_block']}/xcd{cfg['xcd_remap']}"
    if cfg["loop"] == pd.LOOP_PERSISTENT and cfg.get("persistent_blocks", 0):
        base += f"/wg{cfg['persistent_blocks']}"
    return base + "/tiles" if cfg.get("bond_path", pd.BONDS_SLICES) == pd.BONDS_TILES else base


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path: str, table: dict) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return str(getattr(p, "gcnArchName", p.name))


def time_config(sim: "pd.Sim", cfg: Dict[str, int], steps: int) -> float:
    """Seconds per step of cfg (after one warm-up run of the same length)."""
    sim.set_launch(**cfg)
    sim.step(steps)  # warm-up: graph capture, caches (pd_step returns when the GPU is done)
    t0 = time.perf_counter()
    sim.step(steps)
    return (time.perf_counter() - t0) / steps


def tune(sim: "pd.Sim", steps: Optional[int] = None, use_cache: bool = True,
         persistent: bool = True, path: Optional[str] = None) -> Dict:
    """Pick the fastest launch configuration for sim, apply it and return
    {"config": ..., "key": ..., "cached": bool, "times": {...}}."""
    path = path or cache_path()
    info = sim.info()
    key = shape_key(_arch(), info["n_nodes"], info["nnz"], np.diff(sim.wl.grain_begin))
    # the wall-corner pass runs before every evaluation, and an early candidate
    # rebuild is decided on the host between steps: one persistent launch of
    # several steps can host neither
    if getattr(sim.wl.params, "wall_corners", False) or getattr(sim.wl.params, "adaptive_rebuild", False):
        persistent = False
    table = _load(path) if use_cache else {}
    if use_cache and key in table and (persistent or table[key]["config"]["loop"] != pd.LOOP_PERSISTENT):
        cfg = table[key]["config"]
        sim.set_launch(**cfg)
        return {"config": cfg, "key": key, "cached": True, "times": table[key].get("times", {})}
    R = sim.wl.params.rebuild_every
    graph_len = R if R % 2 == 0 else 2 * R
    if steps is None:
        # at least two graph replays, and about 20 ms of work per measurement
        steps = graph_len * max(2, int(math.ceil(0.02 / max(_quick_step_estimate(sim), 1e-6) / graph_len)))
    start = sim.get_state()
    before = sim.get_launch()
    tiles = not any(w.mode == I.WALL_SERVO for w in sim.wl.walls)
    cands = candidates(persistent, tiles)
    times = {}
    try:
        for cfg in cands:
            name = name_of(cfg)
            try:
                times[name] = time_config(sim, cfg, steps)
            except pd.PDError as e:
                if e.status == pd.PD_ERR_UNSTABLE:  # the run itself failed: not a tuning matter
                    raise
                times[name] = float("inf")  # a mode this device cannot launch is skipped
            sim.set_state(start)
    finally:
        sim.set_launch(**before)
        sim.set_state(start)
    best_name = min(times, key=times.get)
    cfg = next(c for c in cands if name_of(c) == best_name)
    sim.set_launch(**cfg)
    if use_cache:
        table = _load(path)
        table[key] = {"config": cfg, "times": times, "steps": steps}
        _store(path, table)
    return {"config": cfg, "key": key, "cached": False, "times": times}


def _quick_step_estimate(sim: "pd.Sim") -> float:
    """Rough seconds per step from the bond count (4e11 bond updates/s)."""
    return max(sim.info()["nnz"] / 4e11, 2e-5)
