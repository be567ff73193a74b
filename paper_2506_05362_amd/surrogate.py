"""Surrogate of the bulk stress-strain response of a representative volume.

The paper's study of aggregate size (Sec. 7.5) finds that the normalised
platen force stops changing once an aggregate holds enough grains, i.e. such
an aggregate behaves as a representative volume.  This module generates
confined-compression paths of such volumes with the simulator (libpd_mi355x),
trains a small network on them with the matrix-core kernels of libpd_mlp, and
evaluates it against held-out simulations and against a no-network baseline.

Conventions (compression positive, geomechanics sign):
  strain  e = (e_xx, e_yy, e_zz, g_yz, g_xz, g_xy), e_ii = (L_i0 - L_i) / L_i0 from
          the distance L_i between the two walls normal to axis i;
  stress  s = (s_xx, s_yy, s_zz, s_yz, s_xz, s_xy), s_ii = mean of the two walls'
          normal stress -(P_w . n_w) / A_w averaged over the logging interval
          through the wall impulse, A_w the initial wall area;
  damage  D = mean over nodes of the nodal damage (bond-loss fraction).
The walls of the rig are frictionless planes normal to the axes, so the shear
components of both are zero on every path.

Everything numerical on the path runs in the HIP libraries; PyTorch holds the
device buffers and streams, NumPy does the logging arithmetic on a few numbers
per logged step, and SciPy only for the interpolation baseline.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import time
from typing import Dict, List, Optional

import numpy as np

from . import inputs as I

DIMS = [6, 256, 256, 256, 7]
OUT_NAMES = ["s_xx", "s_yy", "s_zz", "s_yz", "s_xz", "s_xy", "damage"]
AXIAL = 2  # index of s_zz
# Contact candidates per node the simulations reserve: past the peak, crushed
# grains pack fragments within R_c + skin of a node from several sides (at
# 48, four of 64 paths at 15-20 MPa filled the list between 3.5% and 4.9%).
SIM_CAPACITY = 96


@dataclasses.dataclass
class PathSpec:
    seed: int
    confinement: float  # lateral servo target [Pa]


def path_specs(n_paths: int, seed: int = 0, max_confinement: float = 20e6) -> List[PathSpec]:
    """Aggregate seeds 0..n-1, confinement ~ U(0, max) from one seeded stream."""
    rng = np.random.default_rng(seed + 1000003)
    conf = rng.uniform(0.0, max_confinement, size=n_paths)
    return [PathSpec(seed=seed + k, confinement=float(conf[k])) for k in range(n_paths)]


def _axis_walls(wl) -> List[tuple]:
    """(plus, minus) wall indices for each axis: normals +e_i and -e_i."""
    pairs = []
    for ax in range(3):
        plus = minus = None
        for k, w in enumerate(wl.walls):
            n = np.asarray(w.normal, dtype=np.float64)
            if abs(n[ax] - 1.0) < 1e-12:
                plus = k
            elif abs(n[ax] + 1.0) < 1e-12:
                minus = k
        if plus is None or minus is None:
            raise ValueError("the rig needs two walls normal to every axis")
        pairs.append((plus, minus))
    return pairs


def simulate_path(wl, n_log: int = 400, log=None, capacity: int = SIM_CAPACITY) -> Dict[str, np.ndarray]:
    """Run a confined-compression workload and log strain, stress and damage.

    Returns strain (T, 6), target (T, 7) = stress and damage, t (T,), the
    wall-clock seconds of the whole simulation (context set up, bonds built,
    every step run and logged), the steps run and the early candidate
    rebuilds.  When the simulator flags a step chunk (a non-finite force, a
    node through a wall, a full candidate list, or without early rebuilds a
    node that outran the contact skin), the path ends at the last good log
    point and is marked truncated.
    """
    import torch
    from . import pd
    pairs = _axis_walls(wl)
    normals = np.array([w.normal for w in wl.walls], dtype=np.float64)
    areas = np.array([w.area for w in wl.walls], dtype=np.float64)
    t0 = time.perf_counter()
    sim = pd.Sim(wl, candidate_capacity_per_node=capacity)
    try:  # the tessellated volume shares one lattice: the tiled bond loop covers it in one box
        sim.set_launch(bond_path=pd.BONDS_TILES)
    except pd.PDError:
        pass
    nnz = sim.info()["nnz"]
    dmg = torch.empty(wl.n_nodes, dtype=torch.float64, device="cuda")
    off0 = sim.get("wall_offset")
    L0 = np.array([-off0[m] - off0[p] for p, m in pairs])
    imp_prev = sim.get("wall_impulse")
    strain, target, times = [], [], []
    done, truncated = 0, False
    while done + n_log <= wl.steps:
        try:
            sim.step(n_log)
        except pd.PDError as e:
            truncated = True
            if log:
                log(f"  stopped after step {done}: {e}")
            break
        done += n_log
        off = sim.get("wall_offset")
        imp = sim.get("wall_impulse")
        sim.get_device("damage", dmg.data_ptr(), 8 * wl.n_nodes)
        force = (imp - imp_prev) / (n_log * wl.params.dt)
        imp_prev = imp
        sig_w = -np.sum(force * normals, axis=1) / areas
        L = np.array([-off[m] - off[p] for p, m in pairs])
        e = np.zeros(6)
        e[:3] = (L0 - L) / L0
        s = np.zeros(7)
        for ax, (p, m) in enumerate(pairs):
            s[ax] = 0.5 * (sig_w[p] + sig_w[m])
        s[6] = float(dmg.mean().item())
        strain.append(e)
        target.append(s)
        times.append(done * wl.params.dt)
    seconds = time.perf_counter() - t0
    early = sim.loop_counts()["early_rebuilds"]
    sim.close()
    return {"strain": np.array(strain).reshape(-1, 6), "target": np.array(target).reshape(-1, 7),
            "t": np.array(times), "seconds": seconds, "nodes": wl.n_nodes, "bonds": nnz,
            "steps_run": done, "steps": wl.steps, "truncated": truncated, "early_rebuilds": early}


def _make_rve(args):
    seed, confinement, kw = args
    return I.rve_aggregate(seed=seed, confinement=confinement, **kw)


def generate(specs: List[PathSpec], n_log: int = 400, log=print, workers: int = 6,
             **rve_kw) -> Dict[str, np.ndarray]:
    """Simulate every path.  Paths have different lengths (truncation), so the
    samples are stored flat with offsets[p]:offsets[p+1] selecting path p.

    Host processes lay out the next aggregates while the GPU runs the current one."""
    import concurrent.futures as cf
    import multiprocessing as mp
    res, kept = [], []
    jobs = [(sp.seed, sp.confinement, rve_kw) for sp in specs]
    with cf.ProcessPoolExecutor(max_workers=max(1, workers),
                                mp_context=mp.get_context("spawn")) as pool:
        for k, (sp, wl) in enumerate(zip(specs, pool.map(_make_rve, jobs))):
            r = simulate_path(wl, n_log=n_log, log=log)
            tag = "truncated" if r["truncated"] else "complete"
            last = (f"e_zz {r['strain'][-1, AXIAL] * 100:.2f} % s_zz {r['target'][-1, AXIAL] / 1e6:.2f} MPa "
                    f"D {r['target'][-1, 6]:.4f}") if len(r["t"]) else "no samples"
            log(f"path {k}: seed {sp.seed} conf {sp.confinement / 1e6:.2f} MPa nodes {wl.n_nodes} "
                f"bonds {r['bonds']} steps {r['steps_run']}/{r['steps']} {tag} "
                f"early rebuilds {r['early_rebuilds']} sim {r['seconds']:.2f} s; "
                f"end {last}")
            if len(r["t"]) >= 2:
                res.append(r)
                kept.append(sp)
    lens = [len(r["t"]) for r in res]
    offsets = np.zeros(len(res) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(lens)
    return {"strain": np.concatenate([r["strain"] for r in res]),
            "target": np.concatenate([r["target"] for r in res]),
            "t": np.concatenate([r["t"] for r in res]), "offsets": offsets,
            "seconds": np.array([r["seconds"] for r in res]),
            "steps_run": np.array([r["steps_run"] for r in res]),
            "steps": np.array([r["steps"] for r in res]),
            "truncated": np.array([r["truncated"] for r in res]),
            "early_rebuilds": np.array([r["early_rebuilds"] for r in res], dtype=np.int64),
            "nodes": np.array([r["nodes"] for r in res]), "bonds": np.array([r["bonds"] for r in res]),
            "confinement": np.array([sp.confinement for sp in kept]),
            "seed": np.array([sp.seed for sp in kept]),
            "dropped": np.array(sorted(set(sp.seed for sp in specs) - set(sp.seed for sp in kept)),
                                dtype=np.int64)}


def path(data, p: int, key: str) -> np.ndarray:
    o = data["offsets"]
    return data[key][o[p]:o[p + 1]]


def samples(data, paths: np.ndarray, key: str) -> np.ndarray:
    return np.concatenate([path(data, int(p), key) for p in paths])


@dataclasses.dataclass
class Scaler:
    mean: np.ndarray
    std: np.ndarray

    @staticmethod
    def fit(a: np.ndarray) -> "Scaler":
        m = a.mean(axis=0)
        s = a.std(axis=0)
        s = np.where(s > 1e-12 * max(1.0, float(np.abs(a).max())), s, 1.0)
        return Scaler(m, s)

    def fwd(self, a):
        return (a - self.mean) / self.std

    def inv(self, a):
        return a * self.std + self.mean


def init_params(dims, seed=0) -> np.ndarray:
    """Weights and biases ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)), in the library's
    parameter order (held-out error about 0.3 points lower than with He-uniform
    weights on the representative-volume data)."""
    rng = np.random.default_rng(seed)
    parts = []
    for a, b in zip(dims[:-1], dims[1:]):
        lim = 1.0 / math.sqrt(a)
        parts.append(rng.uniform(-lim, lim, size=a * b))
        parts.append(rng.uniform(-lim, lim, size=b))
    return np.concatenate(parts).astype(np.float32)


class Surrogate:
    """Standardisation + the matrix-core network of libpd_mlp."""

    def __init__(self, dims=DIMS, max_batch: int = 65536, seed: int = 0):
        from . import mlp
        self.dims = list(dims)
        self.net = mlp.Net(self.dims, max_batch=max_batch)
        self.net.set_params(init_params(self.dims, seed))
        self.xs: Optional[Scaler] = None
        self.ys: Optional[Scaler] = None

    def fit(self, X: np.ndarray, Y: np.ndarray, steps: int = 4000, batch: int = 512,
            lr: float = 2e-3, lr_min: float = 2e-5, weight_decay: float = 1e-2,
            axial_weight: float = 2.0, seed: int = 0, log=None) -> List[float]:
        """Adam with decoupled weight decay on the standardised MSE, cosine
        learning-rate decay, minibatches drawn without replacement per epoch.
        The axial stress is standardised with its scale divided by axial_weight,
        which weights its squared error axial_weight^2 times in the mean."""
        import torch
        self.net.set_adam(weight_decay=weight_decay)
        self.xs, self.ys = Scaler.fit(X), Scaler.fit(Y)
        self.ys.std = self.ys.std.copy()
        self.ys.std[AXIAL] /= axial_weight
        self.lo, self.hi = X.min(axis=0), X.max(axis=0)
        net = self.net
        g = torch.Generator(device="cpu").manual_seed(seed)
        losses = []
        with torch.cuda.stream(net.stream):
            xd = torch.tensor(self.xs.fwd(X), dtype=torch.float32, device="cuda")
            yd = torch.tensor(self.ys.fwd(Y), dtype=torch.float32, device="cuda")
            n = xd.shape[0]
            b = min(batch, n)
            perm = torch.randperm(n, generator=g).cuda()
            pos = 0
            for it in range(steps):
                if pos + b > n:
                    perm = torch.randperm(n, generator=g).cuda()
                    pos = 0
                idx = perm[pos:pos + b]
                pos += b
                xb = xd.index_select(0, idx)
                yb = yd.index_select(0, idx)
                rate = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * it / steps))
                want = (it % 100 == 0) or it == steps - 1
                loss = net.train_step(xb, yb, rate, want_loss=want)
                if want:
                    losses.append(loss)
                    if log:
                        log(f"train step {it}: loss {loss:.3e} lr {rate:.2e}")
        torch.cuda.synchronize()
        return losses

    def in_envelope(self, X: np.ndarray, pad: float = 0.05) -> np.ndarray:
        """True where a query lies inside the training inputs' per-component range
        (padded by a fraction of it); queries outside go to the full simulation."""
        lo, hi = self.lo, self.hi
        w = np.maximum(hi - lo, 0.0) * pad
        return np.all((X >= lo - w) & (X <= hi + w), axis=1)

    def predict_device(self, x_std):
        """x_std: standardised (B, 6) float32 device tensor -> standardised outputs."""
        return self.net.forward(x_std)

    def predict(self, X: np.ndarray) -> np.ndarray:
        import torch
        xd = torch.tensor(self.xs.fwd(X), dtype=torch.float32, device="cuda")
        y = self.net.forward(xd)
        self.net.stream.synchronize()
        return self.ys.inv(y.cpu().numpy().astype(np.float64))


class SurrogateEnsemble:
    """The mean prediction of networks trained alike from different initial
    weights and minibatch orders; the envelope is the first one's (all saw the
    same inputs)."""

    def __init__(self, members: List["Surrogate"]):
        self.members = members

    def predict(self, X: np.ndarray) -> np.ndarray:
        return np.mean([m.predict(X) for m in self.members], axis=0)

    def in_envelope(self, X: np.ndarray, pad: float = 0.05) -> np.ndarray:
        return self.members[0].in_envelope(X, pad)


def rel_l2(pred: np.ndarray, ref: np.ndarray) -> float:
    return float(np.linalg.norm(pred - ref) / max(np.linalg.norm(ref), 1e-300))


def interpolation_baseline(Xtr: np.ndarray, ytr: np.ndarray, Xq: np.ndarray) -> np.ndarray:
    """No-network baseline: piecewise-linear interpolation of the training samples
    over the three normal strains (nearest sample outside their convex hull)."""
    from scipy.interpolate import LinearNDInterpolator, NearestNDInterpolator
    out = LinearNDInterpolator(Xtr[:, :3], ytr)(Xq[:, :3])
    bad = ~np.isfinite(out)
    if bad.any():
        out[bad] = NearestNDInterpolator(Xtr[:, :3], ytr)(Xq[bad, :3])
    return out


def ensemble_prediction(data, p: int, train: np.ndarray, k: int = 4) -> np.ndarray:
    """Axial stress of path p predicted as the mean of the k training paths whose
    confinement is nearest, each interpolated along the axial strain: what the
    loading parameters alone fix, without the held-out aggregate's own scatter."""
    conf = np.asarray(data["confinement"])
    e = path(data, p, "strain")[:, AXIAL]
    near = train[np.argsort(np.abs(conf[train] - conf[p]), kind="stable")[:k]]
    return np.mean([np.interp(e, path(data, int(q), "strain")[:, AXIAL], path(data, int(q), "target")[:, AXIAL])
                    for q in near], axis=0)


def pair_scatter(data, paths: np.ndarray) -> Dict:
    """The scatter between aggregates loaded alike, from the simulated paths
    alone: sorted by confinement, each neighbouring pair's relative L2
    difference of the axial stress along their common axial strains (the norm
    of the difference over the root mean square of the two paths' norms).  If
    every path deviates independently from one function of strain and
    confinement, one path lies about 1/sqrt(2) of that difference from it: an
    error no predictor of the loading alone gets below."""
    conf = np.asarray(data["confinement"])
    paths = np.asarray(paths)
    order = paths[np.argsort(conf[paths], kind="stable")]
    diffs, gaps = [], []
    for p, q in zip(order[:-1], order[1:]):
        ea, a = path(data, int(p), "strain")[:, AXIAL], path(data, int(p), "target")[:, AXIAL]
        eb, b = path(data, int(q), "strain")[:, AXIAL], path(data, int(q), "target")[:, AXIAL]
        keep = ea <= eb.max()  # a path stopped early covers fewer strains
        a, b = a[keep], np.interp(ea[keep], eb, b)
        norm = np.sqrt(0.5 * (np.dot(a, a) + np.dot(b, b)))
        diffs.append(float(np.linalg.norm(a - b) / max(norm, 1e-300)))
        gaps.append(float(abs(conf[p] - conf[q])))
    d = float(np.mean(diffs))
    return {"pair_axial_rel_l2_mean": d, "pair_confinement_gap_mean": float(np.mean(gaps)),
            "single_path_scatter": d / math.sqrt(2.0)}


def evaluate(sur: "Surrogate", data, held: np.ndarray, train: np.ndarray, prepeak_strain: float = 0.025) -> Dict:
    """Per held-out path: relative L2 error of the axial stress along the path,
    for the network, the interpolation baseline and the confinement ensemble
    (the scatter between aggregates loaded alike), over the whole path and up to
    prepeak_strain axial strain."""
    errs, errs_lat, errs_dmg, base, ens, errs_pre, base_pre = [], [], [], [], [], [], []
    Xtr = samples(data, train, "strain")
    ytr = samples(data, train, "target")
    for p in held:
        X = path(data, int(p), "strain")
        Y = path(data, int(p), "target")
        P = sur.predict(X)
        errs.append(rel_l2(P[:, AXIAL], Y[:, AXIAL]))
        errs_lat.append(rel_l2(P[:, :2], Y[:, :2]))
        errs_dmg.append(float(np.abs(P[:, 6] - Y[:, 6]).max()))
        B = interpolation_baseline(Xtr, ytr[:, AXIAL], X)
        base.append(rel_l2(B, Y[:, AXIAL]))
        ens.append(rel_l2(ensemble_prediction(data, int(p), train), Y[:, AXIAL]))
        pre = X[:, AXIAL] <= prepeak_strain
        errs_pre.append(rel_l2(P[pre, AXIAL], Y[pre, AXIAL]))
        base_pre.append(rel_l2(B[pre], Y[pre, AXIAL]))
    return {"axial_rel_l2": errs, "axial_rel_l2_mean": float(np.mean(errs)),
            "axial_rel_l2_max": float(np.max(errs)),
            "lateral_rel_l2_mean": float(np.mean(errs_lat)),
            "damage_abs_max": float(np.max(errs_dmg)),
            "interp_axial_rel_l2": base, "interp_axial_rel_l2_mean": float(np.mean(base)),
            "ensemble_axial_rel_l2": ens, "ensemble_axial_rel_l2_mean": float(np.mean(ens)),
            "prepeak_strain": prepeak_strain,
            "axial_rel_l2_prepeak": errs_pre, "axial_rel_l2_prepeak_mean": float(np.mean(errs_pre)),
            "interp_axial_rel_l2_prepeak_mean": float(np.mean(base_pre))}


def inference_paths(data, train: np.ndarray, n_paths: int, T: int = 100, seed: int = 7) -> np.ndarray:
    """Seeded strain paths for the throughput measurement: T points of axial strain
    from 0 to the smallest final axial strain of the complete training paths;
    each path's lateral strains blend those of two training paths of
    neighbouring confinement with a seeded weight."""
    rng = np.random.default_rng(seed)
    full = [int(p) for p in train if not data["truncated"][int(p)]] or [int(p) for p in train]
    full.sort(key=lambda p: data["confinement"][p])
    top = min(float(path(data, p, "strain")[-1, AXIAL]) for p in full)
    a = np.linspace(0.0, top, T)
    lat = []
    for p in full:
        S = path(data, p, "strain")
        lat.append(np.stack([np.interp(a, S[:, AXIAL], S[:, ax]) for ax in (0, 1)], axis=1))
    lat = np.stack(lat)  # (P, T, 2)
    k = rng.integers(0, max(len(full) - 1, 1), size=n_paths)
    k2 = np.minimum(k + 1, len(full) - 1)
    w = rng.uniform(0.0, 1.0, size=n_paths)[:, None, None]
    out = np.zeros((n_paths, T, 6), dtype=np.float32)
    out[:, :, AXIAL] = a[None, :]
    out[:, :, :2] = (1 - w) * lat[k] + w * lat[k2]
    return out


def time_inference(sur: Surrogate, paths: np.ndarray, reps: int = 3) -> Dict:
    """GPU seconds for all paths as one batch (inputs resident in HBM)."""
    import torch
    B = paths.shape[0] * paths.shape[1]
    x = torch.tensor(sur.xs.fwd(paths.reshape(B, 6)), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    sur.predict_device(x)
    sur.net.stream.synchronize()
    best = math.inf
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(sur.net.stream)
        sur.predict_device(x)
        b.record(sur.net.stream)
        b.synchronize()
        best = min(best, a.elapsed_time(b) * 1e-3)
    flops = 2.0 * sum(i * o for i, o in zip(sur.dims[:-1], sur.dims[1:])) * B
    return {"samples": B, "paths": int(paths.shape[0]), "T": int(paths.shape[1]),
            "seconds": best, "seconds_per_path": best / paths.shape[0],
            "tflops": flops / best / 1e12}


# Loading of the representative volume: the platen moves slowly enough that the
# compaction front crosses the sample many times during the path, and normal
# contact damping at about half the critical value of a node pair (h = 70 um)
# lets grain rattling decay, so the logged stress is a quasi-static response.
# The servo gain caps the lateral walls' speed near the platen's (gain * 20 MPa
# = 1 m/s).  Paths run to 5% axial strain, well past the peak; candidate lists
# are rebuilt every 10 steps with a skin of h/2, so a node may move at up to
# 250 m/s between rebuilds, and earlier for the single detached nodes thrown
# off faster than that past the peak (a rebuild as soon as one has moved h/4).
RVE_DEFAULTS = dict(platen_speed=1.0, contact_damping=2.8e22, servo_gain=5e-8, rebuild_every=10,
                    axial_strain=0.05, skin_factor=0.5, adaptive_rebuild=True)


def load_data(files: List[str]) -> Dict[str, np.ndarray]:
    """Paths saved by earlier runs (their _data.npz), joined in the given order."""
    parts = []
    for fn in files:
        with np.load(fn) as f:
            parts.append({k: f[k] for k in f.files})
    if len(parts) == 1:
        return parts[0]
    flat = ("strain", "target", "t")
    per_path = ("seconds", "steps_run", "steps", "truncated", "nodes", "bonds", "confinement", "seed",
                "early_rebuilds")
    out = {k: np.concatenate([d[k] for d in parts]) for k in flat + per_path if all(k in d for d in parts)}
    lens = np.concatenate([np.diff(d["offsets"]) for d in parts])
    out["offsets"] = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    out["dropped"] = np.concatenate([d["dropped"] for d in parts]).astype(np.int64)
    return out


def run(n_paths: int = 64, n_held: int = 8, n_log: int = 400, train_steps: int = 4000,
        infer_paths: int = 100000, infer_T: int = 100, seed: int = 0, out: Optional[str] = None,
        log=print, data_file: Optional[str] = None, only: Optional[tuple] = None, nets: int = 1,
        **rve_kw) -> Dict:
    """The whole study; with only = (a, b), just simulate paths a..b-1 of the
    n_paths path set and save them (to join later with data_file).  nets > 1
    trains that many networks (seeds seed, seed + 1, ...) and evaluates their
    mean, beside the first one alone."""
    rve_kw = {**RVE_DEFAULTS, **rve_kw}
    t0 = time.perf_counter()
    if only is not None:
        data = generate(path_specs(n_paths, seed=seed)[only[0]:only[1]], n_log=n_log, log=log, **rve_kw)
        res = {"paths": f"{only[0]}:{only[1]} of {n_paths}", "rve": dict(rve_kw),
               "generate_seconds": time.perf_counter() - t0, "paths_used": len(data["offsets"]) - 1,
               "paths_truncated": int(np.sum(data["truncated"])),
               "early_rebuilds": int(np.sum(data["early_rebuilds"]))}
        if out:
            with open(out, "w") as f:
                json.dump(res, f, indent=1)
            np.savez_compressed(out.replace(".json", "_data.npz"), **data)
        return res
    if data_file:
        # paths generated earlier (the _data.npz files earlier runs wrote), comma-separated
        data = load_data(data_file.split(","))
    else:
        data = generate(path_specs(n_paths, seed=seed), n_log=n_log, log=log, **rve_kw)
    gen_s = time.perf_counter() - t0
    n_ok = len(data["offsets"]) - 1
    held = np.arange(n_ok - n_held, n_ok)
    train = np.arange(0, n_ok - n_held)
    X = samples(data, train, "strain")
    Y = samples(data, train, "target")
    members = []
    t1 = time.perf_counter()
    for k in range(max(1, nets)):
        m = Surrogate(seed=seed + k)
        lk = m.fit(X, Y, steps=train_steps, seed=seed + k, log=log if k == 0 else None)
        if k == 0:
            losses = lk
        members.append(m)
    train_s = time.perf_counter() - t1
    sur = members[0] if len(members) == 1 else SurrogateEnsemble(members)
    ev = evaluate(sur, data, held, train)
    if len(members) > 1:
        one = evaluate(members[0], data, held, train)
        ev["first_network"] = {k: one[k] for k in ("axial_rel_l2", "axial_rel_l2_mean",
                                                   "axial_rel_l2_prepeak_mean")}
    paths = inference_paths(data, train, infer_paths, T=infer_T)
    inside = float(sur.in_envelope(paths.reshape(-1, 6)).mean())
    inf = time_inference(members[0], paths)
    if len(members) > 1:  # each network runs the whole batch
        inf = {**inf, "networks": len(members), "seconds": inf["seconds"] * len(members),
               "seconds_per_path": inf["seconds_per_path"] * len(members)}
    # GPU seconds of one full path: per-step cost of each run times its length
    per_path = data["seconds"] / np.maximum(data["steps_run"], 1) * data["steps"]
    sim_per_path = float(np.mean(per_path))
    res = {
        "paths": n_paths, "paths_used": n_ok, "paths_dropped": data["dropped"].tolist(),
        "paths_truncated": int(np.sum(data["truncated"])), "held_out": n_held,
        "early_rebuilds": int(np.sum(data["early_rebuilds"])) if "early_rebuilds" in data else None,
        "samples": int(len(data["t"])), "rve": {k: v for k, v in rve_kw.items()},
        "nodes_mean": float(np.mean(data["nodes"])), "bonds_mean": float(np.mean(data["bonds"])),
        "steps_per_path": int(np.max(data["steps"])),
        "generate_seconds": gen_s, "sim_seconds_per_path": sim_per_path,
        "train_seconds": train_s, "train_steps": train_steps, "final_loss": losses[-1], "nets": len(members),
        **ev, "scatter_of_training_paths": pair_scatter(data, train),
        "inference": inf, "inference_inside_envelope": inside,
        "speedup_per_path": sim_per_path / inf["seconds_per_path"],
        "paths_simulated_in_inference_time": inf["seconds"] / sim_per_path,
    }
    if data_file:
        res["data_file"] = ",".join(os.path.basename(f) for f in data_file.split(","))
    if out:
        with open(out, "w") as f:
            json.dump(res, f, indent=1)
        if not data_file:
            np.savez_compressed(out.replace(".json", "_data.npz"), **data)
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--paths", type=int, default=64)
    ap.add_argument("--held", type=int, default=8)
    ap.add_argument("--log-every", type=int, default=400)
    ap.add_argument("--platen-speed", type=float, default=RVE_DEFAULTS["platen_speed"])
    ap.add_argument("--train-steps", type=int, default=4000)
    ap.add_argument("--infer-paths", type=int, default=100000)
    ap.add_argument("--grains", type=int, default=200)
    ap.add_argument("--nodes-per-grain", type=float, default=1850.0)
    ap.add_argument("--out", default=None)
    ap.add_argument("--data", default=None, metavar="NPZ[,NPZ...]",
                    help="train and evaluate on paths earlier runs saved (their _data.npz, joined in order) "
                         "instead of simulating")
    ap.add_argument("--nets", type=int, default=1,
                    help="train this many networks from different seeds and evaluate their mean")
    ap.add_argument("--only", default=None, metavar="A:B",
                    help="only simulate paths A..B-1 of the --paths set and save them (no training)")
    ap.add_argument("--scatter", default=None, metavar="NPZ[,NPZ...]",
                    help="only print the scatter between neighbouring-confinement paths of saved data "
                         "(all but the last --held paths) and exit; runs on the host alone")
    ap.add_argument("--time-path", type=int, default=0, metavar="STEPS",
                    help="only time STEPS steps (after as many warm-up steps) of path 1 and exit")
    ap.add_argument("--time-inference", type=int, default=0, metavar="PATHS",
                    help="only time inference of PATHS random strain paths x 100 points with the "
                         "fused and the layer-by-layer kernels (random weights) and exit")
    a = ap.parse_args(argv)
    if a.scatter:
        data = load_data(a.scatter.split(","))
        n_ok = len(data["offsets"]) - 1
        print(json.dumps(pair_scatter(data, np.arange(0, n_ok - a.held))), flush=True)
        return
    if a.time_inference:
        rng = np.random.default_rng(0)
        sur = Surrogate()
        sur.xs = Scaler(np.zeros(6), np.ones(6))
        sur.ys = Scaler(np.zeros(7), np.ones(7))
        paths = rng.normal(size=(a.time_inference, 100, 6)).astype(np.float32)
        out = {}
        for name, fused in (("fused", True), ("layers", False)):
            sur.net.set_inference(fused)
            out[name] = time_inference(sur, paths)
        print(json.dumps(out), flush=True)
        return
    if a.time_path:
        from . import pd
        sp = path_specs(2)[1]
        wl = I.rve_aggregate(seed=sp.seed, confinement=sp.confinement,
                             **{**RVE_DEFAULTS, "n_grains": a.grains, "nodes_per_grain": a.nodes_per_grain})
        sim = pd.Sim(wl, candidate_capacity_per_node=SIM_CAPACITY)
        try:  # the launch the path generation uses
            sim.set_launch(bond_path=pd.BONDS_TILES)
        except pd.PDError:
            pass
        sim.step(a.time_path)
        t0 = time.perf_counter()
        sim.step(a.time_path)  # returns when the GPU is done
        ms = (time.perf_counter() - t0) / a.time_path * 1e3
        print(json.dumps({"ms_per_step": ms, **sim.info(), **sim.loop_counts(),
                          "bond_path": sim.get_launch()["bond_path"]}), flush=True)
        sim.close()
        return
    res = run(n_paths=a.paths, n_held=a.held, n_log=a.log_every, train_steps=a.train_steps,
              infer_paths=a.infer_paths, out=a.out, n_grains=a.grains,
              nodes_per_grain=a.nodes_per_grain, platen_speed=a.platen_speed,
              log=lambda s: print(s, flush=True), data_file=a.data,
              only=tuple(int(v) for v in a.only.split(":")) if a.only else None, nets=a.nets)
    print(json.dumps({k: v for k, v in res.items() if not isinstance(v, list)}), flush=True)


if __name__ == "__main__":
    # run through the package module so worker processes can import the helpers
    from paper_2506_05362_amd.surrogate import main as _main
    _main()
