"""Python binding of the C ABI in include/pd.h (argument marshalling only).

Every step of the simulation runs in the HIP library libpd_mi355x.so; this
module only converts numpy arrays and dataclasses into the ABI's structs.
PyTorch supplies the device allocator and the HIP stream.  There is no
fallback: when the library is missing, importing this module raises.
"""
from __future__ import annotations

import atexit
import sys
import ctypes as C
import weakref
import os
from typing import Optional

import numpy as np

from . import inputs as _inp

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpd_mi355x.so")

PD_OK, PD_ERR_INVALID, PD_ERR_STATE, PD_ERR_OOM, PD_ERR_HIP, PD_ERR_UNSTABLE = 0, -1, -2, -3, -4, -5
PD_ERR_UNSUPPORTED, PD_ERR_CORRUPT = -6, -7
FLAG_TABLE_LITERAL, FLAG_ABS_STRETCH, FLAG_NO_GRAPH, FLAG_CONIC, FLAG_SELF_CONTACT = 1, 2, 4, 8, 16
FLAG_WALL_CORNERS = 32
FLAG_ADAPTIVE_REBUILD = 64

FIELDS = dict(displacement=0, velocity=1, accel=2, force_density=3, damage=4, intact_count=5,
              initial_count=6, bond_rowptr=7, bond_col=8, bond_broken=9, contact_rowptr=10,
              contact_col=11, wall_force=12, wall_offset=13, energy=14, step=15,
              wall_impulse=16)
_FIELD_DTYPE = dict(displacement=np.float64, velocity=np.float64, accel=np.float64,
                    force_density=np.float64, damage=np.float64, intact_count=np.int32,
                    initial_count=np.int32, bond_rowptr=np.int64, bond_col=np.int32,
                    bond_broken=np.uint8, contact_rowptr=np.int64, contact_col=np.int32,
                    wall_force=np.float64, wall_offset=np.float64, energy=np.float64,
                    step=np.int64, wall_impulse=np.float64)

P = C.c_void_p


class pd_material(C.Structure):
    _fields_ = [("bulk_modulus", C.c_double), ("density", C.c_double),
                ("fracture_energy", C.c_double)]


class pd_grains(C.Structure):
    _fields_ = [("n_grains", C.c_int32), ("node_begin", P), ("material", P), ("h", P),
                ("origin", P)]


class pd_mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("X", P), ("ijk", P), ("u0", P), ("v0", P), ("fixed", P)]


class pd_params(C.Structure):
    _fields_ = [("horizon_factor", C.c_int32), ("flags", C.c_int32),
                ("contact_radius", C.c_double), ("contact_horizon", C.c_double),
                ("skin", C.c_double), ("rebuild_every", C.c_int32),
                ("candidate_capacity_per_node", C.c_int32), ("dt", C.c_double),
                ("gravity", C.c_double * 3), ("contact_damping", C.c_double),
                ("friction", C.c_double)]


class pd_wall(C.Structure):
    _fields_ = [("normal", C.c_double * 3), ("offset", C.c_double), ("velocity", C.c_double),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("mode", C.c_int32),
                ("target_stress", C.c_double), ("servo_gain", C.c_double), ("area", C.c_double)]


class pd_launch(C.Structure):
    _fields_ = [("loop", C.c_int32), ("slices_per_block", C.c_int32), ("xcd_remap", C.c_int32),
                ("persistent_blocks", C.c_int32), ("bond_path", C.c_int32)]


LOOP_GRAPH, LOOP_DIRECT, LOOP_PERSISTENT, LOOP_PER_GRAIN = 0, 1, 2, 3
LOOP_NAMES = {LOOP_GRAPH: "graph", LOOP_DIRECT: "direct", LOOP_PERSISTENT: "persistent",
              LOOP_PER_GRAIN: "per_grain"}
BONDS_SLICES, BONDS_TILES = 0, 1
BOND_PATH_NAMES = {BONDS_SLICES: "slices", BONDS_TILES: "tiles"}


class pd_cut(C.Structure):
    _fields_ = [("kind", C.c_int32), ("grain", C.c_int32), ("plane", C.c_int64 * 4),
                ("lo", C.c_int64 * 3), ("hi", C.c_int64 * 3), ("center", C.c_int64 * 3),
                ("radius2", C.c_int64)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

EXPORTS = ["pd_init", "pd_build_bonds", "pd_step", "pd_field_bytes", "pd_get", "pd_set_wall",
           "pd_get_state", "pd_set_state", "pd_info", "pd_set_timing", "pd_timing", "pd_destroy",
           "pd_last_error", "pd_status_string", "pd_set_launch", "pd_get_launch"]


def load_library(path: str = _LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is not built; run __graft_entry__.build()")
    # PyTorch ships its own HIP runtime with the same soname; loading it first
    # makes the library bind to that one instead of a second runtime instance.
    import torch  # noqa: F401
    L = C.CDLL(path)
    L.pd_init.argtypes = [C.POINTER(P), C.POINTER(pd_grains), C.POINTER(pd_mesh),
                          C.POINTER(pd_material), C.c_int32, C.POINTER(pd_params),
                          C.POINTER(pd_wall), C.c_int32, ALLOC_FN, FREE_FN, P, P]
    L.pd_build_bonds.argtypes = [P, C.POINTER(pd_cut), C.c_int32]
    L.pd_step.argtypes = [P, C.c_int64]
    L.pd_field_bytes.argtypes = [P, C.c_int32, C.POINTER(C.c_int64)]
    L.pd_get.argtypes = [P, C.c_int32, P, C.c_int64, C.c_int32]
    L.pd_set_wall.argtypes = [P, C.c_int32, C.POINTER(pd_wall)]
    L.pd_get_state.argtypes = [P, P, C.POINTER(C.c_int64)]
    L.pd_set_state.argtypes = [P, P, C.c_int64]
    L.pd_info.argtypes = [P, P]
    L.pd_loop_counts.argtypes = [P, P]
    L.pd_energy_noalloc.argtypes = [P, P, C.c_int32]
    L.pd_tile_info.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
    L.pd_set_timing.argtypes = [P, C.c_int32]
    L.pd_timing.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
    L.pd_set_launch.argtypes = [P, C.POINTER(pd_launch)]
    L.pd_get_launch.argtypes = [P, C.POINTER(pd_launch)]
    L.pd_destroy.argtypes = [P]
    L.pd_last_error.argtypes = [P]
    L.pd_last_error.restype = C.c_char_p
    L.pd_status_string.argtypes = [C.c_int32]
    L.pd_status_string.restype = C.c_char_p
    for name in ["pd_init", "pd_build_bonds", "pd_step", "pd_field_bytes", "pd_get",
                 "pd_set_wall", "pd_get_state", "pd_set_state", "pd_info", "pd_loop_counts", "pd_tile_info", "pd_energy_noalloc", "pd_set_timing",
                 "pd_timing", "pd_set_launch", "pd_get_launch"]:
        getattr(L, name).restype = C.c_int32
    return L


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


class PDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(P)


def make_wall(w: "_inp.Wall") -> pd_wall:
    s = pd_wall()
    s.normal[:] = list(w.normal)
    s.offset = w.offset
    s.velocity = w.velocity
    s.lo[:] = [max(x, -1e300) for x in w.lo]
    s.hi[:] = [min(x, 1e300) for x in w.hi]
    s.mode = w.mode
    s.target_stress = w.target_stress
    s.servo_gain = w.servo_gain
    s.area = w.area
    return s


def make_cut(c: "_inp.Cut") -> pd_cut:
    s = pd_cut()
    s.kind = c.kind
    s.grain = c.grain
    s.plane[:] = list(c.plane)
    s.lo[:] = list(c.lo)
    s.hi[:] = list(c.hi)
    s.center[:] = list(c.center)
    s.radius2 = c.radius2
    return s


class TorchPlumbing:
    """Device memory from PyTorch's caching allocator and a PyTorch HIP stream.

    By default each context gets its own stream (default priority): the legacy
    null stream cannot be captured into the library's HIP graphs."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible to PyTorch")
        self.torch = torch
        self.device = device
        torch.cuda.set_device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device)
        self.stream_ptr = self.stream.cuda_stream

        def _alloc(nbytes, user):
            try:
                return self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
            except Exception:  # out of memory -> NULL -> PD_ERR_OOM
                return None

        def _free(ptr, user):
            cuda = getattr(self.torch, "cuda", None)
            if cuda is None:  # interpreter shutdown: the process releases the memory
                return
            cuda.caching_allocator_delete(int(ptr))

        self.alloc = ALLOC_FN(_alloc)
        self.free = FREE_FN(_free)


# Contexts still open when the interpreter exits are destroyed by an exit hook,
# while the HIP runtime (and any profiler attached to it) is still up, rather
# than by garbage collection during interpreter teardown.
_LIVE = weakref.WeakSet()


@atexit.register
def _close_live_contexts():
    for sim in list(_LIVE):
        try:
            sim.close()
        except Exception:
            pass


class Sim:
    """One library context built from a seeded workload (see inputs.py)."""

    def __init__(self, wl: "_inp.Workload", flags: int = 0, plumbing: Optional[TorchPlumbing] = None,
                 torch_allocator: bool = True, candidate_capacity_per_node: int = 0,
                 build: bool = True):
        L = lib()
        self.wl = wl
        self.n = wl.n_nodes
        self.n_walls = len(wl.walls)
        if plumbing is None and torch_allocator:
            plumbing = TorchPlumbing()
        self.plumbing = plumbing
        k = self._keep = dict(
            X=np.ascontiguousarray(wl.X, dtype=np.float64),
            ijk=np.ascontiguousarray(wl.ijk, dtype=np.int32),
            u0=np.ascontiguousarray(wl.u0, dtype=np.float64),
            v0=np.ascontiguousarray(wl.v0, dtype=np.float64),
            fixed=np.ascontiguousarray(wl.fixed, dtype=np.uint8),
            gb=np.ascontiguousarray(wl.grain_begin, dtype=np.int64),
            gm=np.ascontiguousarray(wl.grain_material, dtype=np.int32),
            gh=np.ascontiguousarray(wl.grain_h, dtype=np.float64),
            go=np.ascontiguousarray(wl.grain_origin, dtype=np.float64))
        g = pd_grains(wl.n_grains, _ptr(k["gb"]), _ptr(k["gm"]), _ptr(k["gh"]), _ptr(k["go"]))
        m = pd_mesh(self.n, _ptr(k["X"]), _ptr(k["ijk"]), _ptr(k["u0"]), _ptr(k["v0"]),
                    _ptr(k["fixed"]) if wl.fixed.any() else None)
        mats = (pd_material * len(wl.materials))(
            *[pd_material(x.bulk_modulus, x.density, x.fracture_energy) for x in wl.materials])
        p = wl.params
        prm = pd_params()
        prm.horizon_factor = p.horizon_factor
        prm.flags = flags | (FLAG_CONIC if getattr(p, "micromodulus", "constant") == "conic" else 0)
        if getattr(p, "self_contact", False):
            prm.flags |= FLAG_SELF_CONTACT
        if getattr(p, "wall_corners", False):
            prm.flags |= FLAG_WALL_CORNERS
        if getattr(p, "adaptive_rebuild", False):
            prm.flags |= FLAG_ADAPTIVE_REBUILD
        prm.contact_radius = p.contact_radius
        prm.contact_horizon = p.contact_horizon
        prm.skin = p.skin
        prm.rebuild_every = p.rebuild_every
        prm.candidate_capacity_per_node = candidate_capacity_per_node
        prm.dt = p.dt
        prm.gravity[:] = list(p.gravity)
        prm.contact_damping = getattr(p, "contact_damping", 0.0)
        prm.friction = getattr(p, "friction", 0.0)
        walls = (pd_wall * max(self.n_walls, 1))(*[make_wall(w) for w in wl.walls])
        h = P()
        if plumbing is not None:
            st = L.pd_init(C.byref(h), C.byref(g), C.byref(m), mats, len(wl.materials),
                           C.byref(prm), walls if self.n_walls else None, self.n_walls,
                           plumbing.alloc, plumbing.free, None, P(plumbing.stream_ptr))
        else:
            st = L.pd_init(C.byref(h), C.byref(g), C.byref(m), mats, len(wl.materials),
                           C.byref(prm), walls if self.n_walls else None, self.n_walls,
                           ALLOC_FN(0), FREE_FN(0), None, None)
        self.h = h
        _LIVE.add(self)
        self._check(st)
        if build:
            self.build_bonds()

    # --- ABI calls ---
    def _check(self, st):
        if st != PD_OK:
            msg = lib().pd_last_error(self.h).decode() if self.h else lib().pd_status_string(st).decode()
            raise PDError(st, msg)

    def build_bonds(self, cuts=None):
        cuts = self.wl.cuts if cuts is None else cuts
        arr = (pd_cut * max(len(cuts), 1))(*[make_cut(c) for c in cuts])
        self._check(lib().pd_build_bonds(self.h, arr if cuts else None, len(cuts)))

    def step(self, n: int):
        self._check(lib().pd_step(self.h, int(n)))

    def step_status(self, n: int) -> int:
        """Like step() but returns the status instead of raising."""
        return int(lib().pd_step(self.h, int(n)))

    def field_bytes(self, name: str) -> int:
        b = C.c_int64()
        self._check(lib().pd_field_bytes(self.h, FIELDS[name], C.byref(b)))
        return b.value

    def get(self, name: str) -> np.ndarray:
        nb = self.field_bytes(name)
        dt = _FIELD_DTYPE[name]
        out = np.zeros(max(nb // np.dtype(dt).itemsize, 1), dtype=dt)
        self._check(lib().pd_get(self.h, FIELDS[name], _ptr(out), nb, 0))
        out = out[: nb // np.dtype(dt).itemsize]
        if name in ("displacement", "velocity", "accel", "force_density"):
            return out.reshape(3, self.n)
        if name in ("wall_force", "wall_impulse"):
            return out.reshape(self.n_walls, 3)
        return out

    def get_device(self, name: str, dst_ptr: int, nbytes: int):
        self._check(lib().pd_get(self.h, FIELDS[name], P(dst_ptr), nbytes, 1))

    def info(self) -> dict:
        o = np.zeros(5, dtype=np.int64)
        self._check(lib().pd_info(self.h, _ptr(o)))
        return dict(n_nodes=int(o[0]), nnz=int(o[1]), padded=int(o[2]), candidates=int(o[3]),
                    step=int(o[4]))

    def energy_noalloc(self, out_ptr: Optional[int] = None) -> Optional[np.ndarray]:
        """pd_energy_noalloc: into a new host array, or into device memory at out_ptr."""
        if out_ptr is not None:
            self._check(lib().pd_energy_noalloc(self.h, P(out_ptr), 1))
            return None
        out = np.zeros(4)
        self._check(lib().pd_energy_noalloc(self.h, _ptr(out), 0))
        return out

    def tile_info(self) -> dict:
        n, lat = C.c_int64(), C.c_int32()
        self._check(lib().pd_tile_info(self.h, C.byref(n), C.byref(lat)))
        return dict(tiles=n.value, lattice=bool(lat.value))

    def loop_counts(self) -> dict:
        o = np.zeros(6, dtype=np.int64)
        self._check(lib().pd_loop_counts(self.h, _ptr(o)))
        return dict(graph_replays=int(o[0]), graph_steps=int(o[1]), direct_steps=int(o[2]),
                    persistent_launches=int(o[3]), persistent_steps=int(o[4]), early_rebuilds=int(o[5]))

    def set_launch(self, loop: int = LOOP_GRAPH, slices_per_block: int = 4, xcd_remap: int = 1,
                   persistent_blocks: int = 0, bond_path: int = BONDS_SLICES):
        cfg = pd_launch(int(loop), int(slices_per_block), int(xcd_remap), int(persistent_blocks),
                        int(bond_path))
        self._check(lib().pd_set_launch(self.h, C.byref(cfg)))

    def get_launch(self) -> dict:
        cfg = pd_launch()
        self._check(lib().pd_get_launch(self.h, C.byref(cfg)))
        return dict(loop=cfg.loop, slices_per_block=cfg.slices_per_block, xcd_remap=cfg.xcd_remap,
                    persistent_blocks=cfg.persistent_blocks, bond_path=cfg.bond_path)

    def set_timing(self, enable: bool):
        self._check(lib().pd_set_timing(self.h, 1 if enable else 0))

    def timing(self):
        """(launches, total_ms) of the fused step kernel since timing was enabled."""
        n, ms = C.c_int64(), C.c_double()
        self._check(lib().pd_timing(self.h, C.byref(n), C.byref(ms)))
        return n.value, ms.value

    def bonds(self):
        return self.get("bond_rowptr"), self.get("bond_col"), self.get("bond_broken")

    def candidates(self):
        return self.get("contact_rowptr"), self.get("contact_col")

    def set_wall(self, w: int, wall: "_inp.Wall"):
        s = make_wall(wall)
        self._check(lib().pd_set_wall(self.h, w, C.byref(s)))

    def get_state(self) -> bytes:
        n = C.c_int64()
        self._check(lib().pd_get_state(self.h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._check(lib().pd_get_state(self.h, C.cast(buf, P), C.byref(n)))
        return buf.raw

    def set_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        self._check(lib().pd_set_state(self.h, C.cast(buf, P), len(blob)))

    def close(self):
        if getattr(self, "h", None):
            lib().pd_destroy(self.h)
            self.h = None
        _LIVE.discard(self)

    def __del__(self, _finalizing=sys.is_finalizing):
        # during interpreter teardown the HIP runtime may already be gone: the
        # exit hook closed every context that was still open before that (the
        # check is bound at definition, since module globals may be cleared by then)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
