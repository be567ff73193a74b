"""ctypes wrapper of the plain FP64 CPU oracle (pdref.c).

TEST INFRASTRUCTURE ONLY: used by the tests, the package smoke check and the
benchmark's CPU-baseline leg.  The product library never imports this module.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pdref.c")
LIB = os.path.join(HERE, "libpdref.so")

TABLE_LITERAL = 1
ABS_STRETCH = 2
CELL_LIST = 4
CONIC = 8
SELF_CONTACT = 16
WALL_CORNERS = 32
ADAPTIVE_REBUILD = 64

CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-std=c99", "-fPIC",
          "-shared", "-Wall"]


SANITIZE_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=all", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-std=c99",
                  "-fPIC", "-shared", "-Wall"]


def build_sanitized(out: str) -> str:
    """The oracle with AddressSanitizer and UndefinedBehaviorSanitizer (any
    finding aborts), for a process that preloads the ASan runtime."""
    subprocess.check_call(["gcc", *SANITIZE_FLAGS, SRC, "-o", out, "-lm"])
    return out


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        # PDREF_LIB: another build of the same source (the sanitizer test's)
        path = os.environ.get("PDREF_LIB", LIB)
        if path == LIB and not os.path.exists(LIB):
            build()
        L = C.CDLL(path)
        P = C.c_void_p
        L.pdref_create.restype = P
        L.pdref_create.argtypes = [C.c_int64, P, P, P, P, P, C.c_int32, P, P, P, C.c_int32, P, P,
                                   C.c_int32, P, C.c_int32, P, C.c_int32]
        L.pdref_destroy.argtypes = [P]
        L.pdref_build.argtypes = [P]
        L.pdref_build.restype = C.c_int32
        L.pdref_step.argtypes = [P, C.c_int64]
        L.pdref_step.restype = C.c_int32
        L.pdref_set_threads.argtypes = [C.c_int32]
        L.pdref_nnz.argtypes = [P]
        L.pdref_nnz.restype = C.c_int64
        L.pdref_step_count.argtypes = [P]
        L.pdref_step_count.restype = C.c_int64
        L.pdref_get_bonds.argtypes = [P, P, P, P]
        L.pdref_get_state.argtypes = [P, P, P, P, P]
        L.pdref_get_damage.argtypes = [P, P, P, P]
        L.pdref_get_walls.argtypes = [P, P, P]
        L.pdref_get_wall_impulse.argtypes = [P, P]
        L.pdref_n_candidates.argtypes = [P]
        L.pdref_n_candidates.restype = C.c_int64
        L.pdref_get_candidates.argtypes = [P, P, P]
        L.pdref_energy.argtypes = [P, P]
        L.pdref_min_margin.argtypes = [P]
        L.pdref_min_margin.restype = C.c_double
        L.pdref_bond_margin.argtypes = [P, P]
        L.pdref_skin_exceeded.argtypes = [P]
        L.pdref_skin_exceeded.restype = C.c_int32
        L.pdref_early_rebuilds.argtypes = [P]
        L.pdref_early_rebuilds.restype = C.c_int64
        L.pdref_set_u.argtypes = [P, P]
        L.pdref_rebuild_candidates.argtypes = [P]
        L.pdref_energy_density.argtypes = [P, P]
        L.pdref_constants.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int32,
                                      C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.pdref_contact_stiffness.argtypes = [C.c_double, C.c_double, C.c_double]
        L.pdref_contact_stiffness.restype = C.c_double
        L.pdref_wall_cap.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_double),
                                     C.POINTER(C.c_double)]
        L.pdref_corner_region.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double,
                                          C.POINTER(C.c_double), C.POINTER(C.c_double)]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def constants(K, Gc, delta, flags=0):
    c, s0 = C.c_double(), C.c_double()
    lib().pdref_constants(K, Gc, delta, flags, C.byref(c), C.byref(s0))
    return c.value, s0.value


def contact_stiffness(ka, kb, eps):
    return lib().pdref_contact_stiffness(ka, kb, eps)


def wall_cap(Rc, d):
    v, l = C.c_double(), C.c_double()
    lib().pdref_wall_cap(Rc, d, C.byref(v), C.byref(l))
    return v.value, l.value


def corner_region(R, a, b, c=-np.inf):
    """Volume and centroid of {|x| < R, x_u > a, x_v > b, x_w > c}."""
    v = C.c_double()
    cen = (C.c_double * 3)()
    lib().pdref_corner_region(R, a, b, c, C.byref(v), cen)
    return v.value, np.array(cen[:])


def pack_walls(walls):
    out = np.zeros((max(len(walls), 1), 15), dtype=np.float64)
    for k, w in enumerate(walls):
        out[k] = [*w.normal, w.offset, w.velocity, *w.lo, *w.hi, float(w.mode),
                  w.target_stress, w.servo_gain, w.area]
    return out


def pack_cuts(cuts):
    out = np.zeros((max(len(cuts), 1), 16), dtype=np.int64)
    for k, c in enumerate(cuts):
        out[k] = [c.kind, c.grain, *c.plane, *c.lo, *c.hi, *c.center, c.radius2]
    return out


class Oracle:
    """One oracle simulation of a workload (inputs from the seeded generators)."""

    def __init__(self, wl, flags: int = 0, threads: int = 1, build_now: bool = True):
        L = lib()
        if getattr(wl.params, "micromodulus", "constant") == "conic":
            flags |= CONIC
        if getattr(wl.params, "self_contact", False):
            flags |= SELF_CONTACT
        if getattr(wl.params, "wall_corners", False):
            flags |= WALL_CORNERS
        if getattr(wl.params, "adaptive_rebuild", False):
            flags |= ADAPTIVE_REBUILD
        self.wl = wl
        self.n = wl.n_nodes
        p = wl.params
        self._keep = dict(
            X=np.ascontiguousarray(wl.X, dtype=np.float64),
            ijk=np.ascontiguousarray(wl.ijk, dtype=np.int32),
            u0=np.ascontiguousarray(wl.u0, dtype=np.float64),
            v0=np.ascontiguousarray(wl.v0, dtype=np.float64),
            fixed=np.ascontiguousarray(wl.fixed, dtype=np.uint8),
            gb=np.ascontiguousarray(wl.grain_begin, dtype=np.int64),
            gm=np.ascontiguousarray(wl.grain_material, dtype=np.int32),
            gh=np.ascontiguousarray(wl.grain_h, dtype=np.float64),
            mat=np.array([[m.bulk_modulus, m.density, m.fracture_energy] for m in wl.materials],
                         dtype=np.float64),
            par=np.array([p.horizon_factor, p.contact_radius, p.contact_horizon, p.skin,
                          p.rebuild_every, p.dt, *p.gravity, p.contact_damping,
                          getattr(p, "friction", 0.0)],
                         dtype=np.float64),
            walls=pack_walls(wl.walls), cuts=pack_cuts(wl.cuts))
        k = self._keep
        L.pdref_set_threads(threads)
        self.h = L.pdref_create(self.n, _p(k["X"]), _p(k["ijk"]), _p(k["u0"]), _p(k["v0"]),
                                _p(k["fixed"]), wl.n_grains, _p(k["gb"]), _p(k["gm"]),
                                _p(k["gh"]), len(wl.materials), _p(k["mat"]), _p(k["par"]),
                                len(wl.walls), _p(k["walls"]), len(wl.cuts), _p(k["cuts"]), flags)
        self.status = None
        if build_now:
            self.status = L.pdref_build(self.h)

    def __del__(self):
        if getattr(self, "h", None):
            lib().pdref_destroy(self.h)
            self.h = None

    def build(self):
        self.status = lib().pdref_build(self.h)
        return self.status

    def step(self, n: int) -> int:
        self.status = lib().pdref_step(self.h, int(n))
        return self.status

    @property
    def nnz(self) -> int:
        return int(lib().pdref_nnz(self.h))

    @property
    def step_count(self) -> int:
        return int(lib().pdref_step_count(self.h))

    def bonds(self):
        rp = np.zeros(self.n + 1, dtype=np.int64)
        col = np.zeros(max(self.nnz, 1), dtype=np.int32)
        br = np.zeros(max(self.nnz, 1), dtype=np.uint8)
        lib().pdref_get_bonds(self.h, _p(rp), _p(col), _p(br))
        return rp, col[: self.nnz], br[: self.nnz]

    def state(self):
        u, v, a, F = (np.zeros((3, self.n)) for _ in range(4))
        lib().pdref_get_state(self.h, _p(u), _p(v), _p(a), _p(F))
        return dict(u=u, v=v, a=a, F=F)

    def damage(self):
        d = np.zeros(self.n)
        it = np.zeros(self.n, dtype=np.int32)
        n0 = np.zeros(self.n, dtype=np.int32)
        lib().pdref_get_damage(self.h, _p(d), _p(it), _p(n0))
        return d, it, n0

    def walls(self):
        nw = len(self.wl.walls)
        f = np.zeros((max(nw, 1), 3))
        o = np.zeros(max(nw, 1))
        lib().pdref_get_walls(self.h, _p(f), _p(o))
        return f[:nw], o[:nw]

    def wall_impulse(self):
        nw = len(self.wl.walls)
        f = np.zeros((max(nw, 1), 3))
        lib().pdref_get_wall_impulse(self.h, _p(f))
        return f[:nw]

    def candidates(self):
        nc = int(lib().pdref_n_candidates(self.h))
        rp = np.zeros(self.n + 1, dtype=np.int64)
        col = np.zeros(max(nc, 1), dtype=np.int32)
        lib().pdref_get_candidates(self.h, _p(rp), _p(col))
        return rp, col[:nc]

    def energy(self):
        out = np.zeros(4)
        lib().pdref_energy(self.h, _p(out))
        return dict(kinetic=out[0], elastic=out[1], contact=out[2], gravity=out[3],
                    total=float(out.sum()))

    def energy_density(self):
        W = np.zeros(self.n)
        lib().pdref_energy_density(self.h, _p(W))
        return W

    def min_margin(self) -> float:
        return float(lib().pdref_min_margin(self.h))

    def bond_margin(self) -> np.ndarray:
        """Per directed bond (aligned with bonds()), the smallest |s/s0 - 1| any of
        its break decisions saw (inf for a bond never evaluated)."""
        m = np.zeros(max(self.nnz, 1))
        lib().pdref_bond_margin(self.h, _p(m))
        return m[: self.nnz]

    def skin_exceeded(self) -> bool:
        return bool(lib().pdref_skin_exceeded(self.h))

    def early_rebuilds(self) -> int:
        return int(lib().pdref_early_rebuilds(self.h))

    def set_u(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        lib().pdref_set_u(self.h, _p(u))

    def rebuild_candidates(self):
        lib().pdref_rebuild_candidates(self.h)
