"""Seeded synthetic workloads for the peridynamic grain-aggregate step.

This module only lays out geometry and initial data: lattice nodes of each
grain, initial displacement/velocity, material table, rigid walls and the
bond cuts (notch planes, cavities) as *descriptions*.  It contains none of the
method's arithmetic (no bonds, stretches, forces, contact tests or time
stepping); both the HIP library and the CPU oracle consume its arrays.

Geometry conventions (the paper meshes each grain, Sec. 7.5; here every grain
is meshed on its own axis-aligned cubic lattice of spacing h):

* node n of grain g sits at  X = origin[g] + h[g] * ijk[n]  with integer
  grain-local lattice indices 0 <= ijk < 1024;
* nodes are grouped by grain (grain_begin is a CSR-style offset array) and
  ordered lexicographically inside each grain, slowest axis = longest extent,
  middle axis = shortest extent, so neighbour rows stay close in memory;
* cuts are given in half-lattice integer units: node ijk sits at 2*ijk, so
  planes and cavity centres that fall between nodes are exact integers.

Every random quantity comes from numpy's PCG64 seeded by the caller.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

UNBOUNDED = float("inf")
CUT_NOTCH, CUT_CAVITY_ENDPOINT, CUT_CAVITY_CHORD = 0, 1, 2
WALL_FIXED, WALL_VELOCITY, WALL_SERVO = 0, 1, 2
HALF_UNBOUNDED = 1 << 50  # |lo|,|hi| >= this means "no bound on that axis"


@dataclasses.dataclass
class Material:
    bulk_modulus: float  # K [Pa]
    density: float  # rho [kg/m^3]
    fracture_energy: float  # G_c [J/m^2]


@dataclasses.dataclass
class Wall:
    normal: tuple  # unit normal pointing into the domain
    offset: float  # plane n.p = offset at t = 0
    mode: int = WALL_FIXED
    velocity: float = 0.0  # d(offset)/dt for WALL_VELOCITY
    lo: tuple = (-UNBOUNDED,) * 3  # patch: node acted on iff lo <= p <= hi
    hi: tuple = (UNBOUNDED,) * 3
    target_stress: float = 0.0  # WALL_SERVO
    servo_gain: float = 0.0  # WALL_SERVO [m/s per Pa]
    area: float = 1.0  # reaction force / area = wall stress


@dataclasses.dataclass
class Cut:
    kind: int
    grain: int
    plane: tuple = (0, 0, 0, 0)  # a,b,c,d : a*X+b*Y+c*Z+d = 0 (half-lattice units)
    lo: tuple = (-HALF_UNBOUNDED,) * 3  # crossing point bounds (half-lattice)
    hi: tuple = (HALF_UNBOUNDED,) * 3
    center: tuple = (0, 0, 0)  # cavity centre (half-lattice)
    radius2: int = 0  # cavity squared radius (half-lattice units^2)


@dataclasses.dataclass
class Params:
    horizon_factor: int  # m: delta = m*h
    contact_radius: float  # R_c [m]
    contact_horizon: float  # epsilon in K_n = 18k/(pi eps^5) [m]
    skin: float  # Verlet skin of the contact candidate list [m]
    rebuild_every: int  # candidate rebuild cadence [steps]
    dt: float
    gravity: tuple = (0.0, 0.0, 0.0)
    contact_damping: float = 0.0  # beta_d of the normal damping law [N s/m^7]; 0 = none
    friction: float = 0.0  # mu of the stick-slip friction law; 0 = none
    micromodulus: str = "constant"  # "constant" or "conic" (c0 (1 - |xi|/delta))
    self_contact: bool = False  # contact between nodes of one grain with no intact bond
    wall_corners: bool = False  # inclusion-exclusion of orthogonal walls at box corners
    adaptive_rebuild: bool = False  # rebuild the candidates early once a node moved skin/2


@dataclasses.dataclass
class Workload:
    name: str
    X: np.ndarray  # (3, N) float64
    ijk: np.ndarray  # (3, N) int32
    grain_begin: np.ndarray  # (G+1,) int64
    grain_h: np.ndarray  # (G,) float64
    grain_origin: np.ndarray  # (3, G) float64
    grain_material: np.ndarray  # (G,) int32
    materials: List[Material]
    params: Params
    u0: np.ndarray  # (3, N)
    v0: np.ndarray  # (3, N)
    fixed: np.ndarray  # (N,) uint8
    walls: List[Wall]
    cuts: List[Cut]
    steps: int
    info: Dict = dataclasses.field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.X.shape[1])

    @property
    def n_grains(self) -> int:
        return int(self.grain_h.shape[0])

    def grain_of_node(self) -> np.ndarray:
        return np.repeat(np.arange(self.n_grains, dtype=np.int32), np.diff(self.grain_begin))


# ----------------------------------------------------------------------------
# lattice helpers
# ----------------------------------------------------------------------------

def _order_nodes(ijk: np.ndarray) -> np.ndarray:
    """Lexicographic order: slowest = longest extent, middle = shortest, fastest = the other."""
    ext = ijk.max(axis=1) - ijk.min(axis=1)
    slow = int(np.argmax(ext))
    rest = [a for a in range(3) if a != slow]
    mid = rest[0] if ext[rest[0]] <= ext[rest[1]] else rest[1]
    fast = rest[1] if mid == rest[0] else rest[0]
    return np.lexsort((ijk[fast], ijk[mid], ijk[slow]))


def _grain_block(offsets: np.ndarray, origin_of_zero: np.ndarray, h: float, axes=None):
    """offsets: (3, n) integer lattice points of one grain (any sign).

    Returns (ijk >= 0 ordered, origin) with X = origin + h*ijk.  Nodes are in
    lexicographic order of the axes `axes` (slowest first), or of the grain's
    own longest, shortest and remaining extents when axes is None.
    """
    lo = offsets.min(axis=1)
    ijk = (offsets - lo[:, None]).astype(np.int64)
    if ijk.max() >= 1024:
        raise ValueError("grain lattice extent exceeds 1023 cells")
    if axes is None:
        order = _order_nodes(ijk)
    else:
        order = np.lexsort((ijk[axes[2]], ijk[axes[1]], ijk[axes[0]]))
    ijk = ijk[:, order]
    origin = origin_of_zero + h * lo.astype(np.float64)
    return ijk.astype(np.int32), origin


def _assemble(name, blocks, materials, params, walls, cuts, steps, u0=None, v0=None,
              fixed=None, info=None) -> Workload:
    """blocks: list of (ijk (3,n) int32, origin (3,), h, material)."""
    sizes = [b[0].shape[1] for b in blocks]
    begin = np.zeros(len(blocks) + 1, dtype=np.int64)
    begin[1:] = np.cumsum(sizes)
    ijk = np.concatenate([b[0] for b in blocks], axis=1).astype(np.int32)
    h = np.array([b[2] for b in blocks], dtype=np.float64)
    origin = np.stack([np.asarray(b[1], dtype=np.float64) for b in blocks], axis=1)
    mat = np.array([b[3] for b in blocks], dtype=np.int32)
    X = np.empty((3, begin[-1]), dtype=np.float64)
    for g, b in enumerate(blocks):
        s, e = begin[g], begin[g + 1]
        X[:, s:e] = origin[:, g:g + 1] + h[g] * b[0].astype(np.float64)
    N = int(begin[-1])
    return Workload(
        name=name, X=X, ijk=ijk, grain_begin=begin, grain_h=h, grain_origin=origin,
        grain_material=mat, materials=list(materials), params=params,
        u0=np.zeros((3, N)) if u0 is None else u0,
        v0=np.zeros((3, N)) if v0 is None else v0,
        fixed=np.zeros(N, dtype=np.uint8) if fixed is None else fixed,
        walls=list(walls), cuts=list(cuts), steps=int(steps), info=dict(info or {}))


def sphere_offsets(n: int) -> np.ndarray:
    """Integer points with i^2 + j^2 + k^2 <= n^2 (a lattice-centred ball of radius n*h)."""
    r = np.arange(-n, n + 1)
    I, J, K = np.meshgrid(r, r, r, indexing="ij")
    m = I * I + J * J + K * K <= n * n
    return np.stack([I[m], J[m], K[m]])


def box_offsets(nx: int, ny: int, nz: int) -> np.ndarray:
    I, J, K = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    return np.stack([I.ravel(), J.ravel(), K.ravel()])


# public names for building small custom workloads
grain_block = _grain_block
assemble = _assemble


# ----------------------------------------------------------------------------
# materials used by the workloads
# ----------------------------------------------------------------------------

SAND = Material(bulk_modulus=14.9e9, density=2600.0, fracture_energy=10.0)
# Maraging steel of the Kalthoff-Winkler test: bulk modulus of material M1,
# G_c = K_IC^2 / E with K_IC = 68 MPa sqrt(m), E = 190 GPa.
STEEL = Material(bulk_modulus=159.2e9, density=8000.0, fracture_energy=68e6 ** 2 / 190e9)


def default_params(h: float, dt: float, m: int = 3, rebuild_every: int = 20,
                   gravity=(0.0, 0.0, 0.0)) -> Params:
    return Params(horizon_factor=m, contact_radius=0.95 * h, contact_horizon=m * h,
                  skin=0.25 * h, rebuild_every=rebuild_every, dt=dt, gravity=tuple(gravity))


# ----------------------------------------------------------------------------
# workload 1: two spherical grains
# ----------------------------------------------------------------------------

def two_spheres(seed: int = 0, speed: float = 1.0, radius_cells: int = 10, h: float = 1e-4,
                gap: float = 2e-6, steps: int = 500, dt: float = 1e-8,
                material: Material = SAND, rebuild_every: int = 20) -> Workload:
    """Two lattice balls of radius radius_cells*h; B moves along -x at `speed` into A.

    A is centred at the origin and starts at rest (unconstrained).  B's centre
    gets seeded y/z offsets in [0, h) and an x position chosen so the closest
    inter-grain node distance at t = 0 is R_c + gap.
    """
    rng = np.random.default_rng(seed)
    params = default_params(h, dt, rebuild_every=rebuild_every)
    off = sphere_offsets(radius_cells)
    yz = rng.uniform(0.0, h, size=2)
    XA = off.astype(np.float64) * h
    XB0 = off.astype(np.float64) * h
    XB0[1] += yz[0]
    XB0[2] += yz[1]
    # closest-approach placement along x, facing slabs only
    a = XA[:, XA[0] >= XA[0].max() - 4 * h]
    b = XB0[:, XB0[0] <= XB0[0].min() + 4 * h]
    target = params.contact_radius + gap
    rho2 = (a[1][:, None] - b[1][None, :]) ** 2 + (a[2][:, None] - b[2][None, :]) ** 2
    ok = rho2 < target * target
    need = a[0][:, None] - b[0][None, :] + np.sqrt(np.where(ok, target * target - rho2, 0.0))
    xB = float(np.max(np.where(ok, need, -np.inf)))
    cB = np.array([xB, yz[0], yz[1]])
    ijkA, oA = _grain_block(off, np.zeros(3), h)
    ijkB, oB = _grain_block(off, cB, h)
    wl = _assemble("two_spheres", [(ijkA, oA, h, 0), (ijkB, oB, h, 0)], [material], params,
                   [], [], steps, info={"seed": seed, "speed": speed, "centre_B": cB.tolist()})
    nA = ijkA.shape[1]
    wl.v0[0, nA:] = -speed
    return wl


# ----------------------------------------------------------------------------
# workload 2: double-notched plate hit on its edge by a rigid projectile face
# ----------------------------------------------------------------------------

def notched_plate(nx: int = 200, ny: int = 200, nz: int = 18, h: float = 5e-4,
                  notch_x=(25e-3, 75e-3), notch_len: float = 50e-3, speed: float = 32.0,
                  dt: float = 2.5e-8, steps: int = 4000, material: Material = STEEL,
                  rebuild_every: int = 20, seed: int = 0) -> Workload:
    """Plate [0,nx*h]x[0,ny*h]x[0,nz*h] with node centres at (i+1/2)h.

    Two zero-width notch planes x = notch_x[k] run from the impact edge y = 0 to
    y = notch_len (tip included).  A rigid wall patch covering x in
    [notch_x[0], notch_x[1]] (the projectile face) starts R_c below the lowest
    node row and moves +y at `speed`.
    """
    del seed  # geometry is deterministic
    params = default_params(h, dt, rebuild_every=rebuild_every)
    off = box_offsets(nx, ny, nz)
    ijk, origin = _grain_block(off, np.full(3, 0.5 * h), h)
    cuts = []
    for xn in notch_x:
        # plane x = xn: node i sits at (i + 1/2) h, half-lattice coordinate 2i
        half = 2.0 * (xn / h - 0.5)
        yhalf = 2.0 * (notch_len / h - 0.5)
        if abs(half - round(half)) > 1e-9 or abs(yhalf - round(yhalf)) > 1e-9:
            raise ValueError("notch geometry must fall on half-lattice coordinates")
        cuts.append(Cut(kind=CUT_NOTCH, grain=0, plane=(1, 0, 0, -int(round(half))),
                        lo=(-HALF_UNBOUNDED, -HALF_UNBOUNDED, -HALF_UNBOUNDED),
                        hi=(HALF_UNBOUNDED, int(round(yhalf)), HALF_UNBOUNDED)))
    y0 = 0.5 * h
    wall = Wall(normal=(0.0, 1.0, 0.0), offset=y0 - params.contact_radius, mode=WALL_VELOCITY,
                velocity=speed, lo=(notch_x[0], -UNBOUNDED, -UNBOUNDED),
                hi=(notch_x[1], UNBOUNDED, UNBOUNDED), area=(notch_x[1] - notch_x[0]) * nz * h)
    return _assemble("notched_plate", [(ijk, origin, h, 0)], [material], params, [wall], cuts,
                     steps, info={"nx": nx, "ny": ny, "nz": nz})


# ----------------------------------------------------------------------------
# level-set grains (spheres perturbed by real spherical harmonics, l = 2..6)
# ----------------------------------------------------------------------------

def _real_sph_harm(l: int, m: int, theta: np.ndarray, phi: np.ndarray, p=None) -> np.ndarray:
    """Real spherical harmonic, theta = polar angle, phi = azimuth.  p may carry
    the associated Legendre values P_l^|m|(cos theta) already evaluated."""
    from scipy.special import lpmv
    am = abs(m)
    norm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
    if p is None:
        p = lpmv(am, l, np.cos(theta))
    if m > 0:
        return math.sqrt(2.0) * norm * p * np.cos(m * phi)
    if m < 0:
        return math.sqrt(2.0) * norm * p * np.sin(am * phi)
    return norm * p


class LevelSetShape:
    """r(theta, phi) = R [1 + A S(Q d) / max|S|], S = sum_{l=2..6} sum_m a_lm Y_lm."""

    def __init__(self, rng: np.random.Generator, radius: float, lmax: int = 6):
        self.R = radius
        self.A = rng.uniform(0.05, 0.20)
        self.coef = [(l, m, rng.normal(0.0, 1.0 / l)) for l in range(2, lmax + 1)
                     for m in range(-l, l + 1)]
        # random rotation: QR of a Gaussian matrix with sign fix
        q, r = np.linalg.qr(rng.normal(size=(3, 3)))
        q = q * np.sign(np.diag(r))
        if np.linalg.det(q) < 0:
            q[:, 0] = -q[:, 0]
        self.Q = q
        th = np.linspace(0.0, math.pi, 65)
        ph = np.linspace(0.0, 2 * math.pi, 129)
        T, P = np.meshgrid(th, ph, indexing="ij")
        self.smax = float(np.max(np.abs(self._S(T, P)))) or 1.0

    def _S(self, theta, phi):
        from scipy.special import lpmv
        c = np.cos(theta)
        leg = {}
        s = np.zeros_like(theta)
        for l, m, a in self.coef:
            if (l, abs(m)) not in leg:
                leg[(l, abs(m))] = lpmv(abs(m), l, c)
            s = s + a * _real_sph_harm(l, m, theta, phi, leg[(l, abs(m))])
        return s

    def radius_at(self, d: np.ndarray) -> np.ndarray:
        """d: (3, n) directions (not necessarily unit)."""
        e = self.Q.T @ d
        nrm = np.sqrt(np.sum(e * e, axis=0))
        nrm = np.where(nrm == 0, 1.0, nrm)
        theta = np.arccos(np.clip(e[2] / nrm, -1.0, 1.0))
        phi = np.arctan2(e[1], e[0])
        return self.R * (1.0 + self.A * self._S(theta, phi) / self.smax)


def level_set_grain(rng: np.random.Generator, n_target: float, h: float, hollow: bool):
    """Mesh one level-set grain on a lattice with a seeded sub-cell offset.

    Returns (offsets (3,n) int, centre-relative lattice shift (3,), outer radius,
    cavity radius or 0).  Lattice point (i,j,k) sits at (i+o)h relative to the centre.
    """
    R = h * (3.0 * n_target / (4.0 * math.pi)) ** (1.0 / 3.0)
    shape = LevelSetShape(rng, R)
    o = rng.uniform(0.0, 1.0, size=3)
    nmax = int(math.ceil(R * 1.25 / h)) + 2
    r = np.arange(-nmax, nmax + 1)
    I, J, K = np.meshgrid(r, r, r, indexing="ij")
    pts = np.stack([I.ravel(), J.ravel(), K.ravel()])
    q = (pts + o[:, None]) * h
    d2 = np.sum(q * q, axis=0)
    rr = shape.radius_at(q)
    inside = d2 <= rr * rr
    rin = 0.0
    if hollow:
        rin = 0.5 * R
        inside &= d2 >= rin * rin
    return pts[:, inside], o, float(np.max(rr[inside]) if inside.any() else R), rin


def grain_aggregate(n_grains: int = 100, seed: int = 0, h: float = 1e-4, n_min: float = 2e3,
                    n_max: float = 5e4, hollow_frac: float = 0.2, grid=(5, 5, 4),
                    platen_speed: float = 0.5, dt: float = 1e-8, steps: int = 200,
                    material: Material = SAND, rebuild_every: int = 20,
                    n_targets: Optional[np.ndarray] = None, pitch_factor: float = 2.1) -> Workload:
    """Uneven level-set grains on a grid between two rigid platens.

    Node targets N_g ~ LogUniform(n_min, n_max); a seeded permutation picks
    hollow_frac of the grains to carry a centred cavity of radius R_g/2.  The
    bottom platen sits R_c below the lowest node; the top platen starts R_c/2
    above the highest node and moves down at platen_speed.
    """
    rng = np.random.default_rng(seed)
    params = default_params(h, dt, rebuild_every=rebuild_every)
    if n_targets is None:
        n_targets = np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=n_grains))
    hollow_ids = set(rng.permutation(n_grains)[: int(round(hollow_frac * n_grains))].tolist())
    meshed = []
    for g in range(n_grains):
        off, o, rout, rin = level_set_grain(rng, float(n_targets[g]), h, g in hollow_ids)
        meshed.append((off, o, rout, rin))
    pitch = pitch_factor * max(m[2] for m in meshed)
    gx, gy, gz = grid
    if gx * gy * gz < n_grains:
        raise ValueError("grid too small")
    blocks, cuts, centres = [], [], []
    for g, (off, o, rout, rin) in enumerate(meshed):
        a, b, c = g % gx, (g // gx) % gy, g // (gx * gy)
        centre = np.array([a, b, c], dtype=np.float64) * pitch
        ijk, origin = _grain_block(off, centre + o * h, h)
        blocks.append((ijk, origin, h, 0))
        centres.append(centre)
        if rin > 0:
            # cavity centre in half-lattice units of this grain: centre = origin + h*ijk_c
            ijk_c = (centre - origin) / h
            cen_half = np.rint(2.0 * ijk_c).astype(np.int64)
            # rounding the centre moves it by <= sqrt(3)/2 half-units, so a cut
            # sphere one half-unit smaller stays inside the meshed-out cavity
            r_half = 2.0 * rin / h - 1.0
            cuts.append(Cut(kind=CUT_CAVITY_CHORD, grain=g, center=tuple(int(v) for v in cen_half),
                            radius2=int(math.floor(r_half * r_half))))
    wl = _assemble("grain_aggregate", blocks, [material], params, [], cuts, steps,
                   info={"seed": seed, "n_grains": n_grains, "pitch": pitch,
                         "hollow": sorted(hollow_ids)})
    zmin, zmax = float(wl.X[2].min()), float(wl.X[2].max())
    lo = wl.X.min(axis=1)
    hi = wl.X.max(axis=1)
    area = float((hi[0] - lo[0] + pitch) * (hi[1] - lo[1] + pitch))
    Rc = params.contact_radius
    wl.walls = [
        Wall(normal=(0.0, 0.0, 1.0), offset=zmin - Rc, mode=WALL_FIXED, area=area),
        Wall(normal=(0.0, 0.0, -1.0), offset=-(zmax + 0.5 * Rc), mode=WALL_VELOCITY,
             velocity=platen_speed, area=area),
    ]
    return wl


# ----------------------------------------------------------------------------
# representative volume: a dense tessellated aggregate in a confining box
# ----------------------------------------------------------------------------

def _hard_core_seeds(rng: np.random.Generator, n: int, L: float, dmin: float) -> np.ndarray:
    """Random sequential addition of n points in [0, L]^3 at least dmin apart."""
    pts = np.empty((0, 3))
    tries = 0
    while pts.shape[0] < n:
        c = rng.uniform(0.0, L, size=3)
        if pts.shape[0] == 0 or np.min(np.sum((pts - c) ** 2, axis=1)) >= dmin * dmin:
            pts = np.vstack([pts, c])
        tries += 1
        if tries > 200 * n:
            raise RuntimeError("seed placement did not converge; lower dmin")
    return pts


def rve_aggregate(seed: int = 0, n_grains: int = 200, nodes_per_grain: float = 1850.0,
                  h: float = 7e-5, dt: float = 7e-9, confinement: float = 10e6,
                  platen_speed: float = 10.0, axial_strain: float = 0.05,
                  servo_gain: float = 5e-7, gap_factor: float = 0.0, material: Material = SAND,
                  rebuild_every: int = 20, min_grain_nodes: int = 20,
                  contact_damping: float = 0.0, friction: float = 0.0, skin_factor: float = 0.25,
                  adaptive_rebuild: bool = False) -> Workload:
    """A dense aggregate of polyhedral grains filling a box, confined by six walls.

    The grains are the cells of a Voronoi tessellation of hard-core random
    seeds, meshed on one cubic lattice with node centres at (i + 1/2) h, so
    nodes of different grains are at least h > R_c apart: neighbouring grains
    touch face to face without pressing, and the aggregate needs no settling.
    With gap_factor > 0 a node is kept only when its distance to every
    bisector plane of its cell is at least gap_factor * R_c / 2 (a looser
    packing).  The walls sit one lattice spacing beyond the outermost nodes:
    the bottom wall (normal +z) is fixed, the top wall moves down at
    platen_speed, and the four lateral walls are servo-controlled to the
    confining stress.  steps covers axial_strain of the initial wall spacing.
    """
    rng = np.random.default_rng(seed)
    from scipy.spatial import cKDTree
    params = default_params(h, dt, rebuild_every=rebuild_every)
    params.contact_damping = contact_damping
    params.friction = friction
    params.skin = skin_factor * h
    params.adaptive_rebuild = adaptive_rebuild
    Rc = params.contact_radius
    g = gap_factor * Rc
    n_side = int(math.ceil((n_grains * nodes_per_grain) ** (1.0 / 3.0)))
    L = n_side * h
    spacing = L / n_grains ** (1.0 / 3.0)
    seeds = _hard_core_seeds(rng, n_grains, L, 0.75 * spacing)
    # order grains along a coarse space-filling sweep so neighbours stay close in memory
    cell = np.floor(seeds / (L / 4.0)).clip(0, 3).astype(np.int64)
    seeds = seeds[np.lexsort((seeds[:, 0], cell[:, 0], cell[:, 1], cell[:, 2]))]
    r = np.arange(n_side)
    I, J, K = np.meshgrid(r, r, r, indexing="ij")
    lat = np.stack([I.ravel(), J.ravel(), K.ravel()])
    x = (lat.T + 0.5) * h
    kq = min(16, n_grains)
    dist, idx = cKDTree(seeds).query(x, k=kq)
    own = idx[:, 0]
    keep = np.ones(x.shape[0], dtype=bool)
    if g > 0:
        si = seeds[own]
        margin = np.full(x.shape[0], np.inf)
        for q in range(1, kq):
            sj = seeds[idx[:, q]]
            dsep = np.linalg.norm(sj - si, axis=1)
            margin = np.minimum(margin, (dist[:, q] ** 2 - dist[:, 0] ** 2) / (2.0 * dsep))
        keep = margin >= 0.5 * g
    gid = own[keep]
    lat_k = lat[:, keep]
    blocks = []
    for gr in range(n_grains):
        m = gid == gr
        if int(m.sum()) < min_grain_nodes:
            continue
        ijk, origin = _grain_block(lat_k[:, m], np.full(3, 0.5 * h), h, axes=(0, 1, 2))
        blocks.append((ijk, origin, h, 0))
    wl = _assemble("rve_aggregate", blocks, [material], params, [], [], 1,
                   info={"seed": seed, "n_grains": len(blocks), "box": L})
    lo = wl.X.min(axis=1) - max(g, h)
    hi = wl.X.max(axis=1) + max(g, h)
    span = hi - lo
    area = [span[1] * span[2], span[0] * span[2], span[0] * span[1]]
    wl.walls = [
        Wall(normal=(0.0, 0.0, 1.0), offset=lo[2], mode=WALL_FIXED, area=area[2]),
        Wall(normal=(0.0, 0.0, -1.0), offset=-hi[2], mode=WALL_VELOCITY, velocity=platen_speed,
             area=area[2]),
    ]
    for ax in (0, 1):
        for sgn in (1.0, -1.0):
            nrm = [0.0, 0.0, 0.0]
            nrm[ax] = sgn
            wl.walls.append(Wall(normal=tuple(nrm), offset=lo[ax] if sgn > 0 else -hi[ax],
                                 mode=WALL_SERVO, target_stress=confinement,
                                 servo_gain=servo_gain, area=area[ax]))
    wl.steps = int(math.ceil(axial_strain * span[2] / (platen_speed * dt)))
    wl.info.update({"span0": span.tolist(), "confinement": confinement,
                    "platen_speed": platen_speed, "gap": g})
    return wl


def _sequential_spheres(rng: np.random.Generator, radii: np.ndarray, L: float, frac: float) -> np.ndarray:
    """Centres in [0, L]^3 for spheres of radii frac * radii, placed largest first
    by random sequential addition without overlap (a hashed grid keeps each
    placement test local)."""
    from scipy.spatial import cKDTree
    order = np.argsort(-radii)
    r = frac * radii
    rmax = r.max()
    pts = np.zeros((len(radii), 3))
    placed = []
    tree = None
    since = 0
    for k in order:
        for _ in range(100000):
            c = rng.uniform(r[k], L - r[k], size=3)
            ok = True
            if tree is not None:
                near = tree.query_ball_point(c, r[k] + rmax)
                ok = all(np.sum((pts[j] - c) ** 2) >= (r[j] + r[k]) ** 2 for j in (placed[q] for q in near))
            if ok:
                for j in placed[len(placed) - since:]:
                    if np.sum((pts[j] - c) ** 2) < (r[j] + r[k]) ** 2:
                        ok = False
                        break
            if ok:
                break
        else:
            raise RuntimeError("sphere placement did not converge; lower frac")
        pts[k] = c
        placed.append(k)
        since += 1
        if since >= 64:  # rebuild the tree over everything placed so far
            tree = cKDTree(pts[placed])
            since = 0
    return pts


def large_aggregate(seed: int = 0, n_grains: int = 1000, mean_radius: float = 0.5e-3, sigma: float = 0.3,
                    h: float = 4.1e-5, dt: float = 4.0e-9, platen_speed: float = 10.0, axial_strain: float = 0.05,
                    material: Material = SAND, rebuild_every: int = 20, min_grain_nodes: int = 20) -> Workload:
    """A dense aggregate of n_grains grains with log-normal sizes confined by six walls.

    Radii r ~ LogNormal(ln(mean_radius) - sigma^2/2, sigma) (mean mean_radius);
    the box holds their total volume.  Seeds are spread by random sequential
    addition of spheres of 0.6 r, and every node centre (i + 1/2) h of the box
    joins the seed of least power distance |x - c|^2 - r^2 (a Laguerre
    tessellation), so cell volumes follow the radii and neighbouring grains
    touch face to face without pressing.  Walls one spacing beyond the nodes:
    floor fixed (normal +z), platen moving down at platen_speed, four fixed
    lateral walls; steps cover axial_strain of the box height.
    """
    rng = np.random.default_rng(seed)
    from scipy.spatial import cKDTree
    params = default_params(h, dt, rebuild_every=rebuild_every)
    radii = rng.lognormal(math.log(mean_radius) - 0.5 * sigma * sigma, sigma, size=n_grains)
    L = float(np.sum(4.0 / 3.0 * math.pi * radii ** 3)) ** (1.0 / 3.0)
    n_side = int(round(L / h))
    L = n_side * h
    seeds = _sequential_spheres(rng, radii, L, 0.6)
    # grains in a coarse space-filling order so neighbours stay close in memory
    cell = np.floor(seeds / (L / 8.0)).clip(0, 7).astype(np.int64)
    perm = np.lexsort((seeds[:, 0], cell[:, 0], cell[:, 1], cell[:, 2]))
    seeds, radii = seeds[perm], radii[perm]
    r = np.arange(n_side)
    tree = cKDTree(seeds)
    kq = min(16, n_grains)
    gid = np.empty(n_side ** 3, dtype=np.int64)
    for i0 in range(0, n_side, 16):  # slabs of the lattice keep the query's memory small
        I, J, K = np.meshgrid(r[i0:i0 + 16], r, r, indexing="ij")
        x = (np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1) + 0.5) * h
        d, idx = tree.query(x, k=kq)
        power = d * d - radii[idx] ** 2
        gid[i0 * n_side * n_side:(i0 + I.shape[0]) * n_side * n_side] = idx[np.arange(len(idx)), np.argmin(power, axis=1)]
    I, J, K = np.meshgrid(r, r, r, indexing="ij")
    lat = np.stack([I.ravel(), J.ravel(), K.ravel()]).astype(np.int64)
    order = np.argsort(gid, kind="stable")
    bounds = np.searchsorted(gid[order], np.arange(n_grains + 1))
    blocks = []
    for gr in range(n_grains):
        sel = order[bounds[gr]:bounds[gr + 1]]
        if sel.size < min_grain_nodes:
            continue
        # one node order (x slowest, z fastest) for every grain of the shared lattice
        ijk, origin = _grain_block(lat[:, sel], np.full(3, 0.5 * h), h, axes=(0, 1, 2))
        blocks.append((ijk, origin, h, 0))
    wl = _assemble("large_aggregate", blocks, [material], params, [], [], 1,
                   info={"seed": seed, "n_grains": len(blocks), "box": L})
    lo = wl.X.min(axis=1) - h
    hi = wl.X.max(axis=1) + h
    span = hi - lo
    area = [span[1] * span[2], span[0] * span[2], span[0] * span[1]]
    wl.walls = [
        Wall(normal=(0.0, 0.0, 1.0), offset=lo[2], mode=WALL_FIXED, area=area[2]),
        Wall(normal=(0.0, 0.0, -1.0), offset=-hi[2], mode=WALL_VELOCITY, velocity=platen_speed, area=area[2]),
    ]
    for ax in (0, 1):
        for sgn in (1.0, -1.0):
            nrm = [0.0, 0.0, 0.0]
            nrm[ax] = sgn
            wl.walls.append(Wall(normal=tuple(nrm), offset=lo[ax] if sgn > 0 else -hi[ax], mode=WALL_FIXED,
                                 area=area[ax]))
    wl.steps = int(math.ceil(axial_strain * span[2] / (platen_speed * dt)))
    wl.info.update({"span0": span.tolist(), "platen_speed": platen_speed, "radii_mean": float(radii.mean())})
    return wl


# ----------------------------------------------------------------------------
# shape study: 125 grains of one shape on a cubic grid, compressed by the lid
# ----------------------------------------------------------------------------

SHAPES = ("sphere", "shell", "jack")


def _rotation(rng: np.random.Generator) -> np.ndarray:
    """A uniformly distributed rotation (normalised Gaussian quaternion)."""
    q = rng.normal(size=4)
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def shape_grain(rng: np.random.Generator, shape: str, radius: float, h: float,
                arm_half_width: float = 0.25, cavity: float = 0.5):
    """Lattice points of one grain of the shape study, all within the ball of
    the given radius about the grain centre.

    sphere: the ball; shell: the ball less a concentric cavity of cavity*radius;
    jack: three orthogonal square bars of half-width arm_half_width*radius
    through the centre, clipped to the ball, in a seeded random orientation.
    Every grain gets a seeded sub-cell lattice offset.  Returns (offsets (3,n)
    int, centre-relative lattice shift (3,), cavity radius or 0)."""
    if shape not in SHAPES:
        raise ValueError(f"unknown shape {shape!r}")
    o = rng.uniform(0.0, 1.0, size=3)
    rot = _rotation(rng) if shape == "jack" else None
    nmax = int(math.ceil(radius / h)) + 1
    r = np.arange(-nmax, nmax + 1)
    I, J, K = np.meshgrid(r, r, r, indexing="ij")
    pts = np.stack([I.ravel(), J.ravel(), K.ravel()])
    q = (pts + o[:, None]) * h
    d2 = np.sum(q * q, axis=0)
    inside = d2 <= radius * radius
    rin = 0.0
    if shape == "shell":
        rin = cavity * radius
        inside &= d2 >= rin * rin
    elif shape == "jack":
        a = arm_half_width * radius
        body = np.abs(rot.T @ q) <= a  # coordinates in the jack's own frame
        inside &= np.sum(body, axis=0) >= 2  # inside at least one bar
    return pts[:, inside], o, rin


def shape_study(shape: str = "sphere", seed: int = 0, grid=5, radius: float = 1e-3,
                h: float = 1e-4, gap: float = 1.0, lid_speed: float = 10.0, dt: float = 1e-8,
                duration: float = 5e-4, material: Material = SAND, rebuild_every: int = 5,
                arm_half_width: float = 0.25, cavity: float = 0.5) -> Workload:
    """grid^3 grains of one shape (Sec. 7.6: 125 grains of radius 1 mm on a
    cubic grid, solid spheres, hollow spheres or jacks) in a box of rigid walls
    whose lid moves down at lid_speed (10 m/s in the paper).  grid is the
    number of grains per side, or (nx, ny, nz) (1, 1, 2: two stacked grains,
    the double hollow sphere of Sec. 6).

    Grid pitch 2*radius + gap*h; the floor and the four side walls sit R_c
    beyond the outermost nodes, the lid R_c above the highest node, so no node
    touches a wall at t = 0.  Shell cavities are cut with the chord rule.
    steps cover duration (the paper plots 100 x 5 us)."""
    rng = np.random.default_rng(seed)
    params = default_params(h, dt, rebuild_every=rebuild_every)
    pitch = 2.0 * radius + gap * h
    gx, gy, gz = (grid, grid, grid) if isinstance(grid, int) else tuple(grid)
    blocks, cuts = [], []
    for g in range(gx * gy * gz):
        a, b, c = g % gx, (g // gx) % gy, g // (gx * gy)
        centre = np.array([a, b, c], dtype=np.float64) * pitch
        off, o, rin = shape_grain(rng, shape, radius, h, arm_half_width, cavity)
        ijk, origin = _grain_block(off, centre + o * h, h)
        blocks.append((ijk, origin, h, 0))
        if rin > 0:
            ijk_c = (centre - origin) / h
            cen_half = np.rint(2.0 * ijk_c).astype(np.int64)
            r_half = 2.0 * rin / h - 1.0  # stays inside the unmeshed cavity after rounding
            cuts.append(Cut(kind=CUT_CAVITY_CHORD, grain=g, center=tuple(int(v) for v in cen_half),
                            radius2=int(math.floor(r_half * r_half))))
    steps = int(math.ceil(duration / dt))
    wl = _assemble(f"shape_study_{shape}", blocks, [material], params, [], cuts, steps,
                   info={"seed": seed, "shape": shape, "grid": grid, "radius": radius, "pitch": pitch})
    Rc = params.contact_radius
    lo = wl.X.min(axis=1) - Rc
    hi = wl.X.max(axis=1) + Rc
    span = hi - lo
    area = [span[1] * span[2], span[0] * span[2], span[0] * span[1]]
    wl.walls = [
        Wall(normal=(0.0, 0.0, 1.0), offset=lo[2], mode=WALL_FIXED, area=area[2]),
        Wall(normal=(0.0, 0.0, -1.0), offset=-hi[2], mode=WALL_VELOCITY, velocity=lid_speed, area=area[2]),
    ]
    for ax in (0, 1):
        for sgn in (1.0, -1.0):
            nrm = [0.0, 0.0, 0.0]
            nrm[ax] = sgn
            wl.walls.append(Wall(normal=tuple(nrm), offset=lo[ax] if sgn > 0 else -hi[ax], mode=WALL_FIXED,
                                 area=area[ax]))
    wl.info.update({"span0": span.tolist(), "lid_speed": lid_speed})
    return wl


# ----------------------------------------------------------------------------
# named workloads with the sizes of the paper-scale experiments
# ----------------------------------------------------------------------------

def workload(name: str, **kw) -> Workload:
    if name == "two_spheres":
        return two_spheres(**kw)
    if name == "two_spheres_break":
        kw.setdefault("speed", 50.0)
        return two_spheres(**kw)
    if name == "notched_plate":
        return notched_plate(**kw)
    if name == "grain_aggregate":
        return grain_aggregate(**kw)
    if name == "rve_aggregate":
        return rve_aggregate(**kw)
    if name == "large_aggregate":
        return large_aggregate(**kw)
    if name == "shape_study":
        return shape_study(**kw)
    raise KeyError(name)
