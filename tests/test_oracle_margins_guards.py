"""Pins of the oracle's break-decision margins, its Verlet-skin guard, the
gravity term of its energy and its self-contact candidate search.

Each compares the oracle with something it does not compute itself: a
closed-form stretch, the closed-form trajectory of a linear oscillator, exact
displacements of a free node, the conservation of energy under a constant body
force, or an O(N^2) brute force.
"""
import math

import numpy as np
import pytest

from paper_2506_05362_amd import inputs as I
from test_oracle_pins import two_node

H = 1e-4
K_SAND = 14.9e9


def s0_of(Gc=10.0, flags=0):
    from oracle import pdref
    return pdref.constants(K_SAND, Gc, 3 * H, flags)[1]


# ---------------------------------------------------------------------------
# break-decision margin per bond (Sec. 3.1.1 bond memory)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("alpha,absr", [(0.3, False), (0.9, False), (-0.5, False), (1.2, False), (2.0, False),
                                        (-0.5, True), (-1.3, True), (0.6, True)])
@pytest.mark.parametrize("Gc", [10.0, 160.0])
def test_bond_margin_of_a_prestretched_pair(oracle_lib, alpha, absr, Gc):
    """Two bonded nodes pre-stretched to s = alpha s0: the first evaluation's
    margin is |alpha - 1| (tension test) or ||alpha| - 1| (|s| test) on both
    directed entries, the bond breaks iff alpha (or |alpha|) exceeds 1, and the
    margin is relative: a 16 times larger G_c (4 times larger s0) leaves it
    unchanged."""
    s0 = s0_of(Gc)
    mat = I.Material(bulk_modulus=K_SAND, density=2600.0, fracture_energy=Gc)
    wl = two_node(stretch=alpha * s0, mat=mat)
    o = oracle_lib.Oracle(wl, flags=oracle_lib.ABS_STRETCH if absr else 0)
    m = o.bond_margin()
    expect = abs(abs(alpha) - 1.0) if absr else abs(alpha - 1.0)
    assert len(m) == 2
    assert m == pytest.approx([expect, expect], rel=1e-9)
    assert o.min_margin() == pytest.approx(expect, rel=1e-9)
    broke = (abs(alpha) > 1.0) if absr else (alpha > 1.0)
    assert o.bonds()[2].tolist() == [int(broke)] * 2


def test_bond_margin_is_the_minimum_over_the_trajectory(oracle_lib):
    """A bonded pair at rest length pulled apart by opposite velocities: the
    relative coordinate of position-form velocity Verlet is exactly
    w_n = (dt V / sin theta) sin(n theta), cos theta = 1 - omega^2 dt^2 / 2, so
    the recorded margin after N steps is min over n <= N of |w_n/(h s0) - 1|.
    Taken before and after the peak it tracks the largest stretch so far, and
    it is not lowered by compression."""
    rho = 2600.0
    s0 = s0_of()
    c = 18 * K_SAND / (math.pi * (3 * H) ** 4)
    w2 = 2 * c * H ** 3 / (rho * H)
    dt = 0.15 / math.sqrt(w2)
    th = math.acos(1 - w2 * dt * dt / 2)
    amp = 0.7 * s0 * H  # peak of w
    V = amp * math.sin(th) / dt
    wl = two_node(stretch=0.0, dt=dt)
    wl.v0[0, 0], wl.v0[0, 1] = -V / 2, V / 2
    o = oracle_lib.Oracle(wl)
    assert o.bond_margin() == pytest.approx([1.0, 1.0], abs=1e-15)  # s = 0 at t = 0
    done = 0
    for n_steps in (4, 9, 30):  # before the peak (n theta < pi/2), around it, past a half period
        o.step(n_steps - done)
        done = n_steps
        w = [dt * V / math.sin(th) * math.sin(k * th) for k in range(0, done + 1)]
        expect = min(abs(x / (H * s0) - 1.0) for x in w)
        assert o.bond_margin() == pytest.approx([expect, expect], rel=1e-8)
        if n_steps == 4:
            assert expect > 0.31  # the peak (margin 0.3) has not been reached yet
    assert expect == pytest.approx(0.3, abs=0.01)
    assert o.bonds()[2].sum() == 0


def test_bond_margins_of_a_shaken_ball(oracle_lib):
    """A ball with a random displacement field: after the build each bond's
    margin is |s/s0 - 1| of its stretch s = (|xi + eta| - |xi|)/|xi| computed
    here from the positions, whether the bond broke in that evaluation or not;
    further steps only lower margins (a minimum over evaluations), bonds broken
    at the build keep theirs, and the global margin is the smallest one."""
    off = I.sphere_offsets(4)
    ijk, origin = I.grain_block(off, np.zeros(3), H)
    params = I.default_params(H, 1e-9)
    wl = I.assemble("ball", [(ijk, origin, H, 0)], [I.SAND], params, [], [], 10)
    rng = np.random.default_rng(11)
    wl.u0[:] = rng.normal(0, 2e-3 * H, size=wl.u0.shape)
    s0 = s0_of()
    o = oracle_lib.Oracle(wl)
    rp, col, br0 = o.bonds()
    i = np.repeat(np.arange(wl.n_nodes), np.diff(rp))
    xi = wl.X[:, col] - wl.X[:, i]
    y = xi + (wl.u0[:, col] - wl.u0[:, i])
    l0 = np.sqrt((xi * xi).sum(axis=0))
    s = (np.sqrt((y * y).sum(axis=0)) - l0) / l0
    m0 = o.bond_margin().copy()
    assert m0 == pytest.approx(np.abs(s / s0 - 1.0), rel=1e-6, abs=1e-9)
    assert np.array_equal(br0.astype(bool), s > s0)
    assert 0 < br0.sum() < len(br0)
    o.step(10)
    m = o.bond_margin()
    assert np.all(m <= m0)
    assert np.array_equal(m[br0 > 0], m0[br0 > 0])  # broken bonds are not evaluated again
    assert np.any(m[br0 == 0] < m0[br0 == 0])
    assert o.min_margin() == m.min()


# ---------------------------------------------------------------------------
# Verlet-skin guard (candidate lists rebuilt on a fixed cadence)
# ---------------------------------------------------------------------------

def _drifting_node(frac, rebuild_every=10, n_grains=2, self_contact=False):
    """Two one-node grains 20 h apart; node 1 drifts at constant velocity so
    that at the first rebuild it has moved frac * skin/2 (no force acts: the
    pair is far outside R_c + skin, and no bonds exist)."""
    dt = 1e-9
    params = I.default_params(H, dt, rebuild_every=rebuild_every)
    params.self_contact = self_contact
    skin = params.skin
    off = np.zeros((3, 1), dtype=np.int64)
    blocks = [(*I.grain_block(off, np.zeros(3), H), H, 0)]
    if n_grains == 2:
        blocks.append((*I.grain_block(off, np.array([20 * H, 0.0, 0.0]), H), H, 0))
    wl = I.assemble("drift", blocks, [I.SAND], params, [], [], rebuild_every)
    v = frac * 0.5 * skin / (rebuild_every * dt)
    wl.v0[1, -1] = v
    return wl


@pytest.mark.parametrize("frac,expect", [(0.99, 0), (1.01, -5)])
def test_skin_guard_at_half_the_skin(oracle_lib, frac, expect):
    """A node that moved more than skin/2 since the last rebuild stops the run
    with the instability status at the next rebuild; 1% short of it does not."""
    wl = _drifting_node(frac)
    o = oracle_lib.Oracle(wl, flags=oracle_lib.CELL_LIST)
    assert o.step(wl.params.rebuild_every - 1) == 0
    assert not o.skin_exceeded()  # nine tenths of the way: below skin/2 either way
    assert o.step(1) == expect
    u = o.state()["u"]
    assert u[1, -1] == pytest.approx(frac * 0.5 * wl.params.skin, rel=1e-12)


def test_skin_query_between_rebuilds(oracle_lib):
    """The guard's test itself: nine steps into a drift that reaches 1.2 skin/2 at
    the tenth, the node is already 1.08 skin/2 away from where it was binned."""
    wl = _drifting_node(1.2)
    o = oracle_lib.Oracle(wl, flags=oracle_lib.CELL_LIST)
    assert not o.skin_exceeded()
    assert o.step(9) == 0
    assert o.skin_exceeded()


def test_skin_guard_needs_a_contact_partner(oracle_lib):
    """One grain without self-contact has no contact pairs to miss: no guard.
    With self-contact the same drift trips it."""
    wl = _drifting_node(1.5, n_grains=1)
    o = oracle_lib.Oracle(wl, flags=oracle_lib.CELL_LIST)
    assert o.step(wl.params.rebuild_every) == 0
    wl = _drifting_node(1.5, n_grains=1, self_contact=True)
    o = oracle_lib.Oracle(wl, flags=oracle_lib.CELL_LIST)
    assert o.step(wl.params.rebuild_every) == -5


def test_adaptive_rebuild_counts_the_drift(oracle_lib):
    """With early rebuilds the drift of 0.12 skin/2 per step never stops the
    run: the list is rebuilt at the ninth step after each rebuild (1.08 skin/2;
    the eighth is at 0.96), so once in every cadence of ten steps."""
    wl = _drifting_node(1.2)
    wl.params.adaptive_rebuild = True
    o = oracle_lib.Oracle(wl, flags=oracle_lib.CELL_LIST)
    assert o.step(100) == 0
    assert o.early_rebuilds() == 10
    assert not o.skin_exceeded()  # step 100 is a cadence rebuild
    u = o.state()["u"]
    assert u[1, -1] == pytest.approx(100 * 0.12 * 0.5 * wl.params.skin, rel=1e-12)


def _fast_collision(rebuild_every, adaptive):
    # the closest pair starts 1.2 skins beyond R_c: out of the first list
    wl = I.two_spheres(radius_cells=4, speed=50.0, gap=0.3 * H, rebuild_every=rebuild_every)
    wl.params.adaptive_rebuild = adaptive
    return wl


def test_adaptive_rebuild_equals_a_rebuild_before_every_evaluation(oracle_lib):
    """Two balls closing at 50 m/s move skin/2 in 25 steps.  A rebuild every
    100 steps alone misses the pairs that come within R_c after the first list
    (the velocities differ by metres per second at step 100, where the guard
    stops the run); with early rebuilds the state is bitwise that of a rebuild
    before every evaluation: each list holds every pair within R_c, sorted, and
    the contact sum only takes those."""
    steps = 300
    plain = oracle_lib.Oracle(_fast_collision(100, False), flags=oracle_lib.CELL_LIST, threads=2)
    every = oracle_lib.Oracle(_fast_collision(1, False), flags=oracle_lib.CELL_LIST, threads=2)
    assert plain.step(steps) == -5
    assert plain.step_count == 100  # it stops after the step whose rebuild found the drift
    assert every.step(100) == 0
    assert np.abs(plain.state()["v"] - every.state()["v"]).max() > 1.0
    early = oracle_lib.Oracle(_fast_collision(100, True), flags=oracle_lib.CELL_LIST, threads=2)
    assert early.step(steps) == 0 and every.step(steps - 100) == 0
    assert early.early_rebuilds() >= steps // 25 - 4
    assert every.early_rebuilds() == 0
    se, s1 = early.state(), every.state()
    for k in ("u", "v", "a"):
        assert np.array_equal(se[k], s1[k]), k
    assert np.array_equal(early.bonds()[2], every.bonds()[2])
    # the balls met: the struck one moves along -x
    nA = int(early.wl.grain_begin[1])
    assert se["v"][0, :nA].mean() < -1.0


# ---------------------------------------------------------------------------
# gravity potential of the energy diagnostic (Sec. 5.1 body force)
# ---------------------------------------------------------------------------

def test_gravity_potential_conserves_energy_in_free_fall(oracle_lib):
    """A node thrown upwards under a body force g: velocity Verlet integrates a
    constant acceleration exactly, so kinetic energy plus the gravity potential
    -rho V g.u stays at its initial value to rounding while each changes by
    many times that; a wrong sign or a missing term would not."""
    dt = 1e-8
    params = I.default_params(H, dt)
    g = np.array([3e5, 0.0, -9.81e6])
    params.gravity = tuple(g)
    off = np.zeros((3, 1), dtype=np.int64)
    wl = I.assemble("fall", [(*I.grain_block(off, np.zeros(3), H), H, 0)], [I.SAND], params, [], [], 1)
    wl.v0[:, 0] = [2.0, -1.0, 5.0]
    o = oracle_lib.Oracle(wl)
    e0 = o.energy()
    assert e0["gravity"] == 0.0
    for _ in range(5):
        o.step(200)
        e = o.energy()
        st = o.state()
        rho, V = I.SAND.density, H ** 3
        assert e["gravity"] == pytest.approx(-rho * V * float(g @ st["u"][:, 0]), rel=1e-12)
        assert abs(e["gravity"]) > 0.1 * e0["kinetic"]
        assert e["total"] == pytest.approx(e0["total"], rel=1e-11)
    # the node rose, then fell below its start: the potential took both signs
    assert st["u"][2, 0] < 0


# ---------------------------------------------------------------------------
# self-contact candidate search (Sec. 5)
# ---------------------------------------------------------------------------

def brute_self_candidates(wl, u):
    """Every other node, of any grain, within R_c + skin (self-contact keeps the
    node's own grain; whether a pair is bonded is decided at the force)."""
    X = wl.X
    cut = wl.params.contact_radius + wl.params.skin
    rows = []
    for i in range(wl.n_nodes):
        y = (X - X[:, i:i + 1]) + (u - u[:, i:i + 1])
        d2 = (y[0] * y[0] + y[1] * y[1]) + y[2] * y[2]
        sel = d2 < cut * cut
        sel[i] = False
        rows.append(np.where(sel)[0].tolist())
    return rows


@pytest.mark.parametrize("cell_list", [False, True])
def test_self_contact_candidates_match_brute_force(oracle_lib, cell_list):
    """With self-contact the candidate rows (O(N^2) scan and cell list) are
    exactly the brute-force rows including the node's own grain, for two
    shaken, interpenetrating balls."""
    from test_oracle_lists import assert_rows_equal
    wl = I.two_spheres(radius_cells=4, gap=0.0)
    wl.params.self_contact = True
    wl.params.contact_radius = 0.95 * H
    wl.params.skin = 0.6 * H
    rng = np.random.default_rng(4)
    wl.u0[:] = rng.normal(0, 0.2 * H, size=wl.u0.shape)
    wl.u0[0, wl.grain_begin[1]:] -= 2.5 * H
    flags = oracle_lib.SELF_CONTACT | (oracle_lib.CELL_LIST if cell_list else 0)
    o = oracle_lib.Oracle(wl, flags=flags)
    rp, col = o.candidates()
    rows = brute_self_candidates(wl, wl.u0)
    g = wl.grain_of_node()
    own = sum(int((g[r] == g[i]).sum()) for i, r in enumerate(rows) if r)
    other = sum(len(r) for r in rows) - own
    assert own > wl.n_nodes and other > 50  # both kinds of pair are present
    assert_rows_equal(rp, col, rows)
