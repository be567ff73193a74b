"""Tiled bond loop (u of a tile and its halo in LDS, bond memory in per-node
class masks) against the slice path: bitwise the same node state and bond
state, also across hand-overs between the paths and checkpoints, with wall
reactions equal to rounding; parity with the oracle through the tiles."""
import numpy as np
import pytest

from paper_2506_05362_amd import inputs as I

pytestmark = pytest.mark.gpu

# force_density comes before any field whose read hands the bond memory over to
# the column words, so it checks that its own read does
NODE_FIELDS = ["displacement", "velocity", "accel", "force_density", "bond_broken", "intact_count", "damage",
               "step"]


def cases():
    return {
        "spheres_fracture": I.two_spheres(radius_cells=6, speed=50.0, gap=0.0, rebuild_every=7),
        "plate_notched": I.notched_plate(nx=40, ny=30, nz=6, h=5e-4, notch_x=(10 * 5e-4, 30 * 5e-4),
                                         notch_len=15 * 5e-4, steps=1),
        "aggregate_hollow": I.grain_aggregate(n_grains=6, grid=(3, 2, 1), n_min=800, n_max=3000, seed=2,
                                              platen_speed=5.0, rebuild_every=10),
        # tessellations on one lattice: tiles over one box across all grains
        "lattice_aggregate": I.large_aggregate(seed=2, n_grains=30, h=1.6e-4, platen_speed=50.0),
        "lattice_volume": I.rve_aggregate(seed=3, n_grains=12, nodes_per_grain=300, confinement=15e6,
                                          platen_speed=20.0, rebuild_every=10),
    }


LATTICE_CASES = ("lattice_aggregate", "lattice_volume")


def run(wl, steps, bond_path, loop=0, lattice=None):
    from paper_2506_05362_amd import pd
    sim = pd.Sim(wl)
    sim.set_launch(loop=loop, bond_path=bond_path)
    assert sim.get_launch()["bond_path"] == bond_path
    if lattice is not None:
        assert sim.tile_info()["lattice"] == lattice
    sim.step(steps)
    out = {f: sim.get(f) for f in NODE_FIELDS + ["wall_force"]}
    sim.close()
    return out


def assert_same(a, b, what):
    for f in NODE_FIELDS:
        assert np.array_equal(a[f], b[f]), f"{what}: {f}"
    if a["wall_force"].size:
        scale = max(np.abs(a["wall_force"]).max(), 1e-300)
        assert np.abs(a["wall_force"] - b["wall_force"]).max() <= 1e-12 * scale, what


@pytest.mark.parametrize("case", list(cases()))
def test_tiles_bitwise_equal_to_slices(case):
    from paper_2506_05362_amd import pd
    wl = cases()[case]
    print(f"[{case}] {wl.n_nodes} nodes, {wl.n_grains} grains", flush=True)
    steps = 60
    ref = run(wl, steps, pd.BONDS_SLICES)
    for loop in (pd.LOOP_GRAPH, pd.LOOP_DIRECT):
        got = run(wl, steps, pd.BONDS_TILES, loop, lattice=case in LATTICE_CASES)
        assert_same(ref, got, f"{case} loop {loop}")
    if case == "spheres_fracture":
        assert ref["bond_broken"].any()  # the comparison covered bond breaking


def test_hand_over_between_paths_and_checkpoint():
    from paper_2506_05362_amd import pd
    wl = cases()["spheres_fracture"]
    a = pd.Sim(wl)
    a.step(75)
    b = pd.Sim(wl)
    b.step(20)
    b.set_launch(bond_path=pd.BONDS_TILES)
    b.step(20)
    blob = b.get_state()  # taken on the tile path
    b.set_launch(bond_path=pd.BONDS_SLICES)
    b.step(35)
    for f in NODE_FIELDS:
        assert np.array_equal(a.get(f), b.get(f)), f
    c = pd.Sim(wl)
    c.set_launch(bond_path=pd.BONDS_TILES)
    c.set_state(blob)  # restored onto the tile path
    assert c.info()["step"] == 40
    c.step(35)
    for f in NODE_FIELDS:
        assert np.array_equal(a.get(f), c.get(f)), f


def test_tile_path_matches_oracle(oracle_lib):
    from paper_2506_05362_amd import pd
    wl = I.two_spheres(radius_cells=6, speed=50.0, gap=0.0, rebuild_every=7)
    sim = pd.Sim(wl)
    sim.set_launch(bond_path=pd.BONDS_TILES)
    ora = oracle_lib.Oracle(wl, flags=oracle_lib.CELL_LIST)
    sim.step(80)
    ora.step(80)
    so = ora.state()
    for name, key in (("displacement", "u"), ("velocity", "v")):
        g = sim.get(name)
        assert np.abs(g - so[key]).max() <= 1e-9 * np.abs(so[key]).max(), name
    from test_gpu_parity import assert_broken_sets
    assert_broken_sets(sim, ora, what="tile path")
    assert sim.bonds()[2].any()


def test_tile_path_argument_errors():
    from paper_2506_05362_amd import pd
    wl = I.two_spheres(radius_cells=3)
    s = pd.Sim(wl, build=False)
    with pytest.raises(pd.PDError) as e:
        s.set_launch(bond_path=pd.BONDS_TILES)  # bonds not built yet
    assert e.value.status == pd.PD_ERR_STATE
    s.build_bonds()
    for bad in (dict(loop=pd.LOOP_PERSISTENT, bond_path=pd.BONDS_TILES),
                dict(loop=pd.LOOP_PER_GRAIN, bond_path=pd.BONDS_TILES), dict(bond_path=7)):
        with pytest.raises(pd.PDError) as e:
            s.set_launch(**bad)
        assert e.value.status == pd.PD_ERR_INVALID
    m2 = I.two_spheres(radius_cells=3)
    m2.params.horizon_factor = 2
    s2 = pd.Sim(m2)
    with pytest.raises(pd.PDError) as e:
        s2.set_launch(bond_path=pd.BONDS_TILES)
    assert e.value.status == pd.PD_ERR_UNSUPPORTED
