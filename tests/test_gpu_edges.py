"""Degenerate inputs on the GPU: a mesh without nodes in every step loop, and
a node-free grain among others through both bond paths."""
import numpy as np
import pytest

from test_gpu_parity import assert_state_close, rel_inf
from test_oracle_edges import empty_mesh, spheres

pytestmark = pytest.mark.gpu


def gpu_sim(wl, **kw):
    from paper_2506_05362_amd import pd
    return pd.Sim(wl, **kw)


@pytest.mark.parametrize("loop", [0, 1, 2, 3])
def test_empty_mesh_in_every_step_loop(oracle_lib, loop):
    """No nodes: the steps run (the wall moves as in the oracle, with no
    reaction) and every node field is empty."""
    wl = empty_mesh()
    ora = oracle_lib.Oracle(wl, flags=oracle_lib.CELL_LIST)
    assert ora.step(50) == 0
    sim = gpu_sim(wl)
    sim.set_launch(loop=loop)
    sim.step(50)
    info = sim.info()
    assert (info["n_nodes"], info["nnz"], info["step"]) == (0, 0, 50)
    assert sim.get("displacement").shape == (3, 0)
    assert sim.get("damage").size == 0
    fo, oo = ora.walls()
    assert np.all(sim.get("wall_force") == 0.0)
    assert rel_inf(sim.get("wall_offset"), oo) <= 1e-12
    sim.close()


@pytest.mark.parametrize("loop,bond_path", [(0, 0), (3, 0), (2, 0), (0, 1)])
def test_node_free_grain_between_grains(oracle_lib, loop, bond_path):
    """Two balls meeting at 20 m/s with a node-free grain listed between them:
    state within 1e-9 of the oracle through the contact, and bitwise that of
    the same balls without the empty grain."""
    wl = spheres(True)
    ora = oracle_lib.Oracle(wl, flags=oracle_lib.CELL_LIST, threads=8)
    assert ora.step(300) == 0
    runs = []
    for w in (wl, spheres(False)):
        sim = gpu_sim(w)
        sim.set_launch(loop=loop, bond_path=bond_path)
        sim.step(300)
        runs.append({k: sim.get(k) for k in ("displacement", "velocity", "accel", "force_density", "damage")})
        if w is wl:
            assert_state_close(sim, ora, what=f"node-free grain, loop {loop}, bonds {bond_path}")
        sim.close()
    for k in runs[0]:
        assert np.array_equal(runs[0][k], runs[1][k]), k
