"""Degenerate inputs of the oracle: a mesh without nodes, and a grain without
nodes among others (node-free grains change nothing but the grain ids)."""
import numpy as np
import pytest

from paper_2506_05362_amd import inputs as I

H = 1e-4
DT = 1e-8
SPEED = 20.0


def empty_block():
    return (np.zeros((3, 0), np.int32), np.zeros(3), H, 0)


def empty_mesh():
    """One grain without nodes and a wall moving at 2 m/s."""
    params = I.default_params(H, DT, rebuild_every=5)
    wall = I.Wall(normal=(0.0, 0.0, 1.0), offset=-1e-3, mode=I.WALL_VELOCITY, velocity=2.0)
    return I.assemble("empty", [empty_block()], [I.SAND], params, [wall], [], 1)


def spheres(with_empty_grain: bool):
    """Two balls of radius 3 h closing at 20 m/s (surfaces 1.2 h apart, contact
    from about step 125), listed with or without a node-free grain between them."""
    params = I.default_params(H, DT, rebuild_every=5)
    a = I.grain_block(I.sphere_offsets(3), np.zeros(3), H)
    b = I.grain_block(I.sphere_offsets(3), np.array([7.2 * H, 0.0, 0.0]), H)
    blocks = [(a[0], a[1], H, 0)] + ([empty_block()] if with_empty_grain else []) + [(b[0], b[1], H, 0)]
    wl = I.assemble("spheres", blocks, [I.SAND], params, [], [], 300)
    wl.v0[0, : a[0].shape[1]] = SPEED
    return wl


def test_empty_mesh_steps_and_moves_its_wall(oracle_lib):
    wl = empty_mesh()
    o = oracle_lib.Oracle(wl, flags=oracle_lib.CELL_LIST)
    assert o.nnz == 0
    assert o.step(50) == 0 and o.step_count == 50
    force, offset = o.walls()
    assert np.all(force == 0.0)
    assert offset[0] == pytest.approx(-1e-3 + 50 * DT * 2.0, rel=1e-12)
    assert all(v == 0.0 for v in o.energy().values())


def test_node_free_grain_changes_nothing(oracle_lib):
    """The same two balls with a node-free grain listed between them: bitwise
    the same trajectory through their contact (grain ids only tell grains apart)."""
    runs = []
    for with_empty in (False, True):
        o = oracle_lib.Oracle(spheres(with_empty), flags=oracle_lib.CELL_LIST, threads=2)
        assert o.step(300) == 0
        runs.append(o)
    s0, s1 = runs[0].state(), runs[1].state()
    for k in ("u", "v", "a", "F"):
        assert np.array_equal(s0[k], s1[k]), k
    assert np.array_equal(runs[0].bonds()[2], runs[1].bonds()[2])
    nA = I.sphere_offsets(3).shape[1]
    assert s0["v"][0, nA:].max() > 1.0  # the struck ball moves: the contact happened
