"""GPU tests of the library's guard paths and the remaining state paths: the
instability flags (Verlet skin, candidate capacity, non-finite force) halt the
run at the step that raised them, early candidate rebuilds in their place,
fixed nodes, and pd_get into device memory."""
import zlib

import numpy as np
import pytest

from paper_2506_05362_amd import inputs as I
from test_gpu_parity import assert_state_close, rel_inf
from test_oracle_margins_guards import _drifting_node, _fast_collision

pytestmark = pytest.mark.gpu


def gpu_sim(wl, **kw):
    from paper_2506_05362_amd import pd
    return pd.Sim(wl, **kw)


@pytest.mark.parametrize("frac", [0.99, 1.01])
def test_skin_guard_halts_at_the_flagged_step(oracle_lib, frac):
    """A node drifting frac * skin/2 per rebuild interval: 1% past the limit the
    call returns PD_ERR_UNSTABLE with the context at the first rebuild step
    (the steps after it did nothing), equal to the oracle stopped there; 1% short
    of it all 50 steps run."""
    from paper_2506_05362_amd import pd
    wl = _drifting_node(frac)
    R = wl.params.rebuild_every
    sim = gpu_sim(wl)
    ora = oracle_lib.Oracle(wl, flags=oracle_lib.CELL_LIST)
    st = sim.step_status(50)
    ost = ora.step(50)
    if frac > 1:
        assert st == pd.PD_ERR_UNSTABLE and ost == -5
        assert sim.info()["step"] == R == ora.step_count
        assert "skin" in pd.lib().pd_last_error(sim.h).decode()
    else:
        assert st == pd.PD_OK and ost == 0
        assert sim.info()["step"] == 50 == ora.step_count
    u = sim.get("displacement")
    assert u[1, -1] == pytest.approx(frac * 0.5 * wl.params.skin * sim.info()["step"] / R, rel=1e-12)
    assert_state_close(sim, ora, what=f"skin {frac}")
    # the flag was cleared when reported: stepping on is allowed again
    assert sim.step_status(1) in (pd.PD_OK, pd.PD_ERR_UNSTABLE)
    sim.close()


@pytest.mark.parametrize("loop,bond_path", [(0, 0), (1, 0), (3, 0), (0, 1), (1, 1)])
def test_early_rebuilds_match_the_oracle(oracle_lib, loop, bond_path):
    """Two balls closing at 50 m/s (skin/2 in 25 steps) with a cadence of 100
    steps: without early rebuilds the call stops at step 100 on the skin
    guard; with them all 300 steps run, in every step loop and bond path, and
    the state matches the oracle taking the same early rebuilds."""
    from paper_2506_05362_amd import pd
    plain = gpu_sim(_fast_collision(100, False))
    plain.set_launch(loop=loop, bond_path=bond_path)
    assert plain.step_status(300) == pd.PD_ERR_UNSTABLE
    assert plain.info()["step"] == 100
    plain.close()
    wl = _fast_collision(100, True)
    sim = gpu_sim(wl)
    sim.set_launch(loop=loop, bond_path=bond_path)
    ora = oracle_lib.Oracle(wl, flags=oracle_lib.CELL_LIST, threads=8)
    for _ in range(3):
        sim.step(100)
        assert ora.step(100) == 0
    assert sim.info()["step"] == 300
    assert_state_close(sim, ora, what=f"early rebuilds, loop {loop}, bonds {bond_path}")
    n = sim.loop_counts()["early_rebuilds"]
    # a displacement within rounding of skin/2 may be decided either way; one
    # rebuild more or less does not change the forces
    assert n > 0 and abs(n - ora.early_rebuilds()) <= 1, (n, ora.early_rebuilds())
    sim.close()


def test_early_rebuilds_equal_a_rebuild_every_step_bitwise():
    """The forces do not depend on when the candidates were built, only on
    their holding every pair within R_c: early rebuilds give bitwise the state
    of a rebuild before every evaluation."""
    early = gpu_sim(_fast_collision(100, True))
    every = gpu_sim(_fast_collision(1, False))
    early.step(300)
    every.step(300)
    assert early.loop_counts()["early_rebuilds"] > 0 and every.loop_counts()["early_rebuilds"] == 0
    for name in ("displacement", "velocity", "accel", "force_density", "damage"):
        assert np.array_equal(early.get(name), every.get(name)), name
    early.close()
    every.close()


def test_early_rebuilds_refuse_the_persistent_loop():
    from paper_2506_05362_amd import pd
    sim = gpu_sim(_fast_collision(100, True))
    with pytest.raises(pd.PDError, match="persistent"):
        sim.set_launch(loop=pd.LOOP_PERSISTENT)
    sim.close()


def _closing_blocks():
    """Two 4 x 4 x 4 blocks 2.5 h apart face to face, closing at 50 m/s, with a
    skin of h: the faces come within R_c + skin after about 110 steps and, a
    few rebuilds later, each face node has its opposite node and four diagonal
    ones in range."""
    h = 1e-4
    params = I.default_params(h, 1e-8, rebuild_every=5)
    params.skin = h
    b0 = I.grain_block(I.box_offsets(4, 4, 4), np.zeros(3), h)
    b1 = I.grain_block(I.box_offsets(4, 4, 4), np.array([5.5 * h, 0.0, 0.0]), h)
    wl = I.assemble("blocks", [(b0[0], b0[1], h, 0), (b1[0], b1[1], h, 0)], [I.SAND], params, [], [], 1)
    n0 = int(wl.grain_begin[1])
    wl.v0[0, :n0] = 25.0
    wl.v0[0, n0:] = -25.0
    return wl


def test_candidate_overflow_halts_at_the_rebuild(oracle_lib):
    """Two blocks closing in with a capacity of one candidate per node (rows of
    at most two): the first rebuild whose oracle rows exceed two candidates
    raises PD_ERR_UNSTABLE, and the context stops at that step."""
    from paper_2506_05362_amd import pd
    wl = _closing_blocks()
    ora = oracle_lib.Oracle(wl, flags=oracle_lib.CELL_LIST)
    assert ora.candidates()[1].size == 0
    flagged = None
    for k in range(1, 41):
        ora.step(wl.params.rebuild_every)
        rp, _ = ora.candidates()
        if np.diff(rp).max() > 2:
            flagged = k * wl.params.rebuild_every
            break
    assert flagged is not None
    sim = gpu_sim(wl, candidate_capacity_per_node=1)
    assert sim.step_status(400) == pd.PD_ERR_UNSTABLE
    assert sim.info()["step"] == flagged
    assert "capacity" in pd.lib().pd_last_error(sim.h).decode()
    sim.close()


def test_candidate_overflow_at_the_build():
    from paper_2506_05362_amd import pd
    wl = I.two_spheres(radius_cells=4, gap=0.0)
    wl.u0[0, wl.grain_begin[1]:] -= 2e-4  # interpenetrating: many candidates per node
    sim = gpu_sim(wl, candidate_capacity_per_node=1, build=False)
    with pytest.raises(pd.PDError) as e:
        sim.build_bonds()
    assert e.value.status == pd.PD_ERR_UNSTABLE
    sim.close()


def test_non_finite_force_halts_after_one_step():
    """A checkpoint whose u holds a NaN (its CRC recomputed so it loads): the
    first step's force evaluation raises the non-finite flag; the call returns
    PD_ERR_UNSTABLE at that step and the nine steps after it did nothing."""
    from paper_2506_05362_amd import pd
    wl = I.two_spheres(radius_cells=5, speed=5.0, gap=0.0)
    sim = gpu_sim(wl)
    sim.step(7)
    blob = bytearray(sim.get_state())
    body = len(blob) - 4
    node = 123
    n = wl.n_nodes
    # header of 8 int64, u of the current step, then the drifted u of the next
    # step (the positions the next evaluation reads), each as (x, y, z, w) doubles
    off = 64 + 32 * n + 32 * node
    blob[off:off + 8] = np.array([np.nan]).tobytes()
    blob[body:] = np.uint32(zlib.crc32(bytes(blob[:body]))).tobytes()
    sim.set_state(bytes(blob))
    assert sim.info()["step"] == 7
    assert sim.step_status(10) == pd.PD_ERR_UNSTABLE
    assert sim.info()["step"] == 8
    assert "non-finite" in pd.lib().pd_last_error(sim.h).decode()
    v = sim.get("velocity")
    assert not np.all(np.isfinite(v))
    sim.close()


@pytest.mark.parametrize("bond_path", [0, 1])
def test_fixed_grain_matches_oracle(oracle_lib, bond_path):
    """Grain A clamped (every node fixed: u kept, v = a = 0) and struck by grain B
    at 5 m/s: state 1e-9 after 600 steps through both bond paths, A's nodes
    never moved."""
    wl = I.two_spheres(radius_cells=5, speed=5.0, gap=0.0)
    nA = int(wl.grain_begin[1])
    wl.fixed[:nA] = 1
    ora = oracle_lib.Oracle(wl, flags=oracle_lib.CELL_LIST)
    sim = gpu_sim(wl)
    sim.set_launch(bond_path=bond_path)
    for _ in range(3):
        sim.step(200)
        ora.step(200)
    st = ora.state()
    assert np.abs(st["u"][:, nA:]).max() > 0 and np.all(st["u"][:, :nA] == 0)
    assert ora.energy()["contact"] > 0 or np.abs(st["v"][:, nA:]).max() > 0
    assert_state_close(sim, ora, what=f"fixed grain, bond path {bond_path}")
    g = sim.get("displacement")
    assert np.all(g[:, :nA] == 0) and np.all(sim.get("velocity")[:, :nA] == 0)
    sim.close()


def test_get_into_device_memory():
    """pd_get with a device destination writes the same bytes as into host
    memory; a destination one byte short is refused."""
    import torch
    from paper_2506_05362_amd import pd
    wl = I.two_spheres(radius_cells=4, speed=30.0, gap=0.0)
    sim = gpu_sim(wl)
    sim.step(30)
    for name, dt in (("displacement", torch.float64), ("damage", torch.float64), ("bond_col", torch.int32),
                     ("intact_count", torch.int32), ("bond_broken", torch.uint8)):
        nb = sim.field_bytes(name)
        host = sim.get(name)
        dev = torch.zeros(nb // torch.tensor([], dtype=dt).element_size(), dtype=dt, device="cuda")
        sim.get_device(name, dev.data_ptr(), nb)
        torch.cuda.synchronize()
        assert np.array_equal(dev.cpu().numpy().ravel(), host.ravel()), name
        with pytest.raises(pd.PDError) as e:
            sim.get_device(name, dev.data_ptr(), nb - 1)
        assert e.value.status == pd.PD_ERR_INVALID
    sim.close()
