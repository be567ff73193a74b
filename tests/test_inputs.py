"""Seeded input generators: the shapes and structure they promise."""
import math

import numpy as np

from paper_2506_05362_amd import inputs as I


def test_large_aggregate_tessellation_small():
    """A small instance of the large aggregate: the grains tile the box (every
    lattice cell has exactly one node), sizes spread like the log-normal radii,
    each grain's nodes are in lexicographic lattice order (so the tiled bond
    path applies), the walls sit one spacing outside the nodes and the steps
    cover the requested strain."""
    h = 1.6e-4
    wl = I.large_aggregate(seed=1, n_grains=40, h=h, axial_strain=0.02)
    pos = np.rint((wl.X - wl.X.min(axis=1, keepdims=True)) / h).astype(np.int64)
    n_side = int(pos.max()) + 1
    flat = (pos[0] * n_side + pos[1]) * n_side + pos[2]
    assert np.unique(flat).size == wl.n_nodes  # no cell holds two nodes
    assert wl.n_nodes >= 0.99 * n_side ** 3  # and (up to dropped tiny grains) every cell one
    sizes = np.diff(wl.grain_begin)
    assert sizes.max() > 4 * np.median(sizes) / 2 and wl.n_grains >= 35
    for g in range(wl.n_grains):
        ijk = wl.ijk[:, wl.grain_begin[g]:wl.grain_begin[g + 1]].astype(np.int64)
        keys = [(ijk[a] << 20) | (ijk[b] << 10) | ijk[c] for a, b, c in
                ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))]
        assert any(np.all(np.diff(k) > 0) for k in keys), g
    lo, hi = wl.X.min(axis=1), wl.X.max(axis=1)
    assert math.isclose(wl.walls[0].offset, lo[2] - h) and math.isclose(-wl.walls[1].offset, hi[2] + h)
    span = hi[2] - lo[2] + 2 * h
    assert wl.steps == math.ceil(0.02 * span / (wl.walls[1].velocity * wl.params.dt))


def test_large_aggregate_is_seeded():
    a = I.large_aggregate(seed=3, n_grains=20, h=2e-4)
    b = I.large_aggregate(seed=3, n_grains=20, h=2e-4)
    c = I.large_aggregate(seed=4, n_grains=20, h=2e-4)
    assert np.array_equal(a.X, b.X) and np.array_equal(a.grain_begin, b.grain_begin)
    assert not np.array_equal(a.grain_begin, c.grain_begin)


def test_shape_study_geometry():
    """Shape study (Sec. 7.6): grid^3 grains of one shape, every node within the
    grain radius of its grid centre; shells miss the cavity, jacks fill less of
    the ball than shells; the walls box the nodes R_c out; steps cover the
    duration."""
    h, R = 1e-4, 5e-4
    counts = {}
    for shape in I.SHAPES:
        wl = I.shape_study(shape, seed=1, grid=2, radius=R, h=h, duration=2e-6)
        assert wl.n_grains == 8 and wl.steps == 200
        pitch = wl.info["pitch"]
        for g in range(wl.n_grains):
            x = wl.X[:, wl.grain_begin[g]:wl.grain_begin[g + 1]]
            centre = np.array([g % 2, (g // 2) % 2, g // 4]) * pitch
            r = np.linalg.norm(x - centre[:, None], axis=0)
            assert r.max() <= R * (1 + 1e-12)
            if shape == "shell":
                assert r.min() >= 0.5 * R * (1 - 1e-12)
        counts[shape] = np.diff(wl.grain_begin)
        Rc = wl.params.contact_radius
        lo, hi = wl.X.min(axis=1), wl.X.max(axis=1)
        assert math.isclose(wl.walls[0].offset, lo[2] - Rc) and math.isclose(-wl.walls[1].offset, hi[2] + Rc)
        assert wl.walls[1].velocity == 10.0 and len(wl.walls) == 6
        assert (len(wl.cuts) == 8) == (shape == "shell")
    ball = 4 / 3 * math.pi * (R / h) ** 3
    assert np.all(np.abs(counts["sphere"] / ball - 1) < 0.05)
    assert np.all(np.abs(counts["shell"] / (ball * 7 / 8) - 1) < 0.08)
    assert counts["jack"].max() < 0.5 * counts["shell"].min()


def test_shape_study_jacks_are_three_bars():
    """A jack is three orthogonal bars: in its own frame every node lies within
    the half-width of at least two axes, and it reaches out to the radius along
    all six arm directions."""
    rng = np.random.default_rng(5)
    R, h = 1e-3, 1e-4
    off, o, rin = I.shape_grain(rng, "jack", R, h)
    assert rin == 0.0
    rng = np.random.default_rng(5)
    rng.uniform(size=3)
    rot = I._rotation(rng)
    q = rot.T @ ((off + o[:, None]) * h)
    assert np.all(np.sum(np.abs(q) <= 0.25 * R, axis=0) >= 2)
    for ax in range(3):
        assert q[ax].max() > R - 2 * h and q[ax].min() < -(R - 2 * h)
