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
