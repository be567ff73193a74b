"""Host-side parts of the surrogate study: the data-only scatter estimate and
the joining of saved path sets (no GPU)."""
import math

import numpy as np
import pytest

from paper_2506_05362_amd import surrogate as S


def _paths(factors, confinements, lengths=None):
    e = np.linspace(0.0, 0.05, 11)
    base = 1e6 * np.sin(np.pi * e / 0.05 * 0.8) + 2e5
    strain, target, offsets = [], [], [0]
    for k, f in enumerate(factors):
        n = len(e) if lengths is None else lengths[k]
        X = np.zeros((n, 6))
        X[:, S.AXIAL] = e[:n]
        Y = np.zeros((n, 7))
        Y[:, S.AXIAL] = f * base[:n]
        strain.append(X)
        target.append(Y)
        offsets.append(offsets[-1] + n)
    return {"strain": np.concatenate(strain), "target": np.concatenate(target),
            "offsets": np.array(offsets), "confinement": np.array(confinements, dtype=float)}


def test_pair_scatter_of_scaled_paths():
    """Paths f(e) (1 + 0.1 k) taken in confinement order: each neighbouring
    pair differs by 0.1 ||f|| against the root mean square of their norms."""
    data = _paths([1.2, 1.0, 1.1], [3e6, 1e6, 2e6])
    r = S.pair_scatter(data, np.arange(3))
    want = [0.1 / math.sqrt((1.0 + 1.21) / 2), 0.1 / math.sqrt((1.21 + 1.44) / 2)]
    assert r["pair_axial_rel_l2_mean"] == pytest.approx(np.mean(want), rel=1e-12)
    assert r["single_path_scatter"] == pytest.approx(np.mean(want) / math.sqrt(2), rel=1e-12)
    assert r["pair_confinement_gap_mean"] == pytest.approx(1e6)


def test_pair_scatter_compares_common_strains_only():
    """A path stopped early is compared over the strains it reached."""
    data = _paths([1.0, 1.0], [1e6, 2e6], lengths=[11, 6])
    assert S.pair_scatter(data, np.arange(2))["pair_axial_rel_l2_mean"] == pytest.approx(0.0, abs=1e-15)
    data = _paths([1.0, 2.0], [1e6, 2e6], lengths=[11, 6])
    assert S.pair_scatter(data, np.arange(2))["pair_axial_rel_l2_mean"] == pytest.approx(
        1.0 / math.sqrt(2.5), rel=1e-12)


def test_load_data_joins_parts(tmp_path):
    """Saved parts join in order; per-path fields only some parts carry are left out."""
    a, b = _paths([1.0, 1.1], [1e6, 2e6]), _paths([1.2], [3e6])
    for d, seeds, extra in ((a, [0, 1], True), (b, [2], False)):
        n = len(d["offsets"]) - 1
        d.update(t=np.arange(d["offsets"][-1], dtype=float), seconds=np.ones(n), steps_run=np.ones(n),
                 steps=np.ones(n), truncated=np.zeros(n, bool), nodes=np.ones(n), bonds=np.ones(n),
                 seed=np.array(seeds), dropped=np.zeros(0, np.int64))
        if extra:
            d["early_rebuilds"] = np.zeros(n, np.int64)
    np.savez(tmp_path / "a.npz", **a)
    np.savez(tmp_path / "b.npz", **b)
    j = S.load_data([str(tmp_path / "a.npz"), str(tmp_path / "b.npz")])
    assert list(j["seed"]) == [0, 1, 2]
    assert list(j["offsets"]) == [0, 11, 22, 33]
    assert "early_rebuilds" not in j
    assert np.array_equal(S.path(j, 2, "target"), S.path(b, 0, "target"))
