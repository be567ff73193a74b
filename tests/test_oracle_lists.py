"""Bond and contact-candidate lists of the oracle against O(N^2) brute force.

The brute force below follows the paper's statements directly: bond family =
same-grain points within the horizon (Sec. 3.1, inclusive integer shell),
notch removal with the crossing parameter t of Sec. 6.3.1 computed as an exact
fraction, cavity removal by the endpoint rule of Sec. 6.3.2 (and the chord
variant by the exact closest point of the segment), contact candidates =
other-grain nodes closer than R_c + skin.
"""
from fractions import Fraction

import numpy as np
import pytest

from paper_2506_05362_amd import inputs as I


def brute_bonds(wl):
    n = wl.n_nodes
    m = wl.params.horizon_factor
    g = wl.grain_of_node()
    ijk = wl.ijk.astype(np.int64)
    rows = []
    for i in range(n):
        d = ijk - ijk[:, i:i + 1]
        d2 = (d * d).sum(axis=0)
        cand = np.where((g == g[i]) & (d2 > 0) & (d2 <= m * m))[0]
        keep = [int(j) for j in cand if not brute_removed(wl, g[i], ijk[:, i], ijk[:, j])]
        rows.append(sorted(keep))
    return rows


def _notch(cut, P1, P2):
    a, b, c, d = cut.plane
    f1 = a * P1[0] + b * P1[1] + c * P1[2] + d
    den = a * (P2[0] - P1[0]) + b * (P2[1] - P1[1]) + c * (P2[2] - P1[2])
    if den == 0:
        return False
    t = Fraction(-f1, den)
    if not (0 < t < 1):
        return False
    for q in range(3):
        Q = P1[q] + t * (P2[q] - P1[q])
        if cut.lo[q] > -I.HALF_UNBOUNDED and Q < cut.lo[q]:
            return False
        if cut.hi[q] < I.HALF_UNBOUNDED and Q > cut.hi[q]:
            return False
    return True


def _inside(cut, P):
    return sum((P[q] - cut.center[q]) ** 2 for q in range(3)) < cut.radius2


def _chord(cut, P1, P2):
    D = [P2[q] - P1[q] for q in range(3)]
    DD = sum(x * x for x in D)
    t = Fraction(sum((cut.center[q] - P1[q]) * D[q] for q in range(3)), DD)
    t = min(max(t, Fraction(0)), Fraction(1))
    return sum((P1[q] + t * D[q] - cut.center[q]) ** 2 for q in range(3)) < cut.radius2


def brute_removed(wl, g, a, b):
    P1 = [2 * int(x) for x in a]
    P2 = [2 * int(x) for x in b]
    for cut in wl.cuts:
        if cut.grain != g:
            continue
        if cut.kind == I.CUT_NOTCH and _notch(cut, P1, P2):
            return True
        if cut.kind == I.CUT_CAVITY_ENDPOINT and (_inside(cut, P1) or _inside(cut, P2)):
            return True
        if cut.kind == I.CUT_CAVITY_CHORD and _chord(cut, P1, P2):
            return True
    return False


def assert_rows_equal(rp, col, rows):
    assert rp[-1] == sum(len(r) for r in rows)
    for i, r in enumerate(rows):
        assert col[rp[i]:rp[i + 1]].tolist() == r, f"row {i}"


def small_plate(h=5e-4):
    # 16 x 12 x 4 plate, notch planes between columns 4|5 and 11|12 up to row 5 (tip inclusive)
    return I.notched_plate(nx=16, ny=12, nz=4, h=h, notch_x=(5 * h, 12 * h), notch_len=6 * h,
                           steps=1)


def hollow_ball(kind, include_cavity_nodes):
    h = 1e-4
    off = I.sphere_offsets(6)
    if not include_cavity_nodes:
        keep = (off * off).sum(axis=0) >= 9
        off = off[:, keep]
    ijk, origin = I.grain_block(off, np.zeros(3), h)
    lo = off.min(axis=1)
    centre_half = tuple(int(v) for v in (-2 * lo))
    cut = I.Cut(kind=kind, grain=0, center=centre_half, radius2=33)  # 2.87 cells
    return I.assemble("hollow", [(ijk, origin, h, 0)], [I.SAND], I.default_params(h, 1e-9), [],
                      [cut], 1)


@pytest.mark.parametrize("case", ["ball", "two_grains", "plate_notches", "cavity_endpoint",
                                  "cavity_endpoint_meshed_out", "cavity_chord"])
def test_bond_lists_match_brute_force(oracle_lib, case):
    if case == "ball":
        off = I.sphere_offsets(4)
        ijk, origin = I.grain_block(off, np.zeros(3), 1e-4)
        wl = I.assemble("b", [(ijk, origin, 1e-4, 0)], [I.SAND], I.default_params(1e-4, 1e-9), [],
                        [], 1)
    elif case == "two_grains":
        wl = I.two_spheres(radius_cells=4)
    elif case == "plate_notches":
        wl = small_plate()
    elif case == "cavity_endpoint":
        wl = hollow_ball(I.CUT_CAVITY_ENDPOINT, True)
    elif case == "cavity_endpoint_meshed_out":
        wl = hollow_ball(I.CUT_CAVITY_ENDPOINT, False)
    else:
        wl = hollow_ball(I.CUT_CAVITY_CHORD, False)
    o = oracle_lib.Oracle(wl)
    rp, col, _ = o.bonds()
    rows = brute_bonds(wl)
    assert_rows_equal(rp, col, rows)
    full = sum(len(r) for r in brute_bonds(
        I.assemble("x", [(wl.ijk[:, wl.grain_begin[g]:wl.grain_begin[g + 1]],
                          wl.grain_origin[:, g], wl.grain_h[g], 0) for g in range(wl.n_grains)],
                   wl.materials, wl.params, [], [], 1)))
    if case in ("plate_notches", "cavity_endpoint", "cavity_chord"):
        assert rp[-1] < full  # the cut removed something
    if case == "cavity_endpoint_meshed_out":
        assert rp[-1] == full  # endpoint rule is a no-op when the cavity has no nodes


def test_interior_row_has_122_bonds(oracle_lib):
    wl = I.two_spheres(radius_cells=5)
    o = oracle_lib.Oracle(wl)
    rp, col, _ = o.bonds()
    assert np.diff(rp).max() == 122


def test_notch_tip_is_inclusive(oracle_lib):
    """A bond whose crossing point lies exactly at the notch tip is removed."""
    wl = small_plate()
    cut = wl.cuts[0]
    tip = cut.hi[1]
    # node (4, 5, 0) -> (5, 6, 0): half-lattice (8,10)->(10,12), crosses x=9 at y=11
    assert tip == 11
    o = oracle_lib.Oracle(wl)
    rp, col, _ = o.bonds()
    ijk = wl.ijk

    def idx(a, b, c):
        return int(np.where((ijk[0] == a) & (ijk[1] == b) & (ijk[2] == c))[0][0])

    i, j, k = idx(4, 5, 0), idx(5, 6, 0), idx(5, 7, 0)
    assert j not in col[rp[i]:rp[i + 1]]
    # crossing at y = 12 > tip: kept
    assert k in col[rp[i]:rp[i + 1]]


def brute_candidates(wl, u):
    g = wl.grain_of_node()
    X = wl.X
    cut = wl.params.contact_radius + wl.params.skin
    rows = []
    for i in range(wl.n_nodes):
        y = (X - X[:, i:i + 1]) + (u - u[:, i:i + 1])
        d2 = (y[0] * y[0] + y[1] * y[1]) + y[2] * y[2]
        rows.append(np.where((g != g[i]) & (d2 < cut * cut))[0].tolist())
    return rows


@pytest.mark.parametrize("cell_list", [False, True])
def test_contact_candidates_match_brute_force(oracle_lib, cell_list):
    wl = I.two_spheres(radius_cells=5, gap=0.0)
    rng = np.random.default_rng(1)
    wl.u0[:] = rng.normal(0, 3e-6, size=wl.u0.shape)
    wl.u0[0, wl.grain_begin[1]:] -= 4e-4  # push B into A: many pairs in range
    flags = oracle_lib.CELL_LIST if cell_list else 0
    o = oracle_lib.Oracle(wl, flags=flags)
    rp, col = o.candidates()
    rows = brute_candidates(wl, wl.u0)
    assert sum(len(r) for r in rows) > 50
    assert_rows_equal(rp, col, rows)


def test_contact_candidates_adversarial_ties(oracle_lib):
    """Pairs placed at distances within a few ulps of R_c + skin."""
    h = 1e-4
    params = I.default_params(h, 1e-9)
    cut = params.contact_radius + params.skin
    off = np.zeros((3, 1), dtype=np.int64)
    blocks = []
    for k in range(24):
        blocks.append((*I.grain_block(off, np.array([0.0, 10 * h * k, 0.0]), h), h, 0))
        dx = np.nextafter(cut, cut + (k - 12)) if k != 12 else cut
        for _ in range(abs(k - 12) // 2):
            dx = np.nextafter(dx, 0 if k < 12 else 1)
        blocks.append((*I.grain_block(off, np.array([dx, 10 * h * k, 0.0]), h), h, 0))
    wl = I.assemble("ties", blocks, [I.SAND], params, [], [], 1)
    for flags in (0, oracle_lib.CELL_LIST):
        o = oracle_lib.Oracle(wl, flags=flags)
        rp, col = o.candidates()
        assert_rows_equal(rp, col, brute_candidates(wl, wl.u0))
