"""Invariants of the oracle's dynamics: antisymmetric pair forces, conservation of
linear and angular momentum, and second-order energy behaviour of velocity
Verlet (Sec. 6.2) in the elastic regime."""
import numpy as np
import pytest

from paper_2506_05362_amd import inputs as I


def colliding_pair(speed=2.0, dt=1e-8, push=1.5e-4, seed=0):
    wl = I.two_spheres(radius_cells=5, speed=speed, dt=dt, gap=0.0, seed=seed, rebuild_every=10)
    wl.u0[0, wl.grain_begin[1]:] -= push  # start in contact
    rng = np.random.default_rng(seed + 7)
    wl.v0 += rng.normal(0, 0.05, size=wl.v0.shape)  # plus a random elastic field
    return wl


def momenta(wl, st):
    V = wl.grain_h[0] ** 3
    rho = wl.materials[0].density
    P = (rho * V * st["v"]).sum(axis=1)
    pos = wl.X + st["u"]
    L = (rho * V * np.cross(pos.T, st["v"].T)).sum(axis=0)
    return P, L


def test_total_internal_force_vanishes(oracle_lib):
    wl = colliding_pair()
    rng = np.random.default_rng(2)
    wl.u0 += rng.normal(0, 1e-7, size=wl.u0.shape)
    o = oracle_lib.Oracle(wl, flags=oracle_lib.CELL_LIST)
    F = o.state()["F"]
    V = wl.grain_h[0] ** 3
    tot = (V * F).sum(axis=1)
    scale = (V * abs(F)).sum()
    assert scale > 0
    assert np.all(abs(tot) <= 1e-12 * scale)
    # contact is active and some bonds are loaded
    assert o.energy()["contact"] > 0 and o.energy()["elastic"] > 0


def test_momentum_conservation(oracle_lib):
    wl = colliding_pair()
    o = oracle_lib.Oracle(wl, flags=oracle_lib.CELL_LIST)
    P0, L0 = momenta(wl, o.state())
    o.step(120)
    P1, L1 = momenta(wl, o.state())
    pscale = np.abs(P0).max()
    assert np.all(abs(P1 - P0) <= 1e-11 * pscale)
    lscale = np.abs(L0).max()
    assert np.all(abs(L1 - L0) <= 1e-9 * lscale)
    assert o.energy()["contact"] > 0


def _max_energy_error(oracle_lib, dt, T):
    wl = colliding_pair(dt=dt, speed=1.0, push=2e-6)
    o = oracle_lib.Oracle(wl, flags=oracle_lib.CELL_LIST)
    E0 = o.energy()["total"]
    n = int(round(T / dt))
    err = 0.0
    for _ in range(10):
        o.step(n // 10)
        err = max(err, abs(o.energy()["total"] - E0))
    assert o.bonds()[2].sum() == 0  # elastic regime
    assert o.energy()["contact"] > 0
    return err / E0


def test_energy_error_is_second_order(oracle_lib):
    T = 4e-7
    e1 = _max_energy_error(oracle_lib, 1e-8, T)
    e2 = _max_energy_error(oracle_lib, 5e-9, T)
    assert e1 < 1e-3
    assert e1 / e2 == pytest.approx(4.0, rel=0.05)


def test_break_margin_is_recorded(oracle_lib):
    wl = I.two_spheres(radius_cells=5, speed=50.0, gap=0.0)
    wl.u0[0, wl.grain_begin[1]:] -= 1e-4
    o = oracle_lib.Oracle(wl, flags=oracle_lib.CELL_LIST)
    o.step(40)
    m = o.min_margin()
    assert 0.0 <= m < 1.0
