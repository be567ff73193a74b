"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer, run
over small instances of every workload family and every optional law (contact
with rebuilds, breaking, both stretch tests, the conic micromodulus, notch and
cavity cuts, moving, servo and corner walls, damping, friction, self-contact,
gravity), with the query functions the tests use.  Any finding aborts the
child process; the test then fails with the sanitizer's report.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import numpy as np
from oracle import pdref
from paper_2506_05362_amd import inputs as I

def run(wl, flags, steps):
    o = pdref.Oracle(wl, flags=flags, threads=2)
    o.step(steps)
    st = o.state()
    assert np.isfinite(st["u"]).all() and np.isfinite(st["v"]).all()
    o.bonds(); o.damage(); o.walls(); o.wall_impulse(); o.energy(); o.energy_density()
    o.bond_margin(); o.min_margin(); o.skin_exceeded()
    if flags & pdref.CELL_LIST:
        o.candidates()
    return o

spheres = I.two_spheres(radius_cells=4, speed=50.0, gap=0.0, rebuild_every=5)
for flags in (pdref.CELL_LIST, pdref.CELL_LIST | pdref.ABS_STRETCH, pdref.CELL_LIST | pdref.CONIC, 0):
    run(spheres, flags, 30)
plate = I.notched_plate(nx=24, ny=20, nz=4, h=5e-4, notch_x=(6 * 5e-4, 18 * 5e-4), notch_len=8 * 5e-4, steps=1)
run(plate, pdref.CELL_LIST, 20)
agg = I.grain_aggregate(n_grains=4, grid=(2, 2, 1), n_min=300, n_max=800, seed=3, platen_speed=5.0,
                        rebuild_every=5)
run(agg, pdref.CELL_LIST, 20)
rve = I.rve_aggregate(seed=1, n_grains=6, nodes_per_grain=120, confinement=5e6, platen_speed=20.0,
                      rebuild_every=5, contact_damping=1e22, friction=0.3)
run(rve, pdref.CELL_LIST, 20)
rve.params.self_contact = True
rve.params.wall_corners = True
rve.params.gravity = (0.0, 0.0, -9.81)
o = run(rve, pdref.CELL_LIST, 20)
o.set_u(o.state()["u"])
o.rebuild_candidates()
print("sanitized oracle: done", flush=True)
"""


def _asan_runtime():
    try:
        p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True, check=True)
    except (OSError, subprocess.CalledProcessError):
        return None
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    from oracle import pdref
    asan = _asan_runtime()
    if asan is None:
        pytest.skip("no AddressSanitizer runtime for gcc")
    lib = pdref.build_sanitized(str(tmp_path / "libpdref_san.so"))
    env = dict(os.environ)
    env.update(LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1",
               PDREF_LIB=lib, PYTHONPATH=ROOT, OMP_NUM_THREADS="2")
    p = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    report = p.stdout[-3000:] + p.stderr[-6000:]
    assert p.returncode == 0, report
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr, report
    assert "sanitized oracle: done" in p.stdout, report
