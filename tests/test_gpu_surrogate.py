"""The surrogate pipeline end to end on small aggregates: training data from the
simulator (confined compression with servo walls), the network trained by the
library's own matrix-core kernels, held-out paths checked against the
simulation, and the network's cost per path against the simulation's."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_surrogate_small_rve_end_to_end():
    from paper_2506_05362_amd import surrogate as S
    specs = S.path_specs(10, seed=100)
    kw = dict(S.RVE_DEFAULTS, n_grains=24, nodes_per_grain=300)
    data = S.generate(specs, n_log=200, log=lambda s: print(s, flush=True), workers=2, **kw)
    n = len(data["offsets"]) - 1
    assert n >= 8
    held, train = np.arange(n - 2, n), np.arange(0, n - 2)
    sur = S.Surrogate(max_batch=4096)
    losses = sur.fit(S.samples(data, train, "strain"), S.samples(data, train, "target"), steps=2000)
    assert losses[-1] < 0.1 * losses[0]
    ev = S.evaluate(sur, data, held, train)
    print("held-out axial rel L2", ev["axial_rel_l2"], "interpolation", ev["interp_axial_rel_l2"],
          "confinement ensemble", ev["ensemble_axial_rel_l2"], flush=True)
    assert ev["axial_rel_l2_mean"] <= 0.15
    # the network does at least about as well as interpolating the training samples
    assert ev["axial_rel_l2_mean"] <= 1.25 * ev["interp_axial_rel_l2_mean"]
    paths = S.inference_paths(data, train, 20000, T=50)
    assert sur.in_envelope(paths.reshape(-1, 6)).all()
    inf = S.time_inference(sur, paths)
    sim_per_path = float(np.mean(data["seconds"] / np.maximum(data["steps_run"], 1) * data["steps"]))
    speedup = sim_per_path / inf["seconds_per_path"]
    print(f"simulation {sim_per_path:.3f} s/path, network {inf['seconds_per_path']:.2e} s/path, "
          f"speedup {speedup:.3g}", flush=True)
    assert speedup > 1e4
