"""Batched ensemble: several scenarios of uneven size in one context (one
launch per stage, per-scenario CFL step, time and hydrograph) reproduce
their separate runs bitwise; the autotuner leaves the state and the results
unchanged."""
import numpy as np
import pytest

from gpu_util import lib
from swe_inputs import ensemble_scenarios

pytestmark = pytest.mark.gpu


def _scenarios():
    return ensemble_scenarios(n=4, size_scale=0.02)


def _single(sc, steps):
    swe, prepare_scenario = lib()
    pr = prepare_scenario(sc)
    s = swe.Solver(precision=0, scheme=1, integrator=1, limiter=0)
    s.mesh_upload(pr.mesh)
    s.set_bc_series(*sc.hydrograph)
    l2g = pr.sub.l2g
    s.set_state(sc.h[l2g], sc.hu[l2g], sc.hv[l2g])
    s.step(steps)
    return s.read_state(), s.time()


def _batch(scs, steps, tune=False):
    swe, prepare_scenario = lib()
    preps = [prepare_scenario(sc) for sc in scs]
    s = swe.Solver(precision=0, scheme=1, integrator=1, limiter=0)
    s.mesh_upload_batch([p.mesh for p in preps])
    for i, sc in enumerate(scs):
        s.set_bc_series_scenario(i, *sc.hydrograph)
    h = np.concatenate([sc.h[p.sub.l2g] for sc, p in zip(scs, preps)])
    hu = np.concatenate([sc.hu[p.sub.l2g] for sc, p in zip(scs, preps)])
    hv = np.concatenate([sc.hv[p.sub.l2g] for sc, p in zip(scs, preps)])
    s.set_state(h, hu, hv)
    if tune:
        b, g = s.autotune(5)
        assert b in (64, 128, 256, 512)
        st = s.read_state()
        assert np.array_equal(st[0], h.astype(np.float32))
    s.step(steps)
    return s.read_state(), s.scenario_times(), s.offsets


@pytest.mark.parametrize("tune", [False, True])
def test_batch_equals_separate_runs(tune):
    scs = _scenarios()
    sizes = [sc.n_cells for sc in scs]
    assert len(set(sizes)) > 1
    steps = 40
    (bh, bhu, bhv), times, off = _batch(scs, steps, tune=tune)
    assert len(set(np.round(times, 9))) > 1          # each scenario keeps its own clock
    for i, sc in enumerate(scs):
        (h, hu, hv), t = _single(sc, steps)
        sl = slice(off[i], off[i + 1])
        assert np.array_equal(bh[sl], h) and np.array_equal(bhu[sl], hu) and np.array_equal(bhv[sl], hv)
        assert times[i] == t
