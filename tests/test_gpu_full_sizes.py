"""The full-size workloads, in the launch configuration the benchmark times.

* The 13,000,560-cell river (40 km x 8 km, islands, dam-break start): the
  whole mesh in FP32 MUSCL-minmod-HLLC-RK2 against the FP64 oracle on every
  cell after 10 fixed-dt steps; the largest of 32 greedy-BFS parts with 4
  ghost layers equals the whole-mesh run bitwise on its owned cells after
  one step (the stencil radius of a MUSCL-RK2 step is 4 layers), and its
  on-device pack gathers exactly the send lists.
* The 64-scenario ensemble (38.1M cells in one context): the smallest, the
  median and the largest scenario equal their separate runs bitwise (state
  and clock) after 100 CFL steps, and the smallest and the median one
  follow the oracle (1e-4 per field, their clocks to 1e-5).
"""
import numpy as np
import pytest

from gpu_util import make_pair, state_errors, lib, oracle_side, assert_same_numbering
from swe_inputs import config3, ensemble_scenarios

pytestmark = pytest.mark.gpu

MUSCL_RK2 = dict(precision=0, scheme=1, integrator=1, limiter=0)


def test_config3_full_mesh_and_largest_part():
    import torch
    swe, prepare_scenario = lib()
    sc = config3()
    assert sc.n_cells == 13_000_560
    s, M, par, pr = make_pair(sc, "muscl_minmod_rk2", precision=0)
    l2g = pr.sub.l2g
    dt = M.dt(par, sc.h[l2g], sc.hu[l2g], sc.hv[l2g])
    s.step(1, dt)
    g1 = s.read_state()
    one = [np.empty_like(x) for x in g1]          # global numbering
    for f in range(3):
        one[f][l2g] = g1[f]
    s.step(9, dt)
    g10 = s.read_state()
    r10 = M.run(par, sc.h[l2g], sc.hu[l2g], sc.hv[l2g], 10, dt_fixed=dt)
    errs = state_errors(g10, r10[:3], pr.sub.n_owned)
    print("config3 full mesh, 10 steps, rel errors", errs)
    assert max(errs) <= 1e-4, errs
    del M, s

    nbr = swe.swe_dual_graph(sc.mesh.n_nodes, sc.mesh.tri)
    part = swe.swe_partition_bfs(nbr, 32)
    p = int(np.argmax(np.bincount(part, minlength=32)))
    pp = prepare_scenario(sc, P=32, p=p, k=4, nbr_global=nbr, part=part)
    sub = swe.Solver(**MUSCL_RK2)
    sub.mesh_upload(pp.mesh)
    sl = pp.sub.l2g
    sub.set_state(sc.h[sl], sc.hu[sl], sc.hv[sl])
    n_own = pp.sub.n_owned
    assert n_own > 400_000
    sub.step(1, dt)
    st = sub.read_state()
    for f in range(3):
        assert np.array_equal(st[f][:n_own], one[f][sl[:n_own]]), f
    n_send, n_ghost = sub.ghost_sizes()
    assert n_send == pp.sub.send_idx.size and n_ghost == pp.sub.n_total - n_own
    buf = torch.empty(3 * n_send, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    sub.pack_ghosts(buf)
    sub.sync()
    b = buf.cpu().numpy().reshape(3, n_send)
    for f in range(3):
        assert np.array_equal(b[f], st[f][pp.sub.send_idx])


def test_config5_ensemble():
    from oracle import oracle as O
    swe, prepare_scenario = lib()
    scs = ensemble_scenarios()
    assert len(scs) == 64
    preps = [prepare_scenario(x) for x in scs]
    s = swe.Solver(**MUSCL_RK2)
    s.mesh_upload_batch([p.mesh for p in preps])
    for i, x in enumerate(scs):
        if x.hydrograph is not None:
            s.set_bc_series_scenario(i, *x.hydrograph)
    s.set_state(np.concatenate([x.h[p.sub.l2g] for x, p in zip(scs, preps)]),
                np.concatenate([x.hu[p.sub.l2g] for x, p in zip(scs, preps)]),
                np.concatenate([x.hv[p.sub.l2g] for x, p in zip(scs, preps)]))
    assert s.offsets[-1] == sum(x.n_cells for x in scs)
    s.step(100)
    bst = s.read_state()
    times = s.scenario_times()
    off = s.offsets
    sizes = np.array([x.n_cells for x in scs])
    order = np.argsort(sizes)
    for i in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        x, p = scs[i], preps[i]
        one = swe.Solver(**MUSCL_RK2)
        one.mesh_upload(p.mesh)
        if x.hydrograph is not None:
            one.set_bc_series(*x.hydrograph)
        one.set_state(x.h[p.sub.l2g], x.hu[p.sub.l2g], x.hv[p.sub.l2g])
        one.step(100)
        st = one.read_state()
        sl = slice(off[i], off[i + 1])
        for f in range(3):
            assert np.array_equal(bst[f][sl], st[f]), (i, f)
        assert times[i] == one.time()
        one.close()
    # the smallest and the median scenario against the oracle (each with its
    # own CFL steps)
    for i in (int(order[0]), int(order[len(order) // 2])):
        x, p = scs[i], preps[i]
        l2g = p.sub.l2g
        M, osub = oracle_side(x)
        assert_same_numbering(p.sub, osub)
        par = O.scenario_params(x, scheme=1, integrator=1, limiter=0)
        r = M.run(par, x.h[l2g], x.hu[l2g], x.hv[l2g], 100)
        sl = slice(off[i], off[i + 1])
        errs = state_errors([b[sl] for b in bst], r[:3], p.sub.n_owned)
        print("ensemble scenario", i, x.n_cells, "cells, 100 CFL steps, rel errors", errs,
              "time", times[i], r[3])
        assert max(errs) <= 1e-4, errs
        assert times[i] == pytest.approx(r[3], rel=1e-5)
