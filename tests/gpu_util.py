"""Shared set-up of the GPU tests: the same problem, numbered the same way,
on the HIP library (through the C ABI) and on the oracle.

The oracle side is built from the oracle alone: its own dual graph,
partition, ghost layers and numbering (``oracle/decomp_oracle.c``) and its
own inflow length.  The library's tables are asserted equal to the oracle's
before any state is compared, so no value the library computed ever enters
an oracle call."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O


def lib():
    from paper_2307_16758_amd import swe
    from paper_2307_16758_amd.problem import prepare_scenario
    return swe, prepare_scenario


SCHEME_KW = {
    "hllc1": dict(scheme=0, integrator=0, limiter=0),
    "muscl_minmod_rk2": dict(scheme=1, integrator=1, limiter=0),
    "muscl_superbee_rk2": dict(scheme=1, integrator=1, limiter=1),
    "muscl_vanalbada_rk2": dict(scheme=1, integrator=1, limiter=2),
    "muscl_minmod_euler": dict(scheme=1, integrator=0, limiter=0),
    "waf": dict(scheme=2, integrator=0, limiter=0),
}


def oracle_side(sc, P=1, p=0, k=0, nbr_g=None, part=None):
    """(oracle mesh, oracle sub-domain) of part ``p`` of ``P`` with ``k``
    ghost layers, from the oracle's own decomposition."""
    if nbr_g is None:
        nbr_g = O.neighbors(sc.mesh.n_nodes, sc.mesh.tri)
    if part is None:
        part = O.partition(nbr_g, P) if P > 1 else np.zeros(sc.n_cells, np.int32)
    sub = O.subdomain(sc.mesh.xy, sc.mesh.tri, nbr_g, sc.bc, part, P, p, k)
    l2g = sub.l2g
    M = O.Mesh(sc.mesh.xy, sc.mesh.tri[l2g], sub.nbr, sc.b[l2g], sc.manning[l2g],
               gid=l2g, n_owned=sub.n_owned)
    return M, sub


def assert_same_numbering(lib_sub, osub):
    """The library's sub-domain tables equal the oracle's, entry for entry."""
    assert lib_sub.n_owned == osub.n_owned and lib_sub.n_total == osub.n_total
    assert np.array_equal(lib_sub.l2g, osub.l2g)
    assert np.array_equal(lib_sub.nbr, osub.nbr)


def oracle_params(sc, name=None, **cfg):
    """Oracle parameters of a scenario (inflow length from the oracle's own
    edge lengths) for the scheme ``name`` and the overrides in ``cfg``."""
    kw = dict(SCHEME_KW[name]) if name else {}
    kw.update({k_: v for k_, v in cfg.items() if k_ in ("scheme", "integrator", "limiter")})
    okw = {k_: v for k_, v in kw.items() if k_ in ("scheme", "integrator", "limiter")}
    for k_ in ("waf_limiter", "cfl_rule", "cfl", "dt_max", "eps"):
        if k_ in cfg:
            okw[k_] = cfg[k_]
    if "waf_positivity" in cfg:
        okw["waf_pos"] = cfg["waf_positivity"]
    return O.scenario_params(sc, **okw)


def make_pair(sc, name, precision, P=1, p=0, k=0, prepared=None, **cfg):
    """(solver, oracle mesh, oracle params, prepared) for one scenario.

    With ``prepared`` (a decomposition the caller made with the library) only
    the solver is set up, and the oracle mesh and parameters are None."""
    swe, prepare_scenario = lib()
    pr = prepared if prepared is not None else prepare_scenario(sc, P=P, p=p, k=k)
    kw = dict(SCHEME_KW[name])
    kw.update(cfg)
    s = swe.Solver(precision=precision, **kw)
    s.mesh_upload(pr.mesh)
    if sc.hydrograph is not None:
        s.set_bc_series(*sc.hydrograph)
    l2g = pr.sub.l2g
    s.set_state(sc.h[l2g], sc.hu[l2g], sc.hv[l2g])
    if prepared is not None:
        return s, None, None, pr
    M, osub = oracle_side(sc, P, p, k)
    assert_same_numbering(pr.sub, osub)
    return s, M, oracle_params(sc, name, **cfg), pr


def rel_err(a, r, n_owned=None):
    """Per field: max |a - r| / max |r| over owned cells (0/0 -> 0)."""
    if n_owned is not None:
        a, r = a[:n_owned], r[:n_owned]
    d = np.abs(np.asarray(a, np.float64) - r).max() if r.size else 0.0
    s = np.abs(r).max() if r.size else 0.0
    return d / s if s > 0 else d


def state_errors(gpu_state, ref_state, n_owned):
    return tuple(rel_err(g, r, n_owned) for g, r in zip(gpu_state, ref_state))
