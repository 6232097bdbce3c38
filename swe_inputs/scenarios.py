"""Seeded flood / dam-break problem definitions on the meshes of ``mesh.py``.

A :class:`Scenario` carries everything the solver takes as *input*: mesh,
boundary tag per local edge, bed elevation ``b`` and Manning ``n`` per cell
(sampled at the cell's centroid), the initial state (h, hu, hv) and the
boundary parameters.  Nothing here computes fluxes, geometry of the scheme or
neighbour relations.

Workload recipes (the sizes, seeds and value ranges the measurements use):

* ``config1``: 100 m x 20 m flat channel, 200 x 40 quads (16,000 triangles),
  seed 1, h = 1 m for x_c < 50 m else 0.5 m, still water, walls, n = 0.
* ``config2``: 10 km x 2 km meandering channel, 1582 x 316 quads
  (999,824 triangles), seed 2, 40 Gaussian bumps, dry banks, Manning n drawn
  once in [0.02, 0.05], lake at rest at the outlet stage, 500 m^3/s inflow.
* ``config3``: 40 km x 8 km channel, 5702 x 1140 quads (13,000,560
  triangles), seed 3, 40 bumps plus 12 emerging islands, dam-break start
  (stage +2 m upstream of the middle of the reach, 0 m downstream).
* ``ensemble_scenarios``: 64 channels, sizes log-uniform in [5e4, 2e6]
  triangles, triangular inflow pulses 100 -> [100, 2000] m^3/s.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

from .mesh import (TriMesh, grid_mesh, refine_red, BC_INTERIOR, BC_WALL,
                   BC_TRANSMISSIVE, BC_INFLOW, BC_OUTFLOW, SIDE_NONE,
                   SIDE_LEFT, SIDE_RIGHT, SIDE_BOTTOM, SIDE_TOP)


@dataclass
class Scenario:
    name: str
    mesh: TriMesh
    bc: np.ndarray            # int8 [n, 3]: 0 interior, <0 boundary tag
    b: np.ndarray             # float64 [n] bed elevation at the centroid
    manning: np.ndarray       # float64 [n]
    h: np.ndarray             # float64 [n]
    hu: np.ndarray            # float64 [n]
    hv: np.ndarray            # float64 [n]
    inflow_q: float = 0.0     # total inflow discharge [m^3/s]
    outflow_stage: float = 0.0
    hydrograph: Optional[tuple] = None   # (t[], Q[]) piecewise linear
    bed_fn: Optional[Callable] = field(default=None, repr=False)
    ic_fn: Optional[Callable] = field(default=None, repr=False)
    side_tags: dict = field(default_factory=dict)
    manning_value: Optional[float] = None
    params: dict = field(default_factory=dict)

    @property
    def n_cells(self) -> int:
        return self.mesh.n_cells


def _bc_from_sides(side: np.ndarray, side_tags: dict, wet: np.ndarray) -> np.ndarray:
    """Map rectangle sides to tags.  An inflow or outflow side only opens on
    edges whose cell is wet initially; its dry edges are walls."""
    bc = np.zeros(side.shape, dtype=np.int8)
    for s in (SIDE_LEFT, SIDE_RIGHT, SIDE_BOTTOM, SIDE_TOP):
        tag = side_tags.get(s, BC_WALL)
        on = side == s
        if tag in (BC_INFLOW, BC_OUTFLOW):
            open_ = on & wet[:, None]
            bc[open_] = tag
            bc[on & ~wet[:, None]] = BC_WALL
        else:
            bc[on] = tag
    return bc


def _build(name, mesh, bed_fn, ic_fn, manning, side_tags, inflow_q=0.0,
           outflow_stage=0.0, hydrograph=None, params=None) -> Scenario:
    c = mesh.centroids()
    b = np.asarray(bed_fn(c[:, 0], c[:, 1]), dtype=np.float64)
    h, hu, hv = ic_fn(c[:, 0], c[:, 1], b)
    wet = h > 0.0
    bc = _bc_from_sides(mesh.edge_side, side_tags, wet)
    n = np.full(mesh.n_cells, float(manning), dtype=np.float64)
    return Scenario(name=name, mesh=mesh, bc=bc, b=b, manning=n,
                    h=np.asarray(h, np.float64), hu=np.asarray(hu, np.float64),
                    hv=np.asarray(hv, np.float64), inflow_q=float(inflow_q),
                    outflow_stage=float(outflow_stage), hydrograph=hydrograph,
                    bed_fn=bed_fn, ic_fn=ic_fn, side_tags=dict(side_tags),
                    manning_value=float(manning), params=dict(params or {}))


def refine_scenario(sc: Scenario) -> Scenario:
    """Same problem on the red-refined mesh (bed and initial state resampled
    at the children's centroids, boundary sides inherited)."""
    m = refine_red(sc.mesh)
    return _build(sc.name + "_red", m, sc.bed_fn, sc.ic_fn, sc.manning_value,
                  sc.side_tags, sc.inflow_q, sc.outflow_stage, sc.hydrograph,
                  dict(sc.params, refined=sc.params.get("refined", 0) + 1))


# ---------------------------------------------------------------- flat cases
def _flat_bed(x, y):
    return np.zeros_like(x)


def dam_break_channel(Lx=100.0, Ly=20.0, nx=200, ny=40, seed=1, x_dam=50.0,
                      h_left=1.0, h_right=0.5, jitter=0.2) -> Scenario:
    mesh = grid_mesh(Lx, Ly, nx, ny, seed, jitter=jitter)

    def ic(x, y, b):
        h = np.where(x < x_dam, h_left, h_right).astype(np.float64)
        return h, np.zeros_like(h), np.zeros_like(h)

    return _build("dam_break_channel", mesh, _flat_bed, ic, 0.0,
                  {s: BC_WALL for s in range(4)},
                  params=dict(x_dam=x_dam, h_left=h_left, h_right=h_right))


def strip_riemann(L=10.0, W=1.0, nx=200, ny=4, seed=11, x0=5.0, hL=1.0,
                  hR=0.5, uL=0.0, uR=0.0, jitter=0.2,
                  ends=BC_TRANSMISSIVE) -> Scenario:
    """1D Riemann problem on a thin strip: flat bed, walls on the long sides,
    ``ends`` (transmissive by default) at x = 0 and x = L."""
    mesh = grid_mesh(L, W, nx, ny, seed, jitter=jitter)

    def ic(x, y, b):
        left = x < x0
        h = np.where(left, hL, hR).astype(np.float64)
        u = np.where(left, uL, uR).astype(np.float64)
        return h, h * u, np.zeros_like(h)

    tags = {SIDE_LEFT: ends, SIDE_RIGHT: ends, SIDE_BOTTOM: BC_WALL,
            SIDE_TOP: BC_WALL}
    return _build("strip_riemann", mesh, _flat_bed, ic, 0.0, tags,
                  params=dict(x0=x0, hL=hL, hR=hR, uL=uL, uR=uR))


# --------------------------------------------------------------- river cases
def _river_bed(Lx, Ly, rng, n_bumps=40, n_islands=0, bank_height=3.0,
               rise=1.0):
    """Meandering channel: thalweg y_c(x) = Ly/2 + Ly/4 sin(2 pi x /(Lx/4)),
    half-width 0.15 Ly, parabolic cross-section of depth D(x) in [3, 8] m,
    banks rising to ``bank_height`` above the stage, a bed rising ``rise``
    metres from outlet to inlet, Gaussian bumps (sigma 50..300 m scaled with
    Ly/2 km, amplitude +-2 m) and optional emerging islands."""
    W = 0.15 * Ly
    phi = rng.uniform(0.0, 2.0 * math.pi)
    lam_d = Lx / rng.uniform(4.0, 8.0)
    scale = Ly / 2000.0
    slope = rise / Lx

    def yc(x):
        return 0.5 * Ly + 0.25 * Ly * np.sin(2.0 * math.pi * x / (0.25 * Lx))

    def depth(x):
        return 5.5 + 2.5 * np.sin(2.0 * math.pi * x / lam_d + phi)

    bx = rng.uniform(0.0, Lx, n_bumps)
    by = yc(bx) + rng.uniform(-1.0, 1.0, n_bumps) * W
    bs = rng.uniform(50.0, 300.0, n_bumps) * scale
    ba = rng.uniform(-2.0, 2.0, n_bumps)
    ix = rng.uniform(0.1 * Lx, 0.9 * Lx, n_islands)
    iy = yc(ix) + rng.uniform(-0.5, 0.5, n_islands) * W
    isg = rng.uniform(50.0, 300.0, n_islands) * scale
    ia = depth(ix) + slope * (Lx - ix) + rng.uniform(2.5, 4.0, n_islands)
    gx = np.concatenate([bx, ix])
    gy = np.concatenate([by, iy])
    gs = np.concatenate([bs, isg])
    ga = np.concatenate([ba, ia])

    def bed(x, y):
        d = np.abs(y - yc(x))
        D = depth(x)
        inside = d <= W
        b = np.where(inside, -D * (1.0 - (d / W) ** 2),
                     np.minimum(bank_height, bank_height * (d - W) / (0.25 * W)))
        b = b + slope * (Lx - x)
        for k in range(gx.shape[0]):
            win = np.abs(x - gx[k]) < 6.0 * gs[k]
            if not np.any(win):
                continue
            r2 = (x[win] - gx[k]) ** 2 + (y[win] - gy[k]) ** 2
            b[win] += ga[k] * np.exp(-r2 / (2.0 * gs[k] ** 2))
        return b

    return bed


def _lake_ic(stage):
    def ic(x, y, b):
        h = np.maximum(0.0, stage - b)
        return h, np.zeros_like(h), np.zeros_like(h)
    return ic


def river_channel(Lx=10000.0, Ly=2000.0, nx=1582, ny=316, seed=2,
                  n_bumps=40, n_islands=0, inflow_q=500.0, stage=0.0,
                  manning=None, hydrograph=None, name="river_channel") -> Scenario:
    mesh = grid_mesh(Lx, Ly, nx, ny, seed)
    rng = np.random.default_rng([seed, 202])
    bed = _river_bed(Lx, Ly, rng, n_bumps=n_bumps, n_islands=n_islands)
    if manning is None:
        manning = rng.uniform(0.02, 0.05)
    tags = {SIDE_LEFT: BC_INFLOW, SIDE_RIGHT: BC_OUTFLOW,
            SIDE_BOTTOM: BC_WALL, SIDE_TOP: BC_WALL}
    return _build(name, mesh, bed, _lake_ic(stage), manning, tags,
                  inflow_q=inflow_q, outflow_stage=stage,
                  hydrograph=hydrograph,
                  params=dict(seed=seed, Lx=Lx, Ly=Ly, nx=nx, ny=ny))


def lake_at_rest(Lx=1000.0, Ly=200.0, nx=60, ny=12, seed=21, n_bumps=40,
                 n_islands=2, stage=0.0, manning=0.03) -> Scenario:
    """Still water over bumpy bathymetry with dry banks and islands, closed
    by walls: the exact solution is the initial state."""
    mesh = grid_mesh(Lx, Ly, nx, ny, seed)
    rng = np.random.default_rng([seed, 202])
    bed = _river_bed(Lx, Ly, rng, n_bumps=n_bumps, n_islands=n_islands)
    return _build("lake_at_rest", mesh, bed, _lake_ic(stage), manning,
                  {s: BC_WALL for s in range(4)}, params=dict(seed=seed))


def river_dam_break(Lx=40000.0, Ly=8000.0, nx=5702, ny=1140, seed=3,
                    n_bumps=40, n_islands=12, jump=2.0, stage=0.0,
                    inflow_q=500.0, name="river_dam_break") -> Scenario:
    mesh = grid_mesh(Lx, Ly, nx, ny, seed)
    rng = np.random.default_rng([seed, 202])
    bed = _river_bed(Lx, Ly, rng, n_bumps=n_bumps, n_islands=n_islands)
    manning = rng.uniform(0.02, 0.05)

    def ic(x, y, b):
        eta = np.where(x < 0.5 * Lx, stage + jump, stage)
        h = np.maximum(0.0, eta - b)
        return h, np.zeros_like(h), np.zeros_like(h)

    tags = {SIDE_LEFT: BC_INFLOW, SIDE_RIGHT: BC_OUTFLOW,
            SIDE_BOTTOM: BC_WALL, SIDE_TOP: BC_WALL}
    return _build(name, mesh, bed, ic, manning, tags, inflow_q=inflow_q,
                  outflow_stage=stage,
                  params=dict(seed=seed, Lx=Lx, Ly=Ly, nx=nx, ny=ny))


def config1() -> Scenario:
    return dam_break_channel()


def config2(nx=1582, ny=316) -> Scenario:
    return river_channel(nx=nx, ny=ny, seed=2)


def config3(nx=5702, ny=1140) -> Scenario:
    return river_dam_break(nx=nx, ny=ny, seed=3)


def ensemble_member(s, seed_base=5000, min_cells=5.0e4, max_cells=2.0e6, size_scale=1.0):
    """Scenario s of the seeded flood ensemble (its own random stream, so
    any member can be built alone)."""
    seed = seed_base + s
    rng = np.random.default_rng([seed, 303])
    N = math.exp(rng.uniform(math.log(min_cells), math.log(max_cells)))
    N *= size_scale
    ny = max(2, int(round(math.sqrt(N / 10.0))))
    nx = 5 * ny
    q_peak = rng.uniform(100.0, 2000.0)
    t_peak = rng.uniform(30.0, 90.0)
    width = rng.uniform(0.2, 0.9) * t_peak      # rise starts after t = 0
    manning = rng.uniform(0.02, 0.05)
    hyd = (np.array([0.0, t_peak - width, t_peak, t_peak + width, 1.0e9]),
           np.array([100.0, 100.0, q_peak, 100.0, 100.0]))
    sc = river_channel(nx=nx, ny=ny, seed=seed, manning=manning,
                       inflow_q=100.0, hydrograph=hyd,
                       name=f"ensemble_{s:02d}")
    sc.params.update(q_peak=q_peak, t_peak=t_peak, width=width)
    return sc


def ensemble_scenarios(n=64, seed_base=5000, min_cells=5.0e4, max_cells=2.0e6,
                       size_scale=1.0):
    """Seeded flood ensemble on the 10 km x 2 km channel.  ``size_scale``
    shrinks every mesh (for quick tests); 1.0 is the full recipe."""
    return [ensemble_member(s, seed_base, min_cells, max_cells, size_scale) for s in range(n)]
