"""Seeded triangle meshes: jittered structured grids split along random
diagonals, and red (1 -> 4) refinement of such meshes.

Conventions shared by every consumer of these meshes:

* ``xy``   float64 [n_nodes, 2]  node coordinates.
* ``tri``  int32   [n_cells, 3]  node ids, counter-clockwise.  Local edge
  ``m`` of a triangle joins ``tri[c, m]`` and ``tri[c, (m + 1) % 3]``.
* ``edge_side`` int8 [n_cells, 3]: ``-1`` if the local edge is inside the
  domain, else the side of the rectangle it lies on (0 left, 1 right,
  2 bottom, 3 top).  Scenarios turn sides into boundary-condition tags.
* The global id of a cell is its row index in ``tri``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Boundary-condition tags used for the local edges of a cell (0 = interior).
BC_INTERIOR = 0
BC_WALL = -1
BC_TRANSMISSIVE = -2
BC_INFLOW = -3
BC_OUTFLOW = -4

SIDE_NONE, SIDE_LEFT, SIDE_RIGHT, SIDE_BOTTOM, SIDE_TOP = -1, 0, 1, 2, 3


@dataclass
class TriMesh:
    xy: np.ndarray          # float64 [n_nodes, 2]
    tri: np.ndarray         # int32 [n_cells, 3]
    edge_side: np.ndarray   # int8 [n_cells, 3]
    info: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_cells(self) -> int:
        return int(self.tri.shape[0])

    def centroids(self) -> np.ndarray:
        """Point at which cell data (bed, initial state) is sampled."""
        p = self.xy[self.tri]                       # [n, 3, 2]
        return ((p[:, 0] + p[:, 1]) + p[:, 2]) / 3.0


def grid_mesh(Lx: float, Ly: float, nx: int, ny: int, seed: int,
              jitter: float = 0.2, x0: float = 0.0, y0: float = 0.0) -> TriMesh:
    """nx*ny quads over [x0, x0+Lx] x [y0, y0+Ly], 2*nx*ny triangles.

    Interior nodes move uniformly in +-jitter*dx and +-jitter*dy; boundary
    nodes move only along their side; the four corners stay fixed.  Each quad
    is split along one of its diagonals, chosen by a seeded fair coin.
    Draw order (x jitter, y jitter, diagonals) is part of the recipe.
    """
    rng = np.random.default_rng([seed, 101])
    dx, dy = Lx / nx, Ly / ny
    I, J = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="xy")
    jx = rng.uniform(-jitter, jitter, size=I.shape) * dx
    jy = rng.uniform(-jitter, jitter, size=I.shape) * dy
    diag = rng.integers(0, 2, size=(ny, nx))
    on_lr = (I == 0) | (I == nx)
    on_bt = (J == 0) | (J == ny)
    jx[on_lr] = 0.0
    jy[on_bt] = 0.0
    x = x0 + I * dx + jx
    y = y0 + J * dy + jy
    xy = np.stack([x.ravel(), y.ravel()], axis=1).astype(np.float64)

    qi, qj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    a = (qj * (nx + 1) + qi).ravel()
    b = a + 1
    c = a + (nx + 1) + 1
    d = a + (nx + 1)
    dg = diag.ravel()
    t0 = np.where(dg[:, None] == 0, np.stack([a, b, c], 1), np.stack([a, b, d], 1))
    t1 = np.where(dg[:, None] == 0, np.stack([a, c, d], 1), np.stack([b, c, d], 1))
    tri = np.empty((2 * nx * ny, 3), dtype=np.int32)
    tri[0::2] = t0
    tri[1::2] = t1

    ni = np.arange((nx + 1) * (ny + 1)) % (nx + 1)
    nj = np.arange((nx + 1) * (ny + 1)) // (nx + 1)
    p = tri
    q = np.roll(tri, -1, axis=1)
    side = np.full(tri.shape, SIDE_NONE, dtype=np.int8)
    side[(ni[p] == 0) & (ni[q] == 0)] = SIDE_LEFT
    side[(ni[p] == nx) & (ni[q] == nx)] = SIDE_RIGHT
    side[(nj[p] == 0) & (nj[q] == 0)] = SIDE_BOTTOM
    side[(nj[p] == ny) & (nj[q] == ny)] = SIDE_TOP
    info = dict(kind="grid", Lx=Lx, Ly=Ly, nx=nx, ny=ny, seed=seed,
                jitter=jitter, x0=x0, y0=y0)
    return TriMesh(xy=xy, tri=tri, edge_side=side, info=info)


def refine_red(mesh: TriMesh) -> TriMesh:
    """Red refinement: every triangle -> 4 through its edge midpoints.

    Children of parent ``c`` have global ids ``4c + k``: k = 0, 1, 2 is the
    corner child at parent node k, k = 3 the central child.  Children keep
    the counter-clockwise orientation; child edges lying on a parent edge
    inherit that edge's side.
    """
    n = mesh.n_cells
    tri = mesh.tri.astype(np.int64)
    p = tri
    q = np.roll(tri, -1, axis=1)
    lo = np.minimum(p, q)
    hi = np.maximum(p, q)
    key = lo * np.int64(mesh.n_nodes) + hi            # [n, 3]
    uniq, inv = np.unique(key.ravel(), return_inverse=True)
    inv = inv.reshape(n, 3)
    ulo = uniq // mesh.n_nodes
    uhi = uniq % mesh.n_nodes
    mid = 0.5 * (mesh.xy[ulo] + mesh.xy[uhi])
    xy = np.concatenate([mesh.xy, mid], axis=0)
    m = inv + mesh.n_nodes                             # midpoint node of local edge k
    p0, p1, p2 = tri[:, 0], tri[:, 1], tri[:, 2]
    m01, m12, m20 = m[:, 0], m[:, 1], m[:, 2]
    ch = np.empty((n, 4, 3), dtype=np.int64)
    ch[:, 0] = np.stack([p0, m01, m20], 1)
    ch[:, 1] = np.stack([m01, p1, m12], 1)
    ch[:, 2] = np.stack([m20, m12, p2], 1)
    ch[:, 3] = np.stack([m01, m12, m20], 1)
    s = mesh.edge_side
    cs = np.full((n, 4, 3), SIDE_NONE, dtype=np.int8)
    cs[:, 0, 0] = s[:, 0]
    cs[:, 0, 2] = s[:, 2]
    cs[:, 1, 0] = s[:, 0]
    cs[:, 1, 1] = s[:, 1]
    cs[:, 2, 1] = s[:, 1]
    cs[:, 2, 2] = s[:, 2]
    info = dict(mesh.info)
    info["refined"] = info.get("refined", 0) + 1
    return TriMesh(xy=xy, tri=ch.reshape(4 * n, 3).astype(np.int32),
                   edge_side=cs.reshape(4 * n, 3), info=info)
