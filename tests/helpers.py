"""Small mesh manipulations used by the tests (no solver arithmetic)."""
from __future__ import annotations

import math

import numpy as np

from swe_inputs.mesh import TriMesh, grid_mesh, SIDE_LEFT, SIDE_RIGHT, SIDE_BOTTOM, SIDE_TOP
from swe_inputs.scenarios import Scenario


def mirror_mesh_x(half: TriMesh, x_mirror: float):
    """Mesh of [x0, 2 x_mirror - x0] made of ``half`` and its mirror image in
    x = x_mirror (the nodes on that line are shared).  Returns (mesh, pair)
    where pair[c] is the mirror cell of c."""
    xy = half.xy
    on = np.isclose(xy[:, 0], x_mirror, rtol=0, atol=1e-9 * max(1.0, abs(x_mirror)))
    n0 = xy.shape[0]
    new_id = np.full(n0, -1, np.int64)
    extra = np.where(~on)[0]
    new_id[extra] = n0 + np.arange(extra.shape[0])
    new_id[on] = np.where(on)[0]
    mxy = xy[extra].copy()
    mxy[:, 0] = 2.0 * x_mirror - mxy[:, 0]
    xy2 = np.concatenate([xy, mxy], 0)
    t = half.tri.astype(np.int64)
    mt = new_id[t][:, [0, 2, 1]]            # reflection flips orientation
    tri = np.concatenate([t, mt], 0).astype(np.int32)
    side = half.edge_side.copy()
    # edges of the mirrored cell: (0->2), (2->1), (1->0) = original edges 2, 1, 0
    ms = half.edge_side[:, [2, 1, 0]].copy()
    ms[ms == SIDE_LEFT] = SIDE_RIGHT
    side = side.copy()
    side[side == SIDE_RIGHT] = -1           # the mirror line is interior
    ms_right = half.edge_side[:, [2, 1, 0]] == SIDE_RIGHT
    ms[ms_right] = -1
    es = np.concatenate([side, ms], 0).astype(np.int8)
    n = half.n_cells
    pair = np.concatenate([np.arange(n) + n, np.arange(n)])
    return TriMesh(xy=xy2, tri=tri, edge_side=es, info=dict(kind="mirror")), pair


def rotate_xy(xy, theta):
    c, s = math.cos(theta), math.sin(theta)
    R = np.array([[c, -s], [s, c]])
    return xy @ R.T


def edge_lengths(mesh: TriMesh):
    p = mesh.xy[mesh.tri]
    q = np.roll(p, -1, axis=1)
    return np.sqrt(((q - p) ** 2).sum(-1))


def areas(mesh: TriMesh):
    p = mesh.xy[mesh.tri]
    return 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                  - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))


def python_neighbors(tri):
    """Dual graph by a dictionary keyed on the sorted node pair."""
    owner = {}
    nbr = -np.ones(tri.shape, np.int64)
    for c in range(tri.shape[0]):
        for m in range(3):
            p, q = int(tri[c, m]), int(tri[c, (m + 1) % 3])
            key = (min(p, q), max(p, q))
            if key in owner:
                d, dm = owner[key]
                nbr[c, m] = d
                nbr[d, dm] = c
            else:
                owner[key] = (c, m)
    return nbr


def one_cell_basin(h=1.0, u=0.4, v=-0.2, b=0.1, n=0.03):
    """A single triangle with walls on its three edges (the smallest mesh the
    method accepts): still water or a uniform current in a closed cell."""
    xy = np.array([[0.0, 0.0], [2.0, 0.3], [0.7, 1.8]])
    tri = np.array([[0, 1, 2]], np.int32)
    mesh = TriMesh(xy=xy, tri=tri, edge_side=np.array([[SIDE_BOTTOM, SIDE_RIGHT, SIDE_LEFT]], np.int8),
                   info=dict(kind="one_cell"))
    return Scenario("one_cell", mesh, np.full((1, 3), -1, np.int8), np.array([b]), np.array([n]),
                    np.array([h]), np.array([h * u]), np.array([h * v]))
