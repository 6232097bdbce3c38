"""Problem description -> library mesh, through the library's host toolkit.

Marshalling only: the dual graph, partition, ghost layers, renumbering and
edge lengths are computed by libswe.so's C++ toolkit (include/swe.h).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import swe


@dataclass
class Prepared:
    mesh: swe.MeshArrays
    sub: swe.SubDomain
    nbr_global: np.ndarray
    part: np.ndarray


def prepare(node_xy, cell_nodes, bc, cell_b, cell_manning, inflow_q=0.0, outflow_stage=0.0,
            P: int = 1, p: int = 0, k: int = 0, nbr_global=None, part=None) -> Prepared:
    """Part ``p`` of a ``P``-way greedy partition with ``k`` ghost layers
    (P = 1: the whole mesh in Morton order).  ``bc`` int8 [n, 3] gives the
    boundary tag of each local edge without a neighbour."""
    node_xy = np.ascontiguousarray(node_xy, np.float64)
    cell_nodes = np.ascontiguousarray(cell_nodes, np.int32)
    if nbr_global is None:
        nbr_global = swe.swe_dual_graph(node_xy.shape[0], cell_nodes)
    if part is None:
        part = (swe.swe_partition_bfs(nbr_global, P) if P > 1
                else np.zeros(cell_nodes.shape[0], np.int32))
    sub = swe.swe_subdomain_build(node_xy, cell_nodes, nbr_global, bc, part, P, p, k)
    L_in = swe.swe_edge_length_sum(node_xy, cell_nodes, bc, swe.BC_INFLOW)
    mesh = swe.mesh_from_subdomain(node_xy, cell_nodes, cell_b, cell_manning, sub,
                                   inflow_q=inflow_q, inflow_length=L_in,
                                   outflow_stage=outflow_stage)
    return Prepared(mesh=mesh, sub=sub, nbr_global=nbr_global, part=part)


def prepare_scenario(sc, P: int = 1, p: int = 0, k: int = 0, nbr_global=None, part=None):
    """Same for an object with ``mesh.xy``, ``mesh.tri``, ``bc``, ``b``,
    ``manning``, ``inflow_q`` and ``outflow_stage`` attributes."""
    return prepare(sc.mesh.xy, sc.mesh.tri, sc.bc, sc.b, sc.manning, sc.inflow_q,
                   sc.outflow_stage, P=P, p=p, k=k, nbr_global=nbr_global, part=part)


def prepare_parts(sc, P: int, k: int, nbr_global=None, part=None, threads: int = 0) -> list:
    """All ``P`` parts of a scenario with ``k`` ghost layers, the ghost layers
    and numbering of every part built on ``threads`` host threads; part q
    equals ``prepare_scenario(sc, P, q, k)``."""
    node_xy = np.ascontiguousarray(sc.mesh.xy, np.float64)
    cell_nodes = np.ascontiguousarray(sc.mesh.tri, np.int32)
    if nbr_global is None:
        nbr_global = swe.swe_dual_graph(node_xy.shape[0], cell_nodes)
    if part is None:
        part = swe.swe_partition_bfs(nbr_global, P)
    subs = swe.swe_subdomain_build_all(node_xy, cell_nodes, nbr_global, sc.bc, part, P, k, threads)
    L_in = swe.swe_edge_length_sum(node_xy, cell_nodes, sc.bc, swe.BC_INFLOW)
    return [Prepared(mesh=swe.mesh_from_subdomain(node_xy, cell_nodes, sc.b, sc.manning, sub,
                                                  inflow_q=sc.inflow_q, inflow_length=L_in,
                                                  outflow_stage=sc.outflow_stage),
                     sub=sub, nbr_global=nbr_global, part=part) for sub in subs]
