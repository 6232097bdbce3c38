"""Seeded synthetic inputs for the shallow-water finite-volume step.

This module only *describes problems*: node coordinates, triangles, boundary
tags of the domain edges, bed elevation and Manning coefficient per cell,
initial states and boundary-condition parameters.  It performs none of the
finite-volume method's arithmetic (no geometry of the scheme, no fluxes, no
neighbour search, no partitioning).  Both the CPU oracle and the HIP library
read its output; neither of them is imported here.
"""
from .mesh import TriMesh, grid_mesh, refine_red, BC_INTERIOR, BC_WALL, \
    BC_TRANSMISSIVE, BC_INFLOW, BC_OUTFLOW
from .scenarios import (Scenario, dam_break_channel, river_channel,
                        lake_at_rest, strip_riemann, river_dam_break,
                        ensemble_scenarios, config1, config2, config3,
                        refine_scenario)

__all__ = [
    "TriMesh", "grid_mesh", "refine_red", "Scenario", "dam_break_channel",
    "river_channel", "lake_at_rest", "strip_riemann", "river_dam_break",
    "ensemble_scenarios", "config1", "config2", "config3", "refine_scenario",
    "BC_INTERIOR", "BC_WALL", "BC_TRANSMISSIVE", "BC_INFLOW", "BC_OUTFLOW",
]
