"""Seeded synthetic inputs for the P-NDF evaluation path.

This package only draws random inputs: height fields, the normal maps derived
from them, and query batches.  It holds none of the method's arithmetic (no
triangles, Jacobians, hierarchy or kernel sums), so both the FP64 oracle and the
GPU library can consume what it produces without sharing code.
"""
from .maps import (normals_from_height, bumps_height, powerlaw_height,
                   scratched_normals, make_map, MAP_KINDS)
from .queries import uniform_queries, tile_request, CONFIGS

__all__ = ["normals_from_height", "bumps_height", "powerlaw_height",
           "scratched_normals", "make_map", "MAP_KINDS", "uniform_queries",
           "tile_request", "CONFIGS"]
