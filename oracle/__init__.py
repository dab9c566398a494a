"""FP64 CPU oracle for the manifold P-NDF.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it; the library never imports it.  See pndf_oracle.c for the
definitions it follows and oracle.py for the Python entry points.
"""
from .oracle import (build, load, mesh, cluster_level, cluster_all, fine_contrib,
                     evaluate, sample, projected_area, tri_projected, sample_normals, triangle_id, decode_id, num_threads,
                     set_threads)

__all__ = ["build", "load", "mesh", "cluster_level", "cluster_all", "fine_contrib", "sample", "projected_area", "tri_projected",
           "evaluate", "sample_normals", "triangle_id", "decode_id", "num_threads", "set_threads"]
