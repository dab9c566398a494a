"""MI355X (gfx950) library for batched evaluation of the manifold-based P-NDF.

The compute path is the HIP library libpndf.so (C ABI in include/pndf.h); this
package is its thin Python binding.  Importing it requires the library to be
built (`python -m paper_2505_08985_amd.build`).
"""
from .binding import (Mesh, Hierarchy, PndfError, build_mesh, build_hierarchy, eval_batch, eval_batch_noalloc,
                      sample_batch, projected_area,
                      eval_counts, eval_hits, mesh_info, mesh_export, hier_info, hier_export_level,
                      EXPORTED, LIB_PATH, Plan, default_tuning, autotune, Server)

__all__ = ["Mesh", "Hierarchy", "PndfError", "build_mesh", "build_hierarchy", "eval_batch", "eval_batch_noalloc",
           "sample_batch",
           "projected_area",
           "eval_counts", "eval_hits", "mesh_info", "mesh_export", "hier_info",
           "hier_export_level", "EXPORTED", "LIB_PATH", "Plan", "default_tuning", "autotune", "Server"]
