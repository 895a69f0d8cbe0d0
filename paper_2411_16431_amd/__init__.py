"""MI355X (gfx950) boundary-MPS conditional marginals and branch and bound.

The compute path is libtnbb.so (HIP kernels behind the C ABI in
include/tnbb.h); this package only marshals arguments.  Importing it does
not touch the GPU; the first call that needs the library loads it and fails
loudly if it has not been built.
"""
from .api import (TnbError, energies, Clusters, Env, Beam, EnvOptions, solve, library_path,
                  exported_symbols, profile_enable, profile_query, profile_names, FirstRowLogZ,
                  first_row_layout, diagram_dims, diagram_apply, select_lowest, solve_transformed,
                  autotune, use_torch_allocator, solve_batch)

__all__ = ["TnbError", "energies", "Clusters", "Env", "Beam", "EnvOptions", "solve",
           "library_path", "exported_symbols", "profile_enable", "profile_query", "profile_names",
           "FirstRowLogZ", "first_row_layout", "diagram_dims", "diagram_apply", "select_lowest",
           "solve_transformed", "autotune", "use_torch_allocator", "solve_batch"]
