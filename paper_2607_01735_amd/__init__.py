"""MI355X-native red-black Gauss-Seidel for the 5-point 2D Poisson stencil.

The solver lives in librbgs.so (HIP kernels for gfx950 behind the C ABI of
include/rbgs.h); this package is its Python binding.  Importing the package
fails loudly when the library has not been built.
"""
from .rbgs import (  # noqa: F401
    EXPORTED, BatchPlan, RbgsError, make_grid, rbgs_autotune_batched, rbgs_batch_last_error,
    rbgs_batch_workspace_size, rbgs_last_error, rbgs_residual, rbgs_residual_noalloc,
    rbgs_solve, rbgs_stream_probe,
    rbgs_strerror, rbgs_sweep, rbgs_sweep_batched, rbgs_workspace_size, UNet,
    rbgs_unet_param_count, rbgs_restrict, rbgs_prolong, rbgs_solve_batched,
    rbgs_mg_solve, rbgs_mg_workspace_size, rbgs_mc9_workspace_size, rbgs_mc9_sweep,
    rbgs_mc9_residual, rbgs_mc9_solve, rbgs_rb3_workspace_size, rbgs_rb3_sweep,
    rbgs_rb3_residual, rbgs_rb3_solve, make_grid3, rbgs_split_pitch, rbgs_pack, rbgs_unpack,
    rbgs_sweep_split,
)

__all__ = ["rbgs_split_pitch", "rbgs_pack", "rbgs_unpack", "rbgs_sweep_split",
           "rbgs_rb3_workspace_size", "rbgs_rb3_sweep", "rbgs_rb3_residual", "rbgs_rb3_solve",
           "make_grid3", "rbgs_mc9_workspace_size", "rbgs_mc9_sweep", "rbgs_mc9_residual", "rbgs_mc9_solve",
           "rbgs_mg_solve", "rbgs_mg_workspace_size", "rbgs_restrict", "rbgs_prolong", "rbgs_solve_batched", "UNet", "rbgs_unet_param_count", "rbgs_sweep_batched", "BatchPlan", "rbgs_autotune_batched",
           "rbgs_batch_workspace_size", "rbgs_batch_last_error",
           "rbgs_sweep", "rbgs_residual", "rbgs_residual_noalloc", "rbgs_solve",
           "rbgs_workspace_size",
           "rbgs_stream_probe", "rbgs_strerror", "rbgs_last_error", "make_grid", "RbgsError", "EXPORTED"]
