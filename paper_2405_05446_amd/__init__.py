"""MI355X (gfx950) implementation of the gradient-domain Gaussian splatting
render + Poisson reconstruction path of GDGS (arXiv 2405.05446).

The compute lives in libgdgs.so (hand-written HIP kernels behind the C ABI of
include/gdgs.h); this package marshals torch device tensors into it.
"""
from ._lib import GdgsError, load  # noqa: F401
from . import api  # noqa: F401
from .api import (  # noqa: F401
    DeviceScene, Renderer, alloc_bins, alloc_proj, camera_struct, gdgs_bin_sort,
    gdgs_div_adjoint, gdgs_poisson_solve, gdgs_poisson_solve_rhs, gdgs_project,
    gdgs_project_2d, gdgs_project_backward, gdgs_raster_grad, gdgs_raster_grad_backward,
    gdgs_raster_laplacian, gdgs_raster_laplacian_threshold, gdgs_render, gdgs_render_laplacian,
    gdgs_render_laplacian_sparse, mg_params, new_stats, read_stats,
    render_workspace_size, workspace, FMG, NEUMANN, RESUME, STOP_ETA, WARM_START,
)
from .serve import Server, now_ns  # noqa: F401
