"""FP64 CPU oracle of the gradient-domain render + Poisson path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package; only the tests, the smoke check and the benchmark's CPU
baseline leg may use it.  It shares no code with the HIP kernels.

What it computes, following GDGS (arXiv 2405.05446):

* ``project``   -- Sec. 1.2 (3D Gaussian splatting, Eq. 8-10) and Sec. 2.2
  "Projection" (Eq. 19): Sigma = R S S^T R^T, Sigma2D = J W Sigma W^T J^T with
  W the world-to-camera rotation and J the Jacobian of the pinhole map at the
  splat mean.  The Gaussian exponent has no factor 1/2 (Eq. 9 and Eq. 18).
* ``composite`` -- the alpha blend of Eq. 11 applied to the projected field
  (Eq. 20): out = sum_k v_k a_k prod_{j<k} (1 - a_j), a_k = alpha_k G_k, with k
  ordered front to back along the view direction.  Per-pixel brute force.
* ``binning``   -- the tile/depth ordering the rasteriser consumes, as its
  plain definition (pairs of (tile, splat), lexicographically sorted).
* ``poisson``   -- Sec. 2 (Eq. 13-16) and Sec. 2.2 "Poisson Equation"
  (Eq. 21): divergence of the gradient image, then an exact direct solve of
  the discrete Poisson equation (dense LU on tiny grids, DST-I
  diagonalisation on larger ones).
* ``backward``  -- exact gradients of a squared-error loss on the recovered
  image with respect to the rasteriser inputs (the particle-parameter
  gradients of Sec. 1.1, Eq. 5-7, specialised to this pipeline), plus central
  finite differences.

Readings of points the paper leaves open (exponent without 1/2, support
cut-off E_CUT, depth tie-break, pixel centres, Dirichlet ring, finite
difference scheme) are stated in each module.
"""
from .constants import E_CUT, Z_NEAR, TILE  # noqa: F401
from . import project, composite, binning, poisson, backward, render  # noqa: F401
