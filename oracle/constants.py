"""Conventions the paper leaves open, fixed once for the oracle.

E_CUT: a splat contributes G = exp(-E) only where its exponent E <= ln(1e5);
beyond that G is taken as exactly 0 (the paper gives no cut-off; this one
bounds any disagreement at the support edge by alpha * 1e-5 * |v|).
Z_NEAR: splats whose camera-space depth is <= 0.2 are culled.
TILE: the rasteriser's screen tile edge in pixels (ordering only; the result
of the method does not depend on it).
"""
import math

E_CUT = math.log(1e5)
Z_NEAR = 0.2
TILE = 16
