"""Seeded synthetic inputs shared by the GPU path's tests/bench and the FP64 oracle.

This package only *draws* inputs: spectral cubes, cameras, colour look-up tables and
transfer-function control points.  It holds none of the rendering, filtering or
line-ratio arithmetic of the method; both sides receive the arrays built here.

Stand-ins: the paper's cubes (THINGS NGC 2903, ALMA Antennae CO(3-2), SAMI
GAMA-511867 H-alpha/[NII], Section 5.2) are not available, so every workload is a
seeded synthetic cube with the same kind of content (noise-dominated HI-like cubes with
rotating discs, NaN-masked mosaics, two-line IFU pairs, uniform [0,1] benchmark cubes
as in Appendix B).
"""
from .cubes import (  # noqa: F401
    blob_cube, disc_cube, add_disc, uniform_cube, nan_mosaic_cube, two_line_pair,
    two_line_pair_512x512x32,
    subcube_batch_specs, subcube, blob_cube_64, hi_cube_512x512x1024, disc_cube_256, gradcheck_cube,
    smooth_analytic_cube,
)
from .cameras import (  # noqa: F401
    Camera, ortho_axis, perspective_lookat, perspective_direction, rotation_views,
)
from .tables import lut_ramp, lut_heat, tf_ramp, tf_bumps  # noqa: F401
