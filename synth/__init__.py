"""Seeded synthetic sky catalogues shared by the tests, the smoke check and the
benchmark.

This package only draws input data (RA/Dec in degrees and theta bin edges;
flat-sky galaxy positions and ellipticities).
It holds none of the pair-counting or aperture-mass arithmetic: no unit
vectors, no chord lengths, no binning, no filter.  Both the CPU oracle and the
GPU library receive exactly the arrays produced here.
"""

from .catalogs import (  # noqa: F401
    Patch,
    centred_patch,
    pool_random,
    request_catalog,
    FULL_SKY,
    uniform_patch,
    neyman_scott,
    log_edges,
    linear_edges,
    config_small,
    config_1m,
    config_batched,
    config_large,
    serve_stream,
    paper_shape,
)
from .shear import (  # noqa: F401
    APERTURE_CONFIG,
    PAPER_DENSITY,
    shear_catalog,
    field_grid,
    config_aperture,
)
