"""Seeded synthetic inputs shared by the FP64 oracle and the GPU path.

This package only *draws* inputs: random gauge links of the prescribed
construction, staggered phases folded into them, Gaussian sources and random
gauge transformations.  It performs none of the Dslash / solver arithmetic, so
both sides of every parity test start from the same bytes without sharing any
of the computation under test.
"""

from .fields import (  # noqa: F401
    CFG_IDS,
    STREAM_THIN,
    STREAM_FAT,
    STREAM_SRC,
    STREAM_NN_INIT,
    STREAM_NN_PAIRS,
    STREAM_GAUGE_TF,
    CONFIGS,
    volume,
    site_coords,
    site_parity,
    staggered_eta,
    haar_su3,
    su3_near_identity,
    thin_links,
    hisq_links,
    free_links,
    gaussian_source,
    plane_wave,
    random_gauge_transform,
    shifted_ladder,
)
