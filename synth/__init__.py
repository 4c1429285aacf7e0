"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This package holds only input generation: grid sizes, boundary-condition and
load *descriptions* given as node coordinates (i, j, k) and a component, and
density fields drawn from seeded generators.  It contains none of the
method's arithmetic (no stiffness, no filter, no solver) and flattens nothing
into either side's memory layout: each side turns these descriptions into its
own vectors.
"""

from .problems import (  # noqa: F401
    Problem,
    cantilever,
    bridge,
    patch_test,
    point_loads_on_face,
    Problem2D,
    cantilever2d,
    half_wheel,
    inverter2d,
    batch_sizes,
    serve_trace,
    PRESETS,
)
from .fields import (  # noqa: F401
    uniform_iid, smoothed_field, thresholded_field, perturb, smooth_perturb)
