"""MI355X-native reduced-MBF array solver with the HARP interaction model
(arXiv 1702.03781): HIP kernels for gfx950 behind a C ABI (include/harp.h),
with this thin Python binding.  See ``api`` for the entry points."""
from . import api  # noqa: F401
from .api import (  # noqa: F401
    Model, ModelBatch, harp_fit, pack_model, stack_models, harp_fill, harp_port_rhs,
    harp_port_admittance, reduced_factor, reduced_solve, embedded_patterns, colmajor,
)
