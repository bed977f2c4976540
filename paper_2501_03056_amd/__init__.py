"""MI355X-native particle relaxation of the feature-preserving particle
generation method (arXiv 2501.03056, section 3.3): HIP kernels for gfx950
behind the C ABI of include/fppg.h, with a thin Python binding.
"""
from ._lib import FppgError, lib  # noqa: F401
from .relax import Context, Geometry, Relaxer  # noqa: F401
