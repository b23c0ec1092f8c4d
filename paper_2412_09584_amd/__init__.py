"""MI355X-native CROWN / alpha / beta bound propagation (HIP kernels for gfx950 behind the
C ABI in include/bound.h).  ``binding`` mirrors the C entry points; ``net`` adds a
network handle, the full-CROWN driver, an autograd Function and the Adam loop."""
from . import binding  # noqa: F401
