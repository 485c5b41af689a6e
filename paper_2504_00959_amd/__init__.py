"""MI355X (gfx950) w-stacking imager: HIP kernels behind a C ABI.

``rick`` is the Python binding of ``include/rick.h``; ``_build`` compiles
``csrc/`` into ``librick.so``.
"""
from .rick import Plan, RickError, lib, wstack_image  # noqa: F401
