"""MI355X (gfx950) tangent-space normal baking: HIP kernels behind a C ABI.

The product is ``libbake.so`` (sources in ``csrc/``, ABI in ``include/bake.h``);
``bake`` is its thin Python binding.
"""
from . import bake  # noqa: F401
from .bake import bake_normals, BakeError  # noqa: F401
