"""MI355X (gfx950) implementation of the data-parallel hot path of Global
Tensor Motion Planning with a straight-line local planner.

The compute lives in ``libgtmp.so`` (HIP kernels behind the C ABI declared in
``include/gtmp.h``); ``paper_2608_25830_amd.gtmp`` is its Python binding.
Importing the binding fails if the library has not been built
(``python -m paper_2608_25830_amd.build``).
"""

__all__ = ["gtmp"]
