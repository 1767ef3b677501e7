"""MI355X (gfx950) PST pose search against a TSDF -- ROSEFusion's hot path.

The compute lives in librose.so (HIP kernels behind the C ABI of
include/rose.h); ``paper_2105_05600_amd.rose`` is the thin Python binding.
Build with ``python -m paper_2105_05600_amd.build``.
"""

__all__ = ["rose"]
