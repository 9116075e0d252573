"""MI355X-native tensorial template matching (TTM) engine.

The compute lives in libttm.so (hand-written HIP for gfx950, C ABI in
include/ttm.h); ``paper_2408_02398_amd.ttm`` marshals torch device tensors to
it.  Importing this package does not load the library; the first call does,
and raises if it has not been built.
"""
__all__ = ["ttm", "build"]
