"""MI355X-native exact event-based divergence estimation (arXiv 2209.13168).

The estimator runs in ``libecmd.so`` (hand-written HIP for gfx950, C ABI in
``include/ecmd.h``); ``paper_2209_13168_amd.ecmd`` is its ctypes binding.
"""

__all__ = ["ecmd"]
