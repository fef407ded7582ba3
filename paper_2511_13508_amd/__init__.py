"""MI355X-native parallel-tempering Monte Carlo of the smoothed-cubic
random-laser spin glass (Benedetti & Leuzzi, arXiv 2511.13508).

The compute path is librlpt.so (HIP kernels for gfx950 behind a C ABI,
include/rlpt.h); ``rlpt`` is its thin Python binding.
"""
from . import rlpt  # noqa: F401
from .rlpt import Context, Graph, default_config, tau_int  # noqa: F401

__all__ = ["rlpt", "Context", "Graph", "default_config", "tau_int"]
