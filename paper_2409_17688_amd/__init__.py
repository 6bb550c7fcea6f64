"""Exact (min,+) matrix arithmetic on MI355X and the 2-domination number of
cylinders P_n x C_m by tropical matrix powers (arXiv 2409.17688).

The computation lives in libtropical.so (HIP kernels for gfx950 behind the C
ABI of include/tropical.h); ``_lib`` is its ctypes binding.
"""
from ._lib import *  # noqa: F401,F403
from ._lib import EXPORTED, INF, LIB_PATH, TropicalError, lib  # noqa: F401
