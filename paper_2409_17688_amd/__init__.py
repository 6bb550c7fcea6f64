"""Exact (min,+) matrix arithmetic on MI355X and the 2-domination number of
cylinders P_n x C_m by tropical matrix powers (arXiv 2409.17688).

The computation lives in libtropical.so (HIP kernels for gfx950 behind the C
ABI of include/tropical.h); ``_lib`` is its ctypes binding.  On import the
package loads its tuning table (kernel shapes measured by ``autotune``,
loaded by ``tuning``):
TP_TUNING=0 keeps the library's built-in defaults, TP_TUNING_FILE names
another table.
"""
import os as _os

from ._lib import *  # noqa: F401,F403
from ._lib import EXPORTED, INF, LIB_PATH, TropicalError, lib  # noqa: F401
from .tuning import apply_tuning  # noqa: F401

TUNED = False
if _os.environ.get("TP_TUNING", "1") != "0":
    TUNED = apply_tuning(_os.environ.get("TP_TUNING_FILE"))
