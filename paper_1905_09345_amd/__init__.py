"""MI355X (gfx950) filtered K-means: point-level and group-level triangle-
inequality filters ahead of MFMA / FP32 distance kernels, behind the C ABI of
include/kp.h.  `kp` is the ctypes binding; `build` compiles libkp.so."""
from . import kp  # noqa: F401
from .kp import KMeans, KPError  # noqa: F401
