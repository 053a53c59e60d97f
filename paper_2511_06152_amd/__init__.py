"""MI355X (gfx950) cluster bundle adjustment: HIP kernels behind a C ABI
(include/ba.h, libba.so) and its ctypes binding."""
from .ba import (BA_FP64, BA_MIXED, BAError, Cluster, Context, Geo, load)  # noqa: F401
