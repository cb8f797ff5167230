"""MI355X-native in situ compressor with time-dependent bases (arXiv 2201.06958).

The compute path lives in libtdb.so (hand-written HIP for gfx950, C ABI in
include/tdb.h); `Compressor` is its thin ctypes binding.
"""
from .tdb import Batch, Compressor, Gate, TDBError, load_library  # noqa: F401
