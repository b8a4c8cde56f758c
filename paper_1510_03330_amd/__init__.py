"""MI355X-native parquet hot path: HIP kernels for gfx950 behind a C ABI.

``native`` is the ctypes binding of ``include/parquet.h``; ``ops`` has the
torch-facing stage wrappers and the ``Solver`` context. Nothing here falls
back to the CPU: the built ``_lib/libparquet.so`` is required.
"""
from . import native  # noqa: F401

__all__ = ["native", "ops", "build"]
