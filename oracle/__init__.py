"""FP64 CPU oracle of the parquet hot path (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package; the product path never does.
"""
from . import parquet  # noqa: F401
