"""FP64 CPU oracle of t-FDP (TEST INFRASTRUCTURE ONLY).

Imported only by the tests, the smoke check and the CPU-baseline leg of the
benchmark. The GPU library never imports or calls anything here, and nothing
here calls the GPU library.
"""
from . import metrics, tfdp  # noqa: F401
