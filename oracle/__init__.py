"""FP64 CPU oracle of the local-expansion-move hot path.

Test infrastructure only: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.
"""
from .oracle import Oracle  # noqa: F401
