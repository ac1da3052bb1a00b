"""CPU oracle for the luminaire emission query and its learned surrogate.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library.  It shares no code
with the GPU path; both read the same seeded inputs from the `inputs` package.
"""
from . import core, exact  # noqa: F401
