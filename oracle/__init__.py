"""Plain serial FP64 CPU oracle of the projected-Jacobian Krylov path.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library's product path.
"""
from . import disc, solvers  # noqa: F401
