"""Seeded synthetic inputs shared by the HIP library's tests and the oracle."""
from . import inputs  # noqa: F401
