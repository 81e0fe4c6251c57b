"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

Holds input construction only; none of the path tracker's arithmetic."""
from .systems import *  # noqa: F401,F403
