"""Seeded synthetic inputs (meshes, states, boundary data) shared by the GPU
library's tests and benchmark and by the CPU oracle.  Holds no part of the
solver's arithmetic."""
from . import flow, mesh, problems, rng  # noqa: F401
