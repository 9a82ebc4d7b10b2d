"""FP64 CPU oracle for the SCALE-TRACK per-particle time step.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg; the product package never imports it.
"""
from .oracle import Oracle, MeshParams, load  # noqa: F401
