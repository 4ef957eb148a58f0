"""Plain double-precision reference of the EOS-based pseudo-potential LB step with geometric wetting.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the benchmark's CPU-baseline leg, never
by the GPU library or its Python binding.
"""
from .oracle import *  # noqa: F401,F403
from .measure import measure_contact_angle  # noqa: F401
